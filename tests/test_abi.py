"""The C-ABI library loads, exports every symbol include/kmc.h declares, and
its structs have the layout the Python binding assumes.  CPU only: nothing
here launches a kernel."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "kmc.h")


@pytest.fixture(scope="module")
def kmc():
    from paper_1407_1507_amd import kmc as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1407_1507_amd import build
        build.build()
    m.lib()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports(kmc):
    assert declared_functions() == sorted(kmc.EXPORTS)


def test_library_exports_every_declared_symbol(kmc):
    out = subprocess.check_output(["nm", "-D", "--defined-only", kmc.LIB_PATH], text=True)
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in syms, name
        assert hasattr(kmc.lib(), name)


def test_struct_layout_matches_header(kmc, tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "kmc.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(kmc_reads), sizeof(kmc_params), sizeof(kmc_stats), sizeof(kmc_table));
  printf("%zu %zu %zu %zu\\n", offsetof(kmc_table, keys), offsetof(kmc_table, bin_offsets),
         offsetof(kmc_table, on_device), offsetof(kmc_table, stats));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    lines = subprocess.check_output([str(exe)], text=True).split("\n")
    sizes = [int(x) for x in lines[0].split()]
    offs = [int(x) for x in lines[1].split()]
    assert sizes == [ctypes.sizeof(kmc.Reads), ctypes.sizeof(kmc.Params),
                     ctypes.sizeof(kmc.Stats), ctypes.sizeof(kmc.Table)]
    assert offs == [kmc.Table.keys.offset, kmc.Table.bin_offsets.offset,
                    kmc.Table.on_device.offset, kmc.Table.stats.offset]


def test_status_strings(kmc):
    L = kmc.lib()
    assert L.kmc_status_str(0) == b"ok"
    assert L.kmc_status_str(1) == b"invalid argument"
    assert L.kmc_status_str(4) == b"job too large"


@pytest.mark.parametrize("k,p,n_bins,ci,cx", [
    (3, 4, 16, 1, 5),        # k < 4
    (65, 7, 16, 1, 5),       # k > 64
    (28, 3, 16, 1, 5),       # p < 4
    (28, 13, 16, 1, 5),      # p > 12
    (8, 9, 16, 1, 5),        # p > k
    (28, 4, 258, 1, 5),      # n_bins > 4^p + 1
    (28, 7, 0, 1, 5),        # n_bins = 0
    (28, 7, 16, 6, 5),       # cutoff_min > cutoff_max
])
def test_invalid_arguments_rejected_before_device_work(kmc, k, p, n_bins, ci, cx):
    seq = np.frombuffer(b"ACGTACGTACGTACGTACGTACGTACGTACGTACGT", dtype=np.uint8).copy()
    off = np.array([0, seq.size], dtype=np.uint64)
    reads, keep = kmc.make_reads(seq, off)
    out = ctypes.POINTER(kmc.Table)()
    st = kmc.lib().kmc_count(ctypes.byref(reads), k, p, n_bins, ci, cx, ctypes.byref(out))
    assert st == kmc.KMC_ERR_INVALID_ARG
    assert not out


@pytest.mark.parametrize("off", [[1, 36], [0, 20, 10, 36], [0, 35]])
def test_malformed_offsets_rejected(kmc, off):
    seq = np.frombuffer(b"ACGTACGTACGTACGTACGTACGTACGTACGTACGT", dtype=np.uint8).copy()
    reads, keep = kmc.make_reads(seq, np.array(off, dtype=np.uint64))
    out = ctypes.POINTER(kmc.Table)()
    st = kmc.lib().kmc_count(ctypes.byref(reads), 28, 7, 16, 1, 5, ctypes.byref(out))
    assert st == kmc.KMC_ERR_INVALID_ARG
