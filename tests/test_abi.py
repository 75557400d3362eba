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
  printf("%zu %zu %zu %zu %zu\\n", sizeof(kmc_job), offsetof(kmc_job, params),
         sizeof(kmc_server_cfg), sizeof(kmc_server_stats), offsetof(kmc_server_stats, active));
  printf("%zu %zu\\n", offsetof(kmc_stats, us_kernel), offsetof(kmc_stats, us_latency));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(kmc_knobs), sizeof(kmc_tune_class),
         sizeof(kmc_tune_report), offsetof(kmc_tune_class, us), sizeof(kmc_db_info));
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
    assert [int(x) for x in lines[2].split()] == [
        ctypes.sizeof(kmc.Job), kmc.Job.params.offset, ctypes.sizeof(kmc.ServerCfg),
        ctypes.sizeof(kmc.ServerStats), kmc.ServerStats.active.offset]
    assert [int(x) for x in lines[3].split()] == [kmc.Stats.us_kernel.offset,
                                                  kmc.Stats.us_latency.offset]
    assert [int(x) for x in lines[4].split()] == [
        ctypes.sizeof(kmc.Knobs), ctypes.sizeof(kmc.TuneClass), ctypes.sizeof(kmc.TuneReport),
        kmc.TuneClass.us.offset, ctypes.sizeof(kmc.DbInfo)]


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


def _ws(kmc, n_reads, length, k, p=7, n_bins=512, ci=1, cx=10, flags=0):
    seq = np.full(n_reads * length, ord("A"), dtype=np.uint8)
    off = np.arange(n_reads + 1, dtype=np.uint64) * length
    reads, keep = kmc.make_reads(seq, off)
    params = kmc.Params(k, p, n_bins, ci, cx, flags)
    out = ctypes.c_size_t(0)
    st = kmc.lib().kmc_workspace_size(ctypes.byref(reads), ctypes.byref(params), ctypes.byref(out))
    return st, out.value


def test_workspace_size_is_host_only_and_bounded(kmc):
    # computed from the sizes alone (no device here): grows with the input,
    # about 2x for 2-word keys, and rejects what kmc_count rejects
    st, small = _ws(kmc, 100, 100, 28)
    assert st == kmc.KMC_OK and small > 0
    st, big = _ws(kmc, 10_000, 100, 28)
    assert st == kmc.KMC_OK and big > small
    n = 10_000 * 100
    assert 16 * n < big < 40 * n
    st, big2 = _ws(kmc, 10_000, 100, 55, p=9, n_bins=1024)
    assert st == kmc.KMC_OK and big2 > 1.5 * big
    assert _ws(kmc, 10, 100, 28, ci=11, cx=10)[0] == kmc.KMC_ERR_INVALID_ARG
    assert _ws(kmc, 10, 100, 3, p=4)[0] == kmc.KMC_ERR_INVALID_ARG
    st, empty = _ws(kmc, 0, 100, 28)
    assert st == kmc.KMC_OK and 0 < empty < small
    # ascending order adds a scratch copy of the table beside it in the
    # records' region (24 instead of 16 bytes per window for 1-word keys)
    st, asc = _ws(kmc, 10_000, 100, 28, flags=kmc.FLAG_ASCENDING)
    assert st == kmc.KMC_OK and big + 4 * n < asc < big + 12 * n


def test_batch_and_server_reject_null_handles(kmc):
    L = kmc.lib()
    outs = (ctypes.POINTER(kmc.Table) * 1)()
    job = kmc.Job()
    assert L.kmc_batch_count(None, ctypes.byref(job), 1, outs) == kmc.KMC_ERR_INVALID_ARG
    srv = ctypes.c_void_p()
    assert L.kmc_server_start(None, None, ctypes.byref(srv)) == kmc.KMC_ERR_INVALID_ARG
    assert not srv
    t = ctypes.c_uint64(0)
    assert L.kmc_server_submit(None, ctypes.byref(job), ctypes.byref(t)) == kmc.KMC_ERR_INVALID_ARG
    out = ctypes.POINTER(kmc.Table)()
    assert L.kmc_server_poll(None, 1, 0, ctypes.byref(out)) == kmc.KMC_ERR_INVALID_ARG
    L.kmc_server_stop(None)
