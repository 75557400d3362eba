"""GPU parity of the table in global ascending key order (KMC_FLAG_ASCENDING):
the table equals the oracle's, which lists its entries in ascending key order,
entry for entry and without re-sorting.  Covers both key widths, the segment
groups ordered in LDS, groups above the LDS capacity (one segment of many
keys that share their leading bits: merge rounds through HBM, an odd and an
even number of rounds), device tables and the caller's workspace."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1407_1507_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kmc():
    from paper_1407_1507_amd import kmc as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(kmc):
    c = kmc.Context(0)
    yield c
    c.close()


def to_reads(strs):
    seq = np.frombuffer("".join(strs).encode(), dtype=np.uint8).copy()
    off = np.zeros(len(strs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in strs])
    return seq, off


def exact(res, seq, off, k, ci, cx):
    ok_keys, ok_counts = oracle.count(seq, off, k, ci, cx)
    keys = res.keys
    assert res.n == len(ok_counts)
    assert res.bin_offsets is None
    assert np.array_equal(keys, ok_keys)
    assert np.array_equal(res.counts, ok_counts)


@pytest.mark.parametrize("k,p,nb", [(28, 7, 512), (55, 9, 1024), (15, 5, 64), (32, 8, 256),
                                    (33, 9, 256)])
def test_random_reads(ctx, kmc, k, p, nb):
    rng = np.random.default_rng(k)
    n = 3000
    lens = rng.integers(k - 3, 180, size=n)
    seq = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), size=int(lens.sum()))
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens)
    res = ctx.count(seq, off, k, p, nb, 1, 2**32 - 1, flags=kmc.FLAG_ASCENDING)
    exact(res, seq, off, k, 1, 2**32 - 1)


@pytest.mark.parametrize("name,scale", [("genome-5M-2Mx100", 0.02),
                                        ("repeats-50M-30x150-k55", 0.004)])
def test_workloads(ctx, kmc, name, scale):
    seq, off, p = synth.make(name, scale)
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                    flags=kmc.FLAG_ASCENDING)
    exact(res, seq, off, p["k"], p["cutoff_min"], p["cutoff_max"])
    # the same entries as the bin-major table
    bm = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    assert bm.n == res.n and int(bm.counts.sum()) == int(res.counts.sum())


@pytest.mark.parametrize("k,p,lead,n", [(28, 7, 10, 6000), (28, 7, 10, 10000),
                                        (55, 9, 30, 3000), (55, 9, 30, 5000)])
def test_groups_above_lds(ctx, kmc, k, p, lead, n):
    # n distinct k-mers that all start with `lead` A's (their canonical form
    # is the forward one): one segment far above the LDS group size, beside
    # ordinary random reads
    rng = np.random.default_rng(n + k)
    acgt = np.array(list("ACGT"))
    strs = ["A" * lead + "".join(rng.choice(acgt, size=k - lead)) for _ in range(n)]
    strs += ["".join(rng.choice(acgt, size=120)) for _ in range(500)]
    seq, off = to_reads(strs)
    res = ctx.count(seq, off, k, p, 64, 1, 2**32 - 1, flags=kmc.FLAG_ASCENDING)
    exact(res, seq, off, k, 1, 2**32 - 1)


def test_empty_and_tiny(ctx, kmc):
    for strs in ([], ["ACG"], ["ACGTACGTACGTACGTACGTACGTACGTAC"]):
        seq, off = to_reads(strs) if strs else (np.zeros(0, np.uint8), np.zeros(1, np.uint64))
        res = ctx.count(seq, off, 28, 7, 16, 1, 2**32 - 1, flags=kmc.FLAG_ASCENDING)
        exact(res, seq, off, 28, 1, 2**32 - 1)


def test_device_table_and_workspace(ctx, kmc):
    import torch
    seq, off, p = synth.make("genome-5M-2Mx100", 0.01)
    args = (p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    host = ctx.count(seq, off, *args, flags=kmc.FLAG_ASCENDING)
    exact(host, seq, off, p["k"], p["cutoff_min"], p["cutoff_max"])
    t = ctx.count(seq, off, *args, flags=kmc.FLAG_ASCENDING | kmc.FLAG_DEVICE_TABLE)
    assert t.on_device and t.n == host.n
    hip = ctypes.CDLL("libamdhip64.so")
    k = np.zeros(t.n, dtype=np.uint64)
    c = np.zeros(t.n, dtype=np.uint32)
    assert hip.hipMemcpy(ctypes.c_void_p(k.ctypes.data), ctypes.c_void_p(t.keys_ptr),
                         ctypes.c_size_t(k.nbytes), 2) == 0
    assert hip.hipMemcpy(ctypes.c_void_p(c.ctypes.data), ctypes.c_void_p(t.counts_ptr),
                         ctypes.c_size_t(c.nbytes), 2) == 0
    t.free()
    assert np.array_equal(k, host.keys) and np.array_equal(c, host.counts)
    need = ctx.workspace_size(seq, off, *args, flags=kmc.FLAG_ASCENDING)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    got = ctx.count_ws(seq, off, *args, workspace=ws, flags=kmc.FLAG_ASCENDING)
    assert np.array_equal(got.keys, host.keys) and np.array_equal(got.counts, host.counts)
