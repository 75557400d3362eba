"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (reads resident on the device, table left on the
device and copied back here).

- genome-5M-2Mx100 (2M reads x 100 bp, k = 28): the whole table equals the
  oracle's, entry for entry.
- repeats-50M-30x150-k55 (10M reads x 150 bp, k = 55): the whole table equals
  the oracle's, entry for entry (the oracle enumerates and sorts on 16 host
  threads).
- large-300M-60Mx150 (the served form's large job, 60M reads x 150 bp, 9
  Gbases, k = 28, 2048 bins): exact at 2% scale (same generator and
  parameters); at full size (7.2e9 k-mers, beyond a whole oracle count in a
  test's memory) every entry of one sixteenth of the key space equals the
  oracle's count of that key range, entry for entry, and properties that
  hold at any size cover the rest: the number of k-mers equals the closed
  form; sampled windows of the input are in the table exactly when their
  oracle count passes the cutoffs; sampled keys sit in the bin of their
  signature; bins are disjoint and ascending.
- the batched workload (256 uneven jobs, 10.3 Gbases): every table of one
  kmc_batch_count equals the same job's table counted alone.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_1407_1507_amd import synth

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


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


def run_like_bench(ctx, kmc, seq, off, p):
    """Device reads, device table (as bench.py), then the table copied back."""
    import torch
    dseq = torch.from_numpy(seq).to("cuda:0")
    doff = torch.from_numpy(off.view(np.int64)).to("cuda:0")
    t = ctx.count(dseq, doff, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                  flags=kmc.FLAG_DEVICE_TABLE)
    kw = t.key_words
    keys = np.zeros(t.n * kw, dtype=np.uint64)
    counts = np.zeros(t.n, dtype=np.uint32)
    hip = ctypes.CDLL("libamdhip64.so")
    if t.n:
        assert hip.hipMemcpy(ctypes.c_void_p(keys.ctypes.data), ctypes.c_void_p(t.keys_ptr),
                             ctypes.c_size_t(keys.nbytes), 2) == 0
        assert hip.hipMemcpy(ctypes.c_void_p(counts.ctypes.data), ctypes.c_void_p(t.counts_ptr),
                             ctypes.c_size_t(counts.nbytes), 2) == 0
    stats, bo, s2b = t.stats, t.bin_offsets, t.sig_to_bin
    t.free()
    del dseq, doff
    torch.cuda.empty_cache()
    return (keys.reshape(-1, 2) if kw == 2 else keys), counts, bo, s2b, stats


def check_bins(keys, bo, n):
    assert bo[0] == 0 and bo[-1] == n and np.all(bo[1:] >= bo[:-1])
    for b in range(len(bo) - 1):
        seg = keys[bo[b]:bo[b + 1]]
        if len(seg) > 1:
            if seg.ndim == 2:
                assert np.all((seg[1:, 0] > seg[:-1, 0]) |
                              ((seg[1:, 0] == seg[:-1, 0]) & (seg[1:, 1] > seg[:-1, 1])))
            else:
                assert np.all(seg[1:] > seg[:-1])


def ascending(keys):
    return np.lexsort((keys[:, 1], keys[:, 0])) if keys.ndim == 2 else np.argsort(keys)


@pytest.mark.timeout(600)
def test_genome_full_size_exact(ctx, kmc):
    seq, off, p = synth.make("genome-5M-2Mx100")
    keys, counts, bo, s2b, st = run_like_bench(ctx, kmc, seq, off, p)
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"],
                                      threads=THREADS)
    order = ascending(keys)
    assert len(counts) == len(ok_counts)
    assert np.array_equal(keys[order], ok_keys)
    assert np.array_equal(counts[order], ok_counts)
    check_bins(keys, bo, len(counts))
    assert st["n_kmers"] == oracle.valid_windows(seq, off, p["k"])
    # every entry in the bin of its signature (a sample of the 6M entries)
    rng = np.random.default_rng(7)
    idx = rng.choice(len(counts), 20000, replace=False)
    bin_of = np.searchsorted(bo, idx, side="right") - 1
    sig = oracle.key_signatures(keys[idx], p["k"], p["p"])
    assert np.array_equal(s2b[sig], bin_of)


def window_keys(seq, off, k, rng, n):
    """Canonical keys of n random valid windows (Python integers -> words)."""
    out = []
    code = {65: 0, 67: 1, 71: 2, 84: 3, 97: 0, 99: 1, 103: 2, 116: 3}
    n_reads = off.size - 1
    while len(out) < n:
        r = int(rng.integers(0, n_reads))
        a, b = int(off[r]), int(off[r + 1])
        if b - a < k:
            continue
        j = int(rng.integers(a, b - k + 1))
        w = seq[j:j + k]
        if not all(int(x) in code for x in w):
            continue
        f = 0
        rc = 0
        for t, x in enumerate(w):
            c = code[int(x)]
            f = f * 4 + c
            rc += (3 - c) << (2 * t)
        out.append(min(f, rc))
    if k <= 32:
        return np.array(out, dtype=np.uint64)
    return np.array([[v >> 64, v & (2**64 - 1)] for v in out], dtype=np.uint64)


def member(table_keys, order, q):
    """Index of each query key in the table (or -1)."""
    s = table_keys[order]
    if s.ndim == 1:
        pos = np.minimum(np.searchsorted(s, q), len(s) - 1)
        return np.where(s[pos] == q, order[pos], -1)
    hi, lo = np.ascontiguousarray(s[:, 0]), np.ascontiguousarray(s[:, 1])
    a = np.searchsorted(hi, q[:, 0], side="left")
    b = np.searchsorted(hi, q[:, 0], side="right")
    res = np.full(len(q), -1, dtype=np.int64)
    for i in range(len(q)):
        j = a[i] + int(np.searchsorted(lo[a[i]:b[i]], q[i, 1]))
        if j < b[i] and lo[j] == q[i, 1]:
            res[i] = order[j]
    return res


@pytest.mark.timeout(1200)
def test_repeats_k55_full_size_exact(ctx, kmc):
    step = lambda m: print(f"[repeats k=55] {m}", flush=True)  # progress of a long test
    seq, off, p = synth.make("repeats-50M-30x150-k55")
    step(f"generated {seq.size} bases")
    k, ci, cx = p["k"], p["cutoff_min"], p["cutoff_max"]
    keys, counts, bo, s2b, st = run_like_bench(ctx, kmc, seq, off, p)
    n = len(counts)
    step(f"counted: {n} entries")
    assert n == st["n_out"] and n > 1_000_000
    check_bins(keys, bo, n)
    ok_keys, ok_counts = oracle.count(seq, off, k, ci, cx, threads=THREADS)
    step(f"oracle: {len(ok_counts)} entries")
    order = ascending(keys)
    assert n == len(ok_counts)
    assert np.array_equal(keys[order], ok_keys)
    assert np.array_equal(counts[order], ok_counts)
    del ok_keys, ok_counts
    assert st["n_kmers"] == oracle.valid_windows(seq, off, k)
    # every entry in the bin of its signature (a sample of the entries)
    rng = np.random.default_rng(11)
    idx = rng.choice(n, 20000, replace=False)
    bin_of = np.searchsorted(bo, idx, side="right") - 1
    sig = oracle.key_signatures(keys[idx], k, p["p"])
    assert np.array_equal(s2b[sig], bin_of)


@pytest.mark.timeout(600)
def test_large_job_scaled_exact(ctx, kmc):
    seq, off, p = synth.make("large-300M-60Mx150", 0.02)
    keys, counts, bo, s2b, st = run_like_bench(ctx, kmc, seq, off, p)
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"],
                                      threads=THREADS)
    order = ascending(keys)
    assert np.array_equal(keys[order], ok_keys)
    assert np.array_equal(counts[order], ok_counts)
    check_bins(keys, bo, len(counts))


@pytest.mark.timeout(1200)
def test_large_job_full_size_exact_slice(ctx, kmc):
    step = lambda m: print(f"[large job] {m}", flush=True)  # progress of a long test
    seq, off, p = synth.make("large-300M-60Mx150")
    step(f"generated {seq.size} bases")
    k, ci, cx = p["k"], p["cutoff_min"], p["cutoff_max"]
    keys, counts, bo, s2b, st = run_like_bench(ctx, kmc, seq, off, p)
    n = len(counts)
    step(f"counted: {n} entries")
    assert n == st["n_out"] and n > 100_000_000
    check_bins(keys, bo, n)
    assert st["n_kmers"] == oracle.valid_windows(seq, off, k)
    assert np.all((counts >= ci) & (counts <= cx))
    step("bins and k-mer total checked")
    # every entry of one sixteenth of the key space (the keys whose top four
    # bits are 9) against the oracle's count of that range, entry for entry
    # (the whole count would need some 230 GB of host memory)
    sl = (keys >> np.uint64(2 * k - 4)) == 9
    ok_keys, ok_counts = oracle.count(seq, off, k, ci, cx, threads=THREADS, slice_bits=4,
                                      slice=9)
    o = np.argsort(keys[sl])
    assert len(ok_keys) > 10_000_000
    assert np.array_equal(keys[sl][o], ok_keys) and np.array_equal(counts[sl][o], ok_counts)
    del ok_keys, ok_counts, o
    step(f"key range 9/16 checked: {int(sl.sum())} entries")
    rng = np.random.default_rng(13)
    idx = rng.choice(n, 5000, replace=False)
    bin_of = np.searchsorted(bo, idx, side="right") - 1
    sig = oracle.key_signatures(keys[idx], k, p["p"])
    assert np.array_equal(s2b[sig], bin_of)
    q = window_keys(seq, off, k, rng, 4000)
    qc = oracle.count_keys(seq, off, k, q, threads=THREADS)
    order = np.argsort(keys)
    pos = member(keys, order, q)
    want = (qc >= ci) & (qc <= cx)
    assert np.array_equal(pos >= 0, want)
    assert np.array_equal(counts[pos[pos >= 0]].astype(np.uint64), qc[pos >= 0])


def _batch_job(j):
    from paper_1407_1507_amd import synth as sy
    return sy.batch_job(j, 1.0)


@pytest.mark.timeout(900)
def test_batch_256_full_size_equals_single_runs(ctx, kmc):
    # the batched workload at full size (256 uneven jobs, 10.3 Gbases, k in
    # {21, 25, 31, 47, 55}): every table of one kmc_batch_count equals the
    # table of the same job counted alone, entry for entry
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    import torch
    step = lambda m: print(f"[batch 256] {m}", flush=True)  # progress of a long test
    with ProcessPoolExecutor(THREADS, mp_context=multiprocessing.get_context("spawn")) as ex:
        jobs = list(ex.map(_batch_job, range(256)))
    step(f"generated {sum(s.size for s, _, _ in jobs)} bases")
    dev = [(torch.from_numpy(s).to("cuda:0"), torch.from_numpy(o.view(np.int64)).to("cuda:0"), p)
           for s, o, p in jobs]
    del jobs
    torch.cuda.synchronize()
    c = kmc.Context(0)  # its own buffers, apart from the large job's cached ones
    out = c.batch_count(dev)
    step(f"batch: {sum(r.n for r in out)} entries")
    assert len(out) == 256
    ks = set()
    for (dseq, doff, p), r in zip(dev, out):
        a = c.count(dseq, doff, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
        ks.add(p["k"])
        assert r.n == a.n
        assert np.array_equal(r.keys, a.keys)
        assert np.array_equal(r.counts, a.counts)
        assert np.array_equal(r.bin_offsets, a.bin_offsets)
    assert ks == {21, 25, 31, 47, 55}
    step("all 256 tables equal their single runs")
    c.close()
    del dev, out
    torch.cuda.empty_cache()
