"""Jobs above a memory budget (kmc_ctx_set_budget; the served form's jobs
larger than its budget): bins expanded, counted and assembled in groups
whose keys fit the budget, and super k-mer records spilled to pinned host
memory when they take more than half of it.  The table must be the one the
job gives without a budget (which the parity tests tie to the oracle), entry
for entry and bin for bin."""
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


def args(p):
    return p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"]


def dev(seq, off):
    import torch
    return (torch.from_numpy(seq).to("cuda:0"),
            torch.from_numpy(off.view(np.int64)).to("cuda:0"))


def same(a, b):
    assert a.n == b.n
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.counts, b.counts)
    if a.bin_offsets is not None or b.bin_offsets is not None:
        assert np.array_equal(a.bin_offsets, b.bin_offsets)


def per_kmer(k):
    return 48 if k <= 32 else 72


@pytest.mark.parametrize("name,scale", [("genome-5M-2Mx100", 0.05),
                                        ("repeats-50M-30x150-k55", 0.01)])
def test_groups_with_records_on_device(kmc, name, scale):
    seq, off, p = synth.make(name, scale)
    s, o = dev(seq, off)
    ctx = kmc.Context(0)
    ref = ctx.count(s, o, *args(p))
    n_kmers, n_rec = ref.stats["n_kmers"], ref.stats["n_superkmers"]
    rec_bytes = int(n_rec * (16 if p["k"] <= 32 else 32) * 1.3) + 256 * p["n_bins"] * 32
    ctx.set_budget(2 * rec_bytes + (24 << 20) + per_kmer(p["k"]) * n_kmers // 3)
    got = ctx.count(s, o, *args(p))
    assert got.stats["n_groups"] >= 2 and got.stats["records_spilled"] == 0
    same(got, ref)
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"],
                                      threads=8)
    keys = got.keys
    order = np.lexsort((keys[:, 1], keys[:, 0])) if keys.ndim == 2 else np.argsort(keys)
    assert np.array_equal(keys[order], ok_keys) and np.array_equal(got.counts[order], ok_counts)
    ctx.close()


@pytest.mark.parametrize("name,scale", [("genome-5M-2Mx100", 0.05),
                                        ("repeats-50M-30x150-k55", 0.01)])
def test_records_spilled_to_host(kmc, name, scale):
    import torch
    seq, off, p = synth.make(name, scale)
    s, o = dev(seq, off)
    ctx = kmc.Context(0)
    ref = ctx.count(s, o, *args(p))
    # what the library sets aside besides the keys (fine histograms of
    # 2^fb ranges per bin, 16 MiB for the smaller arrays), then room for the
    # keys of three of the largest bins: the records (about half the budget
    # or more) go to host memory
    mb = ref.stats["max_bin_kmers"]
    cap = 4096 if p["k"] <= 32 else 2048
    fb = max(1, min(int(np.ceil(np.log2(mb * 8 // cap + 1))), 12))
    fixed = (p["n_bins"] << fb) * 6 + (16 << 20)
    ctx.set_budget(fixed + per_kmer(p["k"]) * 3 * mb)
    got = ctx.count(s, o, *args(p))
    assert got.stats["records_spilled"] == 1 and got.stats["n_groups"] >= 4
    same(got, ref)
    # device table and ascending order from the grouped job
    dt = ctx.count(s, o, *args(p), flags=kmc.FLAG_DEVICE_TABLE)
    kw = 1 if p["k"] <= 32 else 2
    k = torch.empty(dt.n * kw, dtype=torch.int64, device="cuda:0")
    c = torch.empty(dt.n, dtype=torch.int32, device="cuda:0")
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(dt.keys_ptr),
                         ctypes.c_size_t(dt.n * kw * 8), 3) == 0
    assert hip.hipMemcpy(ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(dt.counts_ptr),
                         ctypes.c_size_t(dt.n * 4), 3) == 0
    dk = k.cpu().numpy().view(np.uint64)
    assert np.array_equal(dk.reshape(-1, 2) if kw == 2 else dk, ref.keys)
    assert np.array_equal(c.cpu().numpy().view(np.uint32), ref.counts)
    dt.free()
    asc = ctx.count(s, o, *args(p), flags=kmc.FLAG_ASCENDING)
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"],
                                      threads=8)
    assert np.array_equal(asc.keys, ok_keys) and np.array_equal(asc.counts, ok_counts)
    # the same context without the budget: back to one group
    ctx.set_budget(0)
    again = ctx.count(s, o, *args(p))
    assert again.stats["n_groups"] == 1 and again.stats["records_spilled"] == 0
    same(again, ref)
    ctx.close()


def test_bin_above_budget_rejected(kmc):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.01)
    ctx = kmc.Context(0)
    ctx.set_budget(1 << 20)
    with pytest.raises(kmc.KmcError) as e:
        ctx.count(seq, off, *args(p))
    assert e.value.status == kmc.KMC_ERR_TOO_LARGE
    ctx.close()


def test_server_oversize_job_within_budget(kmc):
    # a job whose footprint exceeds the server's budget runs in three
    # quarters of it, grouped and spilled; the same table as alone, and the
    # jobs around it still served
    big = synth.make("genome-5M-2Mx100", 0.05)
    small = synth.make("genome-5M-2Mx100", 0.002)
    ctx = kmc.Context(0)
    refs = [ctx.count(s, o, *args(p)) for s, o, p in (big, small)]
    fp = ctx.workspace_size(big[0], big[1], *args(big[2]))
    budget = 64 << 20
    assert fp > budget and ctx.workspace_size(small[0], small[1], *args(small[2])) < budget
    srv = kmc.Server(ctx, hbm_budget=budget, max_active=2)
    tickets = [srv.submit(s, o, *args(p)) for s, o, p in (small, big, small)]
    outs = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.stop()
    same(outs[0], refs[1])
    same(outs[1], refs[0])
    same(outs[2], refs[1])
    assert outs[1].stats["n_groups"] >= 2
    assert st["peak_admitted_bytes"] <= budget and st["completed"] == 3
    ctx.close()


@pytest.mark.parametrize("name,scale", [("genome-5M-2Mx100", 0.05),
                                        ("repeats-50M-30x150-k55", 0.01)])
def test_server_oversize_job_records_on_device(kmc, name, scale):
    # an oversize served job whose records stay on the device: its buffers
    # come from its region of the server's arena, group after group; host,
    # device and ascending tables equal the job's table counted alone (and
    # the oracle's)
    import torch
    seq, off, p = synth.make(name, scale)
    s, o = dev(seq, off)
    small = synth.make("genome-5M-2Mx100", 0.002)
    ctx = kmc.Context(0)
    ref = ctx.count(s, o, *args(p))
    ref_small = ctx.count(small[0], small[1], *args(small[2]))
    n_kmers, n_rec = ref.stats["n_kmers"], ref.stats["n_superkmers"]
    rec_bytes = int(n_rec * (16 if p["k"] <= 32 else 32) * 1.3) + 256 * p["n_bins"] * 32
    # the job runs in three quarters of the budget
    budget = (2 * rec_bytes + (24 << 20) + per_kmer(p["k"]) * n_kmers // 3) * 4 // 3
    assert ctx.workspace_size(s, o, *args(p)) > budget
    srv = kmc.Server(ctx, hbm_budget=budget, max_active=2)
    tickets = [srv.submit(small[0], small[1], *args(small[2])), srv.submit(s, o, *args(p)),
               srv.submit(s, o, *args(p), flags=kmc.FLAG_ASCENDING),
               srv.submit(s, o, *args(p), flags=kmc.FLAG_DEVICE_TABLE),
               srv.submit(small[0], small[1], *args(small[2]))]
    outs = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.stop()
    same(outs[0], ref_small)
    same(outs[4], ref_small)
    same(outs[1], ref)
    assert outs[1].stats["n_groups"] >= 2 and outs[1].stats["records_spilled"] == 0
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"],
                                      threads=8)
    assert np.array_equal(outs[2].keys, ok_keys) and np.array_equal(outs[2].counts, ok_counts)
    dt = outs[3]
    assert dt.on_device and dt.n == ref.n and dt.stats["n_groups"] >= 2
    kw = 1 if p["k"] <= 32 else 2
    k = torch.empty(dt.n * kw, dtype=torch.int64, device="cuda:0")
    c = torch.empty(dt.n, dtype=torch.int32, device="cuda:0")
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(dt.keys_ptr),
                         ctypes.c_size_t(dt.n * kw * 8), 3) == 0
    assert hip.hipMemcpy(ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(dt.counts_ptr),
                         ctypes.c_size_t(dt.n * 4), 3) == 0
    dk = k.cpu().numpy().view(np.uint64)
    assert np.array_equal(dk.reshape(-1, 2) if kw == 2 else dk, ref.keys)
    assert np.array_equal(c.cpu().numpy().view(np.uint32), ref.counts)
    assert st["completed"] == 5 and st["peak_admitted_bytes"] <= budget
    for r in outs:
        r.free()
    ctx.close()
