"""GPU parity of the many-job forms: caller workspace (kmc_count_ws), the
batch (kmc_batch_count) and the server (kmc_server_*).  Each job's table must
be bit-identical to what kmc_count_ex returns for that job alone, which
test_gpu_parity ties to the oracle; the small jobs here are also checked
against the oracle directly."""
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


def same(a, b):
    assert a.n == b.n
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.bin_offsets, b.bin_offsets)
    assert np.array_equal(a.sig_to_bin, b.sig_to_bin)


def against_oracle(res, seq, off, p):
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"])
    keys = res.keys
    order = np.lexsort((keys[:, 1], keys[:, 0])) if keys.ndim == 2 else np.argsort(keys)
    assert np.array_equal(keys[order], ok_keys)
    assert np.array_equal(res.counts[order], ok_counts)


def args(p):
    return p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"]


def test_count_ws_matches_count(ctx, kmc):
    import torch
    big = synth.make("genome-5M-2Mx100", 0.02)
    small = synth.make("repeats-50M-30x150-k55", 0.002)
    need = max(ctx.workspace_size(s, o, *args(p)) for s, o, p in (big, small))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    # the same workspace twice in a row, the second job smaller and k > 32
    for seq, off, p in (big, small):
        ref = ctx.count(seq, off, *args(p))
        got = ctx.count_ws(seq, off, *args(p), workspace=ws)
        same(got, ref)
        against_oracle(got, seq, off, p)
    # device table inside the workspace; freeing it leaves the workspace alone
    seq, off, p = big
    t = ctx.count_ws(seq, off, *args(p), workspace=ws, flags=kmc.FLAG_DEVICE_TABLE)
    host = ctx.count(seq, off, *args(p))
    base = ws.data_ptr()
    assert base <= t.keys_ptr < base + need and base <= t.counts_ptr < base + need
    o = t.keys_ptr - base
    keys = ws[o:o + t.n * 8].cpu().numpy().view(np.uint64)
    o = t.counts_ptr - base
    counts = ws[o:o + t.n * 4].cpu().numpy().view(np.uint32)
    t.free()
    assert np.array_equal(keys, host.keys) and np.array_equal(counts, host.counts)


def test_count_ws_too_small(ctx, kmc):
    import torch
    seq, off, p = synth.make("genome-5M-2Mx100", 0.005)
    need = ctx.workspace_size(seq, off, *args(p))
    ws = torch.empty(need // 2, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(kmc.KmcError) as e:
        ctx.count_ws(seq, off, *args(p), workspace=ws)
    assert e.value.status == kmc.KMC_ERR_OUT_OF_MEMORY


def test_batch_matches_single_and_oracle(ctx, kmc):
    jobs = [synth.batch_job(j, 0.02) for j in range(10)]
    jobs.append(synth.make("uniform-10k", 0.1))
    jobs.append((np.zeros(0, np.uint8), np.zeros(1, np.uint64), dict(k=28, p=7, n_bins=512,
                                                                      cutoff_min=1,
                                                                      cutoff_max=10)))
    assert len({p["k"] for _, _, p in jobs}) >= 3
    out = ctx.batch_count(jobs)
    assert len(out) == len(jobs)
    for (seq, off, p), res in zip(jobs, out):
        same(res, ctx.count(seq, off, *args(p)))
        against_oracle(res, seq, off, p)
    # a second batch on the same pool, in another order
    again = ctx.batch_count(jobs[::-1])
    for a, b in zip(again, out[::-1]):
        same(a, b)


def test_batch_all_or_nothing(ctx, kmc):
    good = synth.batch_job(0, 0.01)
    bad = (good[0], good[1], dict(good[2], cutoff_min=5, cutoff_max=4))
    with pytest.raises(kmc.KmcError) as e:
        ctx.batch_count([good, bad, good])
    assert e.value.status == kmc.KMC_ERR_INVALID_ARG
    assert ctx.batch_count([]) == []


def test_server_matches_alone_and_respects_budget(ctx, kmc):
    jobs = [synth.served_job(i, 0.01) for i in range(6)] + [synth.batch_job(j, 0.02)
                                                           for j in range(6)]
    fps = [ctx.workspace_size(s, o, *args(p)) for s, o, p in jobs]
    budget = 3 * max(fps)
    srv = kmc.Server(ctx, hbm_budget=budget, max_active=4)
    try:
        tickets = [srv.submit(s, o, *args(p)) for s, o, p in jobs]
        got = [srv.poll(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.stop()
    assert st["submitted"] == len(jobs) and st["completed"] == len(jobs) and st["failed"] == 0
    assert 0 < st["peak_admitted_bytes"] <= st["budget"] <= budget
    assert st["active"] == 0 and st["queued"] == 0
    for (seq, off, p), res in zip(jobs, got):
        same(res, ctx.count(seq, off, *args(p)))
        assert 0 <= res.stats["us_queue"] <= res.stats["us_latency"]
    for (seq, off, p), res in list(zip(jobs, got))[:3]:
        against_oracle(res, seq, off, p)


def test_server_oversize_job_runs_alone(ctx, kmc):
    small = synth.batch_job(1, 0.01)
    large = synth.make("genome-5M-2Mx100", 0.02)
    fp_small = ctx.workspace_size(small[0], small[1], *args(small[2]))
    fp_large = ctx.workspace_size(large[0], large[1], *args(large[2]))
    # room for a small job beside the large one would leave it less than
    # three quarters of the budget, so it takes the whole arena, alone
    budget = 2 * fp_small + 4096
    assert fp_large > budget
    srv = kmc.Server(ctx, hbm_budget=budget, max_active=2)
    try:
        ts = [srv.submit(small[0], small[1], *args(small[2])),
              srv.submit(large[0], large[1], *args(large[2])),
              srv.submit(small[0], small[1], *args(small[2]))]
        res = [srv.poll(t) for t in ts]
        st = srv.stats()
    finally:
        srv.stop()
    assert st["completed"] == 3 and st["peak_admitted_bytes"] <= st["budget"]
    same(res[0], ctx.count(small[0], small[1], *args(small[2])))
    same(res[2], res[0])
    same(res[1], ctx.count(large[0], large[1], *args(large[2])))


def test_server_poll_without_wait_and_device_tables(ctx, kmc):
    seq, off, p = synth.batch_job(2, 0.01)
    srv = kmc.Server(ctx, hbm_budget=1 << 30, max_active=2)
    try:
        t = srv.submit(seq, off, *args(p), flags=kmc.FLAG_DEVICE_TABLE)
        r = srv.poll(t, wait=False)
        if r is None:
            r = srv.poll(t)
        with pytest.raises(kmc.KmcError):
            srv.poll(t)  # the ticket was released
        # a job left unpolled is freed by stop()
        srv.submit(seq, off, *args(p))
    finally:
        srv.stop()
    assert r.on_device and r.n == ctx.count(seq, off, *args(p)).n
    r.free()
