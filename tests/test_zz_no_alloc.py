"""The allocation-free entry point (kmc_count_static): scratch in the
library's static device array, table in the caller's buffers.  Its tables
must equal kmc_count_ex's for the same job (which the parity tests tie to the
oracle), on consecutive calls that share the array, the second one smaller."""
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


def args(p):
    return p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"]


def static_count(ctx, seq, off, p, flags=0, cap=None, device_reads=True):
    import torch
    kw = 1 if p["k"] <= 32 else 2
    cap = int(off[-1]) if cap is None else cap
    keys = torch.full((max(cap, 1) * kw,), -1, dtype=torch.int64, device="cuda:0")
    counts = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda:0")
    if device_reads:
        s = torch.from_numpy(seq).to("cuda:0")
        o = torch.from_numpy(off.view(np.int64)).to("cuda:0")
    else:
        s, o = seq, off
    n, bo, st = ctx.count_static(s, o, *args(p), keys, counts, flags=flags)
    k = keys[:n * kw].cpu().numpy().view(np.uint64)
    c = counts[:n].cpu().numpy().view(np.uint32)
    return (k.reshape(-1, 2) if kw == 2 else k), c, bo, st


def test_static_equals_count_ex_twice(ctx, kmc):
    jobs = [synth.make("genome-5M-2Mx100", 0.02),           # 4 Mbases, k = 28
            synth.make("repeats-50M-30x150-k55", 0.0015)]   # 2.25 Mbases, k = 55: smaller
    for i, (seq, off, p) in enumerate(jobs):
        ref = ctx.count(seq, off, *args(p))
        keys, counts, bo, st = static_count(ctx, seq, off, p)
        assert st["n_out"] == ref.n == len(counts), i
        assert np.array_equal(keys, ref.keys), i
        assert np.array_equal(counts, ref.counts), i
        assert np.array_equal(bo, ref.bin_offsets), i
        assert st["n_kmers"] == ref.stats["n_kmers"], i
    # the smaller job against the oracle as well
    seq, off, p = jobs[1]
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"])
    order = np.lexsort((keys[:, 1], keys[:, 0]))
    assert np.array_equal(keys[order], ok_keys) and np.array_equal(counts[order], ok_counts)


def test_static_ascending_host_reads(ctx, kmc):
    seq, off, p = synth.make("uniform-10k")
    keys, counts, bo, st = static_count(ctx, seq, off, p, flags=kmc.FLAG_ASCENDING,
                                        device_reads=False)
    ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"])
    assert bo is None
    assert np.array_equal(keys, ok_keys) and np.array_equal(counts, ok_counts)
    assert int(counts.sum()) == 730_000


def test_static_rejects_job_above_scratch(ctx, kmc):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.05)  # 10 Mbases: above 256 MiB of scratch
    with pytest.raises(kmc.KmcError) as e:
        static_count(ctx, seq, off, p)
    assert e.value.status == kmc.KMC_ERR_TOO_LARGE
    assert "static scratch holds" in str(e.value)


def test_static_output_too_small(ctx, kmc):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.005)
    ref = ctx.count(seq, off, *args(p))
    with pytest.raises(kmc.KmcError) as e:
        static_count(ctx, seq, off, p, cap=ref.n - 1)
    assert e.value.status == kmc.KMC_ERR_TOO_LARGE and e.value.n_out == ref.n
    keys, counts, bo, st = static_count(ctx, seq, off, p, cap=ref.n)
    assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)
