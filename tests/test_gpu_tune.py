"""Knobs and the autotuner (kmc_ctx_set_knobs, kmc_autotune): every
candidate knob set gives the same table as the defaults, entry for entry and
bin for bin (the defaults are tied to the oracle by the parity tests, and
one case here is checked against the oracle too); a batch counted after
tuning equals the same jobs counted alone on an untuned context."""
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


def same(a, b):
    assert a.n == b.n
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.bin_offsets, b.bin_offsets)


def big_tile_reads():
    ref = synth.random_reference(9, 3000)
    seq, off = synth.sample_reads(10, ref, 40_000, 100, err=0.002, n_rate=0.0)
    return seq, off, dict(k=28, p=7, n_bins=4, cutoff_min=1, cutoff_max=2**32 - 1)


@pytest.mark.parametrize("case", ["genome", "repeats", "bigtiles"])
def test_every_knob_set_gives_the_same_table(kmc, case):
    if case == "genome":
        seq, off, p = synth.make("genome-5M-2Mx100", 0.02)
    elif case == "repeats":
        seq, off, p = synth.make("repeats-50M-30x150-k55", 0.005)
    else:
        seq, off, p = big_tile_reads()
    ctx = kmc.Context(0)
    ref = ctx.count(seq, off, *args(p))
    for knobs in kmc.KNOB_CANDIDATES:
        ctx.set_knobs(knobs)
        same(ctx.count(seq, off, *args(p)), ref)
    ctx.set_knobs(None)
    if case == "repeats":
        ok_keys, ok_counts = oracle.count(seq, off, p["k"], p["cutoff_min"], p["cutoff_max"])
        order = np.lexsort((ref.keys[:, 1], ref.keys[:, 0]))
        assert np.array_equal(ref.keys[order], ok_keys)
        assert np.array_equal(ref.counts[order], ok_counts)
    ctx.close()


def test_knobs_rejected_out_of_range(kmc):
    ctx = kmc.Context(0)
    for bad in ((1, 0, 0), (3, 3, 0), (3, 0, 300)):
        with pytest.raises(kmc.KmcError):
            ctx.set_knobs(bad)
    ctx.close()


def test_autotune_then_batch_equals_alone(kmc):
    jobs = [synth.batch_job(j, 0.03) for j in range(12)]
    tuned = kmc.Context(0)
    rep = tuned.autotune(jobs)
    assert rep["batch_workers"] in (2, 4, 8)
    assert len(rep["classes"]) >= 2
    assert all(tuple(c["knobs"]) in kmc.KNOB_CANDIDATES for c in rep["classes"])
    outs = tuned.batch_count(jobs)
    plain = kmc.Context(0)
    for (s, o, p), got in zip(jobs, outs):
        same(got, plain.count(s, o, *args(p)))
    tuned.close()
    plain.close()
