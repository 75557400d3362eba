"""GPU parity of the (k,x)-mer mode (Methods, "(k,x)-mers"; Fig. 2): the
table equals the plain oracle's (the k-mer counts do not depend on x), and the
number of (k,x)-mers and of distinct (k,x)-mers equals the string-level
oracle's on small inputs.  Cases cover both scans, x = 1..3, cutoffs and
saturation, tiles too large for LDS in both passes (streamed and partitioned,
with weights), and the rejected configurations."""
import numpy as np
import pytest

from oracle import kxmers as KX
from paper_1407_1507_amd import synth
from test_gpu_parity import check_table, ctx, kmc, to_reads  # noqa: F401

pytestmark = pytest.mark.gpu


def rand_reads(seed, n, lo, hi, n_rate=0.0, lower=0.0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        L = int(rng.integers(lo, hi + 1))
        s = rng.choice(list("ACGT"), size=L)
        m = rng.random(L)
        s[m < n_rate] = "N"
        low = rng.random(L) < lower
        s[low] = np.char.lower(s[low])
        out.append("".join(s))
    return out


@pytest.mark.parametrize("k,p,x", [(21, 7, 3), (15, 5, 1), (28, 7, 2), (12, 4, 3)])
def test_kx_entries_match_string_oracle(ctx, kmc, k, p, x):
    reads = rand_reads(100 + k + x, 1500, k - 3, 160, n_rate=0.005, lower=0.01)
    seq, off = to_reads(reads)
    res = ctx.count(seq, off, k, p, 64, 1, 2**32 - 1, flags=kmc.FLAG_KX(x))
    check_table(res, seq, off, k, p, 1, 2**32 - 1)
    n_p, n_d = KX.entry_stats(reads, k, p, x)
    assert res.stats["n_kx_entries"] == n_p
    assert res.stats["n_kx_distinct"] == n_d
    assert res.stats["n_kmers"] // (x + 1) <= n_p <= res.stats["n_kmers"]


@pytest.mark.parametrize("x", [1, 2, 3])
def test_kx_genome_workload(ctx, kmc, x):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.01)
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                    flags=kmc.FLAG_KX(x))
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])
    assert 0 < res.stats["n_kx_entries"] < res.stats["n_kmers"]


def test_kx_lane_scan_workload(ctx, kmc):
    # 300 000 reads: the lane-per-read scan
    seq, off, p = synth.make("genome-5M-2Mx100", 0.15)
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                    flags=kmc.FLAG_KX(3))
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])


@pytest.mark.parametrize("x", [1, 3])
def test_kx_one_huge_bin(ctx, kmc, x):
    # every k-mer in one bin: big tiles in both passes; the second pass's
    # big tiles carry weights (streamed kernel, then partition)
    rng = np.random.default_rng(40 + x)
    n_reads = 100_000
    seq = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), size=n_reads * 100)
    off = np.arange(n_reads + 1, dtype=np.uint64) * 100
    res = ctx.count(seq, off, 28, 7, 1, 1, 2**32 - 1, flags=kmc.FLAG_KX(x))
    assert res.stats["n_big_tiles"] > 0
    check_table(res, seq, off, 28, 7, 1, 2**32 - 1)


def test_kx_skewed_ranges(ctx, kmc):
    # 40x coverage in 16 bins: the k-mers that begin with their bin's
    # signature fill fine ranges beyond LDS even after the first pass merged
    # equal (k,x)-mers, so big tiles of the single-kernel path carry weights
    # in the second pass (runs of one key summed over their weights)
    seq, off, p = synth.make("genome-5M-2Mx100", 0.1)
    res = ctx.count(seq, off, p["k"], p["p"], 16, 2, 10**9, flags=kmc.FLAG_KX(3))
    assert res.stats["n_big_tiles"] > 0
    check_table(res, seq, off, p["k"], p["p"], 2, 10**9)


def test_kx_cutoffs_and_saturation(ctx, kmc):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.02)
    res = ctx.count(seq, off, 25, 7, 128, 3, 40, flags=kmc.FLAG_KX(2))
    check_table(res, seq, off, 25, 7, 3, 40)
    res = ctx.count(seq, off, 25, 7, 128, 1, 2**32 - 1, flags=kmc.FLAG_KX(3), counter_max=30)
    check_table(res, seq, off, 25, 7, 1, 2**32 - 1, cs=30)


def test_kx_rejected(ctx, kmc):
    seq, off = to_reads(rand_reads(9, 50, 40, 80))
    with pytest.raises(kmc.KmcError):
        ctx.count(seq, off, 29, 7, 16, 1, 2**32 - 1, flags=kmc.FLAG_KX(3))  # k + x > 31
    with pytest.raises(kmc.KmcError):
        ctx.count(seq, off, 21, 7, 16, 1, 2**32 - 1,
                  flags=kmc.FLAG_KX(1) | kmc.FLAG_NON_CANONICAL)
    import torch
    ws = torch.empty(ctx.workspace_size(seq, off, 21, 7, 16, 1, 2**32 - 1,
                                        flags=kmc.FLAG_KX(1)), dtype=torch.uint8,
                     device="cuda:0")
    with pytest.raises(kmc.KmcError):
        ctx.count_ws(seq, off, 21, 7, 16, 1, 2**32 - 1, ws, flags=kmc.FLAG_KX(1))
    # the context still counts afterwards
    res = ctx.count(seq, off, 21, 7, 16, 1, 2**32 - 1, flags=kmc.FLAG_KX(1))
    check_table(res, seq, off, 21, 7, 1, 2**32 - 1)
