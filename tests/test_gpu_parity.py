"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact: the GPU table, put in ascending key
order, equals the oracle's table entry for entry; the GPU's per-window
signatures equal the oracle's; every entry lies in the bin its signature maps
to.  Cases span several tiles and ragged tails, word-boundary k, N bases,
lowercase, empty and short reads, tiles too large for LDS, and the paper's
worked examples."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from conftest import read_golden
from oracle import strings as S
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


def ascending(keys, counts):
    if keys.ndim == 2:
        order = np.lexsort((keys[:, 1], keys[:, 0]))
    else:
        order = np.argsort(keys, kind="stable")
    return keys[order], counts[order]


def check_table(res, seq, off, k, p, ci, cx, flt=True, canonical=True, cs=0):
    """Bit-exact against the oracle, plus the bin invariants."""
    ok_keys, ok_counts = oracle.count(seq, off, k, ci, cx, canonical=canonical, counter_max=cs)
    gk, gc = ascending(res.keys, res.counts)
    assert res.n == len(ok_counts)
    assert np.array_equal(gk, ok_keys)
    assert np.array_equal(gc, ok_counts)
    # bins: every entry sits in the bin its signature maps to, ascending inside
    bo = res.bin_offsets
    assert bo[0] == 0 and bo[-1] == res.n and np.all(bo[1:] >= bo[:-1])
    if res.n:
        sig = oracle.key_signatures(res.keys, k, p, filter=flt)
        bin_of_entry = np.repeat(np.arange(res.n_bins), np.diff(bo).astype(np.int64))
        assert np.array_equal(res.sig_to_bin[sig], bin_of_entry)
        for b in range(res.n_bins):
            seg = res.keys[bo[b]:bo[b + 1]]
            if len(seg) > 1:
                if seg.ndim == 2:
                    assert np.all((seg[1:, 0] > seg[:-1, 0]) |
                                  ((seg[1:, 0] == seg[:-1, 0]) & (seg[1:, 1] > seg[:-1, 1])))
                else:
                    assert np.all(seg[1:] > seg[:-1])
    if ci <= 1 and cx >= 2**32 - 1 and not cs:
        assert int(res.counts.sum()) == oracle.valid_windows(seq, off, k)
    assert res.stats["n_kmers"] == oracle.valid_windows(seq, off, k)


# ---------------------------------------------------------- paper examples


def test_fig1_signatures_and_superkmers(ctx):
    rows = read_golden("fig1_split.txt")
    read = rows[0][1]
    k, m = int(rows[1][1]), int(rows[2][1])
    seq, off = to_reads([read])
    for mode, flags in (("signature", 0), ("minimizer", 2)):
        sig, start = ctx.debug_signatures(seq, off, k, m, flags)
        expect_sig, expect_start = [], []
        for sk, s in [(r[1], r[2]) for r in rows if r[0] == mode]:
            n = len(sk) - k + 1
            expect_sig += [S.encode(s)] * n
            expect_start += [1] + [0] * (n - 1)
        n = len(read) - k + 1
        assert list(sig[:n]) == expect_sig
        assert list(start[:n]) == expect_start
        assert all(int(x) == 0xFFFFFFFF for x in sig[n:])


def test_fig2_superkmer_counts(ctx):
    rows = read_golden("fig2_kx_mers.txt")
    sk, k, m = rows[0][1], int(rows[1][1]), int(rows[2][1])
    seq, off = to_reads([sk])
    sig, start = ctx.debug_signatures(seq, off, k, m)
    assert set(int(x) for x in sig[:len(sk) - k + 1]) == {S.encode(rows[3][1])}
    res = ctx.count(seq, off, k, m, 4, 1, 2**32 - 1)
    check_table(res, seq, off, k, m, 1, 2**32 - 1)
    assert res.n == len(sk) - k + 1


def test_supplement_signature(ctx):
    kmer, plen, sigs, val = read_golden("supp_encoding.txt")[0][1:]
    seq, off = to_reads([kmer])
    sig, _ = ctx.debug_signatures(seq, off, len(kmer), int(plen))
    assert int(sig[0]) == int(val)


# ------------------------------------------------------------ random small


def random_reads(rng, n, lo, hi, n_rate=0.0, lower=0.0):
    out = []
    for _ in range(n):
        L = int(rng.integers(lo, hi + 1))
        b = rng.choice(list("ACGT"), size=L)
        if n_rate:
            b[rng.random(L) < n_rate] = "N"
        if lower:
            idx = rng.random(L) < lower
            b[idx] = np.char.lower(b[idx])
        out.append("".join(b))
    return out


@pytest.mark.parametrize("k,p,n_bins", [(4, 4, 3), (5, 4, 16), (15, 4, 7), (21, 5, 64),
                                        (28, 7, 512), (31, 7, 100), (32, 8, 512), (33, 7, 512),
                                        (47, 9, 1024), (55, 9, 1024), (63, 12, 4096),
                                        (64, 11, 2000)])
def test_random_reads_exact(ctx, k, p, n_bins):
    rng = np.random.default_rng(1000 + k)
    reads = random_reads(rng, 700, 0, 260, n_rate=0.01, lower=0.02)
    reads += ["", "A", "ACGT" * 40, "N" * 50, "A" * 200, "ACACACACAC" * 20]
    seq, off = to_reads(reads)
    for ci, cx in ((1, 2**32 - 1), (2, 10**9), (1, 3)):
        res = ctx.count(seq, off, k, p, n_bins, ci, cx)
        check_table(res, seq, off, k, p, ci, cx)


def test_window_signatures_match_oracle(ctx):
    rng = np.random.default_rng(77)
    reads = random_reads(rng, 300, 0, 300, n_rate=0.02, lower=0.01)
    seq, off = to_reads(reads)
    for k, p, flt in ((28, 7, True), (28, 7, False), (55, 9, True), (12, 5, True), (64, 12, True)):
        sig, start = ctx.debug_signatures(seq, off, k, p, 0 if flt else 2)
        assert np.array_equal(sig, oracle.window_signatures(seq, off, k, p, flt))
        # a super k-mer starts wherever the signature changes or a valid run starts
        valid = sig != 0xFFFFFFFF
        prev_valid = np.concatenate([[False], valid[:-1]])
        prev_sig = np.concatenate([[0xFFFFFFFF], sig[:-1]])
        must = valid & (~prev_valid | (sig != prev_sig))
        assert np.all(start[must] == 1)
        assert np.all(start[~valid] == 0)


@pytest.mark.parametrize("k,p,n_reads", [(28, 7, 100_000), (40, 7, 60_000), (28, 7, 200_000)])
def test_one_huge_bin(ctx, k, p, n_reads):
    # every k-mer in one bin: more keys than 4096 tiles of the tile limit hold,
    # so fine ranges above the limit become big tiles (this once returned
    # KMC_ERR_TOO_LARGE); at 200 000 reads ranges hold more distinct keys
    # than the LDS table has slots
    rng = np.random.default_rng(k)
    seq = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), size=n_reads * 100)
    off = np.arange(n_reads + 1, dtype=np.uint64) * 100
    res = ctx.count(seq, off, k, p, 1, 1, 2**32 - 1)
    assert res.stats["n_big_tiles"] > 0
    check_table(res, seq, off, k, p, 1, 2**32 - 1)


def test_merged_big_tiles_streamed(ctx):
    # every k-mer in one bin, reads drawn without errors from a 100 kbp
    # reference (about 70x): each fine range holds more keys than the tile
    # limit but few distinct keys, so big tiles take the following ranges up
    # to four limits and are counted by streaming (mean big tile well above
    # one range)
    rng = np.random.default_rng(77)
    ref = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), size=100_000)
    n_reads = 200_000
    st = rng.integers(0, ref.size - 100, size=n_reads)
    seq = ref[st[:, None] + np.arange(100)].reshape(-1)
    off = np.arange(n_reads + 1, dtype=np.uint64) * 100
    res = ctx.count(seq, off, 28, 7, 1, 1, 2**32 - 1)
    big, keys = res.stats["n_big_tiles"], res.stats["n_big_keys"]
    assert big > 0 and keys / big > 2 * 3072
    check_table(res, seq, off, 28, 7, 1, 2**32 - 1)


def test_skewed_ranges(ctx):
    # reads at 40x coverage in 64 bins: the k-mers that begin with their
    # signature fill fine ranges of several thousand keys (big tiles), about a
    # quarter of them distinct
    seq, off, p = synth.make("genome-5M-2Mx100", 0.1)
    res = ctx.count(seq, off, p["k"], p["p"], 64, p["cutoff_min"], p["cutoff_max"])
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])


def test_long_reads(ctx):
    # a mean read length above 2 kbp takes the position-per-lane scan for every
    # k (split, sample histogram and the per-window audit); reads of a few
    # hundred kbp with N runs, beside short reads
    rng = np.random.default_rng(5)
    acgt = np.array(list("ACGT"))
    reads = ["".join(rng.choice(acgt, size=n)) for n in (300_000, 120_000, 50_001)]
    reads[1] = reads[1][:60_000] + "N" * 40 + reads[1][60_000:]
    reads += random_reads(rng, 40, 0, 200, n_rate=0.01, lower=0.02)
    seq, off = to_reads(reads)
    for k, p, nb in ((28, 7, 512), (21, 5, 64), (33, 7, 256)):
        res = ctx.count(seq, off, k, p, nb, 1, 2**32 - 1)
        check_table(res, seq, off, k, p, 1, 2**32 - 1)
    for k, p in ((28, 7), (55, 9)):
        sig, _ = ctx.debug_signatures(seq, off, k, p, 0)
        assert np.array_equal(sig, oracle.window_signatures(seq, off, k, p, True))


# ------------------------------------------------------------- workloads


def test_uniform_10k_exact(ctx):
    seq, off, p = synth.make("uniform-10k")
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])
    assert int(res.counts.sum()) == 730_000
    assert res.stats["n_tiles"] > 100


@pytest.mark.parametrize("scale", [0.01, 0.05])
def test_genome_exact(ctx, scale):
    seq, off, p = synth.make("genome-5M-2Mx100", scale)
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])


def test_repeats_k55_exact(ctx):
    seq, off, p = synth.make("repeats-50M-30x150-k55", 0.01)
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])


def test_big_tiles(ctx):
    # a tiny reference at very high coverage: tiles far beyond LDS capacity,
    # with many distinct keys (MSD through HBM) and runs of one key
    ref = synth.random_reference(9, 3000)
    seq, off = synth.sample_reads(10, ref, 40_000, 100, err=0.002, n_rate=0.0)
    seq2, off2 = to_reads(["ACGT" * 30] * 3000)
    seq = np.concatenate([seq, seq2])
    off = np.concatenate([off, off2[1:] + off[-1]])
    for k, p, nb in ((28, 7, 4), (55, 9, 4)):
        res = ctx.count(seq, off, k, p, nb, 1, 2**32 - 1)
        assert res.stats["n_big_tiles"] > 0
        check_table(res, seq, off, k, p, 1, 2**32 - 1)


@pytest.mark.parametrize("name,scale", [("genome-5M-2Mx100", 0.15),
                                        ("repeats-50M-30x150-k55", 0.03)])
def test_lane_scan_workloads(ctx, name, scale):
    # 300 000 reads: enough for the lane-per-read scan (smaller jobs take the
    # position-per-lane scan)
    seq, off, p = synth.make(name, scale)
    res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    check_table(res, seq, off, p["k"], p["p"], p["cutoff_min"], p["cutoff_max"])


def test_lane_scan_queue_overflow(ctx):
    # 300 000 reads, one in ten of 600 bp: the mean length keeps the lane
    # scan, and the long reads overflow their lane's queue of super k-mers
    # (the rest go to their bins one by one)
    ref = synth.random_reference(32, 2_000_000)
    seq, off = synth.sample_reads(33, ref, 300_000, 100, err=0.01, n_rate=0.001)
    lseq, loff = synth.sample_reads(34, ref, 30_000, 600, err=0.01, n_rate=0.001)
    seq = np.concatenate([seq[: int(off[270_000])], lseq])
    off = np.concatenate([off[:270_001], loff[1:] + off[270_000]])
    assert off.size == 300_001
    res = ctx.count(seq, off, 55, 9, 1024, 1, 2**32 - 1)
    check_table(res, seq, off, 55, 9, 1, 2**32 - 1)


def test_lane_scan_long_queue_overflow(ctx):
    # 300 000 reads at k = 28, one in twenty of 600 bp, the rest 150 bp: the
    # mean length (172.5) needs the 16-slot queue per lane (about 14 super
    # k-mers per read), and the long reads (about 53 each) overflow it
    ref = synth.random_reference(35, 4_000_000)
    seq, off = synth.sample_reads(36, ref, 300_000, 150, err=0.01, n_rate=0.001)
    lseq, loff = synth.sample_reads(37, ref, 15_000, 600, err=0.01, n_rate=0.001)
    seq = np.concatenate([seq[: int(off[285_000])], lseq])
    off = np.concatenate([off[:285_001], loff[1:] + off[285_000]])
    assert off.size == 300_001
    res = ctx.count(seq, off, 28, 7, 2048, 1, 2**32 - 1)
    check_table(res, seq, off, 28, 7, 1, 2**32 - 1)


def test_plain_minimizers_same_counts(ctx, kmc):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.01)
    res = ctx.count(seq, off, 28, 7, 512, 2, 10**9, flags=kmc.FLAG_PLAIN_MINIMIZERS)
    check_table(res, seq, off, 28, 7, 2, 10**9, flt=False)


@pytest.mark.parametrize("k,p,n_bins", [(15, 5, 64), (28, 7, 512), (33, 7, 256), (55, 9, 1024),
                                        (55, 9, 8192)])
def test_non_canonical(ctx, kmc, k, p, n_bins):
    # k-mers as read (supplement, -b): random reads with N and lowercase, and
    # the genome workload at 1%; both scans (8192 bins do not fit the lane
    # scan's LDS and take the position-per-lane scan)
    rng = np.random.default_rng(900 + k)
    seq, off = to_reads(random_reads(rng, 3000, 0, 160, n_rate=0.01, lower=0.02))
    res = ctx.count(seq, off, k, p, n_bins, 1, 2**32 - 1, flags=kmc.FLAG_NON_CANONICAL)
    check_table(res, seq, off, k, p, 1, 2**32 - 1, canonical=False)
    seq, off, _ = synth.make("genome-5M-2Mx100", 0.01)
    res = ctx.count(seq, off, k, p, n_bins, 2, 10**9, flags=kmc.FLAG_NON_CANONICAL)
    check_table(res, seq, off, k, p, 2, 10**9, canonical=False)


def test_non_canonical_big_tiles(ctx, kmc):
    # tiles beyond LDS (partitioned through HBM) in the as-read mode
    ref = synth.random_reference(9, 3000)
    seq, off = synth.sample_reads(10, ref, 40_000, 100, err=0.002, n_rate=0.0)
    for k, p, nb in ((28, 7, 4), (55, 9, 4)):
        res = ctx.count(seq, off, k, p, nb, 1, 2**32 - 1, flags=kmc.FLAG_NON_CANONICAL)
        assert res.stats["n_big_tiles"] > 0
        check_table(res, seq, off, k, p, 1, 2**32 - 1, canonical=False)


@pytest.mark.parametrize("ci,cx,cs", [(1, 2**32 - 1, 1), (2, 10**9, 3), (1, 6, 5), (2, 10**9, 255)])
def test_counter_saturation(ctx, kmc, ci, cx, cs):
    # counters clipped at cs (supplement, -cs), cutoffs on the exact counts;
    # both key widths and the ascending order
    for name, sc in (("genome-5M-2Mx100", 0.01), ("repeats-50M-30x150-k55", 0.003)):
        seq, off, p = synth.make(name, sc)
        res = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], ci, cx, counter_max=cs)
        check_table(res, seq, off, p["k"], p["p"], ci, cx, cs=cs)
        asc = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], ci, cx, counter_max=cs,
                        flags=kmc.FLAG_ASCENDING)
        ok_keys, ok_counts = oracle.count(seq, off, p["k"], ci, cx, counter_max=cs)
        assert np.array_equal(asc.keys, ok_keys) and np.array_equal(asc.counts, ok_counts)


def test_table6_shape(ctx, kmc):
    # Table 6's shape on 100 bp genome-like reads at m = 7: signatures give
    # fewer super k-mers per read than plain canonical minimizers, at k = 28
    # and k = 55, about 6.7 per read at k = 28 (the paper's 6.728 on G.
    # gallus); the same k-mers are counted either way
    seq, off, _ = synth.make("genome-5M-2Mx100", 0.05)
    n_reads = off.size - 1
    for k in (28, 55):
        per = {}
        for flags in (0, kmc.FLAG_PLAIN_MINIMIZERS):
            r = ctx.count(seq, off, k, 7, 512, 2, 10**9, flags=flags)
            per[flags] = (r.stats["n_superkmers"] / n_reads, r.stats["n_kmers"])
        assert per[0][1] == per[kmc.FLAG_PLAIN_MINIMIZERS][1]
        assert per[0][0] < per[kmc.FLAG_PLAIN_MINIMIZERS][0]
        if k == 28:
            assert 5.5 < per[0][0] < 8.0
        else:
            assert 2.0 < per[0][0] < 3.5


def test_empty_and_degenerate(ctx):
    for reads in ([], [""], ["ACG"], ["N" * 100], ["ACGTN" * 20]):
        seq, off = to_reads(reads)
        res = ctx.count(seq, off, 28, 7, 512, 1, 2**32 - 1)
        assert res.n == 0 and res.stats["n_kmers"] == 0


def test_deterministic(ctx):
    seq, off, p = synth.make("genome-5M-2Mx100", 0.02)
    a = ctx.count(seq, off, 28, 7, 512, 1, 10**9)
    b = ctx.count(seq, off, 28, 7, 512, 1, 10**9)
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.bin_offsets, b.bin_offsets)


def test_device_inputs_and_device_table(ctx, kmc):
    import torch
    seq, off, p = synth.make("genome-5M-2Mx100", 0.01)
    host = ctx.count(seq, off, 28, 7, 512, 2, 10**9)
    dseq = torch.from_numpy(seq).cuda()
    doff = torch.from_numpy(off.view(np.int64)).cuda()
    dev = ctx.count(dseq, doff, 28, 7, 512, 2, 10**9)
    assert np.array_equal(dev.keys, host.keys) and np.array_equal(dev.counts, host.counts)
    # table left in device memory, copied back with hipMemcpy
    t = ctx.count(dseq, doff, 28, 7, 512, 2, 10**9, flags=kmc.FLAG_DEVICE_TABLE)
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


def test_bad_device_offsets_rejected(ctx, kmc):
    import torch
    seq = torch.zeros(100, dtype=torch.uint8, device="cuda")
    off = torch.tensor([0, 60, 40, 100], dtype=torch.int64, device="cuda")
    with pytest.raises(kmc.KmcError) as e:
        ctx.count(seq, off, 28, 7, 16, 1, 10)
    assert e.value.status == kmc.KMC_ERR_INVALID_ARG


# ------------------------------------------------ forced fallbacks (exact)


def hot_unsampled_reads(n_reads, stride, seed):
    """Random reads, except that every read whose index is not a multiple of
    `stride` (the sample histogram scans reads 0, stride, 2 stride, ...) is a
    copy of one read: its signatures are hot in the input and absent from the
    sample, so their bins outgrow the regions sized from the sample."""
    rng = np.random.default_rng(seed)
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    seq = rng.choice(acgt, size=n_reads * 100).reshape(n_reads, 100)
    hot = rng.choice(acgt, size=100)
    mask = (np.arange(n_reads) % stride) != 0
    seq[mask] = hot
    off = np.arange(n_reads + 1, dtype=np.uint64) * 100
    return seq.reshape(-1).copy(), off


@pytest.mark.parametrize("k,p,n_bins", [(28, 7, 512), (55, 9, 1024), (33, 7, 64), (55, 9, 8192)])
def test_split_second_pass(ctx, k, p, n_bins):
    # both scans: 8192 bins take the position-per-lane scan
    # 20 000 reads x 100 bp: the sample takes every 20th read (stride =
    # bases / 1e5); the other 19 000 are one read repeated
    seq, off = hot_unsampled_reads(20_000, 20, k)
    res = ctx.count(seq, off, k, p, n_bins, 1, 2**32 - 1)
    assert res.stats["split_passes"] == 2
    check_table(res, seq, off, k, p, 1, 2**32 - 1)


@pytest.mark.parametrize("k", [33, 47, 55, 64])
def test_fingerprint_clash_fallback(ctx, kmc, k):
    # 128-bit tiles are counted by fingerprint; a tile where two keys share
    # one goes to the exact partition path.  With the fingerprint narrowed to
    # 2 bits nearly every tile clashes: the table must not change.
    seq, off, p = synth.make("repeats-50M-30x150-k55", 0.004)
    pk = 9 if k >= 47 else 7
    base = ctx.count(seq, off, k, pk, 256, 2, 10**6)
    res = ctx.count(seq, off, k, pk, 256, 2, 10**6, flags=kmc.FLAG_TEST_NARROW_FINGERPRINT)
    print(k, {x: (base.stats[x], res.stats[x]) for x in ("n_tiles", "n_big_tiles", "n_big_keys")})
    assert res.stats["n_big_tiles"] >= max(1000, 10 * base.stats["n_big_tiles"])
    assert res.stats["n_big_keys"] > base.stats["n_big_keys"]
    check_table(res, seq, off, k, pk, 2, 10**6)
    assert np.array_equal(res.keys, base.keys) and np.array_equal(res.counts, base.counts)
