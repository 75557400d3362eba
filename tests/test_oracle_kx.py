"""Pins for the (k,x)-mer oracle (Methods, "(k,x)-mers"; Fig. 2 and the
counting from sorted (k,1)-mers): the figure's pieces, sorted order and
subarrays, the k-mer counts against brute force, and the invariants of the
pieces.  CPU only."""
from collections import Counter

import numpy as np
import pytest

from conftest import read_golden
from oracle import kxmers as KX
from oracle import strings as S


def fig2():
    rows = read_golden("fig2_kx_mers.txt")
    d = {}
    for r in rows:
        d.setdefault(r[0], []).append(r[1:])
    return d


def test_fig2_pieces():
    d = fig2()
    sk, k = d["superkmer"][0][0], int(d["k"][0][0])
    assert KX.pieces(sk, k, 1) == [r[0] for r in d["kx"]]


def test_fig2_sorted_and_subarrays():
    d = fig2()
    sk, k = d["superkmer"][0][0], int(d["k"][0][0])
    srt = KX.sort_pieces(KX.pieces(sk, k, 1))
    assert srt == [r[0] for r in d["sorted"]]
    st = KX.streams(srt, k)
    # R0: the 15-mers; R1: the prefixes of the 16-mers (stream x'=1, j=0);
    # R_X: the 16-mers beginning with X (stream x'=1, j=1, X)
    r0 = [s for s in srt if len(s) == k]
    assert r0 == d["R0"][0]
    r1 = [s for s in srt if len(s) == k + 1]
    assert r1 == d["R1"][0]
    assert st[(1, 0, "")] == [s[:k] for s in r1]
    for x, tag in zip("ACGT", ("RA", "RC", "RG", "RT")):
        group = [s for s in r1 if s[0] == x]
        assert group == d[tag][0]
        assert st.get((1, 1, x), []) == [s[1:] for s in group]


def test_fig2_counts_every_kmer_once():
    d = fig2()
    sk, k = d["superkmer"][0][0], int(d["k"][0][0])
    got = KX.count_sorted(KX.sort_pieces(KX.pieces(sk, k, 1)), k)
    want = sorted(Counter(S.canonical(sk[i:i + k]) for i in range(len(sk) - k + 1)).items())
    assert got == want and all(c == 1 for _, c in got)


def brute(reads, k, ci=1, cx=2**32 - 1):
    c = Counter()
    for r in reads:
        r = r.upper()
        for i in range(len(r) - k + 1):
            w = r[i:i + k]
            if all(ch in "ACGT" for ch in w):
                c[S.canonical(w)] += 1
    return sorted((y, n) for y, n in c.items() if ci <= n <= cx)


def rand_reads(seed, n, lo, hi, n_rate=0.0, repeat=None):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        L = int(rng.integers(lo, hi + 1))
        if repeat is not None and rng.random() < 0.5:
            a = int(rng.integers(0, max(1, len(repeat) - L)))
            s = list(repeat[a:a + L])
        else:
            s = list(rng.choice(list("ACGT"), size=L))
        for i in range(L):
            if rng.random() < n_rate:
                s[i] = "N"
        out.append("".join(s))
    return out


@pytest.mark.parametrize("k,p,x", [(5, 4, 1), (9, 4, 2), (15, 5, 3), (21, 7, 3), (12, 5, 1)])
def test_counts_equal_brute_force(k, p, x):
    rng = np.random.default_rng(k * 10 + x)
    rep = "".join(rng.choice(list("ACGT"), size=400))
    reads = rand_reads(k + x, 120, k - 2, 90, n_rate=0.01, repeat=rep)
    reads.append("ACGT" * 30)  # palindromic k-mers for even k
    assert KX.count(reads, k, p, x) == brute(reads, k)
    assert KX.count(reads, k, p, x, 2, 5) == brute(reads, k, 2, 5)


@pytest.mark.parametrize("k,p,x", [(15, 5, 1), (21, 7, 3), (28, 7, 3)])
def test_pieces_invariants(k, p, x):
    reads = rand_reads(7 + x, 60, 60, 150)
    for r in reads:
        for sk in KX.superkmers(r, k, p):
            ps = KX.pieces(sk, k, x)
            # every k-mer of the super k-mer in exactly one piece, canonical
            ks = [y for q in ps for y in (q[j:j + k] for j in range(len(q) - k + 1))]
            assert sorted(ks) == sorted(S.canonical(sk[i:i + k])
                                        for i in range(len(sk) - k + 1))
            assert all(S.canonical(y) == y for y in ks)
            assert all(k <= len(q) <= k + x for q in ps)
            # the fewest pieces: a piece only ends where the direction of the
            # next k-mer changes or the piece is full
            dirs = [KX.is_reverse(sk[i:i + k]) for i in range(len(sk) - k + 1)]
            pos = 0
            for q in ps:
                n = len(q) - k + 1
                assert len(set(dirs[pos:pos + n])) == 1
                if pos + n < len(dirs) and n < x + 1:
                    assert dirs[pos + n] != dirs[pos]
                pos += n


def test_superkmers_closed_after_w():
    # a run of one signature longer than w k-mers is cut into pieces of w
    k, p = 12, 4
    read = "ACGT" * 20  # repeats its minimal m-mer: long runs of one signature
    sks = KX.superkmers(read, k, p)
    assert all(len(s) - k + 1 <= k - p + 1 for s in sks)
    assert sum(len(s) - k + 1 for s in sks) == len(read) - k + 1


def test_sorted_fraction_about_half_at_x3():
    # random sequence: directions of neighbouring k-mers are near coin flips,
    # so pieces of up to four k-mers number about half the k-mers (the paper
    # reports ~0.5 at x = 3 on real reads)
    reads = rand_reads(3, 200, 150, 150)
    n_k = sum(len(r) - 28 + 1 for r in reads)
    n_p, _ = KX.entry_stats(reads, 28, 7, 3)
    assert 0.4 < n_p / n_k < 0.7
