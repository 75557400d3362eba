"""(k,x)-mers, at the string level, for worked examples and small inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
paper: Methods, "(k,x)-mers", and the counting from sorted (k,1)-mers that
follows Fig. 2, generalized to x <= 3 as the paper states its real
implementation does.

- direction of a k-mer: reverse when its reverse complement is smaller, else
  forward (a palindrome is forward);
- pieces of a super k-mer: walking its k-mers in order, a piece grows while
  the next k-mer has the direction of the piece's first k-mer and the piece
  holds at most x + 1 k-mers; a forward piece is kept as read, a reverse
  piece as its reverse complement, so all k-mers inside a piece are
  canonical, no k-mer is in two neighbouring pieces and every k-mer is in one
  (the fewest pieces: a piece can only end where the direction changes or the
  size limit is reached);
- sorted order: the k-mers first (R0), then the (k+1)-mers, and so on, each
  group lexicographically (Fig. 2: R0 above R1 = R_A, R_C, R_G, R_T);
- streams: within the group of (k+x')-mers, the pieces that begin with the
  same j symbols are consecutive, and their k-mers at offset j come in sorted
  order; the k-mers of all pieces are the union of these streams (for x = 1:
  R0, R1 for the prefixes, R_A .. R_T for the suffixes, the six subarrays);
- counting: a merge of the streams, counting runs of equal k-mers.

Super k-mers come from oracle.strings (maximal runs of k-mers of one
signature); as in the build, a run is also closed after w = k - p + 1 k-mers
(the cut points do not change any k-mer count, but they decide the pieces),
and bases other than A/C/G/T (either case) end a run.
"""
from __future__ import annotations

import heapq
from collections import Counter

from . import strings


def is_reverse(kmer: str) -> bool:
    return strings.revcomp(kmer) < kmer


def pieces(superkmer: str, k: int, x: int) -> list[str]:
    """The (k,x)-mers of one super k-mer, in order along it."""
    n = len(superkmer) - k + 1
    rev = [is_reverse(superkmer[i:i + k]) for i in range(n)]
    out = []
    i = 0
    while i < n:
        j = i + 1
        while j < n and j - i < x + 1 and rev[j] == rev[i]:
            j += 1
        s = superkmer[i:j - 1 + k]
        out.append(strings.revcomp(s) if rev[i] else s)
        i = j
    return out


def sort_pieces(ps: list[str]) -> list[str]:
    return sorted(ps, key=lambda s: (len(s), s))


def streams(sorted_ps: list[str], k: int) -> dict:
    """(x', j, first j symbols) -> the offset-j k-mers of those pieces, in the
    order of sorted_ps."""
    st: dict = {}
    for s in sorted_ps:
        xp = len(s) - k
        for j in range(xp + 1):
            st.setdefault((xp, j, s[:j]), []).append(s[j:j + k])
    return st


def count_sorted(sorted_ps: list[str], k: int) -> list[tuple[str, int]]:
    """k-mer counts from sorted pieces: merge of the streams, runs counted.
    Raises if a stream is out of order (the property the merge relies on)."""
    st = streams(sorted_ps, k)
    for key, seq in st.items():
        if any(a > b for a, b in zip(seq, seq[1:])):
            raise AssertionError(f"stream {key} is not sorted")
    out: list[tuple[str, int]] = []
    for y in heapq.merge(*st.values()):
        if out and out[-1][0] == y:
            out[-1] = (y, out[-1][1] + 1)
        else:
            out.append((y, 1))
    return out


def superkmers(read: str, k: int, p: int, filter: bool = True) -> list[str]:
    """Super k-mers of a read as the build cuts them (see the module note)."""
    w = k - p + 1
    out = []
    seg = []
    for ch in read.upper() + "N":
        if ch in "ACGT":
            seg.append(ch)
            continue
        if len(seg) >= k:
            for sk, _ in strings.superkmers("".join(seg), k, p, filter):
                n = len(sk) - k + 1
                for a in range(0, n, w):
                    b = min(n, a + w)
                    out.append(sk[a:b - 1 + k])
        seg = []
    return out


def read_pieces(reads: list[str], k: int, p: int, x: int) -> list[str]:
    return [q for r in reads for s in superkmers(r, k, p) for q in pieces(s, k, x)]


def count(reads: list[str], k: int, p: int, x: int, cutoff_min: int = 1,
          cutoff_max: int = 2**32 - 1) -> list[tuple[str, int]]:
    """Canonical k-mer counts of the reads through (k,x)-mers, cutoffs
    applied, ascending."""
    ps = sort_pieces(read_pieces(reads, k, p, x))
    return [(y, c) for y, c in count_sorted(ps, k) if cutoff_min <= c <= cutoff_max]


def entry_stats(reads: list[str], k: int, p: int, x: int) -> tuple[int, int]:
    """(pieces, distinct pieces) of the reads."""
    ps = read_pieces(reads, k, p, x)
    return len(ps), len(Counter(ps))
