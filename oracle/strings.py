"""String-level definitions from the paper, for worked examples and tiny inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Everything here works on
Python strings over A/C/G/T, so it shares no representation with either the C
oracle or the HIP path.

- reverse complement: reverse, then swap A<->T and C<->G (Fig. 1 pairs such as
  CGTT -> AACG);
- canonical form: the lexicographically smaller of a string and its reverse
  complement (Methods, "Minimizers of k-mers");
- signature: the smallest canonical m-mer of the k-mer that neither starts
  with AAA nor with ACA and holds no AA except at its start (Methods, "From
  minimizers to signatures"); plain canonical minimizers drop that filter;
- super k-mer: a maximal run of consecutive k-mers of a read that share one
  signature, written as one string (Methods, "Sketch of the algorithm", Fig. 1).
"""
from __future__ import annotations

_COMP = str.maketrans("ACGT", "TGCA")
CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def revcomp(s: str) -> str:
    return s.translate(_COMP)[::-1]


def canonical(s: str) -> str:
    r = revcomp(s)
    return s if s <= r else r


def allowed(mmer: str) -> bool:
    """Filter applied to a canonical m-mer (Methods, signatures)."""
    if mmer.startswith("AAA") or mmer.startswith("ACA"):
        return False
    return "AA" not in mmer[1:]


def signature(kmer: str, m: int, filter: bool = True) -> str | None:
    """Smallest allowed canonical m-mer of kmer; None if no m-mer is allowed."""
    cands = [canonical(kmer[i:i + m]) for i in range(len(kmer) - m + 1)]
    if filter:
        cands = [c for c in cands if allowed(c)]
    return min(cands) if cands else None


def encode(s: str) -> int:
    """Pack a string, leftmost symbol most significant, A=0 C=1 G=2 T=3."""
    v = 0
    for ch in s:
        v = v * 4 + CODE[ch]
    return v


def superkmers(read: str, k: int, m: int, filter: bool = True):
    """Split read (A/C/G/T only) into maximal runs of k-mers of equal signature.

    Returns a list of (super k-mer string, signature string)."""
    out = []
    start = 0
    cur = None
    n = len(read) - k + 1
    for j in range(n):
        s = signature(read[j:j + k], m, filter)
        if j == 0:
            cur = s
        elif s != cur:
            out.append((read[start:j - 1 + k], cur))
            start, cur = j, s
    if n > 0:
        out.append((read[start:n - 1 + k], cur))
    return out
