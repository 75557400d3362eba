"""Plain parsers of FASTQ and FASTA text (the input the paper's distribution
phase reads: Methods, "Sketch of the algorithm"; Additional features).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Line by line over
Python bytes, with the readings the library states: lines end with b"\\n" and
a b"\\r" before it is dropped; the last line may lack its b"\\n"; trailing
empty lines are ignored.  FASTQ: records of four lines (b"@" header, sequence,
b"+" line, quality of the sequence's length), one read per sequence line.
FASTA: a line starting with b">" opens a record whose read is its following
lines joined, up to the next header.  Returns (seq, offsets) in the
library's CSR form, or raises ValueError for malformed input.
"""
from __future__ import annotations

import numpy as np


def _lines(text: bytes):
    lines = text.split(b"\n")
    if text.endswith(b"\n"):
        lines.pop()  # the terminator of the last line, not an empty line
    lines = [ln[:-1] if ln.endswith(b"\r") else ln for ln in lines]
    while lines and lines[-1] == b"":
        lines.pop()
    return lines


def _csr(reads):
    off = np.zeros(len(reads) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(r) for r in reads]) if reads else []
    seq = np.frombuffer(b"".join(reads), dtype=np.uint8).copy()
    return seq, off


def parse_fastq(text: bytes):
    lines = _lines(text)
    if len(lines) % 4:
        raise ValueError("FASTQ text ends inside a record")
    reads = []
    for r in range(0, len(lines), 4):
        head, s, plus, qual = lines[r:r + 4]
        if not head.startswith(b"@") or not plus.startswith(b"+") or len(qual) != len(s):
            raise ValueError(f"malformed FASTQ record at line {r + 1}")
        reads.append(s)
    return _csr(reads)


def parse_fasta(text: bytes):
    reads = []
    for i, ln in enumerate(_lines(text)):
        if ln.startswith(b">"):
            reads.append([])
        elif ln:
            if not reads:
                raise ValueError(f"FASTA sequence before a header at line {i + 1}")
            reads[-1].append(ln)
    return _csr([b"".join(parts) for parts in reads])
