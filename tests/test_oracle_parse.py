"""Pins for the oracle's FASTQ / FASTA parsers: literal records whose reads
are written out here, and round trips of generated read sets through
FASTQ and wrapped multi-FASTA text.  CPU only."""
import numpy as np
import pytest

from oracle import parse as P
from paper_1407_1507_amd import synth


def reads_of(seq, off):
    return [bytes(seq[int(off[i]):int(off[i + 1])]) for i in range(off.size - 1)]


def test_fastq_literal():
    text = (b"@r1 first\nACGTN\n+\nIIIII\n"
            b"@r2\r\nacgt\r\n+r2\r\n####\r\n"
            b"@r3\n\n+\n\n"            # an empty read
            b"@r4\nGGGA\n+\n!!!!")     # no final newline
    assert reads_of(*P.parse_fastq(text)) == [b"ACGTN", b"acgt", b"", b"GGGA"]
    assert reads_of(*P.parse_fastq(text + b"\n\n\n")) == [b"ACGTN", b"acgt", b"", b"GGGA"]
    assert reads_of(*P.parse_fastq(b"")) == []


@pytest.mark.parametrize("bad", [
    b"@r1\nACGT\n+\nIII\n",           # quality shorter than the sequence
    b"r1\nACGT\n+\nIIII\n",           # no '@'
    b"@r1\nACGT\n-\nIIII\n",          # no '+'
    b"@r1\nACGT\n+\n",                # ends inside a record
])
def test_fastq_malformed(bad):
    with pytest.raises(ValueError):
        P.parse_fastq(bad)


def test_fasta_literal():
    text = (b">chr1 desc\nACGT\nNNAC\r\n\nGG\n"
            b">empty\n"
            b">chr2\nTTTT")
    assert reads_of(*P.parse_fasta(text)) == [b"ACGTNNACGG", b"", b"TTTT"]
    assert reads_of(*P.parse_fasta(b"\n>a\nC\n\n\n")) == [b"C"]
    with pytest.raises(ValueError):
        P.parse_fasta(b"ACGT\n>a\nC\n")


def fastq_text(seq, off, rng, crlf=False):
    nl = b"\r\n" if crlf else b"\n"
    parts = []
    for i, r in enumerate(reads_of(seq, off)):
        q = bytes(rng.integers(33, 74, size=len(r), dtype=np.uint8))
        parts += [b"@read%d" % i, r, b"+", q]
    return nl.join(parts) + nl


def fasta_text(seq, off, width):
    parts = []
    for i, r in enumerate(reads_of(seq, off)):
        parts.append(b">rec%d some description" % i)
        parts += [r[j:j + width] for j in range(0, len(r), width)]
    return b"\n".join(parts) + b"\n"


@pytest.mark.parametrize("crlf", [False, True])
def test_fastq_round_trip(crlf):
    seq, off, _ = synth.make("genome-5M-2Mx100", 0.001)
    text = fastq_text(seq, off, np.random.default_rng(1), crlf)
    s2, o2 = P.parse_fastq(text)
    assert np.array_equal(s2, seq) and np.array_equal(o2, off)


@pytest.mark.parametrize("width", [60, 80, 1000])
def test_fasta_round_trip(width):
    seq, off = synth.sample_reads(3, synth.random_reference(2, 20_000), 40, (100, 3000), 0.01,
                                  0.01)
    s2, o2 = P.parse_fasta(fasta_text(seq, off, width))
    assert np.array_equal(s2, seq) and np.array_equal(o2, off)
