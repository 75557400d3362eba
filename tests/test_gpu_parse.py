"""Parsing on the device (kmc_parse): FASTQ, FASTA and multi-FASTA text into
CSR reads, equal to the oracle's parsers byte for byte, from host and device
text; malformed records rejected; parsed reads counted like the same reads
given directly."""
import numpy as np
import pytest

import oracle
from oracle import parse as P
from paper_1407_1507_amd import synth
from test_oracle_parse import fasta_text, fastq_text

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


def parse_both(ctx, kmc, text, fmt, on_device=False):
    import torch
    src = torch.from_numpy(np.frombuffer(text, dtype=np.uint8).copy()).to("cuda:0") \
        if on_device and text else text
    p = kmc.Parsed(ctx, src, fmt)
    seq, off = p.to_host()
    p.free()
    want = (P.parse_fastq if fmt == kmc.FORMAT_FASTQ or (fmt == kmc.FORMAT_AUTO and
                                                           text.lstrip()[:1] == b"@")
            else P.parse_fasta)(text)
    return (seq, off), want


LITERALS = [
    (1, b"@r1 first\nACGTN\n+\nIIIII\n@r2\r\nacgt\r\n+r2\r\n####\r\n@r3\n\n+\n\n@r4\nGGGA\n+\n!!!!"),
    (1, b"@r1\nACGT\n+\nIIII\n\n\n\n"),
    (2, b">chr1 desc\nACGT\nNNAC\r\n\nGG\n>empty\n>chr2\nTTTT"),
    (2, b"\n>a\nC\n\n\n"),
    (0, b"\n\n>a\nCCCC\n>b\nGG\n"),
    (0, b"@x\nAC\n+\n!!\n"),
    (2, b""),
    # trailing empty lines beyond the backward walk's 64 x 64 lines, and
    # texts of empty lines only
    (1, b"@r1\nACGT\n+\nIIII\n" + b"\n" * 5000),
    (2, b">a\nACGT\n" + b"\r\n" * 4200 + b"\r"),
    (2, b"\n" * 70),
    (2, b"\n" * 9000),
]


@pytest.mark.parametrize("fmt,text", LITERALS)
@pytest.mark.parametrize("on_device", [False, True])
def test_literal_records(ctx, kmc, fmt, text, on_device):
    (seq, off), (ws, wo) = parse_both(ctx, kmc, text, fmt, on_device)
    assert np.array_equal(seq, ws) and np.array_equal(off, wo)


@pytest.mark.parametrize("fmt,text", [
    (1, b"@r1\nACGT\n+\nIII\n"), (1, b"r1\nACGT\n+\nIIII\n"), (1, b"@r1\nACGT\n-\nIIII\n"),
    (1, b"@r1\nACGT\n+\n"), (2, b"ACGT\n>a\nC\n"), (0, b"ACGT\n")])
def test_malformed_rejected(ctx, kmc, fmt, text):
    with pytest.raises(kmc.KmcError) as e:
        kmc.Parsed(ctx, text, fmt)
    assert e.value.status == kmc.KMC_ERR_INVALID_ARG


@pytest.mark.parametrize("crlf", [False, True])
def test_fastq_workload(ctx, kmc, crlf):
    # 40 000 reads of the genome workload as FASTQ (several 16 KB chunks), from
    # host and from device text; the parsed reads count like the reads
    seq, off, p = synth.make("genome-5M-2Mx100", 0.02)
    text = fastq_text(seq, off, np.random.default_rng(3), crlf)
    for on_device in (False, True):
        (s2, o2), (ws, wo) = parse_both(ctx, kmc, text, kmc.FORMAT_FASTQ, on_device)
        assert np.array_equal(s2, seq) and np.array_equal(o2, off)
        assert np.array_equal(ws, seq) and np.array_equal(wo, off)
    parsed = kmc.Parsed(ctx, text)
    a = ctx.count(parsed, None, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    b = ctx.count(seq, off, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.counts, b.counts)
    parsed.free()


@pytest.mark.parametrize("width", [60, 80, 4096])
def test_multi_fasta(ctx, kmc, width):
    # records of 100 bp to 30 kbp (long reads take the position-per-lane scan
    # when their mean passes 2 kbp), wrapped at `width`
    seq, off = synth.sample_reads(5, synth.random_reference(6, 200_000), 300, (100, 30_000),
                                  0.01, 0.001)
    text = fasta_text(seq, off, width)
    (s2, o2), (ws, wo) = parse_both(ctx, kmc, text, kmc.FORMAT_AUTO, True)
    assert np.array_equal(s2, seq) and np.array_equal(o2, off)
    parsed = kmc.Parsed(ctx, text, kmc.FORMAT_FASTA)
    res = ctx.count(parsed, None, 28, 7, 256, 1, 2**32 - 1)
    ok_keys, ok_counts = oracle.count(seq, off, 28)
    order = np.argsort(res.keys)
    assert np.array_equal(res.keys[order], ok_keys)
    assert np.array_equal(res.counts[order], ok_counts)
    parsed.free()
