"""Seeded synthetic read sets shaped like the paper's workloads.

This module only makes inputs: random references and reads sampled from them
(with substitution errors, N bases and random strand).  It computes nothing
of the counting method and is shared by the tests, the benchmark and the
smoke check.  All randomness comes from numpy's PCG64 with the stated seed,
and read sets are returned as the library's CSR form: ``seq`` (uint8 ASCII,
upper case) and ``offsets`` (uint64, n_reads + 1, offsets[0] = 0).

Workloads (reads ~100-150 bp, ~30-40x coverage, k = 28 / 55 as in the paper's
experiments; the paper's own datasets are not used, these stand in for them):

- ``uniform``: i.i.d. uniform A/C/G/T reads, no reference, no N.
- ``genome``: uniform random reference; each read takes a uniform start,
  a fair-coin strand (reverse complemented if set), then each base is
  substituted with probability ``err`` by one of the other three uniformly,
  then set to N with probability ``n_rate`` -- in that order.
- ``repeat_reference``: a uniform reference with a fraction overwritten by
  repeat families (unit length U{1000..5000}; half interspersed with 2-10
  copies, half tandem arrays of 2-20 adjacent copies; each copy diverged by
  d ~ U[0, 0.10] substitutions).
- ``batch_job`` / ``served_job``: the uneven jobs of the batched form and the
  arrivals of the served form.
- ``large-300M-60Mx150``: the served form's large job, 60M reads x 150 bp
  (9 Gbases) from a uniform 300 Mbp reference, drawn in chunks of 2^20
  reads, chunk c with seed (500, 1, c).
"""
from __future__ import annotations

import hashlib

import numpy as np

GENERATOR_VERSION = 1
_ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)
_N = ord("N")


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, (tuple, list)):
        return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    return np.random.Generator(np.random.PCG64(seed))


def _substitute(rng, codes: np.ndarray, rate: float) -> None:
    """In place: each entry replaced with probability rate by another symbol."""
    if rate <= 0:
        return
    hit = rng.random(codes.shape, dtype=np.float32) < rate
    shift = rng.integers(1, 4, size=int(hit.sum()), dtype=np.uint8)
    codes[hit] = (codes[hit] + shift) & 3


def random_reference(seed, length: int) -> np.ndarray:
    """Uniform i.i.d. reference as 2-bit codes (uint8 0..3)."""
    return _rng(seed).integers(0, 4, size=length, dtype=np.uint8)


def repeat_reference(seed, length: int, repeat_fraction: float = 0.2) -> np.ndarray:
    """Uniform reference with repeat_fraction of it overwritten by repeat families."""
    rng = _rng(seed)
    ref = rng.integers(0, 4, size=length, dtype=np.uint8)
    target = int(repeat_fraction * length)
    written = 0
    fam = 0
    while written < target:
        ulen = int(rng.integers(1000, 5001))
        unit = rng.integers(0, 4, size=ulen, dtype=np.uint8)
        tandem = (fam % 2) == 1
        ncopy = int(rng.integers(2, 21)) if tandem else int(rng.integers(2, 11))
        if tandem:
            span = ulen * ncopy
            if span >= length:
                ncopy = max(1, length // ulen - 1)
                span = ulen * ncopy
            start = int(rng.integers(0, length - span + 1))
            starts = [start + c * ulen for c in range(ncopy)]
        else:
            starts = [int(rng.integers(0, length - ulen + 1)) for _ in range(ncopy)]
        for s in starts:
            copy = unit.copy()
            _substitute(rng, copy, float(rng.uniform(0.0, 0.10)))
            ref[s:s + ulen] = copy
            written += ulen
        fam += 1
    return ref


def sample_reads(seed, ref: np.ndarray, n_reads: int, read_len, err: float,
                 n_rate: float, chunk: int = 1 << 20):
    """Reads sampled from ref (2-bit codes).  read_len: int or (lo, hi) inclusive."""
    rng = _rng(seed)
    if isinstance(read_len, tuple):
        lens = rng.integers(read_len[0], read_len[1] + 1, size=n_reads).astype(np.uint64)
    else:
        lens = np.full(n_reads, read_len, dtype=np.uint64)
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    seq = np.empty(int(offsets[-1]), dtype=np.uint8)
    L = ref.size
    for c0 in range(0, n_reads, chunk):
        c1 = min(n_reads, c0 + chunk)
        cl = lens[c0:c1].astype(np.int64)
        maxl = int(cl.max()) if cl.size else 0
        starts = rng.integers(0, np.maximum(L - cl + 1, 1))
        strand = rng.random(c1 - c0) < 0.5
        idx = starts[:, None] + np.arange(maxl)[None, :]
        np.minimum(idx, L - 1, out=idx)
        reads = ref[idx]
        # reverse strand: reverse the read's own bases, complement (code 3 - c)
        if strand.any():
            rs = reads[strand]
            rl = cl[strand]
            ridx = (rl[:, None] - 1 - np.arange(maxl)[None, :])
            ridx = np.where(ridx >= 0, ridx, 0)
            reads[strand] = 3 - np.take_along_axis(rs, ridx, axis=1)
        _substitute(rng, reads, err)
        ascii_ = _ASCII[reads]
        if n_rate > 0:
            ascii_[rng.random(reads.shape, dtype=np.float32) < n_rate] = _N
        valid = np.arange(maxl)[None, :] < cl[:, None]
        seq[int(offsets[c0]):int(offsets[c1])] = ascii_[valid]
    return seq, offsets


_SHARED_REF = None  # reference of the chunked generator, inherited by forked workers


def _reads_chunk(task):
    seed, c, n, read_len, err, n_rate = task
    return sample_reads((*seed, c), _SHARED_REF, n, read_len, err, n_rate)


def sample_reads_chunked(seed, ref: np.ndarray, n_reads: int, read_len: int, err: float,
                         n_rate: float, chunk: int = 1 << 20, workers: int = 0):
    """Reads like sample_reads, in chunks of ``chunk`` reads, chunk c drawn
    with seed (*seed, c) (so the chunks can be drawn by parallel processes);
    the read set is the chunks in order."""
    global _SHARED_REF
    import os
    workers = workers or min(16, os.cpu_count() or 1)
    tasks = [(tuple(seed), c, min(chunk, n_reads - c0), read_len, err, n_rate)
             for c, c0 in enumerate(range(0, n_reads, chunk))]
    _SHARED_REF = ref
    try:
        if workers > 1 and len(tasks) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(min(workers, len(tasks))) as pool:
                parts = pool.map(_reads_chunk, tasks, chunksize=1)
        else:
            parts = [_reads_chunk(t) for t in tasks]
    finally:
        _SHARED_REF = None
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    seq = np.empty(sum(int(pt[1][-1]) for pt in parts), dtype=np.uint8)
    r = b = 0
    for ps, po in parts:
        m = po.size - 1
        offsets[r + 1:r + m + 1] = po[1:] + np.uint64(b)
        seq[b:b + ps.size] = ps
        r += m
        b += ps.size
    return seq, offsets


def uniform_reads(seed, n_reads: int, read_len: int):
    rng = _rng(seed)
    codes = rng.integers(0, 4, size=n_reads * read_len, dtype=np.uint8)
    offsets = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(read_len)
    return _ASCII[codes], offsets


def digest(seq: np.ndarray, offsets: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets).tobytes())
    h.update(np.ascontiguousarray(seq).tobytes())
    return h.hexdigest()


# Named workloads: (generator, counting parameters).
CONFIGS = {
    "uniform-10k": dict(k=28, p=7, n_bins=512, cutoff_min=1, cutoff_max=10**9),
    "genome-5M-2Mx100": dict(k=28, p=7, n_bins=512, cutoff_min=2, cutoff_max=10**9),
    "repeats-50M-30x150-k55": dict(k=55, p=9, n_bins=1024, cutoff_min=2, cutoff_max=10**6),
    # the served form's large job: 3.5M keys per bin on average at 2048 bins,
    # but the most frequent signatures alone hold up to 19M each
    "large-300M-60Mx150": dict(k=28, p=7, n_bins=2048, cutoff_min=2, cutoff_max=10**9),
}


def batch_job(j: int, scale: float = 1.0):
    """Job j of the batch of uneven jobs: n_reads = floor(10^U(4,6)) (times
    scale), read lengths U{100..250}, a uniform reference of
    max(10^4, n_reads * 175 / 30) bases (about 30x), 1% substitutions, no N;
    k drawn from {21, 25, 31, 47, 55}, p = 7, 512 bins, cutoffs 2..10^9.
    Seeds (4, j, 0..2).  Returns (seq, offsets, params)."""
    rng = _rng((4, j, 0))
    n_reads = max(1, int(10 ** rng.uniform(4, 6) * scale))
    k = int(rng.choice([21, 25, 31, 47, 55]))
    ref = random_reference((4, j, 1), max(10_000, int(n_reads * 175 / 30)))
    seq, off = sample_reads((4, j, 2), ref, n_reads, (100, 250), err=0.01, n_rate=0.0)
    return seq, off, dict(k=k, p=7, n_bins=512, cutoff_min=2, cutoff_max=10**9)


def served_job(i: int, scale: float = 1.0):
    """Served job i: the repeat-rich generator with a reference whose length
    is log-uniform in [5, 50] Mbp (times scale), 30x of 150 bp reads, 0.5%
    substitutions, 0.1% N; k = 55, p = 9, 1024 bins, cutoffs 2..10^6.
    Seeds (5, i, 0..2).  Returns (seq, offsets, params)."""
    rng = _rng((5, i, 0))
    length = max(20_000, int(10 ** rng.uniform(np.log10(5e6), np.log10(5e7)) * scale))
    ref = repeat_reference((5, i, 1), length)
    seq, off = sample_reads((5, i, 2), ref, max(1, length * 30 // 150), 150,
                            err=0.005, n_rate=0.001)
    return seq, off, dict(CONFIGS["repeats-50M-30x150-k55"])


def make(name: str, scale: float = 1.0):
    """Build a named workload.  scale < 1 shrinks read count and reference
    (same generator, same shape) for quick tests.  Returns (seq, offsets, params)."""
    params = dict(CONFIGS[name])
    if name == "uniform-10k":
        n = max(1, int(10_000 * scale))
        seq, off = uniform_reads(1, n, 100)
    elif name == "genome-5M-2Mx100":
        ref = random_reference((2, 0), max(1000, int(5_000_000 * scale)))
        seq, off = sample_reads((2, 1), ref, max(1, int(2_000_000 * scale)), 100,
                                err=0.01, n_rate=0.0005)
    elif name == "repeats-50M-30x150-k55":
        ref = repeat_reference((3, 0), max(20_000, int(50_000_000 * scale)))
        seq, off = sample_reads((3, 1), ref, max(1, int(10_000_000 * scale)), 150,
                                err=0.005, n_rate=0.001)
    elif name == "large-300M-60Mx150":
        ref = random_reference((500, 0), max(1000, int(300_000_000 * scale)))
        seq, off = sample_reads_chunked((500, 1), ref, max(1, int(60_000_000 * scale)), 150,
                                        err=0.005, n_rate=0.001)
    else:
        raise KeyError(name)
    return seq, off, params
