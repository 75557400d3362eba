"""Plain CPU oracle for canonical k-mer counting (KMC 2, Deorowicz et al.).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
It shares no code with the HIP path.

``count`` is the plain definition the paper's method reaches exactly: every
window of every read that holds only A/C/G/T gives its canonical k-mer (the
smaller of the k-mer and its reverse complement, Methods, "Minimizers of
k-mers"); keys are sorted, run-length counted and kept iff
``cutoff_min <= count <= cutoff_max`` (supplement, -ci/-cx options), in
ascending key order.  Symbols are coded A=0 C=1 G=2 T=3, leftmost symbol most
significant (supplement, database [map] example).

``key_signatures`` / ``window_signatures`` compute the signature of a k-mer
(Methods, "From minimizers to signatures") at the level of its symbols, to
audit where the GPU path placed each k-mer.  ``strings`` holds the same
definitions over Python strings, for the paper's worked examples.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmc_oracle.c")
_LIB = os.path.join(_HERE, "libkmc_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/libkmc_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.kmc_oracle_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(u64p), ctypes.POINTER(u32p)]
        lib.kmc_oracle_count.restype = ctypes.c_int
        lib.kmc_oracle_count_slice.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                               ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_uint32, ctypes.c_uint64,
                                               ctypes.POINTER(ctypes.c_uint64),
                                               ctypes.POINTER(u64p), ctypes.POINTER(u32p)]
        lib.kmc_oracle_count_slice.restype = ctypes.c_int
        lib.kmc_oracle_valid_windows.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_uint64, ctypes.c_uint32]
        lib.kmc_oracle_valid_windows.restype = ctypes.c_uint64
        lib.kmc_oracle_key_signatures.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                                  ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        lib.kmc_oracle_key_signatures.restype = ctypes.c_int
        lib.kmc_oracle_window_signatures.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                                     ctypes.c_uint64, ctypes.c_uint32,
                                                     ctypes.c_uint32, ctypes.c_int,
                                                     ctypes.c_void_p]
        lib.kmc_oracle_window_signatures.restype = ctypes.c_int
        lib.kmc_oracle_count_keys.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        lib.kmc_oracle_count_keys.restype = ctypes.c_int
        lib.kmc_oracle_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _reads(seq, offsets):
    seq = np.ascontiguousarray(np.asarray(seq, dtype=np.uint8))
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if offsets.ndim != 1 or offsets.size < 1 or offsets[0] != 0:
        raise ValueError("offsets must start at 0")
    if np.any(offsets[1:] < offsets[:-1]) or int(offsets[-1]) > seq.size:
        raise ValueError("offsets must be non-decreasing and within seq")
    return seq, offsets


def count(seq, offsets, k: int, cutoff_min: int = 1, cutoff_max: int = 2**32 - 1,
          threads: int = 1, canonical: bool = True, counter_max: int = 0,
          slice_bits: int = 0, slice: int = 0):
    """Return (keys, counts): keys is uint64 [n] (k <= 32) or [n, 2] (hi, lo).
    canonical=False counts k-mers as read (supplement, -b); counter_max > 0
    stores min(count, counter_max), the cutoffs applying to the exact count
    (supplement, -cs).  slice_bits > 0 keeps only the keys whose top
    slice_bits bits (of the 2k-bit key) equal slice: that part of the whole
    count, in memory proportional to it."""
    seq, offsets = _reads(seq, offsets)
    lib = _load()
    n = ctypes.c_uint64(0)
    kp = ctypes.POINTER(ctypes.c_uint64)()
    cp = ctypes.POINTER(ctypes.c_uint32)()
    rc = lib.kmc_oracle_count_slice(seq.ctypes.data, offsets.ctypes.data, offsets.size - 1, k,
                                    cutoff_min, cutoff_max, int(canonical), threads, slice_bits,
                                    slice, ctypes.byref(n), ctypes.byref(kp), ctypes.byref(cp))
    if rc != 0:
        raise ValueError(f"oracle count failed ({rc})")
    kw = 1 if k <= 32 else 2
    m = n.value
    keys = np.ctypeslib.as_array(kp, shape=(max(m * kw, 1),))[: m * kw].copy()
    counts = np.ctypeslib.as_array(cp, shape=(max(m, 1),))[:m].copy()
    lib.kmc_oracle_free(ctypes.cast(kp, ctypes.c_void_p))
    lib.kmc_oracle_free(ctypes.cast(cp, ctypes.c_void_p))
    if kw == 2:
        keys = keys.reshape(m, 2)
    if counter_max:
        counts = np.minimum(counts, np.uint32(counter_max))
    return keys, counts


def count_keys(seq, offsets, k: int, keys, threads: int = 1) -> np.ndarray:
    """Occurrences (over every valid window, canonical form) of each given key
    (uint64 [n] or [n, 2]); for sampled checks of tables too large to sort."""
    seq, offsets = _reads(seq, offsets)
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    kw = 1 if k <= 32 else 2
    n = keys.shape[0] if keys.ndim > 0 else 0
    out = np.zeros(max(n, 1), dtype=np.uint64)
    rc = _load().kmc_oracle_count_keys(seq.ctypes.data, offsets.ctypes.data, offsets.size - 1,
                                       k, keys.ctypes.data if n else None, n, kw, threads,
                                       out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle count_keys failed ({rc})")
    return out[:n]


def valid_windows(seq, offsets, k: int) -> int:
    """Closed form: sum over maximal valid runs of length L of max(0, L-k+1)."""
    seq, offsets = _reads(seq, offsets)
    return int(_load().kmc_oracle_valid_windows(seq.ctypes.data, offsets.ctypes.data,
                                                offsets.size - 1, k))


def key_signatures(keys, k: int, m: int, filter: bool = True) -> np.ndarray:
    """Signature of every packed canonical key (uint64 [n] or [n, 2])."""
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    kw = 1 if k <= 32 else 2
    n = keys.shape[0] if keys.ndim > 0 else 0
    out = np.zeros(max(n, 1), dtype=np.uint32)
    rc = _load().kmc_oracle_key_signatures(keys.ctypes.data, n, kw, k, m, int(filter),
                                           out.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return out[:n]


def window_signatures(seq, offsets, k: int, m: int, filter: bool = True) -> np.ndarray:
    """Signature of the window starting at each byte (0xFFFFFFFF if invalid)."""
    seq, offsets = _reads(seq, offsets)
    nb = int(offsets[-1])
    out = np.zeros(max(nb, 1), dtype=np.uint32)
    rc = _load().kmc_oracle_window_signatures(seq.ctypes.data, offsets.ctypes.data,
                                              offsets.size - 1, k, m, int(filter),
                                              out.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return out[:nb]
