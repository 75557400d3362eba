"""The batched form at full size: the 256 uneven jobs of the batch workload
(n_reads = 10^U(4,6), reads of 100-250 bp from ~30x uniform references, 1%
substitutions, k drawn from {21, 25, 31, 47, 55}, p = 7, 512 bins, cutoffs
2..1e9; about 10 Gbases in all), counted in one batch call with device tables
as the benchmark runs it, each table equal entry for entry to the table of
the same job counted alone (kmc_count_ex, which the parity tests tie to the
oracle)."""
import ctypes
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from paper_1407_1507_amd import synth

pytestmark = pytest.mark.gpu

N_JOBS = 256


def _job(j):
    return synth.batch_job(j, 1.0)


@pytest.fixture(scope="module")
def kmc():
    from paper_1407_1507_amd import kmc as m
    m.lib()
    return m


def device_table(t):
    """Keys and counts of a device table, copied to host arrays."""
    hip = ctypes.CDLL("libamdhip64.so")
    keys = np.zeros(t.n * t.key_words, dtype=np.uint64)
    counts = np.zeros(t.n, dtype=np.uint32)
    if t.n:
        assert hip.hipMemcpy(ctypes.c_void_p(keys.ctypes.data), ctypes.c_void_p(t.keys_ptr),
                             ctypes.c_size_t(keys.nbytes), 2) == 0
        assert hip.hipMemcpy(ctypes.c_void_p(counts.ctypes.data), ctypes.c_void_p(t.counts_ptr),
                             ctypes.c_size_t(counts.nbytes), 2) == 0
    return (keys.reshape(-1, 2) if t.key_words == 2 else keys), counts


@pytest.mark.timeout(1200)
def test_batch_256_full_size_equals_single(kmc):
    import torch
    step = lambda m: print(f"[batch 256] {m}", flush=True)  # progress of a long test
    # inputs drawn in fresh interpreters (this process already holds the GPU)
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        jobs = list(ex.map(_job, range(N_JOBS)))
    bases = sum(int(o[-1]) for _, o, _ in jobs)
    step(f"generated {len(jobs)} jobs, {bases} bases")
    assert bases > 5e9 and len({p["k"] for _, _, p in jobs}) == 5
    ctx = kmc.Context(0)
    djobs = [(torch.from_numpy(s).to("cuda:0"), torch.from_numpy(o.view(np.int64)).to("cuda:0"),
              dict(p, flags=kmc.FLAG_DEVICE_TABLE)) for s, o, p in jobs]
    torch.cuda.synchronize()
    out = ctx.batch_count(djobs)
    step("batch counted")
    assert len(out) == N_JOBS
    for i, ((s, o, p), res) in enumerate(zip(djobs, out)):
        alone = ctx.count(s, o, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                          flags=kmc.FLAG_DEVICE_TABLE)
        assert res.n == alone.n and res.n > 0, i
        assert res.stats["n_kmers"] == alone.stats["n_kmers"], i
        assert np.array_equal(res.bin_offsets, alone.bin_offsets), i
        assert np.array_equal(res.sig_to_bin, alone.sig_to_bin), i
        a_keys, a_counts = device_table(alone)
        b_keys, b_counts = device_table(res)
        assert np.array_equal(a_keys, b_keys), i
        assert np.array_equal(a_counts, b_counts), i
        alone.free()
        res.free()
        if i % 32 == 31:
            step(f"{i + 1} jobs compared")
    ctx.close()
