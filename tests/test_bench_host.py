"""Host-side logic of bench.py (no GPU): the algorithmic bytes it attributes
to each kernel add up to the job's B_alg as the library computes it (input
once, 2-bit payload written and read once, keys written and read once, output
written once), the committed counter summaries are used only for the kernel
sources they were taken on, and runs on more than one GPU are refused."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def job_stats(k, n_reads, read_len, n_super, n_out, n_big_keys, n_big_out):
    n_kmers = n_reads * (read_len - k + 1)
    return {"n_bases": n_reads * read_len, "n_reads": n_reads, "n_superkmers": n_super,
            "n_kmers": n_kmers, "n_out": n_out, "n_big_keys": n_big_keys, "n_big_out": n_big_out}


def b_alg(st, k):
    # the library's figure (kmc_stats.bytes_alg), restated
    w = 8 if k <= 32 else 16
    payload = st["n_superkmers"] * 2 + (st["n_kmers"] + st["n_superkmers"] * (k - 1)) // 4
    return (st["n_bases"] + 8 * (st["n_reads"] + 1) + 2 * payload + 2 * w * st["n_kmers"]
            + (w + 4) * st["n_out"])


@pytest.mark.parametrize("k", [21, 28, 32, 33, 55, 64])
def test_kernel_bytes_add_up_to_the_job(k):
    st = job_stats(k, 1_000_000, 150, 2_600_000, 5_000_000, 20_000_000, 700_000)
    kb = lambda n: bench.kernel_bytes(n, st, k)
    # split, expansion and the two counting kernels move every byte of B_alg
    # once; the fine histogram re-reads the payload and the gather re-reads
    # the output, which B_alg does not count
    assert kb("split") + kb("expand_scatter") + kb("tile_sort") + kb("big_tiles") == b_alg(st, k)
    w = 8 if k <= 32 else 16
    assert kb("tile_sort") + kb("big_tiles") == w * st["n_kmers"] + (w + 4) * st["n_out"]
    assert kb("big_tiles") == w * st["n_big_keys"] + (w + 4) * st["n_big_out"]
    assert kb("assemble") == 2 * (w + 4) * st["n_out"]
    assert kb("no such kernel") == 0


def test_measured_traffic_follows_the_sources():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    recs = json.load(open(path))
    assert recs
    for key, rec in recs.items():
        workload, kernel = key.split(":")
        got = bench.measured_traffic(kernel, workload)
        if rec["source_sha256_16"] == bench.source_digest(kernel):
            assert got == rec["bytes_per_launch"] > 0
        else:
            assert got is None
    assert bench.measured_traffic("expand_scatter", "no-such-workload") is None
    assert bench.source_digest("no-such-kernel") == ""


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
