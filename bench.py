"""Benchmark: one k-mer counting job per step on one MI355X.

A step is one whole pass of the counting path (signature histogram and map,
split and scatter of super k-mers into bins, per-bin key expansion, tile sort,
run-length counting with cutoffs, table assembly) over one synthetic read set
already resident in HBM; the table is left in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("input bases/sec and k-mers/sec per MI355X; achieved HBM GB/s; "
          "p50/p99 job latency")
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "repeats-50M-30x150-k55"
ALSO = ["genome-5M-2Mx100"]
DESCRIPTION = {
    "genome-5M-2Mx100": ("2,000,000 reads x 100 bp sampled (random strand) from a uniform "
                         "5 Mbp reference, 1% substitutions, 0.05% N; k=28, p=7, 512 bins, "
                         "cutoff_min=2, cutoff_max=1e9 (about 40x coverage)"),
    "uniform-10k": "10,000 i.i.d. uniform reads x 100 bp; k=28, p=7, 512 bins, cutoff_min=1",
    "repeats-50M-30x150-k55": ("10,000,000 reads x 150 bp from a 50 Mbp reference with 20% "
                               "repeat families, 0.5% substitutions, 0.1% N; k=55, p=9, "
                               "1024 bins, cutoff_min=2, cutoff_max=1e6"),
    "large-300M-60Mx150": ("60,000,000 reads x 150 bp (9 Gbases) from a uniform 300 Mbp "
                           "reference, 0.5% substitutions, 0.1% N; k=28, p=7, 2048 bins, "
                           "cutoff_min=2, cutoff_max=1e9 (the served form's large job, "
                           "alone)"),
}


def kernel_bytes(name: str, st: dict, k: int) -> int:
    """Algorithmic HBM bytes of one launch of a kernel (what the method must
    move through it, not what the implementation happens to move)."""
    w = 8 if k <= 32 else 16
    inp = st["n_bases"] + 8 * (st["n_reads"] + 1)
    payload = 2 * st["n_superkmers"] + (st["n_kmers"] + st["n_superkmers"] * (k - 1)) // 4
    keys = w * st["n_kmers"]
    out = (w + 4) * st["n_out"]
    # the tile kernel reads the keys of the LDS tiles and writes their entries;
    # the big-tile kernel those of the tiles counted through HBM
    big_keys, big_out = w * st["n_big_keys"], (w + 4) * st["n_big_out"]
    return {
        "split": inp + payload,
        "fine_hist": payload,
        "expand_scatter": payload + keys,
        "tile_sort": keys - big_keys + out - big_out,
        "big_tiles": big_keys + big_out,
        "assemble": 2 * out,
    }.get(name, 0)


# the source files of each timed kernel (for staleness of traffic counters):
# its own file(s) and the shared device headers
_SHARED = ("kmc_device.h", "kmc_internal.h")
KERNEL_SOURCE = {
    "split": ("kmc_split.hip", "kmc_scan_wide.hip"), "sig_hist": ("kmc_split.hip",),
    "fine_hist": ("kmc_expand.hip",), "plan_tiles": ("kmc_expand.hip",),
    "expand_scatter": ("kmc_expand.hip",), "tile_sort": ("kmc_sort.hip",),
    "big_tiles": ("kmc_sort.hip",), "assemble": ("kmc_sort.hip",),
}


def source_digest(kernel: str) -> str:
    """First 16 hex digits of the SHA-256 of the kernel's source files."""
    import hashlib
    files = KERNEL_SOURCE.get(kernel)
    if not files:
        return ""
    h = hashlib.sha256()
    for f in files + _SHARED:
        path = os.path.join(ROOT, "paper_1407_1507_amd", "csrc", f)
        if not os.path.isfile(path):
            return ""
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None if absent or taken on a different version of the kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.isfile(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}:{kernel}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256_16") != source_digest(kernel):
        return None
    return rec.get("bytes_per_launch")


def copy_calibration(nbytes: int):
    """A plain device-to-device copy of nbytes (one kernel), for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


def host_cpu() -> str:
    """The host CPU's model name and logical core count."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model or 'unknown CPU'}, {os.cpu_count()} logical cores"


def _oracle_rate(seq, off, p, threads: int, budget_s: float):
    """Bases/s of the oracle on a prefix of the reads sized to about budget_s."""
    import oracle
    n_reads = off.size - 1
    # calibrate on a small prefix, then run the sized sample once
    n0 = max(1, min(n_reads, 20_000 if threads == 1 else n_reads // 100))
    t = time.perf_counter()
    oracle.count(seq[: int(off[n0])], off[: n0 + 1], p["k"], p["cutoff_min"], p["cutoff_max"],
                 threads=threads)
    dt0 = time.perf_counter() - t
    n = int(min(n_reads, max(n0, n0 * budget_s / max(dt0, 1e-3))))
    s, o = seq[: int(off[n])], off[: n + 1]
    t = time.perf_counter()
    oracle.count(s, o, p["k"], p["cutoff_min"], p["cutoff_max"], threads=threads)
    dt = time.perf_counter() - t
    return float(o[-1]) / dt, n, int(o[-1]), dt


def cpu_baseline(seq, off, p, budget_s: float = 15.0):
    """The oracle, as it stands, on a prefix of the same read set sized to
    about budget_s of CPU time on all host cores, and on one thread (a smaller
    prefix, about budget_s / 3)."""
    import oracle
    oracle.build(force=False)
    cores = os.cpu_count() or 1
    n_reads = off.size - 1
    v, n, b, dt = _oracle_rate(seq, off, p, cores, budget_s)
    v1, n1, b1, dt1 = _oracle_rate(seq, off, p, 1, budget_s / 3)
    return {"value": v, "unit": "bases/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {n_reads} reads ({b} bases), {dt:.2f} s, "
                      f"{cores} threads",
            "host": host_cpu(),
            "one_thread": {"value": v1, "unit": "bases/s", "cores": 1,
                           "sample": f"first {n1} of {n_reads} reads ({b1} bases), "
                                     f"{dt1:.2f} s, 1 thread"}}


def copy_peak(nbytes: int = 2 << 30, reps: int = 10) -> float:
    """Measured HBM rate of a plain device-to-device copy (GB/s, read + write
    bytes), beside the nominal peak."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _gen(task):
    from paper_1407_1507_amd import synth
    kind, i, scale = task
    return (synth.batch_job if kind == "batch" else synth.served_job)(i, scale)


def generate(kind: str, n: int, scale: float):
    """Jobs 0..n-1 of a generator, built in parallel host processes (before
    this process touches the GPU)."""
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1, n))
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_gen, [(kind, i, scale) for i in range(n)]))


def to_device(jobs):
    import torch
    out = []
    for seq, off, p in jobs:
        out.append((torch.from_numpy(seq).to("cuda:0"),
                    torch.from_numpy(off.view(np.int64)).to("cuda:0"), p))
    torch.cuda.synchronize()
    return out


def bench_batch(args):
    """The batched form: one step = one kmc_batch_count over every job."""
    jobs = generate("batch", args.batch_jobs, args.batch_scale)
    import torch
    from paper_1407_1507_amd import kmc
    djobs = to_device(jobs)
    bases = int(sum(int(o[-1]) for _, o, _ in jobs))
    ctx = kmc.Context(0)
    prm = [dict(p, flags=kmc.FLAG_DEVICE_TABLE) for _, _, p in djobs]
    batch = [(s, o, q) for (s, o, _), q in zip(djobs, prm)]

    def timed_batches():
        for _ in range(args.warmup):
            for r in ctx.batch_count(batch):
                r.free()
        torch.cuda.synchronize()
        times, kmers = [], 0
        for _ in range(args.steps):
            t = time.perf_counter()
            res = ctx.batch_count(batch)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            kmers = sum(r.stats["n_kmers"] for r in res)
            for r in res:
                r.free()
        return times, kmers

    untuned_times, _ = timed_batches()
    # the autotuner picks knobs per job class (the largest job of each class
    # counted with every candidate) and the pool's stream count, outside the
    # timed region; then the batch is timed again
    t = time.perf_counter()
    tune = ctx.autotune(batch)
    tune_s = time.perf_counter() - t
    times, kmers = timed_batches()
    # the plain per-job launch: the same jobs one after another on one
    # stream, on a context with the default knobs (a warm pass, then timed)
    plain = kmc.Context(0)
    for rep in range(2):
        t = time.perf_counter()
        for s, o, q in batch:
            plain.count(s, o, q["k"], q["p"], q["n_bins"], q["cutoff_min"], q["cutoff_max"],
                        flags=q["flags"]).free()
        torch.cuda.synchronize()
        serial = time.perf_counter() - t
    plain.close()
    ctx.close()
    ms = float(np.mean(times)) * 1e3
    ks = sorted({p["k"] for _, _, p in jobs})
    return {
        "metric": METRIC, "value": bases / (ms * 1e-3), "unit": "bases/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64/u128",
        "data": "synthetic (seeded generator)",
        "config": {"workload": f"batch of {len(jobs)} uneven jobs (scale {args.batch_scale}): "
                               "n_reads = 10^U(4,6), read length U{100..250}, ~30x uniform "
                               "references, 1% substitutions, k in {21,25,31,47,55}, p=7, "
                               "512 bins, cutoffs 2..1e9",
                   "n_jobs": len(jobs), "n_bases": bases, "k_values": ks},
        "kmers_per_s": kmers / (ms * 1e-3),
        "serial_ms": serial * 1e3,
        "speedup_vs_serial": serial * 1e3 / ms,
        "untuned_ms": float(np.mean(untuned_times)) * 1e3,
        "autotune": {"seconds": tune_s, "batch_workers": tune["batch_workers"],
                     "classes": tune["classes"]},
    }


def bench_serve(args):
    """The served form: closed-loop saturation rate, then Poisson arrivals at
    fractions of it; p50 / p99 of each job's submit-to-ready latency."""
    import queue
    import threading
    pool = generate("serve", args.serve_pool, args.serve_scale)
    import torch
    from paper_1407_1507_amd import kmc
    djobs = to_device(pool)
    ctx = kmc.Context(0)
    out = {"metric": METRIC, "unit": "jobs/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic (seeded generator)", "dtype": "u128",
           "config": {"workload": f"served jobs: {len(pool)} distinct read sets (scale "
                                  f"{args.serve_scale}) of the repeat-rich generator, "
                                  "references log-uniform in [5, 50] Mbp x scale, 30x of "
                                  "150 bp, k=55, p=9, 1024 bins, cutoffs 2..1e6",
                      "pool_bases": int(sum(int(o[-1]) for _, o, _ in pool)),
                      "max_active": args.max_active},
           "budgets": {}}

    def job(i):
        s, o, p = djobs[i % len(djobs)]
        return s, o, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"]

    for label, budget in (("full", 0), ("24GB", 24 << 30)):
        srv = kmc.Server(ctx, hbm_budget=budget, max_active=args.max_active)
        for i in range(len(djobs)):  # warm every worker stream and shape
            srv.poll(srv.submit(*job(i))).free()
        # closed loop: every job queued at once (once to warm the table
        # pools with as many tables alive as the loop keeps, then timed)
        n_sat = max(6 * len(djobs), 64)
        for rep in range(2):
            t = time.perf_counter()
            tickets = [srv.submit(*job(i)) for i in range(n_sat)]
            for tk in tickets:
                srv.poll(tk).free()
            sat = n_sat / (time.perf_counter() - t)
        rows = []
        rng = np.random.default_rng(5)
        for frac in args.serve_lambdas:
            lam = frac * sat
            n = args.serve_arrivals
            gaps = rng.exponential(1.0 / lam, size=n)
            tickets = queue.Queue()
            results = []

            def poller():
                for _ in range(n):
                    r = srv.poll(tickets.get())
                    results.append((r.stats["us_latency"], r.stats["us_queue"],
                                    r.stats["n_bases"]))
                    r.free()

            th = threading.Thread(target=poller)
            th.start()
            t0 = time.perf_counter()
            nxt = t0
            for i in range(n):
                nxt += gaps[i]
                d = nxt - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets.put(srv.submit(*job(i)))
            th.join()
            span = time.perf_counter() - t0
            lat = np.array([x[0] for x in results]) * 1e-3
            q = np.array([x[1] for x in results]) * 1e-3
            rows.append({"lambda_frac": frac, "lambda_jobs_s": lam, "arrivals": n,
                         "achieved_jobs_s": n / span,
                         "bases_per_s": sum(x[2] for x in results) / span,
                         "latency_ms_p50": float(np.percentile(lat, 50)),
                         "latency_ms_p99": float(np.percentile(lat, 99)),
                         "queue_ms_p50": float(np.percentile(q, 50)),
                         "queue_ms_p99": float(np.percentile(q, 99))})
            print(f"serve {label} lambda {frac}: {rows[-1]}", file=sys.stderr, flush=True)
        st = srv.stats()
        srv.stop()
        out["budgets"][label] = {"budget_bytes": st["budget"], "saturation_jobs_s": sat,
                                 "peak_admitted_bytes": st["peak_admitted_bytes"],
                                 "points": rows}
    # the plain per-job launch on the same pool: one host thread counts the
    # jobs one after another (kmc_count_ex), at the same arrival rates
    n_sat = max(6 * len(djobs), 64)
    for rep in range(2):
        t = time.perf_counter()
        for i in range(n_sat):
            ctx.count(*job(i)).free()
        plain_sat = n_sat / (time.perf_counter() - t)
    rows = []
    rng = np.random.default_rng(5)
    sat = out["budgets"]["full"]["saturation_jobs_s"]
    for frac in args.serve_lambdas:
        lam = frac * sat
        n = args.serve_arrivals
        gaps = rng.exponential(1.0 / lam, size=n)
        arrive = np.cumsum(gaps)
        lat, bases = [], 0
        t0 = time.perf_counter()
        for i in range(n):
            d = t0 + arrive[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            r = ctx.count(*job(i))
            done = time.perf_counter()
            lat.append((done - (t0 + arrive[i])) * 1e3)
            bases += r.stats["n_bases"]
            r.free()
        span = time.perf_counter() - t0
        rows.append({"lambda_frac": frac, "lambda_jobs_s": lam, "arrivals": n,
                     "achieved_jobs_s": n / span, "bases_per_s": bases / span,
                     "latency_ms_p50": float(np.percentile(lat, 50)),
                     "latency_ms_p99": float(np.percentile(lat, 99))})
        print(f"plain lambda {frac}: {rows[-1]}", file=sys.stderr, flush=True)
    out["plain"] = {"saturation_jobs_s": plain_sat, "points": rows,
                    "served_over_plain_saturation": sat / plain_sat}
    if args.serve_large:
        out["large_in_mix"] = serve_large_mix(ctx, kmc, djobs, job, sat, args)
    ctx.close()
    full = out["budgets"]["full"]
    out["value"] = full["saturation_jobs_s"]
    return out


def serve_large_mix(ctx, kmc, djobs, job, sat, args):
    """The served form's large job (60M reads x 150 bp, 9 Gbases, k = 28)
    beside Poisson arrivals of the pool's jobs at half the saturation rate,
    for each budget: submitted first, and submitted after the 20th arrival
    (pool jobs running and queued); the large job's table must equal its
    table counted alone."""
    import queue
    import threading
    import torch
    from paper_1407_1507_amd import synth
    seq, off, p = load_workload("large-300M-60Mx150", args.input_cache)
    dl = (torch.from_numpy(seq).to("cuda:0"), torch.from_numpy(off.view(np.int64)).to("cuda:0"))
    del seq, off
    largs = (dl[0], dl[1], p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"])

    def digest(r):
        # entries, sum of counts, and the wrapped sums of keys and of
        # key * count: equal tables give equal digests
        k = r.keys.astype(np.uint64)
        c = r.counts.astype(np.uint64)
        return (int(r.n), int(c.sum()), int(k.sum(dtype=np.uint64)),
                int((k * c).sum(dtype=np.uint64)))

    alone = ctx.count(*largs)
    ref = digest(alone)
    alone_ms = alone.stats["us_total"] * 1e-3
    alone.free()
    res = {"large_job": {"n_bases": int(dl[0].numel()), "alone_device_ms": alone_ms,
                         "entries": ref[0]}}
    for label, budget, at in (("full", 0, 0), ("24GB", 24 << 30, 0), ("full, mid-stream", 0, 20),
                              ("24GB, mid-stream", 24 << 30, 20)):
        srv = kmc.Server(ctx, hbm_budget=budget, max_active=args.max_active)
        n = args.serve_arrivals
        rng = np.random.default_rng(9)
        gaps = rng.exponential(1.0 / (0.5 * sat), size=n)
        tickets = queue.Queue()
        lat = []

        def poller():
            for _ in range(n):
                r = srv.poll(tickets.get())
                lat.append(r.stats["us_latency"] * 1e-3)
                r.free()

        th = threading.Thread(target=poller)
        th.start()
        t0 = time.perf_counter()
        big = srv.submit(*largs) if at == 0 else None
        nxt = t0
        for i in range(n):
            nxt += gaps[i]
            d = nxt - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.put(srv.submit(*job(i)))
            if i + 1 == at:
                big = srv.submit(*largs)
        r = srv.poll(big)
        big_ms = r.stats["us_latency"] * 1e-3
        big_queue_ms = r.stats["us_queue"] * 1e-3
        same = digest(r) == ref
        groups, spilled = r.stats["n_groups"], r.stats["records_spilled"]
        r.free()
        th.join()
        span = time.perf_counter() - t0
        st = srv.stats()
        srv.stop()
        res[label] = {"budget_bytes": st["budget"], "large_after_arrivals": at,
                      "large_latency_ms": big_ms, "large_queue_ms": big_queue_ms,
                      "peak_admitted_bytes": st["peak_admitted_bytes"],
                      "large_n_groups": groups, "large_records_spilled": spilled,
                      "large_table_as_alone": same, "small_jobs": n,
                      "small_latency_ms_p50": float(np.percentile(lat, 50)),
                      "small_latency_ms_p99": float(np.percentile(lat, 99)),
                      "span_s": span}
        print(f"large in mix {label}: {res[label]}", file=sys.stderr, flush=True)
    return res


def bench_table6(args):
    """Super k-mers per read and the largest bin, signatures against plain
    canonical minimizers (the shape of the paper's Table 6), on the 2M-read
    genome-like read set, k = 28 and 55, m = 7, 512 bins."""
    import torch
    from paper_1407_1507_amd import kmc, synth
    seq, off, p = synth.make("genome-5M-2Mx100", args.table6_scale)
    dseq = torch.from_numpy(seq).to("cuda:0")
    doff = torch.from_numpy(off.view(np.int64)).to("cuda:0")
    ctx = kmc.Context(0)
    n_reads = int(off.size - 1)
    rows = []
    for k in (28, 55):
        for label, flags in (("signatures", 0), ("minimizers", kmc.FLAG_PLAIN_MINIMIZERS)):
            r = ctx.count(dseq, doff, k, 7, 512, 2, 10**9, flags=flags | kmc.FLAG_DEVICE_TABLE)
            st = r.stats
            r.free()
            rows.append({"k": k, "m": 7, "kind": label,
                         "superkmers_per_read": st["n_superkmers"] / n_reads,
                         "largest_bin_kmers": st["max_bin_kmers"],
                         "largest_bin_frac": st["max_bin_kmers"] / max(1, st["n_kmers"]),
                         "n_kmers": st["n_kmers"]})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    ctx.close()
    return {"metric": "super k-mers per read and largest bin (Table 6 shape)",
            "value": None, "unit": "super k-mers per read", "n_gpus": 1,
            "data": "synthetic (seeded generator)",
            "config": {"workload": f"genome-5M-2Mx100 at scale {args.table6_scale}: "
                                   f"{n_reads} reads x 100 bp, 512 bins",
                       "n_reads": n_reads},
            "rows": rows}


def bench_kx(args):
    """(k,x)-mers against plain k-mers (the shape of the paper's Table 7): per
    x = 0..3, time per job on device-resident reads, the sorted fraction
    ((k,x)-mers sorted / k-mers) and the distinct (k,x)-mers, on a k = 28
    workload (k + x <= 31)."""
    import torch
    from paper_1407_1507_amd import kmc
    seq, off, p = load_workload(args.workload, args.input_cache)
    if p["k"] + 3 > 31:
        raise SystemExit("--mode kx needs a workload with k <= 28")
    dseq = torch.from_numpy(seq).to("cuda:0")
    doff = torch.from_numpy(off.view(np.int64)).to("cuda:0")
    ctx = kmc.Context(0)
    rows = []
    for x in (0, 1, 2, 3):
        flags = kmc.FLAG_DEVICE_TABLE | kmc.FLAG_KX(x)
        run = lambda: ctx.count(dseq, doff, p["k"], p["p"], p["n_bins"], p["cutoff_min"],
                                p["cutoff_max"], flags=flags)
        for _ in range(args.warmup):
            run().free()
        torch.cuda.synchronize()
        t = []
        st = None
        for _ in range(args.steps):
            t0 = time.perf_counter()
            r = run()
            t.append(time.perf_counter() - t0)
            st = r.stats
            r.free()
        ms = 1e3 * float(np.median(t))
        rows.append({"x": x, "ms_per_job": ms, "bases_per_s": int(off[-1]) / (ms / 1e3),
                     "sorted_fraction": (st["n_kx_entries"] / st["n_kmers"]) if x else 1.0,
                     "distinct_kx": st["n_kx_distinct"], "n_kmers": st["n_kmers"],
                     "n_out": st["n_out"], "n_big_tiles": st["n_big_tiles"],
                     "kernel_us": {k: round(v, 1) for k, v in st["us_kernel"].items()}})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    ctx.close()
    return {"metric": "time per job and sorted fraction, (k,x)-mers against k-mers (Table 7 shape)",
            "value": None, "unit": "ms per job", "n_gpus": 1,
            "data": "synthetic (seeded generator)",
            "config": {"workload": args.workload, "k": p["k"], "p": p["p"],
                       "n_bins": p["n_bins"], "steps": args.steps, "warmup": args.warmup},
            "rows": rows}


def fastq_bytes(seq, off, read_len: int) -> np.ndarray:
    """FASTQ text of equal-length reads ("@r<i>" headers, constant quality),
    built with array operations."""
    n = off.size - 1
    head = np.frombuffer(b"@r\n", dtype=np.uint8)
    mid = np.frombuffer(b"\n+\n", dtype=np.uint8)
    rec = np.empty((n, 3 + read_len + 3 + read_len + 1), dtype=np.uint8)
    rec[:, :3] = head
    rec[:, 3:3 + read_len] = seq.reshape(n, read_len)
    rec[:, 3 + read_len:6 + read_len] = mid
    rec[:, 6 + read_len:6 + 2 * read_len] = ord("I")
    rec[:, -1] = ord("\n")
    return rec.reshape(-1)


def bench_parse(args):
    """Device parsing of FASTQ text (kmc_parse): the 2M-read genome workload
    as FASTQ (one read per record), text resident in HBM."""
    import torch
    from paper_1407_1507_amd import kmc, synth
    seq, off, p = synth.make("genome-5M-2Mx100")
    text = fastq_bytes(seq, off, 100)
    dtext = torch.from_numpy(text).to("cuda:0")
    ctx = kmc.Context(0)
    for _ in range(args.warmup):
        kmc.Parsed(ctx, dtext, kmc.FORMAT_FASTQ).free()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t = time.perf_counter()
        pr = kmc.Parsed(ctx, dtext, kmc.FORMAT_FASTQ)
        times.append(time.perf_counter() - t)
        assert pr.n_reads == off.size - 1 and pr.n_bases == seq.size
        pr.free()
    ms = float(np.median(times)) * 1e3
    ctx.close()
    return {"metric": "FASTQ bytes parsed per second on the device", "value": text.size / (ms * 1e-3),
            "unit": "bytes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "data": "synthetic (seeded generator)",
            "dtype": "u8",
            "config": {"workload": "genome-5M-2Mx100 as FASTQ (2,000,000 records of 100 bp)",
                       "text_bytes": int(text.size)},
            "bases_per_s": seq.size / (ms * 1e-3),
            "hbm_gbs_alg": (text.size + seq.size + 8 * off.size) / (ms * 1e-3) / 1e9}


def bench_query(args):
    """Batched device lookups (kmc_db_query) in the KMC 2 database of the
    genome workload's table: half the queries present (in either
    orientation), half random k-mers."""
    import torch
    from paper_1407_1507_amd import kmc, synth
    seq, off, p = synth.make("genome-5M-2Mx100")
    ctx = kmc.Context(0)
    dseq = torch.from_numpy(seq).to("cuda:0")
    doff = torch.from_numpy(off.view(np.int64)).to("cuda:0")
    res = ctx.count(dseq, doff, p["k"], p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                    flags=kmc.FLAG_DEVICE_TABLE)
    t = time.perf_counter()
    db = kmc.Db.build(ctx, res, 4, 4)
    build_ms = (time.perf_counter() - t) * 1e3
    keys = torch.zeros(res.n, dtype=torch.int64, device="cuda:0")
    counts = torch.zeros(res.n, dtype=torch.int32, device="cuda:0")
    db.decode(keys, counts)
    n_q = args.query_n
    g = torch.Generator(device="cuda:0").manual_seed(7)
    present = keys[torch.randint(0, res.n, (n_q // 2,), device="cuda:0", generator=g)]
    rnd = torch.randint(0, 2**56, (n_q - n_q // 2,), device="cuda:0", generator=g,
                        dtype=torch.int64)
    q = torch.cat([present, rnd])
    out = torch.zeros(n_q, dtype=torch.int32, device="cuda:0")
    for _ in range(args.warmup):
        db.query(q, out)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t = time.perf_counter()
        db.query(q, out)
        times.append(time.perf_counter() - t)
    hit = float((out[: n_q // 2] > 0).float().mean())
    ms = float(np.median(times)) * 1e3
    info = db.info
    db.free()
    res.free()
    ctx.close()
    return {"metric": "k-mer lookups per second in the device database", "value": n_q / (ms * 1e-3),
            "unit": "lookups/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "data": "synthetic (seeded generator)",
            "dtype": "u64",
            "config": {"workload": f"genome-5M-2Mx100 table ({info['total_kmers']} k-mers, "
                                   "k=28, lut_prefix_length 4, 4-byte counters), "
                                   f"{n_q} queries, half present",
                       "queries": n_q},
            "present_hit_rate": hit, "db_build_ms": build_ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["single", "batch", "serve", "table6", "parse", "query",
                                       "kx"],
                    default="single")
    ap.add_argument("--query-n", type=int, default=50_000_000)
    ap.add_argument("--table6-scale", type=float, default=1.0)
    ap.add_argument("--batch-jobs", type=int, default=256)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--serve-scale", type=float, default=0.25)
    ap.add_argument("--serve-arrivals", type=int, default=200)
    ap.add_argument("--serve-lambdas", type=float, nargs="+",
                    default=[0.25, 0.5, 0.7, 0.85, 1.0, 1.2])
    ap.add_argument("--max-active", type=int, default=4)
    ap.add_argument("--serve-large", action="store_true",
                    help="serve mode: also the 9-Gbase large job beside the arrivals")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--also", nargs="*", default=ALSO,
                    help="other workloads measured with a few steps each (extra keys)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--order", choices=["bin", "ascending"], default="bin",
                    help="table order: grouped by bin, or ascending over the whole table")
    ap.add_argument("--input-cache", default="",
                    help="folder holding the generated read sets (made on first use)")
    ap.add_argument("--generate-only", action="store_true",
                    help="with --input-cache: only write the read sets")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every job of the counting path runs on a single "
              "MI355X (jobs are independent; several GPUs would each take whole jobs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.mode != "single":
        line = {"batch": bench_batch, "serve": bench_serve,
                "table6": bench_table6, "parse": bench_parse,
                "query": bench_query, "kx": bench_kx}[args.mode](args)
        print(json.dumps(line), flush=True)
        return

    import torch

    if args.input_cache and args.generate_only:
        for w in [args.workload] + list(args.also):
            load_workload(w, args.input_cache)
        return
    line, data = bench_single(args.workload, args.steps, args.warmup, args.order,
                              args.input_cache)
    line["roofline"]["copy_peak_gbs"] = copy_peak()
    line["roofline"]["frac_vs_copy"] = line["roofline"]["achieved"] / line["roofline"]["copy_peak_gbs"]
    line["job_roofline"]["frac_vs_copy"] = (line["job_roofline"]["achieved"] /
                                            line["roofline"]["copy_peak_gbs"])
    # the other single-job workloads, a few steps each (not the headline value)
    also = {}
    for w in args.also:
        if w == args.workload:
            continue
        other, _ = bench_single(w, max(3, min(args.steps, 5)), 1, args.order, args.input_cache)
        also[w] = {key: other[key] for key in ("value", "unit", "ms_per_step", "kmers_per_s",
                                               "device_ms", "hbm_gbs_alg", "job_roofline",
                                               "roofline", "kernel_us", "job", "config")}
    if also:
        line["also"] = also
    if not args.no_cpu_baseline:
        seq, off, p = data
        line["cpu_baseline"] = cpu_baseline(seq, off, p)
    print(json.dumps(line), flush=True)


def load_workload(workload: str, cache: str = ""):
    """The named synthetic read set; with a cache folder, taken from (or saved
    to) <cache>/<workload>.seq.npy and .off.npy, so that a profiler run need
    not generate it (the large set's parallel generator under a counter
    profiler profiles every worker process)."""
    from paper_1407_1507_amd import synth

    fs, fo = (os.path.join(cache, f"{workload}.{x}.npy") for x in ("seq", "off"))
    if cache and os.path.exists(fs) and os.path.exists(fo):
        return np.load(fs), np.load(fo), dict(synth.CONFIGS[workload])
    seq, off, p = synth.make(workload)
    if cache:
        os.makedirs(cache, exist_ok=True)
        np.save(fs, seq)
        np.save(fo, off)
    return seq, off, p


def bench_single(workload: str, steps: int, warmup: int, order: str, input_cache: str = ""):
    """One job per step on one read set resident in HBM; returns the bench
    line (without the CPU baseline) and the read set."""
    import torch
    from paper_1407_1507_amd import kmc, synth

    seq, off, p = load_workload(workload, input_cache)
    print(f"generated {workload}: {seq.size} bases", file=sys.stderr, flush=True)
    dseq = torch.from_numpy(seq).to("cuda:0")
    doff = torch.from_numpy(off.view(np.int64)).to("cuda:0")
    torch.cuda.synchronize()
    ctx = kmc.Context(0)
    flags = kmc.FLAG_DEVICE_TABLE | (kmc.FLAG_ASCENDING if order == "ascending" else 0)
    run = lambda: ctx.count(dseq, doff, p["k"], p["p"], p["n_bins"], p["cutoff_min"],
                            p["cutoff_max"], flags=flags)
    for _ in range(warmup):
        run().free()
    torch.cuda.synchronize()
    # each step's table is freed once the call returns: its block goes back to
    # the library's pool and holds the next step's table, as in a stream of jobs
    lat, stats = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        r = run()
        lat.append(time.perf_counter() - s)
        stats.append(r.stats)
        r.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    st = stats[-1]
    n_bases, n_kmers = st["n_bases"], st["n_kmers"]
    # dominant kernel: largest mean device time (HIP events on the library's stream)
    names = kmc.KERNELS
    mean_us = {n: float(np.mean([x["us_kernel"][n] for x in stats])) for n in names}
    dom = max(mean_us, key=mean_us.get)
    dom_bytes = kernel_bytes(dom, st, p["k"])
    achieved = dom_bytes / (mean_us[dom] * 1e-6) / 1e9 if mean_us[dom] > 0 else 0.0
    dev_us = float(np.mean([x["us_total"] for x in stats]))
    job_gbs = st["bytes_alg"] / (dev_us * 1e-6) / 1e9 if dev_us > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": n_bases / (ms * 1e-3),
        "unit": "bases/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64" if p["k"] <= 32 else "u128",
        "data": "synthetic (seeded generator; stands in for the paper's read sets)",
        "config": {"workload": f"{workload}: {DESCRIPTION.get(workload, '')}",
                   "k": p["k"], "p": p["p"], "n_bins": p["n_bins"],
                   "cutoff_min": p["cutoff_min"], "cutoff_max": p["cutoff_max"],
                   "n_reads": int(off.size - 1), "n_bases": int(n_bases),
                   "order": order},
        "kmers_per_s": n_kmers / (ms * 1e-3),
        "hbm_gbs_alg": st["bytes_alg"] / (ms * 1e-3) / 1e9,
        "device_ms": dev_us * 1e-3,
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "kernel_us": {n: round(v, 2) for n, v in mean_us.items()},
        "phase_us": {n: round(float(np.mean([x["us_" + n] for x in stats])), 2)
                     for n in ("map", "split", "expand", "sort", "assemble")},
        "job": {key: st[key] for key in ("n_kmers", "n_superkmers", "n_distinct", "n_out",
                                         "n_tiles", "n_big_tiles", "n_big_keys", "bytes_alg",
                                         "max_bin_kmers")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, workload),
                     "alg_bytes_per_launch": dom_bytes},
        # the whole job: algorithmic bytes over device time (first kernel to last)
        "job_roofline": {"achieved": job_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": job_gbs / HBM_PEAK_GBS},
    }
    ctx.close()
    del dseq, doff
    torch.cuda.empty_cache()
    return line, (seq, off, p)


if __name__ == "__main__":
    main()
