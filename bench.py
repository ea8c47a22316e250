"""Benchmark of the per-barrier-interval SIMT race check on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one rv_check of the whole workload (count, expansion, sort +
segmented scan, finish, result copy), inputs resident on the device.  Prints
one JSON line on stdout; diagnostics go to stderr.

Workloads (synthetic, seeded descriptions from ``workloads``):
  matmul16   tiled-matmul access pattern, blockDim (32,32), gridDim (16,16),
             64 K-iterations, dynamic barrier 64 dropped: 1,141,112,832
             records (the 1e9-record configuration; default)
  matmul64   the same pattern at gridDim (64,64): 18,257,805,312 records
  tree       shared-memory tree reduction, blockDim 1024, gridDim 128, 11
             variants checked as one batch (4,321,152 records)
  tiny       the fixed 64-thread kernel and 32 seeded random affine kernels
             of one 64-thread block, checked as one batch
  batch      4096 random affine 2-D kernels (seed 4, records log-uniform in
             [1e2, 1e6], 432,085,651 records) checked by one rv_check_batch
             per step; also times one rv_check per kernel for comparison
  gespmm     the shared-memory staging pattern of Ge-SpMM's Algorithm 2
             (the paper's case study) across sizes (M rows, N columns, T
             chunks, K candidate B rows): the race-free kernel is timed at
             each size and its two barrier-dropped mutants are checked
             against their closed forms
  serve      a server over a 64 GiB budget fed 10,000 random affine jobs
             (seed 5, records log-uniform in [1e3, 1e7]) at Poisson arrival
             times, rate 0.7 x the measured closed-loop capacity, after 500
             warm-up jobs; reports per-job latency p50/p99
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per record of each kernel, as the path defines a
# record: a 12-byte (u64 location key, u32 instance id) pair that the
# expansion writes and the sort + segmented scan reads once.  The count pass
# only evaluates instances (no record traffic).
ALG_BYTES = {"expand": 12.0, "sort_scan": 12.0}
# What this implementation actually moves per record: keys and ids packed
# into one 8-byte word (31-bit location, rw bit, 32-bit id).
PACKED_BYTES = 8.0
# the grouping stage's kernels (fold: buckets of one slice, medium and hot
# buckets; their HIP-event time is taken together)
GROUP_KERNEL = {"fold": "k_fold+k_mid+k_hot", "sort_scan": "k_bucket"}
# Block-local units checked on chip (k_direct): no record reaches HBM; each
# record is folded into its location's 12-byte summary in LDS (smallest id,
# largest 2 id + rw, smallest write id).  Algorithmic LDS bytes per record:
# one read-modify-write of that summary, 12 bytes.  LDS peak: 256 CUs x 32
# banks x 4 bytes per clock x 2.4 GHz.
UNIT_ALG_BYTES = 12.0
LDS_PEAK_GBS = 256 * 32 * 4 * 2.4


def roofline_units(stages, unit_records_timed):
    """The on-chip units' kernel against the LDS roofline: the 12-byte
    summary update per record x records per launch / average launch time
    (HIP events on the stream it runs on)."""
    launches = stages["direct"][1]
    if not launches or stages["direct"][0] <= 0:
        return None
    avg_ms = stages["direct"][0] / launches
    recs = unit_records_timed / launches
    achieved = UNIT_ALG_BYTES * recs / (avg_ms * 1e-3) / 1e9
    return {"bound": "lds", "kernel": "k_direct", "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1),
            "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBS, 4),
            "traffic": traffic_for("k_direct", int(recs)), "avg_launch_ms": round(avg_ms, 4),
            "alg_bytes_per_record": UNIT_ALG_BYTES, "records_per_launch": int(recs),
            "note": "records of block-local units never reach HBM; traffic is the kernel's measured HBM bytes"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    from workloads import kernels as K
    if name == "matmul16":
        d = K.tiled_matmul(grid=16, k_iters=64, drop_dynamic=64)
        return [d], ("tiled-matmul access pattern, blockDim (32,32), gridDim (16,16), 64 K-iterations, "
                     "dynamic barrier 64 dropped")
    if name == "matmul64":
        d = K.tiled_matmul(grid=64, k_iters=64, drop_dynamic=64)
        return [d], ("tiled-matmul access pattern, blockDim (32,32), gridDim (64,64), 64 K-iterations, "
                     "dynamic barrier 64 dropped")
    if name == "tree":
        return [K.tree_reduction(k) for k in range(-1, 10)], \
            "shared-memory tree reduction, blockDim 1024, gridDim 128, correct + 10 barrier-deleted variants"
    if name == "tiny":
        return [K.tiny_fixed()] + K.tiny_random(seed=1, count=32), \
            "tiny kernels: the fixed 64-thread kernel and 32 seeded random affine ones, checked as one batch"
    raise SystemExit(f"unknown workload {name}")


def _host_threads():
    """Threads for the parallel oracle leg: the CPUs this process may run
    on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_pool(jobs, threads):
    """Run oracle.check over jobs [(desc, ilo, ihi)] on a thread pool (the C
    oracle keeps no global state and ctypes releases the interpreter lock
    during the call); returns (records, seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda j: oracle.check(j[0], max_witnesses=1, ilo=j[1], ihi=j[2]), jobs))
    return sum(r.n_records for r in res), time.perf_counter() - t0


def cpu_baseline_units(units, max_seconds):
    """The oracle as it stands, timed on the host: first single-threaded on
    the first units until about max_seconds / 2, then on `threads` threads
    (one unit per task, a kernel or one interval) over a sample sized to take
    about as long.  `units` is a list of (desc, ilo, ihi, label)."""
    import oracle
    oracle.build(force=False)
    recs1, n1 = 0, 0
    t0 = time.perf_counter()
    while n1 < len(units) and time.perf_counter() - t0 < max_seconds / 2:
        d, lo, hi, _ = units[n1]
        recs1 += oracle.check(d, max_witnesses=1, ilo=lo, ihi=hi).n_records
        n1 += 1
    dt1 = time.perf_counter() - t0
    rate1 = recs1 / dt1
    threads = _host_threads()
    per_unit = dt1 / max(1, n1)
    m = max(threads, min(len(units), int(threads * (max_seconds / 2) / max(per_unit, 1e-6))))
    recsN, dtN = _oracle_pool([(d, lo, hi) for d, lo, hi, _ in units[:m]], threads)
    return {"value": recsN / dtN, "unit": "records/s", "cores": threads, "kind": "oracle",
            "sample": f"{units[0][3]} 0..{m - 1} of {len(units)} ({recsN} records, {dtN:.1f} s, "
                      f"{threads} threads, one {units[0][3].rstrip('s')} per task)",
            "single_thread": {"value": rate1, "cores": 1,
                              "sample": f"{units[0][3]} 0..{n1 - 1} ({recs1} records, {dt1:.1f} s)"},
            "host_cpu": _cpu_model(), "host_cpus_visible": os.cpu_count()}


def cpu_baseline_kernels(descs, max_seconds):
    """The oracle on whole kernels of the batch, in order."""
    return cpu_baseline_units([(d, 0, 1 << 62, "kernels") for d in descs], max_seconds)


def cpu_baseline(desc, max_seconds):
    """The oracle on the intervals of one kernel, in order."""
    import oracle
    oracle.build(force=False)
    n_iv = oracle.n_intervals(desc)
    return cpu_baseline_units([(desc, iv, iv + 1, "intervals") for iv in range(n_iv)], max_seconds)


def traffic_for(kernel_name, records_per_launch):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2503_08946_amd", "csrc", "kernels.hip")
    try:
        t = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        ent = t["kernels"][kernel_name]
        if t.get("kernels_hip_sha256") != sha or ent.get("records") != records_per_launch:
            return None
        return ent["fetch_bytes"] + ent["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def roofline_from(stages, n_records_timed, group_kernel="k_fold"):
    """Dominant kernel (by GPU time, among those with a byte count) and its
    algorithmic bandwidth: bytes per record x records per launch / average
    launch time (HIP events on the stream the kernel runs on).  The bytes
    per record are the path's 12-byte record; `achieved_packed` is the same
    launch at the 8 bytes per record this implementation moves."""
    dom = max(ALG_BYTES, key=lambda k: stages[k][0])
    launches = max(1, stages[dom][1])
    avg_ms = stages[dom][0] / launches
    if not stages[dom][1] or avg_ms <= 0:
        # every pass was checked on chip (k_small): no record reaches HBM
        return {"bound": "alu", "kernel": "k_small", "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None,
                "note": "all passes checked on chip by k_small: no HBM record traffic to put against a roofline"}
    recs_per_launch = n_records_timed / launches
    achieved = ALG_BYTES[dom] * recs_per_launch / (avg_ms * 1e-3) / 1e9
    packed = PACKED_BYTES * recs_per_launch / (avg_ms * 1e-3) / 1e9
    kname = {"expand": "k_scatter", "sort_scan": group_kernel}[dom]
    traffic = traffic_for(kname, int(recs_per_launch))
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
            "alg_bytes_per_record": ALG_BYTES[dom], "records_per_launch": int(recs_per_launch),
            "achieved_packed": round(packed, 1), "frac_packed": round(packed / HBM_PEAK_GBS, 4),
            "packed_bytes_per_record": PACKED_BYTES}


def percentile(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]


def bench_batch(args, rv, torch):
    from workloads import random_affine as RA
    t0 = time.perf_counter()
    descs = RA.batch_kernels(seed=4, count=4096)
    log(f"[bench] generated 4096 kernels in {time.perf_counter() - t0:.1f} s")
    ctx = rv.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)))
    ctx.group = args.group
    ctx.target = args.target
    ctx.small_cap = args.small_cap
    ctx.direct = bool(args.direct)
    ks = [ctx.load(d) for d in descs]
    log(f"[bench] loaded 4096 kernels")
    batch = rv.Batch(ctx, ks)
    for i in range(args.warmup):
        batch.run()
        log(f"[bench] warmup {i}: records={sum(r.n_records for r in batch.results())}")
    # per-kernel plain launches, one pass over the batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single = [ctx.check(k) for k in ks] if not args.no_per_kernel else None
    t_single = time.perf_counter() - t0
    if single is None:
        batch.run()
        single = batch.results()
    n_records = sum(r.n_records for r in single)
    log(f"[bench] one rv_check per kernel: {t_single * 1e3:.1f} ms for the batch")
    ctx.timing(reset=True)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        batch.run()
        lat.append(time.perf_counter() - s0)
        log(f"[bench] step {i}: {lat[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    stages = ctx.timing(reset=True)
    small_records = stages.pop("small_records") // max(1, args.steps)
    direct_records = stages.pop("direct_records") // max(1, args.steps)
    counted_records = stages.pop("counted_records") // max(1, args.steps)
    res = batch.results()
    assert [(r.n_records, r.n_conflicts) for r in res] == [(r.n_records, r.n_conflicts) for r in single]
    per_step = {k: v[0] / args.steps for k, v in stages.items()}
    log("[bench] GPU ms per step by stage: " + ", ".join(f"{k}={v:.3f}" for k, v in per_step.items()))
    value = n_records * args.steps / elapsed
    out = {
        "metric": "access records race-checked/sec + % HBM peak; p50/p99 verify latency",
        "value": value, "unit": "records/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "4096 random affine 2-D kernels, seed 4, records log-uniform in [1e2, 1e6], "
                               "one batched check per step",
                   "records": n_records, "kernels": len(ks),
                   "buckets": sum(k.info().n_buckets for k in ks),
                   "kernels_with_conflicts": sum(1 for r in res if r.n_conflicts),
                   "small_cap": ctx.small_cap, "direct": int(ctx.direct),
                   "records_on_chip": small_records + direct_records,
                   "records_counted_without_writes": counted_records},
        "latency_ms": {"p50": round(percentile(lat, 0.5) * 1e3, 3), "p99": round(percentile(lat, 0.99) * 1e3, 3)},
        "per_kernel_launches": None if args.no_per_kernel else {
            "ms_per_batch": round(t_single * 1e3, 2), "value": n_records / t_single,
            "batched_speedup": round(t_single / (elapsed / args.steps), 2)},
        "stage_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        # the HBM kernels see only the records outside the on-chip passes and
        # units and the passes without writes
        "roofline": roofline_from(stages, (n_records - small_records - direct_records - counted_records) * args.steps,
                                  GROUP_KERNEL[ctx.group]),
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_kernels(descs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def gespmm_expected(M, N, T, K):
    """Hand-derived counts of the Ge-SpMM staging kernel (B read over the
    candidate rows only): records, and conflicts with both barriers (the
    paper's verdict: race-free), without the middle barrier and without the
    trailing one; the first witness of each mutant sits at sm_k[0] of block 0."""
    threads, blocks = M * N, M * (N // 32)
    return {"records": threads * T * (4 + 32 * (4 + K)),
            "both": 0, "no_middle": 64 * T * blocks, "no_trailing": 64 * (T - 1) * blocks}


def bench_gespmm(args, rv, torch):
    from workloads import kernels as K
    ctx = rv.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)))
    ctx.group = args.group
    ctx.target = args.target
    sweep, total_records, total_s, stage_acc = [], 0, 0.0, None
    for (M, N, T, Kb) in K.GESPMM_SWEEP:
        exp = gespmm_expected(M, N, T, Kb)
        # the two mutants: counted once, against their closed forms
        mut = {}
        for tag, mid, trail in (("no_middle", False, True), ("no_trailing", True, False)):
            km = ctx.load(K.gespmm_crc(M, N, T, Kb, middle_barrier=mid, trailing_barrier=trail, kb_on_all=False))
            r = ctx.check(km)
            km.free()
            w = r.witness
            ok = (r.n_records == exp["records"] and r.n_conflicts == exp[tag] and w is not None
                  and (w.space, w.block, w.array, w.address) == (0, 0, 4, 0)
                  and (w.first.tid, w.first.is_write, w.second.tid, w.second.is_write) == (0, 1, 31, 0))
            if not ok:
                raise SystemExit(f"gespmm {M}x{N} T={T} K={Kb} {tag}: {r} differs from the closed form {exp}")
            mut[tag] = r.n_conflicts
        k = ctx.load(K.gespmm_crc(M, N, T, Kb, kb_on_all=False))
        for i in range(args.warmup):
            r = ctx.check(k)
        ctx.timing(reset=True)
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            r = ctx.check(k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.set_timing(False)
        stages = ctx.timing(reset=True)
        stages.pop("small_records")
        stages.pop("direct_records")
        stages.pop("counted_records")
        k.free()
        if (r.n_records, r.n_conflicts) != (exp["records"], 0):
            raise SystemExit(f"gespmm {M}x{N} T={T} K={Kb}: {r} differs from the closed form {exp}")
        stage_acc = stages if stage_acc is None else {
            n: (stage_acc[n][0] + v[0], stage_acc[n][1] + v[1]) for n, v in stages.items()}
        total_records += r.n_records * args.steps
        total_s += dt
        ms = dt / args.steps * 1e3
        sweep.append({"M": M, "N": N, "T": T, "K": Kb, "records": r.n_records, "ms": round(ms, 3),
                      "records_per_s": r.n_records / (ms * 1e-3), "conflicts": r.n_conflicts,
                      "verdict": "race-free" if r.n_conflicts == 0 else "races",
                      "mutant_conflicts": mut})
        log(f"[bench] gespmm M={M} N={N} T={T} K={Kb}: {r.n_records} records, {ms:.2f} ms, "
            f"{r.n_records / (ms * 1e-3):.3g} records/s, conflicts 0 (mutants {mut})")
    per_step = {n: v[0] / args.steps for n, v in stage_acc.items()}
    out = {
        "metric": "access records race-checked/sec + % HBM peak; p50/p99 verify latency",
        "value": total_records / total_s, "unit": "records/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_s / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "Ge-SpMM Algorithm 2 shared-memory staging (coalesced row caching), superset "
                               "domain, B read over K candidate rows; one step = one check of each size in turn",
                   "records": total_records // args.steps, "sizes": len(sweep)},
        "sweep": sweep,
        "stage_ms_per_step": {n: round(v, 4) for n, v in per_step.items()},
        "roofline": roofline_from(stage_acc, total_records, GROUP_KERNEL[ctx.group]),
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        M, N, T, Kb = K.GESPMM_SWEEP[0]
        out["cpu_baseline"] = cpu_baseline(K.gespmm_crc(M, N, T, Kb, kb_on_all=False), args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_serve(args, rv, torch):
    import numpy as np
    from workloads import random_affine as RA
    n_warm, n_jobs = 500, args.serve_jobs
    t0 = time.perf_counter()
    descs = list(RA.serving_stream(seed=5, count=n_warm + n_jobs))
    log(f"[bench] generated {len(descs)} jobs in {time.perf_counter() - t0:.1f} s")
    ctx = rv.Context(0, workspace_bytes=1 << 30)
    ctx.group = args.group
    ctx.direct = bool(args.direct)
    ctx.target = args.target
    ks = [ctx.load(d) for d in descs]
    log(f"[bench] loaded {len(ks)} jobs")
    srv = rv.Server(ctx, budget_bytes=int(args.budget_gb * (1 << 30)), max_batch_records=args.batch_records)
    # closed-loop capacity: the warm-up jobs submitted at once
    t0 = time.perf_counter()
    for k in ks[:n_warm]:
        srv.submit(k)
    srv.drain(600000)
    cap_jobs = n_warm / (time.perf_counter() - t0)
    warm = srv.poll(cap=n_warm)
    assert len(warm) == n_warm and all(r.status == 0 for r in warm)
    rate = args.serve_load * cap_jobs
    log(f"[bench] closed-loop capacity {cap_jobs:.0f} jobs/s; Poisson rate {rate:.0f} jobs/s")
    arrivals = RA.poisson_arrivals(seed=5, count=n_jobs, rate_per_s=rate)
    done = []
    lag = []
    t0 = time.perf_counter()
    for i, k in enumerate(ks[n_warm:]):
        target = t0 + arrivals[i]
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            if target - now > 2e-4:
                time.sleep((target - now) * 0.5)
        lag.append(time.perf_counter() - target)
        srv.submit(k)
        if i % 256 == 255:
            done += srv.poll()
            log(f"[bench] submitted {i + 1} jobs, {len(done)} done")
    srv.drain(600000)
    t_end = time.perf_counter()
    done += srv.poll(cap=n_jobs)
    assert len(done) == n_jobs and all(r.status == 0 for r in done)
    stats = srv.stats()
    srv.close()
    lat = np.array([r.latency_ns for r in done], dtype=np.float64) / 1e6
    queue = np.array([r.t_start_ns - r.t_submit_ns for r in done], dtype=np.float64) / 1e6
    run = np.array([r.t_done_ns - r.t_start_ns for r in done], dtype=np.float64) / 1e6
    t_first = min(r.t_submit_ns for r in done)
    slow = sorted(done, key=lambda r: -r.latency_ns)[:8]
    for r in slow:
        log(f"[bench] slow job {r.job_id}: submitted at {(r.t_submit_ns - t_first) / 1e6:.1f} ms, "
            f"queued {(r.t_start_ns - r.t_submit_ns) / 1e6:.2f} ms, ran {(r.t_done_ns - r.t_start_ns) / 1e6:.2f} ms, "
            f"{r.result.n_records} records")
    n_records = sum(r.result.n_records for r in done)
    elapsed = t_end - t0
    out = {
        "metric": "access records race-checked/sec + % HBM peak; p50/p99 verify latency",
        "value": n_records / elapsed, "unit": "records/s", "n_gpus": 1, "steps": n_jobs, "warmup": n_warm,
        "ms_per_step": elapsed / n_jobs * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "served check: random affine 2-D jobs, seed 5, records log-uniform in "
                               f"[1e3, 1e7], Poisson arrivals at {args.serve_load} x closed-loop capacity, "
                               f"{args.budget_gb:g} GiB budget, batches of at most {args.batch_records} records",
                   "records": n_records, "jobs": n_jobs},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "p90": round(float(np.percentile(lat, 90)), 3),
                       "max": round(float(lat.max()), 3),
                       "queue_p50": round(float(np.percentile(queue, 50)), 3),
                       "queue_p99": round(float(np.percentile(queue, 99)), 3),
                       "run_p99": round(float(np.percentile(run, 99)), 3)},
        "arrival_rate_jobs_per_s": round(rate, 1),
        "closed_loop_capacity_jobs_per_s": round(cap_jobs, 1),
        "submit_lag_ms_p99": round(float(np.percentile(lag, 99)) * 1e3, 3),
        "server": stats,
    }
    print(json.dumps(out), flush=True)


def bandwidth_anchor(gib, reps=10):
    """Achievable-bandwidth anchor: torch's own streaming kernels over a
    buffer far larger than the last-level cache, timed with HIP events."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    out = {"bytes": 4 * n}
    for name, fn, moved in (("read", lambda: a.sum(), 4 * n), ("write", lambda: b.fill_(2.0), 4 * n),
                            ("copy", lambda: b.copy_(a), 8 * n)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 4), "GB/s": round(moved / (ms * 1e-3) / 1e9, 1),
                     "frac_of_8TBs": round(moved / (ms * 1e-3) / 8e12, 4)}
        log(f"[anchor] {name}: {out[name]}")
    print(json.dumps({"bandwidth_anchor": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="matmul16")
    ap.add_argument("--workspace-gb", type=float, default=16.0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-kernel", action="store_true",
                    help="batch workload: skip the one-rv_check-per-kernel comparison")
    ap.add_argument("--group", choices=("fold", "sort_scan"), default="fold",
                    help="per-bucket grouping kernel")
    ap.add_argument("--target", type=int, default=2048, help="planner: mean records per location bucket")
    ap.add_argument("--direct", type=int, choices=(0, 1), default=1,
                    help="rv_check: group block-local (shared-array) locations on chip (1) or send every "
                         "record through the HBM pipeline (0)")
    ap.add_argument("--small-cap", type=int, default=2048,
                    help="batched checks: passes of at most this many instances run on chip (0: off)")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="server budget (serve workload)")
    ap.add_argument("--serve-jobs", type=int, default=10000)
    ap.add_argument("--batch-records", type=int, default=1 << 26, help="server: records per batch at most")
    ap.add_argument("--serve-load", type=float, default=0.7, help="arrival rate / closed-loop capacity")
    ap.add_argument("--bandwidth-anchor", type=float, default=0.0, metavar="GIB",
                    help="only time plain streaming kernels over GIB gibibytes (read-only reduction, write-only "
                         "fill, copy) and exit: what this device's HBM delivers to simple kernels")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only copy GIB gibibytes device-to-device (a plain copy kernel of known size, "
                         "to scale the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.bandwidth_anchor:
        return bandwidth_anchor(args.bandwidth_anchor)
    if args.copy_calibration:
        import torch
        n = int(args.copy_calibration * (1 << 30))
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the checker runs on a single GPU and has no multi-GPU path",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_2503_08946_amd as rv

    if args.workload == "batch":
        return bench_batch(args, rv, torch)
    if args.workload == "serve":
        return bench_serve(args, rv, torch)
    if args.workload == "gespmm":
        return bench_gespmm(args, rv, torch)
    descs, wl_text = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: {wl_text}")
    ctx = rv.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)))
    ctx.group = args.group
    ctx.target = args.target
    ctx.direct = bool(args.direct)
    ks = [ctx.load(d) for d in descs]
    batch = len(ks) > 1

    def step():
        return ctx.check_batch(ks) if batch else [ctx.check(ks[0])]

    for i in range(args.warmup):
        res = step()
        log(f"[bench] warmup {i}: records={sum(r.n_records for r in res)} "
            f"conflicts={sum(r.n_conflicts for r in res)}")
    n_records = sum(r.n_records for r in res) if args.warmup else sum(r.n_records for r in step())
    ctx.timing(reset=True)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        res = step()
        lat.append(time.perf_counter() - s0)
        log(f"[bench] step {i}: {lat[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    stages = ctx.timing(reset=True)
    small_records = stages.pop("small_records") // args.steps
    direct_records = stages.pop("direct_records") // args.steps
    counted_records = stages.pop("counted_records") // args.steps
    assert sum(r.n_records for r in res) == n_records
    value = n_records * args.steps / elapsed
    p50 = percentile(lat, 0.5)
    p99 = percentile(lat, 0.99)
    per_step = {k: v[0] / args.steps for k, v in stages.items()}
    log("[bench] GPU ms per step by stage: " + ", ".join(f"{k}={v:.3f}" for k, v in per_step.items()))
    roofline = roofline_from(stages, (n_records - small_records - direct_records - counted_records) * args.steps,
                             GROUP_KERNEL[ctx.group])
    roofline_hbm = None
    if direct_records:
        # the units' kernel dominates when its launch time exceeds every HBM
        # stage's; the HBM pipeline's own roofline is reported beside it
        ru = roofline_units(stages, direct_records * args.steps)
        hbm_ms = max(stages["expand"][0], stages["sort_scan"][0])
        if ru is not None and stages["direct"][0] >= hbm_ms:
            roofline, roofline_hbm = ru, roofline
        elif ru is not None:
            roofline_hbm = ru
    out = {
        "metric": "access records race-checked/sec + % HBM peak; p50/p99 verify latency",
        "value": value,
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl_text, "records": n_records, "kernels": len(ks),
                   "conflicts": sum(r.n_conflicts for r in res), "direct": int(ctx.direct),
                   "records_on_chip": small_records + direct_records,
                   "records_counted_without_writes": counted_records},
        "latency_ms": {"p50": round(p50 * 1e3, 3), "p99": round(p99 * 1e3, 3)},
        "stage_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "roofline": roofline,
    }
    if roofline_hbm is not None:
        out["roofline_other"] = roofline_hbm
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = (cpu_baseline_kernels(descs, args.cpu_seconds) if len(descs) > 1
                               else cpu_baseline(descs[0], args.cpu_seconds))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
