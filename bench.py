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
# Algorithmic HBM bytes per record of each kernel: the expansion writes one
# 8-byte record, the sort + segmented scan reads it once.  The count pass
# only evaluates instances (no record traffic).
ALG_BYTES = {"expand": 8.0, "sort_scan": 8.0}


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
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(desc, max_seconds):
    """The oracle (single-threaded C) on the first intervals of the workload,
    adding intervals until about max_seconds of CPU time."""
    import oracle
    oracle.build(force=False)
    n_iv = oracle.n_intervals(desc)
    recs = 0
    t0 = time.perf_counter()
    iv = 0
    while iv < n_iv and time.perf_counter() - t0 < max_seconds:
        r = oracle.check(desc, max_witnesses=1, ilo=iv, ihi=iv + 1)
        recs += r.n_records
        iv += 1
    dt = time.perf_counter() - t0
    return {"value": recs / dt, "unit": "records/s", "cores": 1, "kind": "oracle",
            "sample": f"intervals 0..{iv - 1} of {n_iv} ({recs} records, {dt:.1f} s, single thread)"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="matmul16")
    ap.add_argument("--workspace-gb", type=float, default=16.0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only copy GIB gibibytes device-to-device (a plain copy kernel of known size, "
                         "to scale the HBM byte counters) and exit")
    args = ap.parse_args()
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
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_2503_08946_amd as rv

    descs, wl_text = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: {wl_text}")
    ctx = rv.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)))
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
    assert sum(r.n_records for r in res) == n_records
    value = n_records * args.steps / elapsed
    lat.sort()
    p50 = lat[len(lat) // 2]
    p99 = lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]
    per_step = {k: v[0] / args.steps for k, v in stages.items()}
    log("[bench] GPU ms per step by stage: " + ", ".join(f"{k}={v:.3f}" for k, v in per_step.items()))
    # dominant kernel among those with a defined byte count
    dom = max(ALG_BYTES, key=lambda k: stages[k][0])
    launches = max(1, stages[dom][1])
    avg_ms = stages[dom][0] / launches
    recs_per_launch = n_records * args.steps / launches
    achieved = ALG_BYTES[dom] * recs_per_launch / (avg_ms * 1e-3) / 1e9
    kname = {"expand": "k_scatter", "sort_scan": "k_bucket"}[dom]
    traffic = traffic_for(kname, int(recs_per_launch))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
                "alg_bytes_per_record": ALG_BYTES[dom]}
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
                   "conflicts": sum(r.n_conflicts for r in res)},
        "latency_ms": {"p50": round(p50 * 1e3, 3), "p99": round(p99 * 1e3, 3)},
        "stage_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(descs[0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
