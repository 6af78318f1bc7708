#!/usr/bin/env python3
"""Benchmark: full FMM throughput (particles/s) and M2L GFLOP/s on one MI355X.

Workload (default): N = 2^24 particles uniform in the unit cube, charges
U(-1,1), uniform octree of depth 7 (128^3 leaves), expansion order p = 10,
ws = 1.  One step = one whole evaluation (keys, sort, P2M, M2M, M2L, L2L,
L2P, P2P) with inputs resident in HBM.  The chosen M2L precision is timed
next to plain FP64 on the same input, and the relative force error of the
chosen mode against FP64 is reported.

    python bench.py [--steps K] [--warmup W] [--precision fp64|fp32|bf16x3]

Prints one JSON line.  M2L roofline: algorithmic flops 2*S(p) per cell pair,
S(p) = (p+1)(p+2)((p+1)^2+(p+1)+1)/6 (non-zero entries of the traceless
operator), over the M2L kernel time measured with HIP events on the
library's stream during the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/s full FMM + M2L GFLOP/s at rel. force err 1e-6 (chosen vs plain FP64)"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16"}
DEFAULT_PRECISION = "fp32"


def s_of_p(p: int) -> int:
    q = p + 1
    return q * (q + 1) * (q * q + q + 1) // 6


def run_leg(F, torch, X, Q, p, depth, precision, steps, warmup):
    f = F.FMM(p, depth, precision)
    n = int(Q.shape[0])
    phi = torch.empty(n, dtype=torch.float64, device=Q.device)
    grad = torch.empty((n, 3), dtype=torch.float64, device=Q.device)
    for _ in range(warmup):
        f.evaluate(X, Q, phi, grad)
    F.ctfmm_sync(f.ctx)
    F.ctfmm_set_timing(f.ctx, True)
    F.ctfmm_reset_stats(f.ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        f.evaluate(X, Q, phi, grad)
        print(f"[bench] {precision} step {i + 1}/{steps}", file=sys.stderr, flush=True)
    F.ctfmm_sync(f.ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = F.ctfmm_stats(f.ctx)
    f.close()
    ms = (t1 - t0) * 1e3 / steps
    flops_pair = 2 * s_of_p(p)
    m2l_flops = st["m2l_pairs"] * flops_pair  # over all timed steps
    m2l_s = st["ms_m2l"] * 1e-3
    leg = {
        "precision": precision,
        "ms_per_step": ms,
        "particles_per_s": n / (ms * 1e-3),
        "m2l_gflops": m2l_flops / m2l_s / 1e9 if m2l_s > 0 else None,
        "phase_ms_per_step": {k[3:]: st[k] / steps for k in st if k.startswith("ms_")},
        "m2l_launches_per_step": st["m2l_launches"] // steps,
        "m2l_pairs_per_step": st["m2l_pairs"] // steps,
        "m2l_avg_launch_ms": st["ms_m2l"] / st["m2l_launches"] if st["m2l_launches"] else None,
    }
    return leg, phi, grad


def m2l_traffic(precision: str):
    """HBM bytes per M2L launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record, or None when it does not describe the kernel source built now."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", f"m2l_{precision}_uniform16M_p10_traffic.json")
    src = os.path.join(ROOT, "paper_1811_06332_amd", "csrc", "ctfmm_kernels.hip")
    if not os.path.exists(rec_path):
        return None
    rec = json.load(open(rec_path))
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != rec.get("kernel_source_sha256_16"):
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(p: int, depth_full: int):
    """The oracle on a 1/64 sub-volume of the same workload: a uniform cube at
    the same density (8 particles per leaf), same p and ws, depth - 2."""
    import numpy as np  # noqa: F401
    import oracle
    from paper_1811_06332_amd import workloads as W
    depth = depth_full - 2
    n = 8 * 8 ** depth
    xyz, q = W.uniform_cube(n, 1002, -1.0, 1.0)
    threads = len(os.sched_getaffinity(0))
    oracle.fmm_uniform(xyz[:64], q[:64], 1, 1, nthreads=threads)  # load and set threads
    used = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.fmm_uniform(xyz, q, p, depth, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "particles/s", "cores": used, "kind": "oracle",
            "sample": f"full oracle FMM of N={n} uniform particles (a 1/64 sub-volume of the workload at the "
                      f"same 8/leaf density: depth {depth}, p={p}, ws=1), one run of {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default=DEFAULT_PRECISION, choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--depth", type=int, default=7)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build evaluates on exactly one GPU; multi-GPU sharding is designed (DESIGN.md) "
              "but not implemented, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1811_06332_amd import ctfmm as F
    from paper_1811_06332_amd import workloads as W

    F.load()
    dev = torch.device("cuda:0")
    xyz, q = W.uniform_cube(args.n, 1002, -1.0, 1.0)
    X = torch.from_numpy(xyz).to(dev)
    Q = torch.from_numpy(q).to(dev)
    del xyz, q
    torch.cuda.synchronize()
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {a.numel() * 8} bytes done", file=sys.stderr, flush=True)
        del a, b
    print(f"[bench] N={args.n} p={args.p} depth={args.depth} precision={args.precision}", file=sys.stderr, flush=True)

    chosen, phi_c, grad_c = run_leg(F, torch, X, Q, args.p, args.depth, args.precision, args.steps, args.warmup)
    plain = None
    err = {"rel_force_err_vs_fp64": 0.0, "rel_potential_err_vs_fp64": 0.0}
    if args.precision != "fp64" and not args.no_fp64_leg:
        plain, phi_p, grad_p = run_leg(F, torch, X, Q, args.p, args.depth, "fp64", args.steps, args.warmup)
        err = {
            "rel_force_err_vs_fp64": float(torch.linalg.norm(grad_c - grad_p) / torch.linalg.norm(grad_p)),
            "rel_potential_err_vs_fp64": float(torch.linalg.norm(phi_c - phi_p) / torch.linalg.norm(phi_p)),
        }
    elif args.precision == "fp64":
        plain = chosen

    peak = PEAK_TFLOPS[args.precision]
    flops_launch = chosen["m2l_pairs_per_step"] * 2 * s_of_p(args.p) / max(1, chosen["m2l_launches_per_step"])
    achieved = flops_launch / (chosen["m2l_avg_launch_ms"] * 1e-3) / 1e12 if chosen["m2l_avg_launch_ms"] else None
    traffic = m2l_traffic(args.precision) if (args.n, args.p, args.depth) == (1 << 24, 10, 7) else None
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak if achieved else None, "traffic": traffic,
                "kernel": "M2L (all levels; algorithmic 2*S(p) flops per cell pair)",
                "flops_per_launch": flops_launch, "avg_launch_ms": chosen["m2l_avg_launch_ms"]}
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.p, args.depth)
    out = {
        "metric": METRIC,
        "value": chosen["particles_per_s"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chosen["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"uniform{args.n}_p{args.p}_d{args.depth}", "n": args.n, "p": args.p,
                   "depth": args.depth, "ws": 1, "charges": "U(-1,1)", "precision": args.precision},
        "m2l_gflops": chosen["m2l_gflops"],
        "chosen": chosen,
        "plain_fp64": plain,
        **err,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
