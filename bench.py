"""Benchmark: operator-apply throughput (GDOF/s) of the Chebyshev collocation
operator at 129^3 on one MI355X, plus the FP64 vs mixed-precision solve at the
same grid, the roofline of the axis-pass kernel and the CPU oracle baseline.

Contract: ``python bench.py --gpus N --steps K --warmup W`` prints ONE JSON line.
A step is one application of the reduced collocation operator (three axis
passes: DCT-I via the FFT of the even extension, derivative recurrence,
back-transform, flux K * du, divergence, boundary elimination) to one input
field of the 129^3 two-phase workload; inputs rotate over 16 (u, y) pairs so
the working set (>550 MB) exceeds the 256 MB Infinity Cache.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_ROT = 16


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(P, seconds_budget=20.0):
    """Time the oracle's reduced-operator apply (np.tensordot with dense D) on
    the host on a bounded sample: as many applies of the same 129^3 input as fit
    in the budget (at least one)."""
    import numpy as np
    from oracle import cheb_oracle as O
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    from paper_2606_21410_amd import workloads as W
    u = W.random_field(P.grid.n, 3)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    reps = 0
    while True:
        O.apply_reduced(G, P.K, u)
        reps += 1
        el = time.perf_counter() - t0
        if el > seconds_budget or reps >= 50:
            break
    npts = float(np.prod(P.grid.n))
    return {"value": npts * reps / el / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} reduced-operator applies of one 129^3 field (dense-D tensordot, FP64), "
                      f"{el:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=129)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is a "
                                   "design note only)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan, SolveOptions, prolong

    assert torch.cuda.is_available(), "bench needs a GPU"
    n = args.n
    dev = torch.device("cuda:0")
    _log(f"generating two-phase workload {n}^3")
    P = W.two_phase_problem(n, seed=1002, n_finest=n)
    shape = P.grid.n
    npts = float(np.prod(shape))

    def d(a, dt=torch.float64):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)

    res = {}
    stream = torch.cuda.current_stream(dev)
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        plan = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, prec, device=dev)
        K = d(P.K, dt)
        us = [d(W.random_field(shape, 100 + i), dt) for i in range(N_ROT)]
        ys = [torch.empty_like(us[0]) for _ in range(N_ROT)]
        for i in range(args.warmup):
            plan.apply(K, us[i % N_ROT], ys[i % N_ROT], "reduced")
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for i in range(args.steps):
            plan.apply(K, us[i % N_ROT], ys[i % N_ROT], "reduced")
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1) / args.steps
        res[prec] = {"ms_per_apply": ms, "gdofs": npts / (ms * 1e-3) / 1e9, "wall_s": wall}
        _log(f"apply {prec}: {ms * 1e3:.1f} us/apply, {res[prec]['gdofs']:.2f} GDOF/s")
        del us, ys, K, plan
        torch.cuda.empty_cache()

    # roofline of the dominant kernel (the axis pass): its own I/O per launch is
    # read u + read K + write y (24 B/pt) for the first pass and + read y (32 B/pt)
    # for the two accumulating passes -> 29.33 B/pt averaged over the 3 launches
    ms = res["f64"]["ms_per_apply"]
    launch_s = ms * 1e-3 / 3.0
    bytes_per_launch = (24.0 + 32.0 + 32.0) / 3.0 * npts
    achieved = bytes_per_launch / launch_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_axis_pass<double,128,REDUCED> (one axis pass; 3 launches per apply)",
                "apply_level_frac": round(24.0 * npts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    solve = None
    if not args.no_solve and n == 129:
        solve = {}
        _log("solve chain 33 -> 65 -> 129 (warm starts)")
        coarse = {m: W.two_phase_problem(m, seed=1002, n_finest=129) for m in (33, 65)}
        pl33 = Plan(coarse[33].grid.n, coarse[33].grid.lo, coarse[33].grid.hi, coarse[33].grid.bc, "f64", dev)
        pl65 = Plan(coarse[65].grid.n, coarse[65].grid.lo, coarse[65].grid.hi, coarse[65].grid.bc, "f64", dev)
        pl129 = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, "f64", dev)
        c33, c65 = coarse[33], coarse[65]
        u33, _ = pl33.solve(d(c33.K), d(c33.f), d(c33.g), opts=SolveOptions(rtol=1e-11, maxiter=40000))
        u65_0, _ = prolong(pl33, pl65, u33)
        u65, _ = pl65.solve(d(c65.K), d(c65.f), d(c65.g), u0=u65_0, opts=SolveOptions(rtol=1e-11, maxiter=40000))
        u0, _ = prolong(pl65, pl129, u65)
        K, f, g = d(P.K), d(P.f), d(P.g)
        sols = {}
        for label, prec, opts in (("fp64", "f64", SolveOptions(rtol=1e-10, maxiter=40000)),
                                  ("mixed", "mixed", SolveOptions(rtol=1e-10, maxiter=40000,
                                                                  ir_inner_rtol=1e-2))):
            pl = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, prec, dev)
            pl.ensure_workspace(opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, info = pl.solve(K, f, g, u0=u0, opts=opts)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            sols[label] = u.clone()
            solve[label] = {"seconds": round(el, 4), "matvecs": info["matvecs"],
                            "matvecs_f32": info["matvecs_f32"], "relres": info["relres_final"],
                            "status": info["status"]}
            _log(f"solve {label}: {el:.3f} s {info}")
            del pl
        solve["rel_diff_mixed_vs_fp64"] = float((sols["mixed"] - sols["fp64"]).norm() / sols["fp64"].norm())
        solve["speedup_mixed"] = round(solve["fp64"]["seconds"] / solve["mixed"]["seconds"], 3)
        solve["tolerance"] = "relative residual 1e-10 of the reduced system, warm start from prolonged 65^3"

    cpu = None
    if not args.no_cpu:
        _log("cpu baseline (oracle)")
        cpu = cpu_baseline(P)

    out = {
        "metric": "GDOF/s operator apply + time-to-1e-8 solve @129^3, mixed vs FP64, 1 GPU",
        "value": round(res["f64"]["gdofs"], 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["f64"]["ms_per_apply"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"two-phase conductivity {n}^3 CGL (spheres R=0.15, vf=0.2, contrast 10, "
                               f"tanh width 2h, seed 1002), u=-1/+1 on x faces, zero flux elsewhere; "
                               f"reduced operator apply", "grid": list(shape), "rotating_buffers": N_ROT},
        "f32_apply_gdofs": round(res["f32"]["gdofs"], 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "solve_129": solve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
