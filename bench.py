"""Benchmark: operator-apply throughput (GDOF/s) of the Chebyshev collocation
operator at 129^3 on one MI355X, plus the FP64 vs mixed-precision solve at the
same grid, the roofline of the axis-pass kernel and the CPU oracle baseline.

Contract: ``python bench.py --gpus N --steps K --warmup W`` prints ONE JSON line.
A step is one application of the reduced collocation operator (per axis:
derivative, flux K * du, divergence, boundary elimination; the derivative by
the DCT-I of the even extension on the FFT route or as a dense contraction on
the matrix-core route, whichever the autotuner picks) to one input field of
the 129^3 two-phase workload; inputs rotate over 16 (u, y) pairs so the
working set (>550 MB) exceeds the 256 MB Infinity Cache.
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
# the method's minimum HBM bytes per point of one FP64 operator apply: read u and
# K, write y
ALG_BYTES_PER_POINT_F64 = 24.0


def _traffic_record(route):
    """HBM bytes per apply measured with rocprofv3 for the apply's kernels
    (profiles/k_dense_pass_f64_129cubed_hbm_bytes.txt), or None when the
    kernel sources or the chosen tile shape differ from the profiled ones."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_dense_pass_f64_129cubed_hbm_bytes.txt")
    if not os.path.exists(path) or route not in ("matrix0", "matrix1"):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
    if rec is None:
        return None
    for f, h in rec["sources"].items():
        cur = hashlib.sha1(open(os.path.join(ROOT, "paper_2606_21410_amd", "csrc", f), "rb").read()).hexdigest()[:12]
        if cur != h:
            return None
    if rec.get("variant") != int(route[-1]):
        return None
    return rec


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _blas_threads():
    from threadpoolctl import threadpool_info
    return max((i.get("num_threads") or 0 for i in threadpool_info()), default=0)


def cpu_baseline(P, reps=5):
    """Time the oracle's reduced-operator apply (np.tensordot with dense D) on
    the host: one warm-up, then the median of ``reps`` applies to the same 129^3
    input, with the BLAS pool set to every core of the affinity mask (the
    count used is recorded)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import cheb_oracle as O
    from paper_2606_21410_amd import workloads as W
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    u = W.random_field(P.grid.n, 3)
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        threads = _blas_threads()
        O.apply_reduced(G, P.K, u)
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            O.apply_reduced(G, P.K, u)
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    npts = float(np.prod(P.grid.n))
    return {"value": round(npts / med / 1e9, 5), "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": f"median of {reps} reduced-operator applies of one 129^3 field after one warm-up "
                      f"(dense-D tensordot, FP64), {med:.3f} s each; BLAS threads {threads} of "
                      f"{cores} cores in the affinity mask"}


def oracle_reference(P):
    """The oracle's solution of the 129^3 collocation system (FDM-preconditioned
    GMRES to relative residual 1e-13), the reference every time-to-1e-8 error is
    measured against; its host wall time is reported next to the GPU solves."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import cheb_oracle as O
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        threads = _blas_threads()
        t0 = time.perf_counter()
        rt = O.reduced_rhs(G, P.K, P.f, P.g)
        x, its, rel = O.solve_interior_system(G, P.K, rt, tol=1e-13)
        U = O.lift(G, x, P.g)
        el = time.perf_counter() - t0
    return U, {"seconds": round(el, 2), "gmres_iterations": int(its), "relres": float(rel),
               "blas_threads": threads, "kind": "oracle: FDM-preconditioned GMRES to relative residual 1e-13"}


def cpu_detail(P, seconds_budget=4.0):
    """More oracle timings on the host: the same 129^3 reduced apply with one
    BLAS thread (median of three after a warm-up), and the oracle's solve of the
    33^3 two-phase problem (spheres R = 0.15, vf 0.2, contrast 10, seed 1002;
    FDM-preconditioned GMRES to 1e-13), median of three, with all threads."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import cheb_oracle as O
    from paper_2606_21410_amd import workloads as W
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    u = W.random_field(P.grid.n, 3)
    with threadpool_limits(limits=1):
        O.apply_reduced(G, P.K, u)
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            O.apply_reduced(G, P.K, u)
            times.append(time.perf_counter() - t0)
    one = float(np.prod(P.grid.n)) / float(np.median(times)) / 1e9
    Q = W.two_phase_problem(33, seed=1002, n_finest=33)
    Gq = O.Grid3(Q.grid.n, Q.grid.lo, Q.grid.hi, Q.grid.bc)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.solve(Gq, Q.K, Q.f, Q.g, tol=1e-13)
        times.append(time.perf_counter() - t0)
    return {"apply_1thread_gdofs": round(one, 5), "apply_1thread_sample": "median of 3 applies",
            "solve_33_seconds_median": round(sorted(times)[1], 3),
            "solve_33_kind": "oracle FDM-preconditioned GMRES to 1e-13, all threads"}


def _solve_once(P, shape, prec, opts, K, f, g, u0, dev):
    """One timed solve on a fresh plan: the plan is created and its workspace
    allocated before the timed region; the preconditioner's set-up (its host
    eigen-decompositions and tables, done on first use) and the solve are
    inside it."""
    import torch
    from paper_2606_21410_amd.api import Plan
    pl = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, prec, dev)
    pl.ensure_workspace(opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, info = pl.solve(K, f, g, u0=u0, opts=opts)
    torch.cuda.synchronize()
    return u, info, time.perf_counter() - t0


def _solve_warm(P, shape, prec, opts, K, f, g, u0, dev, repeats):
    """Median time of ``repeats`` solves on one plan after an untimed first
    solve (the plan's preconditioner set-up and autotuning are then done): the
    cost of a solve for a caller that keeps its plan."""
    import numpy as np
    import torch
    from paper_2606_21410_amd.api import Plan
    pl = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, prec, dev)
    pl.ensure_workspace(opts)
    pl.solve(K, f, g, u0=u0, opts=opts)
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.solve(K, f, g, u0=u0, opts=opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return float(np.median(times))


# residual tolerances tried for the preconditioned solves, loosest first, on a 1-2-5 grid so that
# the first rung meeting the error bar does not overshoot it by a decade
PRE_LADDER = (1e-8, 5e-9, 2e-9, 1e-9, 5e-10, 2e-10, 1e-10, 1e-11)
# inner tolerance of the preconditioned MIXED solve (measured at 129^3: 7e-5 reaches error 2.6e-9
# in two refinement steps, 9.8 ms; 1e-4 gave 1.1e-8, on the edge of the bar)
PRE_MIXED_INNER = 7e-5


def _time_to_error(P, shape, prec, mk_opts, ladder, K, f, g, u0, uref, dev, target=1e-8, repeats=1):
    """Walk a ladder of relative-residual tolerances and stop at the first whose
    solution is within ``target`` (relative L2) of ``uref``; report its time
    (median of ``repeats`` runs) and every rung tried."""
    import numpy as np
    rungs = []
    for rt in ladder:
        u, info, el = _solve_once(P, shape, prec, mk_opts(rt), K, f, g, u0, dev)
        err = float((u - uref).norm() / uref.norm())
        rungs.append({"rtol": rt, "seconds": round(el, 4), "matvecs": info["matvecs"],
                      "matvecs_f32": info["matvecs_f32"], "ir_steps": info["ir_steps"],
                      "relres": info["relres_final"], "status": info["status"], "rel_err": err})
        _log(f"  {prec} rtol {rt:g}: {el:.3f} s, err {err:.3e}, {info}")
        if err <= target:
            times = [el] + [_solve_once(P, shape, prec, mk_opts(rt), K, f, g, u0, dev)[2]
                            for _ in range(repeats - 1)]
            rec = {"reached": True, "seconds": round(float(np.median(times)), 4), "rtol": rt,
                   "rel_err": err, "matvecs": info["matvecs"], "matvecs_f32": info["matvecs_f32"],
                   "rungs": rungs}
            if repeats > 1:
                rec["seconds_plan_reused"] = round(_solve_warm(P, shape, prec, mk_opts(rt), K, f, g, u0, dev,
                                                               repeats), 4)
            return rec
        if info["status"] == 2:
            break  # stagnated: a tighter tolerance cannot help
    return {"reached": False, "best_rel_err": min(r["rel_err"] for r in rungs), "rungs": rungs}


def solve_section(P, d, dev, shape, uref_host, ref_info):
    """Time-to-1e-8 at 129^3 for the plain FP64 LGMRES solver of the method
    (hierarchical warm start 33 -> 65 -> 129), its mixed FP32/FP64 refinement,
    and the same two with the fast-diagonalisation preconditioner (cold start:
    a fresh plan per timed solve; also timed with the plan kept across solves).
    The accuracy reference is the oracle's 129^3 solution (computed on the host
    in the CPU-baseline leg)."""
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan, SolveOptions, prolong
    K, f, g = d(P.K), d(P.f), d(P.g)
    out = {}
    uref = d(uref_host)
    out["reference"] = ref_info
    _log("hierarchical chain 33 -> 65 -> 129 (plain FP64 LGMRES)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    coarse = {m: W.two_phase_problem(m, seed=1002, n_finest=129) for m in (33, 65)}
    pls = {m: Plan(coarse[m].grid.n, coarse[m].grid.lo, coarse[m].grid.hi, coarse[m].grid.bc, "f64", dev)
           for m in (33, 65)}
    c33, c65 = coarse[33], coarse[65]
    u33, _ = pls[33].solve(d(c33.K), d(c33.f), d(c33.g), opts=SolveOptions(rtol=1e-11, maxiter=40000))
    u65_0, _ = prolong(pls[33], pls[65], u33)
    u65, _ = pls[65].solve(d(c65.K), d(c65.f), d(c65.g), u0=u65_0, opts=SolveOptions(rtol=1e-11, maxiter=40000))
    pl129 = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, "f64", dev)
    u0, _ = prolong(pls[65], pl129, u65)
    torch.cuda.synchronize()
    chain_s = time.perf_counter() - t0
    out["chain_33_65_seconds"] = round(chain_s, 4)
    out["prolonged_start_rel_err"] = float((u0 - uref).norm() / uref.norm())

    plain = lambda rt: SolveOptions(rtol=rt, maxiter=200000)
    mixed = lambda rt: SolveOptions(rtol=rt, maxiter=200000, ir_inner_rtol=1e-3)
    # preconditioned runs: restart length 20 (a sweep over 10..30 at 129^3 was fastest there for
    # FP64 and flat for MIXED; the library default stays 30)
    pre = lambda rt: SolveOptions(rtol=rt, maxiter=5000, precond=True, inner_m=20)
    # the preconditioned MIXED run refines with inner solves to PRE_MIXED_INNER: two refinement
    # steps then leave an error well under the bar (1e-4 left it on the bar's edge)
    pre_mixed = lambda rt: SolveOptions(rtol=rt, maxiter=5000, precond=True, inner_m=20,
                                        ir_inner_rtol=PRE_MIXED_INNER)
    _log("time to 1e-8: plain FP64 (warm)")
    out["fp64_plain"] = _time_to_error(P, shape, "f64", plain, (1e-12, 1e-13, 1e-14), K, f, g, u0, uref, dev)
    _log("time to 1e-8: plain mixed (warm)")
    out["mixed_plain"] = _time_to_error(P, shape, "mixed", mixed, (1e-10, 1e-12), K, f, g, u0, uref, dev)
    _log("time to 1e-8: preconditioned FP64 (cold)")
    out["fp64_precond"] = _time_to_error(P, shape, "f64", pre, PRE_LADDER, K, f, g, None, uref, dev, repeats=5)
    _log("time to 1e-8: preconditioned mixed (cold)")
    out["mixed_precond"] = _time_to_error(P, shape, "mixed", pre_mixed, PRE_LADDER, K, f, g, None, uref, dev,
                                          repeats=5)
    fp = out["fp64_plain"]
    if fp["reached"]:
        out["fp64_plain"]["seconds_incl_chain"] = round(fp["seconds"] + chain_s, 4)
        # against the paper's plain FP64 solver: these ratios change the precision and
        # (for the preconditioned runs) the solver at once
        for k in ("mixed_plain", "fp64_precond", "mixed_precond"):
            if out[k]["reached"]:
                out[k]["speedup_vs_paper_plain_fp64"] = round(fp["seconds"] / out[k]["seconds"], 2)
    if out["fp64_precond"]["reached"] and out["mixed_precond"]["reached"]:
        # precision alone: the same preconditioned solver in FP64 and in mixed precision
        out["mixed_precond"]["speedup_vs_fp64_precond"] = round(
            out["fp64_precond"]["seconds"] / out["mixed_precond"]["seconds"], 3)
        # the same with each plan kept across solves (no set-up in the timed solve)
        out["mixed_precond"]["speedup_vs_fp64_precond_plan_reused"] = round(
            out["fp64_precond"]["seconds_plan_reused"] / out["mixed_precond"]["seconds_plan_reused"], 3)
    out["target"] = "relative L2 error <= 1e-8 to the oracle's 129^3 solution"
    return out


def _homog_inputs(dev, n_struct=32, rtol=1e-10):
    """The homogenisation workload's microstructures (sizes from {33, 49, 65, 97}^3, seed 1004,
    log-normal sigma 1, length 0.2) on the GPU and the solver options of its batch."""
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import SolveOptions
    r = W.rng(1004)
    sizes = [int(v) for v in r.choice([33, 49, 65, 97], size=n_struct)]
    Ks = []
    for i, n in enumerate(sizes):
        grid = W.Grid((n, n, n), (0, 0, 0), (1, 1, 1), W.MIXED_X_BC)
        Ks.append(torch.from_numpy(W.lognormal_conductivity(grid, (1004, i), 1.0, 0.2)).to(dev))
    # restart length 20 and (MIXED) inner tolerance 1e-4, as for the preconditioned 129^3 runs
    # (a sweep on this batch: FP64 1.30 -> 1.20 s, MIXED 1.36 -> 1.21 s against 30 / 1e-3)
    opts = SolveOptions(rtol=rtol, maxiter=20000, precond=True, inner_m=20, ir_inner_rtol=1e-4)
    return sizes, Ks, opts


def homogenisation_section(dev, n_struct=32, rtol=1e-10):
    """Batched homogenisation workload: 32 log-normal microstructures (sigma 1,
    correlation length 0.2) on grids drawn uniformly from {33, 49, 65, 97}^3
    (seed 1004), three load cases each = 96 systems, FP32 inner / FP64
    refinement with the fast-diagonalisation preconditioner, solved as one
    batch; against the same solver looped over the 96 systems one by one."""
    import torch
    from paper_2606_21410_amd.api import Plan, homogenize, load_case
    sizes, Ks, opts = _homog_inputs(dev, n_struct, rtol)
    out = {"structures": n_struct, "systems": 3 * n_struct, "sizes": sizes,
           "points": int(sum(3 * n ** 3 for n in sizes)), "rtol": rtol}
    for label, prec in (("batched_mixed", "mixed"), ("batched_fp64", "f64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        det = {}
        Kapp, infos, _ = homogenize(Ks, precision=prec, opts=opts, details=det)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[label] = {"seconds": round(el, 3), "max_matvecs": max(i["matvecs"] for i in infos),
                      "matvecs_per_system": [i["matvecs"] for i in infos],
                      "all_converged": all(i["status"] == 0 for i in infos),
                      "max_relres": max(i["relres_final"] for i in infos)}
        batch = det.pop("batch")
        out[label]["tile_shapes"] = det
        # the same batch again: plans, preconditioner factors and tile shapes set up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        homogenize(Ks, precision=prec, opts=opts, batch=batch)
        torch.cuda.synchronize()
        out[label]["seconds_batch_reused"] = round(time.perf_counter() - t0, 3)
        del batch
        if label == "batched_mixed":
            out["K_app_first"] = [[round(v, 6) for v in row] for row in Kapp[0]]
        _log(f"homogenisation {label}: {el:.3f} s")
    # the same solver looped over the systems
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mvs = []
    for K in Ks:
        n = tuple(K.shape)
        for a in range(3):
            bc, g = load_case(n, a, dev)
            pl = Plan(n, (0, 0, 0), (1, 1, 1), bc, "mixed", dev)
            u, info = pl.solve(K, torch.zeros(n, dtype=torch.float64, device=dev), g, opts=opts)
            mvs.append(info["matvecs"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["looped_mixed"] = {"seconds": round(el, 3), "max_matvecs": max(mvs)}
    out["speedup_batched_vs_looped"] = round(el / out["batched_mixed"]["seconds"], 2)
    # both warm: one plan per (size, load case) made beforehand, solves timed
    plans = {}
    for K in Ks:
        n = tuple(K.shape)
        for a in range(3):
            if (n, a) not in plans:
                bc, g = load_case(n, a, dev)
                pl = Plan(n, (0, 0, 0), (1, 1, 1), bc, "mixed", dev)
                pl.solve(K, torch.zeros(n, dtype=torch.float64, device=dev), g, opts=opts)
                plans[(n, a)] = (pl, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for K in Ks:
        n = tuple(K.shape)
        for a in range(3):
            pl, g = plans[(n, a)]
            pl.solve(K, torch.zeros(n, dtype=torch.float64, device=dev), g, opts=opts)
    torch.cuda.synchronize()
    el2 = time.perf_counter() - t0
    out["looped_mixed"]["seconds_plans_reused"] = round(el2, 3)
    out["speedup_batched_vs_looped_both_reused"] = round(el2 / out["batched_mixed"]["seconds_batch_reused"], 2)
    del plans
    _log(f"homogenisation looped: {el:.3f} s")
    return out


def inclusion_section(dev, n=129, n_plain=33, rtol=1e-10):
    """Section 3.3's spherical-inclusion study: one sphere of radius 0.2 at the
    box centre (phi = 0.0335), or its eighths at the eight corners, sampled
    sharply at the nodes; u = -1 / +1 on the x faces, zero flux elsewhere;
    contrast k_i/k_m = 1e-4 .. 1e4.  Per contrast: the preconditioned FP64
    solve at n^3 (matvecs, seconds, K_num = <K du/dx>/G, Maxwell's dilute
    estimate, their relative difference) and the plain LGMRES iteration count
    at n_plain^3 to rtol 1e-6 (the paper's solver)."""
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan, SolveOptions

    def d(a):
        return torch.from_numpy(a).to(dev, torch.float64)

    out = {"n": n, "n_plain": n_plain, "rtol": rtol, "radius": 0.2}
    for layout in ("center", "corner"):
        rows = []
        for k in range(-4, 5):
            c = 10.0 ** k
            P = W.inclusion_problem(n, c, layout)
            pl = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "f64", dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, info = pl.solve(d(P.K), d(P.f), d(P.g), opts=SolveOptions(rtol=rtol, maxiter=20000, precond=True))
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            knum = pl.flux_average(d(P.K), u)[0] / P.meta["G"]
            km = W.maxwell_keff(P.meta["phi"], c)
            Pp = W.inclusion_problem(n_plain, c, layout)
            pp = Plan(Pp.grid.n, Pp.grid.lo, Pp.grid.hi, Pp.grid.bc, "f64", dev)
            _, pinfo = pp.solve(d(Pp.K), d(Pp.f), d(Pp.g), opts=SolveOptions(rtol=1e-6, maxiter=30000))
            rows.append({"contrast": c, "matvecs": info["matvecs"], "status": info["status"], "seconds": round(el, 4),
                         "K_num": round(knum, 7), "K_maxwell": round(km, 7), "rel_diff": float(abs(knum - km) / km),
                         "plain_matvecs": pinfo["matvecs"], "plain_status": pinfo["status"]})
            _log(f"  {layout} contrast {c:g}: {rows[-1]}")
        out[layout] = rows
    out["phi"] = 4.0 / 3.0 * 3.141592653589793 * 0.2 ** 3
    return out


def picard_chain_section(dev, levels=(33, 65, 129, 257)):
    """Nonlinear two-phase workload: spheres at volume fraction 0.3 (seed 1003),
    contrast 100, tanh width 2/256, K = K0 (1 + u^2/2), u = -1/+1 on the x faces;
    Picard iterations of mixed FP32 / FP64 solves with the preconditioner,
    hierarchical 33 -> 65 -> 129 -> 257 with modal prolongation as warm start.
    Per level: time, Picard steps, matvecs and the refinement indicator e_ref."""
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan, SolveOptions, prolong
    opts = SolveOptions(rtol=1e-10, maxiter=20000, precond=True)
    out = []
    prev = None
    for n in levels:
        P = W.two_phase_problem(n, seed=1003, volume_fraction=0.3, contrast=100.0, n_finest=levels[-1])
        K0 = torch.from_numpy(P.K).to(dev)
        f = torch.from_numpy(P.f).to(dev)
        g = torch.from_numpy(P.g).to(dev)
        plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "mixed", dev)
        plan.ensure_workspace(opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u0 = prolong(prev[0], plan, prev[1])[0] if prev else None
        u, info = plan.picard(K0, f, g, u0=u0, tol=1e-10, max_steps=60, opts=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec = {"n": n, "seconds": round(el, 3), "picard_steps": info["picard_steps"], "matvecs": info["matvecs"],
               "status": info["rc"]}
        if prev:
            _, e = prolong(prev[0], plan, prev[1], uf_solved=u)
            rec["e_ref"] = e
        _log(f"picard chain {rec}")
        out.append(rec)
        prev = (plan, u)
    return out


def _thermal_plan(N, dev):
    """The Section 3.4 problem at N with its flux rows k(T) dT/dn = h on the
    Neumann faces (per-node Robin rows dT/dn - alpha h T = h), its inputs on the
    GPU and its plan."""
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan
    P = W.thermal_nonlinear(N + 1, flux_form=True)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "f64", dev, robin=P.grid.robin,
                robin_nodes=P.grid.robin_nodes)
    t = lambda a: torch.from_numpy(a).to(dev)
    return P, plan, t(P.K), t(P.f), t(P.g)


def thermal_newton_section(dev, levels=(4, 8, 16, 32, 64, 128, 256), tol=1e-11, max_steps=20, maxiter=2000):
    """Section 3.4 nonlinear thermal problem, k(T) = 1 / (1 + T/2) on (0,1)^3
    with the analytic T = (exp(Phi/2) - 1) * 2, Phi = sin(pi x) sin(pi y) sin(pi z),
    and the flux condition on the Neumann faces: Newton-LGMRES (FP64,
    fast-diagonalisation preconditioner) along Table 1's chain
    N = 4 -> 8 -> ... -> 256 with the modal prolongation as warm start.  Per
    level: Newton updates, LGMRES products (total and per update), max error
    against the analytic T, e_ref and the time of prolongation + Newton
    (inputs already on the GPU)."""
    import torch
    from paper_2606_21410_amd.api import SolveOptions, prolong
    opts = SolveOptions(rtol=1e-10, maxiter=maxiter, precond=True)
    out = []
    prev = None
    for N in levels:
        P, plan, K0, f, g = _thermal_plan(N, dev)
        plan.ensure_workspace(opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u0 = prolong(prev[0], plan, prev[1])[0] if prev else None
        u, info = plan.newton(K0, f, g, alpha=P.meta["alpha"], u0=u0, tol=tol, max_steps=max_steps,
                              opts=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        err = float((u - torch.from_numpy(P.u_exact).to(dev)).abs().max().item())
        rec = {"N": N, "newton_steps": info["newton_steps"], "lgmres_total": sum(info["mv_per_step"]),
               "lgmres_per_step": info["mv_per_step"], "max_error": err, "seconds": round(el, 4),
               "status": info["rc"]}
        if prev:
            rec["e_ref"] = prolong(prev[0], plan, prev[1], uf_solved=u)[1]
        _log(f"thermal newton {rec}")
        out.append(rec)
        prev = (plan, u)
        del K0, f, g
    return out


def thermal_newton_cold(dev, levels=(128, 256), tol=1e-11, max_steps=20, maxiter=2000):
    """The Section 3.4 problem solved by Newton-LGMRES from a cold start
    (T_0 = lift(0, g)) at the large levels, so that their time is Newton work
    (the refinement chain reaches them with the prolonged solution already at
    the stopping rule)."""
    import torch
    from paper_2606_21410_amd.api import SolveOptions
    opts = SolveOptions(rtol=1e-10, maxiter=maxiter, precond=True)
    out = []
    for N in levels:
        P, plan, K0, f, g = _thermal_plan(N, dev)
        plan.ensure_workspace(opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = plan.newton(K0, f, g, alpha=P.meta["alpha"], tol=tol, max_steps=max_steps, opts=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        err = float((u - torch.from_numpy(P.u_exact).to(dev)).abs().max().item())
        # one Jacobian call (coefficients k, c_a at the solution, then J v),
        # event-timed: the per-product cost, which does not move with the
        # LGMRES counts near the tolerance floor
        v = torch.randn(P.grid.n, device=dev, dtype=torch.float64)
        y = torch.empty_like(v)
        for _ in range(3):
            plan.newton_jacobian(K0, u, v, alpha=P.meta["alpha"], out=y)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            plan.newton_jacobian(K0, u, v, alpha=P.meta["alpha"], out=y)
        ev1.record()
        torch.cuda.synchronize()
        rec = {"N": N, "start": "cold", "newton_steps": info["newton_steps"],
               "lgmres_total": sum(info["mv_per_step"]), "lgmres_per_step": info["mv_per_step"],
               "max_error": err, "seconds": round(el, 4), "status": info["rc"],
               "jacobian_call_us": round(ev0.elapsed_time(ev1) * 1e3 / 10, 1)}
        _log(f"thermal newton cold {rec}")
        out.append(rec)
        del K0, f, g, u, v, y, plan
        torch.cuda.empty_cache()
    return out


def refinement_stop_section(dev, levels=(33, 65, 129, 257), tol=2e-3):
    """Hierarchical refinement with its stopping rule (Algorithm 4) on the
    two-phase generator (spheres R 0.15, vf 0.2, contrast 10, width 2/256):
    preconditioned FP64 solves level by level until the refinement indicator
    e_ref <= tol, then the prolongation alone; against the same chain with
    every level solved."""
    import numpy as np
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan, SolveOptions, refine
    probs = [W.two_phase_problem(n, seed=1002, n_finest=levels[-1]) for n in levels]
    plans = [Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "f64", dev) for P in probs]
    d = lambda a: torch.from_numpy(a).to(dev)
    Ks, fs, gs = [d(P.K) for P in probs], [d(P.f) for P in probs], [d(P.g) for P in probs]
    opts = SolveOptions(rtol=1e-10, maxiter=5000, precond=True, inner_m=20)
    out = {"levels": list(levels), "tol": tol}
    for label, t in (("every_level", 0.0), ("with_stop", tol)):
        refine(plans, Ks, fs, gs, t, opts)  # warm-up (plans, preconditioner set-up)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        us, e, solved, infos = refine(plans, Ks, fs, gs, t, opts)
        torch.cuda.synchronize()
        out[label] = {"seconds": round(time.perf_counter() - t0, 4), "solved": solved,
                      "e_ref": [None if np.isnan(v) else float(v) for v in e],
                      "matvecs": [i["matvecs"] for i in infos]}
        if label == "every_level":
            ufull = us[-1].clone()
        else:
            out[label]["finest_rel_diff_to_every_level"] = float((us[-1] - ufull).norm() / ufull.norm())
        _log(f"refinement {label}: {out[label]}")
    del us, ufull, Ks, fs, gs, plans
    torch.cuda.empty_cache()
    return out


def precond_section(dev, P, reps=50, warmup=5):
    """One application of the fast-diagonalisation preconditioner
    (cheb_precond_apply) on the 129^3 workload's grid with Kc = mean K, FP64 and
    FP32 fields, event-timed on the plan's stream.  Bytes: each of the five
    launches (x, y, the fused z pair, y, x) reads and writes one field of the
    interior nodes, 10 x m^3 x sizeof(T)."""
    import numpy as np
    import torch
    from paper_2606_21410_amd.api import Plan
    from paper_2606_21410_amd import workloads as W
    out = {}
    m = [v - 2 for v in P.grid.n]
    kc = float(np.mean(P.K))
    r = W.random_field(P.grid.n, 5)
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        pl = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, prec, dev)
        rd = torch.from_numpy(r).to(dev, dt)
        yd = torch.empty_like(rd)
        for _ in range(warmup):
            pl.precond(rd, kc, out=yd)
        stream = torch.cuda.current_stream(dev)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            pl.precond(rd, kc, out=yd)
        ev1.record(stream)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / reps
        nbytes = 10 * m[0] * m[1] * m[2] * (8 if prec == "f64" else 4)
        out[prec] = {"us_per_application": round(us, 2), "launches": 5,
                     "mb_moved": round(nbytes / 1e6, 1), "gbs": round(nbytes / us / 1e3, 1)}
        del pl, rd, yd
    torch.cuda.empty_cache()
    return out


def copy_reference(dev, n=64 * 1024 * 1024, reps=20):
    """Attainable HBM bandwidth: the library's stream-copy kernel (cheb_debug_copy)
    moving n doubles (512 MiB read + 512 MiB written, far beyond the 256 MB
    Infinity Cache), event-timed on the current stream.  GB/s counts read plus
    write bytes."""
    import ctypes
    import torch
    from paper_2606_21410_amd import _lib as L
    lib = L.load()
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream(dev)
    h = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(3):
        L.check(lib.cheb_debug_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, h))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        L.check(lib.cheb_debug_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, h))
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    torch.cuda.empty_cache()
    return {"gbs": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1), "bytes_moved": 2 * n * 8, "ms": round(ms, 4),
            "copy_checked": ok}


def apply_257(dev, steps=40, warmup=5, rot=4):
    """FP64 reduced apply on the 257^3 two-phase grid (the FFT route: the
    matrix-core route covers N <= 128), rotating buffers, event-timed."""
    import numpy as np
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan
    P = W.two_phase_problem(257, seed=1002, n_finest=257)
    shape = P.grid.n
    plan = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, "f64", device=dev)
    K = torch.from_numpy(P.K).to(dev)
    us = [torch.from_numpy(W.random_field(shape, 200 + i)).to(dev) for i in range(rot)]
    ys = [torch.empty_like(us[0]) for _ in range(rot)]
    for i in range(warmup):
        plan.apply(K, us[i % rot], ys[i % rot], "reduced")
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(steps):
        plan.apply(K, us[i % rot], ys[i % rot], "reduced")
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    npts = float(np.prod(shape))
    alg = ALG_BYTES_PER_POINT_F64 * npts / (ms * 1e-3) / 1e9
    del us, ys, K, plan
    torch.cuda.empty_cache()
    return {"ms_per_apply": round(ms, 4), "gdofs": round(npts / (ms * 1e-3) / 1e9, 3),
            "algorithmic_gbs": round(alg, 1), "frac": round(alg / HBM_PEAK_GBS, 4), "route": "fft"}


def robin_section(dev, P, steps=100, warmup=10):
    """Robin rows on the metric workload: the 129^3 two-phase K with
    du/dn + u = 0 on its four former zero-flux faces (sigma = 1), reduced FP64
    applies timed with events; and the sin(pi x) cos(pi y) e^z field on
    [-1,1]^3 (Dirichlet x faces, Robin sigma = 1.5, 0.5, 2, 0.25 on the y and z
    faces) solved at 129^3 by preconditioned FP64 LGMRES, with its max error
    against the analytic field."""
    import numpy as np
    import torch
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import Plan, SolveOptions
    robin = tuple(0.0 if b == W.DIRICHLET else 1.0 for b in P.grid.bc)
    shape = P.grid.n
    plan = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, "f64", device=dev, robin=robin)
    K = torch.from_numpy(P.K).to(dev)
    us = [torch.from_numpy(W.random_field(shape, 100 + i)).to(dev) for i in range(4)]
    ys = [torch.empty_like(us[0]) for _ in range(4)]
    for i in range(warmup):
        plan.apply(K, us[i % 4], ys[i % 4], "reduced")
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(steps):
        plan.apply(K, us[i % 4], ys[i % 4], "reduced")
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    out = {"apply_ms": round(ms, 5), "apply_gdofs": round(float(np.prod(shape)) / (ms * 1e-3) / 1e9, 3),
           "robin": list(robin)}
    sig = (0.0, 0.0, 1.5, 0.5, 2.0, 0.25)
    M = W.manufactured_sincos(shape[0], robin=sig)
    pm = Plan(M.grid.n, M.grid.lo, M.grid.hi, M.grid.bc, "f64", device=dev, robin=sig)
    opts = SolveOptions(rtol=1e-10, precond=True)
    pm.ensure_workspace(opts)
    Km, fm, gm = (torch.from_numpy(a).to(dev) for a in (M.K, M.f, M.g))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, info = pm.solve(Km, fm, gm, opts=opts)
    torch.cuda.synchronize()
    out["sincos_solve"] = {"seconds": round(time.perf_counter() - t0, 4), "matvecs": info["matvecs"],
                           "status": info["status"], "robin": list(sig),
                           "max_error": float((u - torch.from_numpy(M.u_exact).to(dev)).abs().max().item())}
    _log(f"robin {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=129)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--profile-apply", action="store_true",
                    help="for profiler runs: 4 plain device copies of one FP64 field (the byte-counter "
                         "calibration), then the FP64 applies only")
    ap.add_argument("--profile-newton", action="store_true",
                    help="for profiler runs: the Section 3.4 Newton solve from a cold start at N = 128, then "
                         "the refinement chain N = 4 .. 128 (flux rows on the Neumann faces)")
    ap.add_argument("--profile-precond", action="store_true",
                    help="for profiler runs: the preconditioner applications of the bench's precond section "
                         "only")
    ap.add_argument("--profile-batch", action="store_true",
                    help="for profiler runs: the 96-system homogenisation batch (MIXED), solved twice on "
                         "one batch (the first with set-up and tile tuning)")
    ap.add_argument("--profile-solve", action="store_true",
                    help="for profiler runs: the preconditioned FP64 and mixed solves only, each twice on "
                         "one plan (the first with plan and preconditioner set-up)")
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

    if args.profile_newton:
        T, pl, K0t, ft, gt = _thermal_plan(128, dev)
        opts = SolveOptions(rtol=1e-10, precond=True)
        pl.ensure_workspace(opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = pl.newton(K0t, ft, gt, alpha=T.meta["alpha"], tol=1e-11, max_steps=20, opts=opts)
        torch.cuda.synchronize()
        cold = {"seconds": round(time.perf_counter() - t0, 4), "newton_steps": info["newton_steps"],
                "mv_per_step": info["mv_per_step"], "status": info["rc"],
                "max_error": float((u - d(T.u_exact)).abs().max().item())}
        _log(f"cold Newton N=128: {cold}")
        chain = thermal_newton_section(dev, levels=(4, 8, 16, 32, 64, 128))
        print(json.dumps({"profile_newton": {"cold_128": cold, "chain": chain}}), flush=True)
        return

    if args.profile_batch:
        from paper_2606_21410_amd.api import homogenize
        _, Ks, hopts = _homog_inputs(dev)
        rec = {}
        det = {}
        for label in ("first", "second"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos, _ = homogenize(Ks, precision="mixed", opts=hopts, details=det, batch=det.get("batch"))
            torch.cuda.synchronize()
            rec[label] = {"seconds": round(time.perf_counter() - t0, 4),
                          "max_matvecs": max(i["matvecs"] for i in infos),
                          "all_converged": all(i["status"] == 0 for i in infos)}
        print(json.dumps({"profile_batch": rec}), flush=True)
        return

    if args.profile_precond:
        print(json.dumps({"profile_precond": precond_section(dev, P)}), flush=True)
        return

    if args.profile_solve:
        K, f, g = d(P.K), d(P.f), d(P.g)
        out = {}
        # the settings the time-to-1e-8 section reaches the bar with
        for prec, rt in (("f64", 5e-9), ("mixed", 1e-8)):
            opts = SolveOptions(rtol=rt, maxiter=5000, precond=True, inner_m=20,
                                ir_inner_rtol=PRE_MIXED_INNER if prec == "mixed" else 1e-3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, prec, device=dev)
            pl.ensure_workspace(opts)
            _, info = pl.solve(K, f, g, opts=opts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = pl.solve(K, f, g, opts=opts)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            out[prec] = {"cold_s": round(t1 - t0, 4), "warm_s": round(t2 - t1, 4), "matvecs": info["matvecs"],
                         "matvecs_f32": info["matvecs_f32"], "status": info["status"]}
            _log(f"profile solve {prec}: {out[prec]}")
        print(json.dumps({"profile_solve": out}), flush=True)
        return

    def time_applies(plan, K, us, ys, steps, warmup):
        for i in range(warmup):
            plan.apply(K, us[i % N_ROT], ys[i % N_ROT], "reduced")
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for i in range(steps):
            plan.apply(K, us[i % N_ROT], ys[i % N_ROT], "reduced")
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, time.perf_counter() - t0

    if args.profile_apply:
        args.no_solve = args.no_cpu = True
        src = d(P.K)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log(f"calibration copies: 4 x {src.numel() * 8} bytes read and written")
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        if args.profile_apply and prec == "f32":
            continue
        plan = Plan(shape, P.grid.lo, P.grid.hi, P.grid.bc, prec, device=dev)
        K = d(P.K, dt)
        us = [d(W.random_field(shape, 100 + i), dt) for i in range(N_ROT)]
        ys = [torch.empty_like(us[0]) for _ in range(N_ROT)]
        tune = plan.autotune(K, us[0])[prec]
        _log(f"autotune {prec}: {tune}")
        ms, wall = time_applies(plan, K, us, ys, args.steps, args.warmup)
        res[prec] = {"ms_per_apply": ms, "gdofs": npts / (ms * 1e-3) / 1e9, "wall_s": wall,
                     "autotune_us": tune, "route": tune["chosen"]}
        _log(f"apply {prec} ({tune['chosen']}): {ms * 1e3:.1f} us/apply, {res[prec]['gdofs']:.2f} GDOF/s")
        # the same applies replayed from a HIP graph (16 applies per replay)
        graph = plan.capture_applies(K, us, ys, "reduced")
        reps = max(args.steps // N_ROT, 1)
        graph.replay()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            graph.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_g = ev0.elapsed_time(ev1) / (reps * N_ROT)
        res[prec]["graph_ms_per_apply"] = ms_g
        res[prec]["graph_gdofs"] = npts / (ms_g * 1e-3) / 1e9
        _log(f"apply {prec} (graph replay): {ms_g * 1e3:.1f} us/apply")
        del graph
        plan.set_route("fft")
        ms_fft, _ = time_applies(plan, K, us, ys, max(args.steps // 4, 10), 5)
        res[prec]["fft_route_gdofs"] = npts / (ms_fft * 1e-3) / 1e9
        _log(f"apply {prec} (fft route): {ms_fft * 1e3:.1f} us/apply")
        del us, ys, K, plan
        torch.cuda.empty_cache()

    # roofline of the operator apply (the method's algorithmic bytes, 24 B/pt in
    # FP64: read u, read K, write y) over the event-timed apply, i.e. its
    # axis-pass launches together; the traffic the design actually moves (and
    # its ratio to the algorithmic bytes) comes from the rocprofv3 counters
    if args.profile_apply:
        print(json.dumps({"profile_apply": res["f64"]["ms_per_apply"], "route": res["f64"]["route"]}), flush=True)
        return
    ms = res["f64"]["ms_per_apply"]
    apply_s = ms * 1e-3
    bytes_per_apply = ALG_BYTES_PER_POINT_F64 * npts
    achieved = bytes_per_apply / apply_s / 1e9
    route = res["f64"]["route"]
    kname = (f"k_dense_pass<double,128,REDUCED,*,{route[-1]},*> (matrix-core route" if route != "fft"
             else "k_axis_pass<double,128,REDUCED> (FFT route")
    rec = _traffic_record(route)
    traffic = rec["traffic_bytes_per_apply"] if rec else None
    # matrix-core route on this cube: the x and y passes share one launch and
    # the z pass adds both partial sums; FFT route: three axis passes
    launches = 2 if route != "fft" else 3
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic / 1e6, 2) if traffic else None,
                "traffic_unit": "MB per apply (rocprofv3 TCC request counters, copy-calibrated, "
                                f"{launches} launches)",
                "traffic_over_algorithmic": round(traffic / bytes_per_apply, 3) if traffic else None,
                # what the passes must move (u and K per axis, the partial sums
                # written and read back once): the measured traffic against it
                # shows whether the kernels re-read anything
                "traffic_over_design_minimum": (round(traffic / rec["design_min_bytes_per_apply"], 3)
                                                if rec and "design_min_bytes_per_apply" in rec else None),
                "algorithmic_mb_per_apply": round(bytes_per_apply / 1e6, 2),
                "algorithmic_bytes_per_point": ALG_BYTES_PER_POINT_F64,
                "kernel": kname + f"; {launches} launches per apply)",
                "apply_us": round(ms * 1e3, 2)}
    if res["f64"]["route"] != "fft":
        # utilisation of the matrix cores by the dense contractions this route
        # chose (not the method's work): the even-odd split does 2 (n/2)(n/2 + 1)
        # multiply-adds per pencil per derivative, two derivatives per axis, on
        # the (n-2)^2 interior-transverse pencils of each axis
        nn = shape[0]
        flops = 3 * 2 * 2 * 2 * (nn // 2) * (nn // 2 + 1) * (nn - 2) ** 2
        roofline["dense_contraction_mfma_tflops"] = round(flops / apply_s / 1e12, 2)
        roofline["dense_contraction_mfma_frac"] = round(flops / apply_s / 78.6e12, 4)
        roofline["dense_contraction_floor_us"] = round(flops / 78.6e12 * 1e6, 2)
    _log("stream-copy reference and the 257^3 apply")
    copy = copy_reference(dev)
    roofline["copy_gbs"] = copy["gbs"]
    roofline["frac_of_copy"] = round(achieved / copy["gbs"], 4)
    a257 = apply_257(dev)
    _log(f"copy {copy}; apply 257^3 {a257}")
    _log("preconditioner applications")
    precond = precond_section(dev, P)
    _log(f"preconditioner {precond}")
    # CPU-baseline leg: the oracle on the host -- its apply rate, and its
    # solution of the 129^3 system, which the time-to-1e-8 errors are measured
    # against
    cpu = None
    cpu_more = None
    uref_host = None
    ref_info = None
    if not args.no_cpu:
        _log("cpu baseline (oracle)")
        cpu = cpu_baseline(P)
        cpu_more = cpu_detail(P)
        if not args.no_solve and n == 129:
            _log("oracle reference solve at 129^3")
            uref_host, ref_info = oracle_reference(P)
            cpu_more["oracle_solve_129"] = ref_info
        _log(f"cpu baseline {cpu}; detail {cpu_more}")

    solve = None
    if uref_host is not None:
        solve = solve_section(P, d, dev, shape, uref_host, ref_info)

    chain = None
    if not args.no_solve and n == 129:
        _log("hierarchical Picard chain 33 -> 65 -> 129 -> 257")
        chain = picard_chain_section(dev)

    inclusion = None
    if not args.no_solve and n == 129:
        _log("spherical inclusion, contrast sweep 1e-4 .. 1e4")
        inclusion = inclusion_section(dev)

    robin_rows = None
    if not args.no_solve and n == 129:
        _log("Robin rows: apply rate and a manufactured solve at 129^3")
        robin_rows = robin_section(dev, P)

    thermal = None
    thermal_cold = None
    if not args.no_solve and n == 129:
        _log("nonlinear thermal problem (flux rows), Newton-LGMRES chain N = 4 .. 256")
        thermal = thermal_newton_section(dev)
        _log("nonlinear thermal problem, cold-start Newton at N = 128 and 256")
        thermal_cold = thermal_newton_cold(dev)

    refinement = None
    if not args.no_solve and n == 129:
        _log("hierarchical refinement with the e_ref stop, 33 -> 257")
        refinement = refinement_stop_section(dev)

    batch = None
    if not args.no_batch and not args.profile_apply:
        _log("batched homogenisation (32 microstructures x 3 load cases)")
        batch = homogenisation_section(dev)

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
        "apply_detail": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()
                             if kk != "wall_s"} for k, v in res.items()},
        "roofline": roofline,
        "precond_apply": precond,
        "cpu_baseline": cpu,
        "cpu_baseline_detail": cpu_more,
        "time_to_1e-8_129": solve,
        "homogenisation_batch": batch,
        "picard_chain": chain,
        "inclusion_contrast_sweep": inclusion,
        "thermal_newton_chain": thermal,
        "thermal_newton_cold": thermal_cold,
        "refinement_stop": refinement,
        "stream_copy": copy,
        "apply_257": a257,
        "robin_rows": robin_rows,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
