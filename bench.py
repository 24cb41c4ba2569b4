"""Benchmark: elements/s of batched HDG condensation + recovery on one MI355X.

One step = one implicit DIRK stage of the 3D acoustic workload (unit cube, 24^3 x 6 = 82,944
jittered tetrahedra, k = 3, c ~ U[1,2], dt = 0.01, stage coefficient a = 1/(gamma dt)) through
every step of the path: condensation (form, factor, Schur complement, condensed right-hand
side), face-row assembly, FP64 trace solve, recovery, and -- in mixed precision -- the FP64
refinement loop.  Inputs (L2-projected plane-wave state, stage right-hand side, projected
Dirichlet data) are resident in HBM before timing starts.

value        = elements * steps / (time in the element kernels: condensation + recovery
               [+ refinement element work]), HIP events on the library stream
ms_per_step  = wall time of one whole stage (all of the above, including the trace solve)

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--precision fp64|mixed_fp32]
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

GAMMA = 0.43586652150845899942
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def dimp(k, d):
    return {1: k + 1, 2: (k + 1) * (k + 2) // 2, 3: (k + 1) * (k + 2) * (k + 3) // 6}[d]


def acoustic_counts(D, K, R, elt_bytes):
    """Algorithmic HBM bytes and executed flops per element of the acoustic condensation
    kernel (see condense_acoustic.hip) and bytes of the recovery GEMV."""
    N, NF, NFACE = dimp(K, D), dimp(K, D - 1), D + 1
    TT, NLOC = NFACE * NF, (D + 1) * N
    C = TT + R
    npair = D * (D + 1) // 2
    fma = (N * N * (NFACE + npair) + NFACE * N * N * D + D * N * R * D + N * TT * N + N * R * D * N
           + N ** 3 / 3 + N * N * C + D * N * C * N + TT * D * N * D + NFACE * N * C * 2 * D
           + NFACE * NF * C * N)
    flops = 2.0 * fma
    reads = NLOC * R * 8 + 32 * 8 + NFACE * 4
    writes = (TT * TT + TT * R + NLOC * TT + NLOC * R) * elt_bytes
    cond_bytes = reads + writes
    rec_bytes = NLOC * TT * elt_bytes + NLOC * R * elt_bytes + TT * R * 8 + NLOC * R * 8 + NFACE * 4
    return dict(cond_bytes=cond_bytes, cond_flops=flops, rec_bytes=rec_bytes, rec_flops=2.0 * NLOC * TT * R)


def cpu_baseline(problem, a, budget_s=15.0):
    """The oracle's per-element condense + recover (quadrature forming, dense solve, Schur
    complement, recovery) on a seeded sample of elements, single BLAS thread."""
    from threadpoolctl import threadpool_limits

    from oracle import hdg as ohdg
    from synth import random_vector
    d = ohdg.make_discretisation(problem)
    f = random_vector(d.loc_off[-1], problem.cfg_id, 91)
    lam = random_vector(d.tr_off[-1], problem.cfg_id, 92)
    rng = np.random.default_rng(7)
    order = rng.permutation(problem.n_elem)
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for e in order:
            e = int(e)
            A, B, Cm, Dm, _ = ohdg.element_system(d, e, a)
            li, ti = d.elem_local_dofs(e), d.elem_trace_dofs(e)
            Z = np.linalg.solve(A, B)
            z = np.linalg.solve(A, f[li])
            Ke = Dm - Cm @ Z
            re = -Cm @ z
            u = z - Z @ lam[ti]
            d.quad.pop(e, None)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    del Ke, re, u
    return dict(value=done / el, unit="elements/s", cores=1, kind="oracle",
                sample=f"{done} seeded-random elements of the {problem.n_elem}-element mesh, "
                       f"{el:.1f} s, 1 BLAS thread, per-element form+factor+Schur+recover")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed_fp32"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the element kernels shard "
                                   "by element partition, see the design notes", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1807_00086_amd import Solver
    from synth import make_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    p = make_problem(2)
    k = int(p.degree[0])
    a = 1.0 / (GAMMA * p.dt)
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=k, precision=args.precision)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")

    # inputs: projected plane wave p0 = sin(2 pi x), v0 = (p0, 0, 0); Dirichlet p = sin 2pi(x - t)
    vp = s.volume_points()
    p0 = np.sin(2 * np.pi * vp[:, 0])
    u0 = s.project_volume(np.stack([p0, 0 * p0, 0 * p0, p0], 1))
    bp = s.boundary_points()
    lb = s.project_boundary(np.sin(2 * np.pi * (bp[:, 0] - GAMMA * p.dt))[:, None])
    u0_d = torch.as_tensor(u0, device="cuda")
    f_d = torch.zeros(nl, dtype=torch.float64, device="cuda")
    s.apply_mass(a, u0_d, f_d)
    lb_d = torch.as_tensor(lb, device="cuda")
    lam = torch.zeros(nt, dtype=torch.float64, device="cuda")
    u = torch.zeros(nl, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def stage():
        s.condense(a, f_d, lb_d)
        lam.zero_()
        it, rr = s.trace_solve(lam)
        s.recover(lam, u)
        return it, rr

    for _ in range(args.warmup):
        stage()
    torch.cuda.synchronize()
    t_cond = t_rec = t_asm = t_sol = t_ref = 0.0
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        it, rr = stage()
        iters.append(it)
        t_cond += s.timing("condense")
        t_rec += s.timing("recover")
        t_asm += s.timing("assemble")
        t_sol += s.timing("solve")
        t_ref += s.timing("refine_elem")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    elem_ms = t_cond + t_rec + t_ref
    value = p.n_elem * args.steps / (elem_ms * 1e-3)

    eb = 8 if args.precision == "fp64" else 4
    cnt = acoustic_counts(3, k, 1, eb)
    cond_avg_s = t_cond / args.steps * 1e-3
    achieved_gbs = cnt["cond_bytes"] * p.n_elem / cond_avg_s / 1e9
    achieved_tf = cnt["cond_flops"] * p.n_elem / cond_avg_s / 1e12
    rec_gbs = cnt["rec_bytes"] * p.n_elem / (t_rec / args.steps * 1e-3) / 1e9
    out = {
        "metric": "elements/s for batched HDG condensation+recovery, mixed vs FP64 at equal error",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "acoustic3d_kuhn24_k3_dirk33_stage", "elements": p.n_elem, "k": k,
                   "local_unknowns": 80, "trace_unknowns": 40, "precision": args.precision,
                   "parallelism": "single GPU"},
        "value_basis": "element kernels only (condense + recover [+ refinement element work]); "
                       "ms_per_step includes assembly and the FP64 trace solve",
        "ms_condense": t_cond / args.steps,
        "ms_recover": t_rec / args.steps,
        "ms_assemble": t_asm / args.steps,
        "ms_trace_solve": t_sol / args.steps,
        "ms_refine_elem": t_ref / args.steps,
        "krylov_iters": float(np.mean(iters)),
        "stage_elements_per_s": p.n_elem / (ms_step * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "condense_acoustic_kernel<3,3,1>",
                     "bytes_per_element": cnt["cond_bytes"], "flops_per_element": cnt["cond_flops"],
                     "flop_frac_fp64": achieved_tf / FP64_PEAK_TFLOPS},
        "recover_roofline": {"bound": "hbm", "achieved": rec_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": rec_gbs / HBM_PEAK_GBS, "bytes_per_element": cnt["rec_bytes"]},
    }
    s.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, a, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
