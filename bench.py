"""Benchmark: elements/s of batched HDG condensation + recovery on one MI355X.

One step = one implicit DIRK stage of the 3D acoustic workload (unit cube, 24^3 x 6 = 82,944
jittered tetrahedra, k = 3, c ~ U[1,2], dt = 0.01, stage coefficient a = 1/(gamma dt)) through
every step of the path: condensation (form, factor, Schur complement, condensed right-hand
side), face-row assembly, FP64 trace solve (CG with the multicolour block SSOR preconditioner),
recovery, and -- in mixed precision -- the FP64 refinement loop.  Inputs (L2-projected plane-wave state, stage right-hand side, projected
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
FP32_PEAK_TFLOPS = 157.3

# Mixed-precision settings of the timed stage: the first trace solve to 1e-8 (the refinement's
# corrections remove its error with the rest), refinement until the FP64 residual of the full
# stage system is at most 1e-11 of its right-hand side (one correction reaches 3e-13 on the
# acoustic workload, 3e-12 on the elastic and Maxwell workloads).  The GPU parity tests run these
# settings against the oracle.
MIXED_OPTS = dict(krylov_tol=1e-8, refine_tol=1e-11)
# Trace-CG preconditioner of the timed stages (block Jacobi is timed as a secondary figure)
STAGE_PRECOND = "ssor"


def dimp(k, d):
    return {1: k + 1, 2: (k + 1) * (k + 2) // 2, 3: (k + 1) * (k + 2) * (k + 3) // 6}[d]


def acoustic_counts(D, K, R, elt_bytes, mixed=False):
    """Algorithmic HBM bytes and executed flops per element of the acoustic kernels
    (condense_acoustic.hip).  Condensation: closed-form velocity elimination, B~ and W_f by
    MFMA tiles, the pressure Schur block S (upper triangle) from reference tables, elimination
    of [S | B~ | f~] without pivoting (mixed precision also stores the factor U of S),
    K_e = D - B_v^T B_v / (a rho |J|) + W^T W formed and stored by its tiles on and above the
    diagonal.  Recovery:
    p = z_p - Z_p lam, v in closed form.  Reads of the degree-dependent reference tables hit
    the caches and are not counted as HBM traffic; padding of MFMA tiles is not counted."""
    N, NF, NFACE = dimp(K, D), dimp(K, D - 1), D + 1
    TT, NLOC = NFACE * NF, (D + 1) * N
    C = TT + R
    npair = D * (D + 1) // 2
    k_stored = sum(1 for r in range(TT) for c in range(TT) if r // 16 <= c // 16)
    fma = (D * D * N * R + D * N * N * R     # condensed pressure rhs
           + NFACE * N * N * D               # W_f = tau I + sum_r beta_fr Sr_r (MFMA operand)
           + NFACE * N * NF * N              # B~_f = -s_f W_f E_f
           + N * (N + 1) / 2.0 * (NFACE + npair)   # upper triangle of S from reference tables
           + N ** 3 / 3.0 + N * N * C / 2.0  # forward elimination
           + N * N * C / 2.0                 # back substitution
           + 2 * k_stored * N                # W^T W and E^T E on the stored tiles
           + TT * R * 2 * N + NFACE * N * R * D)     # r_e
    reads = NLOC * R * 8 + 32 * 8 + NFACE * 4
    writes = (k_stored + TT * R + N * TT + NLOC * R + (N * N if mixed else 0)) * elt_bytes
    rec_bytes = (N * TT + NLOC * R) * elt_bytes + TT * R * 8 + 32 * 8 + 2 * NFACE * 4 + NLOC * R * 8
    rec_fma = N * TT * R + NFACE * N * NF * R + D * N * N * R + D * N * R * (D + NFACE)
    return dict(cond_bytes=reads + writes, cond_flops=2.0 * fma, rec_bytes=rec_bytes,
                rec_flops=2.0 * rec_fma)


def acoustic_pass_bytes(D, K):
    """Algorithmic HBM bytes per element of the two element passes of the mixed-precision
    refinement (refine_acoustic_kernel<float>, one right-hand side).  F0: recovery from the
    FP32 factors fused with the FP64 residual and the correction right-hand side (reads the
    geometry record, face ids and orientations, lam, Z_p, z_p, f, U; writes u, re64, z'_p and two
    norms).  R: the correction and the check of the FP64 residual at the corrected iterate (reads
    lam, dlam, Z_p, z'_p, u, f; writes u, re64 = -t_e and two norms)."""
    N, NF, NFACE = dimp(K, D), dimp(K, D - 1), D + 1
    TT, NLOC = NFACE * NF, (D + 1) * N
    common = 32 * 8 + 2 * NFACE * 4 + N * TT * 4 + N * 4 + NLOC * 8 + NLOC * 8 + 2 * 8
    f0 = common + TT * 8 + N * N * 4 + TT * 8 + N * 4
    r = common + 2 * TT * 8 + NLOC * 8 + TT * 8
    return {"F0": f0, "R": r}


def general_counts(phys, k, kf, R, elt_bytes, mixed):
    """Algorithmic HBM bytes per element of the block-structured condensation and recovery
    (condense_general.hip, recover_mrhs.hip): the condensation reads f, the geometry record, face
    ids and orientations (Maxwell: face frames) and writes K_e (full), r_e, the Schur rows of Z,
    z and, in mixed precision, the Schur block's factor; the recovery reads Z, z, the element's
    traces and its geometry and writes u.  Reference tables hit the caches."""
    m_local, m_trace = {0: 4, 1: 9, 2: 6, 3: 7}[phys], {0: 1, 1: 3, 2: 2, 3: 2}[phys]
    N, NF = dimp(k, 3), dimp(kf, 2)
    n, t = m_local * N, 4 * m_trace * NF
    ns = {0: N, 1: 3 * N, 2: 3 * N, 3: 4 * N}[phys]
    geo = 32 * 8 + 2 * 4 * 4 + (24 * 8 if phys >= 2 else 0)
    cond = n * R * 8 + geo + (t * t + t * R + ns * t + n * R + (ns * ns if mixed else 0)) * elt_bytes
    rec = (ns * t + n * R) * elt_bytes + t * R * 8 + geo + n * R * 8
    return cond, rec


def hbm_probes(reps=10):
    """Achieved HBM bandwidth of the library's own streaming read and copy passes over a 1 GiB
    buffer (hdg_hbm_probe, the best of a few grid sizes) and of torch's device copy, GB/s."""
    import torch

    from paper_1807_00086_amd.hdg import hbm_probe
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for name, d, nbytes in (("read", None, 8 * n), ("copy", dst, 16 * n)):
        best = None
        for bpc in (2, 4, 8, 16):
            ms = hbm_probe(src, d, reps=reps, blocks_per_cu=bpc)
            gbs = nbytes / (ms * 1e-3) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, bpc)
        out[f"hip_{name}_GBs"] = best[0]
        out[f"hip_{name}_blocks_per_cu"] = best[1]
    del src, dst
    torch.cuda.empty_cache()
    out["torch_copy_GBs"] = copy_bandwidth(reps)
    return out


def copy_bandwidth(reps=10):
    """Achieved HBM bandwidth of a plain 1 GiB device-to-device copy (torch copy_, timed with
    HIP events): the practical ceiling a streaming kernel meets on this GPU, for context."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * 8 * n / (ms * 1e-3) / 1e9


def _profile_record(fname, tag, kernel):
    """Machine-readable record `<tag>: {json}` of `kernel` in a committed rocprofv3 summary
    under profiles/, or None when it is missing or was taken on a different version of the
    kernel source (the record carries the first 16 hex digits of the source's SHA-256)."""
    import hashlib
    import re as _re
    path = os.path.join(ROOT, "profiles", fname)
    src = os.path.join(ROOT, "paper_1807_00086_amd", "csrc", "condense_acoustic.hip")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    for m in _re.finditer(r"^" + tag + r": (\{.*\})$", text, _re.M):
        rec = json.loads(m.group(1))
        if rec.get("kernel") == kernel and rec.get("source_sha256_16") == digest:
            return rec
    return None


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE scaled by the plain-copy calibration), or None (see _profile_record)."""
    rec = _profile_record("hbm_traffic_acoustic_k3.md", "traffic", kernel)
    return None if rec is None else rec["bytes_per_launch"]


def measured_mfma_busy(kernel):
    """Fraction of the matrix cores' cycles busy during `kernel` from the committed PMC summary
    (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE per XCD x 256 CUs x 4 SIMDs), or None."""
    rec = _profile_record("mfma_utilisation_condense.md", "mfma", kernel)
    return None if rec is None else rec["busy"]


def ssor_iteration_bytes(n_elem, n_faces, bs):
    """Algorithmic HBM bytes of one iteration of the block-SSOR trace CG on a tetrahedral mesh:
    every off-diagonal block of the scaled matrix once (one per ordered pair of distinct faces of
    an element: 12 per element, bs x bs FP64), the gathers of the neighbours' bs-vectors (one per
    block), and 14 passes over a trace vector (backward sweeps: p and r read, p and t written;
    their colour-0 launch: u and q written; forward sweeps: p and t read, u and q written; CG
    update: y, p, r, q read, y and r written)."""
    nblk = 12 * n_elem
    nt = n_faces * bs
    return nblk * bs * bs * 8 + nblk * bs * 8 + 14 * nt * 8


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


def _oracle_worker(args):
    """One worker process of the all-cores oracle rate: elements w, w + W, w + 2W, ... of the
    seeded order, for budget_s seconds, one BLAS thread."""
    w, nw, a, budget_s = args
    from threadpoolctl import threadpool_limits

    from oracle import hdg as ohdg
    from synth import make_problem, random_vector
    problem = make_problem(2)
    d = ohdg.make_discretisation(problem)
    f = random_vector(d.loc_off[-1], problem.cfg_id, 91)
    lam = random_vector(d.tr_off[-1], problem.cfg_id, 92)
    order = np.random.default_rng(7).permutation(problem.n_elem)[w::nw]
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for e in order:
            e = int(e)
            A, B, Cm, Dm, _ = ohdg.element_system(d, e, a)
            li, ti = d.elem_local_dofs(e), d.elem_trace_dofs(e)
            Z = np.linalg.solve(A, B)
            z = np.linalg.solve(A, f[li])
            _ = (Dm - Cm @ Z, -Cm @ z, z - Z @ lam[ti])
            d.quad.pop(e, None)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    return done, el


def cpu_baseline_all_cores(a, budget_s=10.0, max_workers=16):
    """The same oracle work on disjoint strided shares of the seeded element order, one worker
    process per core (at most max_workers), each with one BLAS thread: total elements over the
    slowest worker's time (elements are independent, so the rate extrapolates to the mesh)."""
    import multiprocessing as mp
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    nw = max(1, min(max_workers, ncpu))
    with mp.get_context("spawn").Pool(nw) as pool:
        res = pool.map(_oracle_worker, [(w, nw, a, budget_s) for w in range(nw)])
    done = sum(r[0] for r in res)
    el = max(r[1] for r in res)
    return dict(value=done / el, unit="elements/s", cores=nw, kind="oracle",
                sample=f"{done} seeded-random elements of the 82944-element mesh on {nw} worker "
                       f"processes (disjoint shares), {el:.1f} s, 1 BLAS thread each, per-element "
                       f"form+factor+Schur+recover")


def run_precision(p, prec, steps, warmup, keep_solution=False, precond=STAGE_PRECOND):
    """Time `steps` whole stages in one precision; returns timings and (optionally) the
    final stage solution on the host."""
    import torch

    from paper_1807_00086_amd import Solver
    k = int(p.degree[0])
    a = 1.0 / (GAMMA * p.dt)
    kw = dict(krylov_tol=1e-13) if prec == "fp64" else dict(MIXED_OPTS)
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=k, precision=prec, precond=precond, **kw)
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
        it, _ = s.trace_solve(lam)
        s.recover(lam, u)
        return it

    for _ in range(warmup):
        stage()
    torch.cuda.synchronize()
    tm = dict(condense=0.0, recover=0.0, assemble=0.0, solve=0.0, refine_elem=0.0, refine_solve=0.0)
    iters, refs, elem_ms, res = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        iters.append(stage())
        refs.append(s.query("last_refine"))
        st = {key: s.timing(key) for key in tm}
        for key in tm:
            tm[key] += st[key]
        elem_ms.append(st["condense"] + st["recover"] + st["refine_elem"])
        if prec != "fp64":
            res.append(float(s.last_residual().max()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(ms_step=1e3 * wall / steps, iters=float(np.mean(iters)), refine=float(np.mean(refs)),
               elem_ms_median=float(np.median(elem_ms)), elem_ms_min=float(np.min(elem_ms)), n_trace_dofs=nt,
               **{k2: v / steps for k2, v in tm.items()})
    if res:
        out["refine_residual_max"] = max(res)
    if keep_solution:
        out["u"] = u.cpu().numpy()
        out["lam"] = lam.cpu().numpy()
    s.close()
    del f_d, u0_d, lb_d, lam, u
    torch.cuda.empty_cache()
    return out


def run_cached(p, prec, steps, warmup):
    """Secondary figure: stage throughput with the factors kept across stages (the DIRK(3,3)
    stages share the stage coefficient).  One hdg_condense factors; each timed stage is then
    hdg_condense_rhs + trace solve + recover (+ refinement in mixed precision)."""
    import torch

    from paper_1807_00086_amd import Solver
    k = int(p.degree[0])
    a = 1.0 / (GAMMA * p.dt)
    kw = dict(krylov_tol=1e-13) if prec == "fp64" else dict(MIXED_OPTS)
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=k, precision=prec, cache_factors=True,
               precond=STAGE_PRECOND, **kw)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
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
    s.condense(a, f_d, lb_d)

    def stage():
        s.condense_rhs(a, f_d, lb_d)
        lam.zero_()
        it, _ = s.trace_solve(lam)
        s.recover(lam, u)
        return it

    for _ in range(warmup):
        stage()
    torch.cuda.synchronize()
    tm = dict(condense=0.0, recover=0.0, assemble=0.0, solve=0.0, refine_elem=0.0, refine_solve=0.0)
    t0 = time.perf_counter()
    for _ in range(steps):
        stage()
        for key in tm:
            tm[key] += s.timing(key)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    del f_d, u0_d, lb_d, lam, u
    torch.cuda.empty_cache()
    out = dict(ms_step=1e3 * wall / steps, **{k2: v / steps for k2, v in tm.items()})
    out["rhs_condense"] = out.pop("condense")
    out["elements_per_s"] = p.n_elem / ((out["rhs_condense"] + out["recover"] + out["refine_elem"]) * 1e-3)
    return out


def run_step_graph(p, steps, warmup):
    """Secondary figure: whole DIRK(3,3) steps (hdg_step, FP64, factors kept across the stages)
    run eagerly, with a host synchronisation per CG iteration, against the same steps replayed
    as one hipGraph with the CG convergence test on the device (options.graph_step), both with
    the block-Jacobi trace CG (the final states agree to the last bits), and the same pair with
    the block-SSOR trace CG (eager_ssor, graph_ssor: equal to the CG tolerance, the captured CG
    stops on its estimate and checks the true residual at the end)."""
    import torch

    from paper_1807_00086_amd import Solver
    k = int(p.degree[0])
    out = {}
    finals = {}
    for mode in ("eager", "graph", "eager_ssor", "graph_ssor"):
        s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=k, precision="fp64", krylov_tol=1e-13,
                   cache_factors=True, graph_step=mode.startswith("graph"),
                   precond="ssor" if mode.endswith("ssor") else "jacobi")
        nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
        vp = s.volume_points()
        p0 = np.sin(2 * np.pi * vp[:, 0])
        u = torch.as_tensor(s.project_volume(np.stack([p0, 0 * p0, 0 * p0, p0], 1)), device="cuda")
        bp = s.boundary_points()
        lbs = torch.as_tensor(np.stack([s.project_boundary(np.sin(2 * np.pi * (bp[:, 0] - c * p.dt))[:, None])
                                        for c in (GAMMA, 0.5 * (1 + GAMMA), 1.0)]), device="cuda")
        lam = torch.zeros(nt, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            s.step(0.0, p.dt, "dirk33", u, lam, lbs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        replays = 0
        for _ in range(steps):
            s.step(0.0, p.dt, "dirk33", u, lam, lbs)
            replays += s.query("step_graph")
        torch.cuda.synchronize()
        out[f"{mode}_ms_step"] = 1e3 * (time.perf_counter() - t0) / steps
        out[f"{mode}_iters_last_stage"] = s.query("last_iters")
        if mode.startswith("graph"):
            out[f"{mode}_replays"] = replays
            out[f"{mode}_cg_iters_per_stage"] = s.query("step_graph_iters")
        finals[mode] = u.cpu().numpy()
        s.close()
        del u, lbs, lam
        torch.cuda.empty_cache()
    out["graph_vs_eager_max_rel"] = float(np.abs(finals["graph"] - finals["eager"]).max() /
                                          np.abs(finals["eager"]).max())
    # the same steps with the block-SSOR trace CG (eager): equal to the block-Jacobi steps to
    # the CG tolerance
    out["eager_ssor_vs_eager_max_rel"] = float(np.abs(finals["eager_ssor"] - finals["eager"]).max() /
                                               np.abs(finals["eager"]).max())
    out["graph_ssor_vs_eager_ssor_max_rel"] = float(np.abs(finals["graph_ssor"] - finals["eager_ssor"]).max() /
                                                    np.abs(finals["eager_ssor"]).max())
    out["speedup"] = out["eager_ms_step"] / out["graph_ms_step"]
    return out


def run_workload(cfg, prec, steps, warmup, physics=None):
    """Element-kernel throughput of one of the other workloads at full size (secondary figures,
    not the headline): elastic k = 4 (3), p-heterogeneous acoustics with 32 point-source
    right-hand sides (4), Maxwell k = 3 (5).  Seeded random stage right-hand side (point
    sources for workload 4) and homogeneous Dirichlet data; the trace solves run to 1e-10 (the
    element kernels do not depend on it) with the timed stages' preconditioner (block SSOR with
    one right-hand side, block Jacobi with 32)."""
    import torch

    from paper_1807_00086_amd import Solver
    from synth import make_problem, random_vector
    p = make_problem(cfg)
    if physics is not None:
        p.physics = physics
    a = 1.0 / (GAMMA * p.dt) if p.scheme == "dirk33" else 1.0 / p.dt
    kw = dict(krylov_tol=1e-10, krylov_maxit=20000)
    if prec != "fp64":
        kw.update(refine_tol=MIXED_OPTS["refine_tol"])
    uk = p.uniform_k
    # launch schedules picked by the library's autotuner on the first (warm-up) stage; on the
    # mesh of variable degree the degree classes run as one hipGraph
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=uk, degree=None if uk else p.degree,
               precision=prec, nrhs=p.nrhs, autotune=True, use_graph=not uk, precond=STAGE_PRECOND, **kw)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    if p.nrhs > 1:
        f = torch.as_tensor(s.point_sources(p.sources), device="cuda")
    else:
        f = torch.as_tensor(random_vector(nl, cfg, 1), device="cuda")
    lb = torch.zeros(nt * p.nrhs, dtype=torch.float64, device="cuda")
    lam = torch.zeros_like(lb)
    u = torch.zeros(nl * p.nrhs, dtype=torch.float64, device="cuda")

    def stage():
        s.condense(a, f, lb)
        lam.zero_()
        it, _ = s.trace_solve(lam)
        s.recover(lam, u)
        return it

    for _ in range(warmup):
        stage()
    torch.cuda.synchronize()
    tm = dict(condense=0.0, recover=0.0, assemble=0.0, solve=0.0, refine_elem=0.0, refine_solve=0.0)
    its = []
    for _ in range(steps):
        its.append(stage())
        for key in tm:
            tm[key] += s.timing(key)
    torch.cuda.synchronize()
    refine = s.query("last_refine")
    schedules = s.schedules()
    s.close()
    del f, lb, lam, u
    torch.cuda.empty_cache()
    out = {k2: v / steps for k2, v in tm.items()}
    out.update(workload=p.name, elements=p.n_elem, nrhs=p.nrhs, iters=float(np.mean(its)), refine=refine,
               schedules=schedules,
               elements_per_s=p.n_elem / ((out["condense"] + out["recover"] + out["refine_elem"]) * 1e-3))
    # rooflines of the two element kernels (HBM, algorithmic bytes summed over the elements)
    phys = {"acoustic": 0, "elastic": 1, "maxwell": 2, "maxwell_glm": 3}[p.physics]
    eb = 8 if prec == "fp64" else 4
    cb = rb = 0.0
    for kk, cnt in zip(*np.unique(p.degree, return_counts=True)):
        c1, r1 = general_counts(phys, int(kk), 5 if uk is None else int(kk), p.nrhs, eb, prec != "fp64")
        cb += c1 * cnt
        rb += r1 * cnt
    for name, nbytes, ms in (("condense", cb, out["condense"]), ("recover", rb, out["recover"])):
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[f"{name}_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": gbs / HBM_PEAK_GBS, "bytes": nbytes}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed_fp32"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the element-kernel timings of the other workloads (elastic k=4, "
                         "p-heterogeneous 32-rhs acoustics, Maxwell k=3) at full size")
    ap.add_argument("--workload", type=int, choices=[3, 4, 5], default=None,
                    help="time only the element kernels of one of the other workloads (elastic k = 4, "
                         "p-heterogeneous acoustics with 32 right-hand sides, Maxwell k = 3) and print them")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 1 << 27                                   # 2^27 doubles = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_read": 8 * n, "calibration_copy_bytes_written": 8 * n}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: the library has no multi-GPU "
                                   "path (the element kernels would shard by element partition)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload is not None:
        precs = ["fp64", "mixed_fp32"] if args.precision == "both" else [args.precision]
        res = {}
        for pr in precs:
            res[pr] = run_workload(args.workload, pr, args.steps, args.warmup)
            print(f"workload {args.workload} {pr}: {res[pr]['elements_per_s']:.4g} elements/s", file=sys.stderr,
                  flush=True)
        print(json.dumps({"workload": args.workload, "steps": args.steps, "warmup": args.warmup, "results": res}))
        return

    import torch

    from synth import make_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    p = make_problem(2)
    k = int(p.degree[0])
    a = 1.0 / (GAMMA * p.dt)
    precs = ["fp64", "mixed_fp32"] if args.precision == "both" else [args.precision]
    res = {pr: run_precision(p, pr, args.steps, args.warmup, keep_solution=(len(precs) == 2))
           for pr in precs}

    def elem_rate(r):
        return p.n_elem / ((r["condense"] + r["recover"] + r["refine_elem"]) * 1e-3)

    equal_error = None
    if len(precs) == 2:
        u64, u32 = res["fp64"]["u"].reshape(p.n_elem, 4, -1), res["mixed_fp32"]["u"].reshape(p.n_elem, 4, -1)
        X = p.xyz[p.elem_vert]
        dj = np.abs(np.linalg.det(np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))))[:, None, None]
        errs = {}
        for name, comps in (("v", [0, 1, 2]), ("p", [3])):
            num = np.sqrt(np.sum(dj * (u32[:, comps] - u64[:, comps]) ** 2))
            den = np.sqrt(np.sum(dj * u64[:, comps] ** 2))
            errs[name] = float(num / den)
        equal_error = errs
        ok = max(errs.values()) <= 1e-10
        head = "mixed_fp32" if ok and elem_rate(res["mixed_fp32"]) > elem_rate(res["fp64"]) else "fp64"
    else:
        head = precs[0]
    r = res[head]
    value = elem_rate(r)
    eb = 8 if head == "fp64" else 4
    cnt = acoustic_counts(3, k, 1, eb, mixed=head != "fp64")
    kname = f"condense_acoustic_kernel<3,{k},1,{'double' if head == 'fp64' else 'float'}>"
    cond_s = r["condense"] * 1e-3
    achieved_gbs = cnt["cond_bytes"] * p.n_elem / cond_s / 1e9
    achieved_tf = cnt["cond_flops"] * p.n_elem / cond_s / 1e12
    # The condensation's dominant work is the element elimination and its products, issued on the
    # vector units and the matrix cores alike; FP64 vector and matrix peaks coincide (78.6 TF), so
    # the FP64 kernel is measured against that; FP32 against its own 157.3 TF.
    flop_peak = FP64_PEAK_TFLOPS if head == "fp64" else FP32_PEAK_TFLOPS

    def rec_entry(prec_name):
        rr = res[prec_name]
        if prec_name == "fp64":
            b = acoustic_counts(3, k, 1, 8)["rec_bytes"]
            gbs = b * p.n_elem / (rr["recover"] * 1e-3) / 1e9
            return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "bytes_per_element": b, "ms": rr["recover"],
                    "kernel": f"refine_acoustic_kernel<3,{k},1,double,8,0>", "precision": "fp64"}
        # mixed precision: the recovery is fused with the FP64 residual (pass F0); each correction
        # pass applies the correction and checks the residual (pass R)
        pb = acoustic_pass_bytes(3, k)
        b = pb["F0"] + pb["R"] * rr["refine"]
        ms = rr["recover"] + rr["refine_elem"]
        gbs = b * p.n_elem / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                "bytes_per_element": b, "ms": ms, "kernel": f"refine_acoustic_kernel<3,{k},1,float,8,1>",
                "precision": "mixed_fp32",
                "passes": {name: {"ms": ms2, "bytes_per_element": b2,
                                  "frac": b2 * p.n_elem / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS}
                           for name, ms2, b2 in (("F0_recovery_residual", rr["recover"], pb["F0"]),
                                                 ("R_correction_check", rr["refine_elem"] / max(rr["refine"], 1),
                                                  pb["R"]))}}
    probes = hbm_probes()
    out = {
        "metric": "elements/s for batched HDG condensation+recovery, mixed vs FP64 at equal error",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "acoustic3d_kuhn24_k3_dirk33_stage", "elements": p.n_elem, "k": k,
                   "local_unknowns": 80, "trace_unknowns": 40, "precision": head,
                   "trace_preconditioner": "multicolour block SSOR (Eisenstat form)",
                   "parallelism": "single GPU"},
        "value_basis": "element kernels only (condense + recover + refinement element work) per stage, mean "
                       "over the timed steps; ms_per_step is the whole stage including assembly and FP64 "
                       "trace solves",
        "elements_per_s_median": p.n_elem / (r["elem_ms_median"] * 1e-3),
        "elements_per_s_max": p.n_elem / (r["elem_ms_min"] * 1e-3),
        "per_precision": {pr: {kk: vv for kk, vv in rr.items() if kk not in ("u", "lam")} | {
            "elements_per_s": elem_rate(rr)} for pr, rr in res.items()},
        "mixed_vs_fp64_rel_l2": equal_error,
        "mixed_settings": MIXED_OPTS,
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": flop_peak, "unit": "TFLOP/s",
                     "frac": achieved_tf / flop_peak, "traffic": measured_traffic(kname),
                     "kernel": kname, "flops_per_element": cnt["cond_flops"],
                     "bytes_per_element": cnt["cond_bytes"], "hbm_achieved_GBs": achieved_gbs,
                     "hbm_frac": achieved_gbs / HBM_PEAK_GBS, "mfma_busy": measured_mfma_busy(kname)},
        "recover_roofline": rec_entry(head),
        "recover_roofline_by_precision": {pr: rec_entry(pr) for pr in res},
        "hbm_probes": probes,
    }
    out["cached_factor_stage"] = {
        "basis": "secondary: per-stage element kernels with the factors kept across stages "
                 "(right-hand-side condensation + recover [+ refinement element passes]); "
                 "one factorisation per dt, not per stage",
        **{pr: run_cached(p, pr, args.steps, args.warmup) for pr in precs}}
    if "fp64" in res:
        # whole FP64 solves (setup, the scaled matrix, the final true residual included) against
        # the iterations' algorithmic bytes: a lower bound of the sweeps' own rate
        r64 = res["fp64"]
        bs = (k + 1) * (k + 2) // 2
        it_bytes = ssor_iteration_bytes(p.n_elem, r64["n_trace_dofs"] // bs, bs)
        gbs = it_bytes * r64["iters"] / (r64["solve"] * 1e-3) / 1e9
        out["trace_solve_roofline"] = {
            "basis": "secondary: FP64 block-SSOR trace solve of the timed stage, algorithmic bytes of its "
                     "iterations over the whole solve time (setup, scaling and final residual included)",
            "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "bytes_per_iteration": it_bytes, "iters": r64["iters"], "solve_ms": r64["solve"],
            "kernel": "ssor_sweep_kernel<10, ...>, cg_update_kernel"}
    jj = run_precision(p, "fp64", args.steps, args.warmup, precond="jacobi")
    out["trace_solve_jacobi"] = {
        "basis": "secondary: the FP64 stage with block Jacobi in the trace CG instead of the multicolour "
                 "block SSOR of the timed stages; same element kernels",
        "solve_ms": jj["solve"], "iters": jj["iters"], "ms_step": jj["ms_step"],
        "ssor_solve_ms": res["fp64"]["solve"] if "fp64" in res else None,
        "ssor_iters": res["fp64"]["iters"] if "fp64" in res else None}
    print(f"trace solve: jacobi {jj['solve']:.2f} ms ({jj['iters']:.0f} it), ssor "
          f"{out['trace_solve_jacobi']['ssor_solve_ms']} ms", file=sys.stderr, flush=True)
    out["step_graph"] = {"basis": "secondary: whole DIRK(3,3) steps (hdg_step, FP64, cached factors) eager "
                                  "against one hipGraph replay per step, with block Jacobi and with "
                                  "block SSOR", **run_step_graph(p, 3, 1)}
    print(f"step graph: {out['step_graph']['eager_ms_step']:.2f} ms eager, "
          f"{out['step_graph']['graph_ms_step']:.2f} ms graph, "
          f"{out['step_graph']['eager_ssor_ms_step']:.2f} ms eager with SSOR, "
          f"{out['step_graph']['graph_ssor_ms_step']:.2f} ms graph with SSOR", file=sys.stderr, flush=True)
    if not args.no_workloads:
        # the other workloads at full size, element kernels of one stage (secondary figures)
        out["other_workloads"] = {}
        both, three = ("fp64", "mixed_fp32"), ("fp64", "mixed_fp32", "mixed_bf16")
        for cfg, phys, precs_w in ((3, None, three), (4, None, both), (5, None, three), (5, "maxwell_glm", three)):
            for pr in precs_w:
                key = f"{cfg}{'_glm' if phys else ''}_{pr}"
                out["other_workloads"][key] = w = run_workload(cfg, pr, 2, 1, physics=phys)
                print(f"workload {key}: {w['elements_per_s']:.4g} elements/s", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, a, args.cpu_budget)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(a, budget_s=min(args.cpu_budget, 10.0))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
