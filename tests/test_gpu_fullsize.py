"""GPU parity of the elastic, Maxwell and p-heterogeneous workloads at full size, in the launch
configuration the benchmark times (autotuned launch schedules; the degree classes of the
variable-degree mesh as one graph).

At these sizes the oracle cannot solve the global system, so the checks are element by element
on seeded samples (the oracle builds each sampled element's stage system by quadrature in
physical coordinates, independently of the library's reference tables):
  * K_e of sampled elements against D - C A^{-1} B (relative 1e-11, FP64);
  * the local equations A u_e + B lam_e = f_e of sampled elements hold for the recovered fields
    (relative 1e-11);
  * the trace equations sum_K (C u_K + D lam_K) = 0 on sampled interior faces (relative 1e-10)
    and lam = the Dirichlet data on sampled boundary faces;
  * mixed precision (FP32 factors + FP64 refinement) equals the FP64 path to 1e-10 per field.
"""
import time

import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GAMMA = 0.43586652150845899
BS_VAR = 21   # face space of degree 5: trace padding on meshes of variable degree


_T0 = [0.0]


def _step(msg):
    """Progress line per step (flushed), so a long host-side check is visibly alive."""
    now = time.time()
    print(f"  [{now - _T0[0]:7.1f} s] {msg}", flush=True)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(p, prec, **kw):
    from paper_1807_00086_amd import Solver
    uk = p.uniform_k
    return Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=uk, degree=None if uk else p.degree,
                  precision=prec, nrhs=p.nrhs, autotune=True, use_graph=not uk, **kw)


def _stage(s, a, f, lb):
    fd = torch.as_tensor(np.ascontiguousarray(f), device="cuda")
    lbd = torch.as_tensor(np.ascontiguousarray(lb), device="cuda")
    s.condense(a, fd, lbd)
    lam = torch.zeros_like(lbd)
    it, rr = s.trace_solve(lam)
    u = torch.zeros_like(fd)
    s.recover(lam, u)
    torch.cuda.synchronize()
    out = u.cpu().numpy(), lam.cpu().numpy(), rr
    del fd, lbd, lam, u
    torch.cuda.empty_cache()
    return out


def _check_local_and_trace(ohdg, d, p, a, u, lam, f, lb, tmap, n_elem_sample, n_face_sample, seed,
                           faces=None, elems=None):
    """Local equations on sampled elements (or on the given elements) and trace equations on
    sampled faces (or on the given faces).  u, f are [n_local][r]; lam, lb are in the library's
    trace layout, tmap maps the oracle's trace dof index to the library's."""
    rng = np.random.default_rng(seed)
    if elems is None:
        elems = np.unique(np.concatenate([[0, p.n_elem - 1], rng.integers(0, p.n_elem, n_elem_sample)]))
    elems = np.asarray(elems, dtype=np.int64)
    _step(f"local equations on {elems.size} elements")
    for e in elems:
        A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
        li, ti = d.elem_local_dofs(e), tmap[d.elem_trace_dofs(e)]
        res = A @ u[li] + B @ lam[ti] - f[li]
        assert np.linalg.norm(res) <= 1e-11 * max(np.linalg.norm(f[li]), np.linalg.norm(A @ u[li])), int(e)
    if faces is None:
        faces = rng.integers(0, d.skel.n_faces, n_face_sample)
    _step(f"trace equations on {len(faces)} faces")
    for F in faces:
        cols = tmap[np.arange(d.tr_off[F], d.tr_off[F + 1])]
        if d.skel.is_boundary[F]:
            assert np.allclose(lam[cols], lb[cols], rtol=0, atol=1e-14)
            continue
        acc, scale = 0.0, 0.0
        for e in d.skel.face_elems[F]:
            A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
            li, ti = d.elem_local_dofs(e), d.elem_trace_dofs(e)
            rows = np.nonzero(np.isin(ti, np.arange(d.tr_off[F], d.tr_off[F + 1])))[0]
            acc = acc + (Cm[rows] @ u[li] + Dm[rows] @ lam[tmap[ti]])
            scale = max(scale, np.abs(Cm[rows] @ u[li]).max())
        assert np.abs(acc).max() <= 1e-10 * scale, int(F)


@pytest.mark.parametrize("cfg,precond", [(3, "jacobi"), (3, "ssor"), (5, "jacobi"), (5, "ssor"), ("glm", "ssor")])
def test_full_size_uniform_sampled(cfg, precond):
    """Elastic k = 4 (24,576 tets), Maxwell and GLM-Maxwell k = 3 (196,608 tets), FP64 and
    mixed, with either trace preconditioner (the benchmark runs these workloads with block SSOR
    and the autotuned launch schedules)."""
    _need_gpu()
    from oracle import hdg as ohdg
    _T0[0] = time.time()
    glm = cfg == "glm"
    cfg = 5 if glm else cfg
    p = make_problem(cfg)
    if glm:
        p.physics = "maxwell_glm"
    print(f"case fullsize cfg={cfg} {p.physics} precond={precond} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    _step("oracle discretisation built")
    s = _solver(p, "fp64", krylov_tol=1e-12, krylov_maxit=4000, precond=precond)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    assert nl == d.loc_off[-1] and nt == d.tr_off[-1]
    f = random_vector(nl, cfg, 11)[:, None]
    lb = (random_vector(nt, cfg, 12) * ohdg.boundary_trace_mask(d))[:, None]
    u, lam, rr = _stage(s, a, f, lb)
    _step(f"FP64 stage done ({s.query('last_iters')} trace iterations, relres {rr:.2e})")
    assert rr <= 1e-12
    t = d.elem_trace_dofs(0).size
    rng = np.random.default_rng(7)
    for e in np.unique(np.concatenate([[0, p.n_elem - 1], rng.integers(0, p.n_elem, 60)])):
        A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
        Ke_ref = Dm - Cm @ np.linalg.solve(A, B)
        Ke = s.element_data("K", int(e), 1, t * t).reshape(t, t)
        assert np.abs(Ke - Ke_ref).max() <= 1e-11 * np.abs(Ke_ref).max(), int(e)
    s.close()
    _step("sampled K_e match the oracle")
    _check_local_and_trace(ohdg, d, p, a, u, lam, f, lb, np.arange(nt), 60, 40, cfg)

    # mixed precision at equal error: within 1e-10 of the FP64 path, per field
    sm = _solver(p, "mixed_fp32", krylov_tol=1e-12, krylov_maxit=4000, refine_tol=1e-11, precond=precond)
    um, lamm, _ = _stage(sm, a, f, lb)
    _step(f"mixed stage done ({sm.query('last_refine')} refinement passes)")
    sm.close()
    # relative L2(Omega) error per field: with the orthonormal basis and affine elements the
    # |J|-weighted coefficient 2-norm (the oracle's l2_norm_fields, vectorised over elements)
    groups = {"elastic": [list(range(6)), [6, 7, 8]], "maxwell": [[0, 1, 2], [3, 4, 5]],
              "maxwell_glm": [[0, 1, 2], [3, 4, 5], [6]]}[d.physics]
    X = p.xyz[p.elem_vert]
    dj = np.abs(np.linalg.det(np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))))[:, None, None]
    m = len(sum(groups, []))
    uf, umf = u[:, 0].reshape(p.n_elem, m, -1), um[:, 0].reshape(p.n_elem, m, -1)
    for g in groups:
        num = np.sqrt(np.sum(dj * (umf[:, g] - uf[:, g]) ** 2))
        den = np.sqrt(np.sum(dj * uf[:, g] ** 2))
        assert num <= 1e-10 * den, (g, num / den)
        _step(f"mixed vs FP64, components {g}: relative L2 {num / den:.2e}")
    assert np.linalg.norm(lamm - lam) <= 1e-10 * np.linalg.norm(lam)


def test_full_size_pvar_sampled():
    """p-heterogeneous acoustics (200,000 tets, k_e in 1..5, 32 point-source right-hand sides),
    FP64 with the degree classes as one graph and the benchmark's trace preconditioner."""
    _need_gpu()
    import bench
    from oracle import hdg as ohdg
    _T0[0] = time.time()
    p = make_problem(4)
    print(f"case fullsize pvar n_elem={p.n_elem} degrees={np.bincount(p.degree)}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / p.dt
    _step("oracle discretisation built")
    s = _solver(p, "fp64", krylov_tol=1e-12, krylov_maxit=4000, precond=bench.STAGE_PRECOND)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    assert nl == d.loc_off[-1] and nt == d.skel.n_faces * BS_VAR
    f = s.point_sources(p.sources)
    lb = np.zeros((nt, p.nrhs))
    _step("point sources built")
    u, lam, rr = _stage(s, a, f, lb)
    _step(f"FP64 stage done ({s.query('last_iters')} trace iterations, relres {rr:.2e})")
    assert set(s.schedules()) == set(int(k) for k in np.unique(p.degree))
    s.close()
    assert rr <= 1e-12
    # oracle trace dof i of face F sits at F * 21 + (i - tr_off[F]) in the library's layout
    face_of = np.repeat(np.arange(d.skel.n_faces), np.diff(d.tr_off))
    tmap = face_of * BS_VAR + (np.arange(d.tr_off[-1]) - d.tr_off[face_of])
    # the sources' elements first: their right-hand sides are nonzero
    hit = np.unique(np.nonzero(np.abs(f).sum(axis=1))[0])
    src_elems = np.unique(np.searchsorted(d.loc_off, hit, side="right") - 1)
    _step(f"local equations on {min(40, src_elems.size)} source elements")
    for e in src_elems[:40]:
        A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
        li, ti = d.elem_local_dofs(e), tmap[d.elem_trace_dofs(e)]
        res = A @ u[li] + B @ lam[ti] - f[li]
        assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(f[li]), int(e)
    # trace equations on the faces of the source elements (away from the sources the fields
    # are many orders smaller than the global residual the trace solve controls)
    faces = np.unique(np.concatenate([list(d.skel.elem_faces[e]) for e in src_elems[:40]]))
    _check_local_and_trace(ohdg, d, p, a, u, lam, f, lb, tmap, 60, 0, 4, faces=faces)


def test_full_size_acoustic_mixed_bench_settings_sampled():
    """The benchmark workload (3D acoustics, k = 3, 82,944 tets) in mixed precision exactly as
    the benchmark runs it: sampled local and trace equations against the oracle's element
    systems, and the reported FP64 residual at or below refine_tol."""
    _need_gpu()
    import bench
    from oracle import hdg as ohdg
    _T0[0] = time.time()
    p = make_problem(2)
    print(f"case fullsize acoustic mixed bench settings n_elem={p.n_elem} {bench.MIXED_OPTS}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    from paper_1807_00086_amd import Solver
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=3, precision="mixed_fp32",
               precond=bench.STAGE_PRECOND, **bench.MIXED_OPTS)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    f = random_vector(nl, 2, 31)[:, None]
    lb = (random_vector(nt, 2, 32) * ohdg.boundary_trace_mask(d))[:, None]
    u, lam, rr = _stage(s, a, f, lb)
    res = s.last_residual()
    _step(f"mixed stage done ({s.query('last_refine')} corrections, residual {res[0]:.2e})")
    s.close()
    assert np.all(res <= bench.MIXED_OPTS["refine_tol"]), res
    _check_local_and_trace(ohdg, d, p, a, u, lam, f, lb, np.arange(nt), 60, 40, 2)


def test_full_size_acoustic_fp64_bench_settings_sampled():
    """The benchmark workload in FP64 exactly as the benchmark runs it (its trace preconditioner,
    multicolour block SSOR, to krylov_tol 1e-13): sampled local and trace equations against the
    oracle's element systems, the trace solve converged on the true residual."""
    _need_gpu()
    import bench
    from oracle import hdg as ohdg
    _T0[0] = time.time()
    p = make_problem(2)
    print(f"case fullsize acoustic fp64 bench settings n_elem={p.n_elem} {bench.STAGE_PRECOND}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    from paper_1807_00086_amd import Solver
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=3, precision="fp64", krylov_tol=1e-13,
               precond=bench.STAGE_PRECOND)
    assert s.query("n_colors") == 4
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    f = random_vector(nl, 2, 33)[:, None]
    lb = (random_vector(nt, 2, 34) * ohdg.boundary_trace_mask(d))[:, None]
    u, lam, rr = _stage(s, a, f, lb)
    _step(f"FP64 stage done ({s.query('last_iters')} trace iterations, relres {rr:.2e})")
    s.close()
    assert rr <= 1e-13
    _check_local_and_trace(ohdg, d, p, a, u, lam, f, lb, np.arange(nt), 60, 40, 3)


def test_full_size_pvar_mixed_sampled():
    """p-heterogeneous acoustics at full size (200,000 tets, 32 point-source columns) in mixed
    precision with the degree classes as one graph: per-column residuals at or below refine_tol
    and the local and trace equations of the source elements against the oracle."""
    _need_gpu()
    import bench
    from oracle import hdg as ohdg
    _T0[0] = time.time()
    p = make_problem(4)
    print(f"case fullsize pvar mixed n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / p.dt
    tol_res = 1e-12
    s = _solver(p, "mixed_fp32", krylov_tol=1e-10, krylov_maxit=4000, refine_tol=tol_res,
                precond=bench.STAGE_PRECOND)
    nt = s.query("n_trace_dofs")
    f = s.point_sources(p.sources)
    lb = np.zeros((nt, p.nrhs))
    u, lam, rr = _stage(s, a, f, lb)
    res = s.last_residual()
    _step(f"mixed stage done ({s.query('last_refine')} corrections, worst residual {res.max():.2e})")
    s.close()
    assert res.shape == (32,) and np.all(res <= tol_res), res
    face_of = np.repeat(np.arange(d.skel.n_faces), np.diff(d.tr_off))
    tmap = face_of * BS_VAR + (np.arange(d.tr_off[-1]) - d.tr_off[face_of])
    hit = np.unique(np.nonzero(np.abs(f).sum(axis=1))[0])
    src_elems = np.unique(np.searchsorted(d.loc_off, hit, side="right") - 1)
    _step(f"local equations on {min(40, src_elems.size)} source elements")
    for e in src_elems[:40]:
        A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
        li, ti = d.elem_local_dofs(e), tmap[d.elem_trace_dofs(e)]
        r = A @ u[li] + B @ lam[ti] - f[li]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(f[li]), int(e)
    # trace equations on the faces of the source elements (elsewhere the fields are many orders
    # below the scale the residual test controls)
    faces = np.unique(np.concatenate([list(d.skel.elem_faces[e]) for e in src_elems[:40]]))
    _check_local_and_trace(ohdg, d, p, a, u, lam, f, lb, tmap, 0, 0, 4, faces=faces, elems=[])


@pytest.mark.parametrize("cfg", [3, 5, "glm"])
def test_full_size_bf16_equals_fp64(cfg):
    """Elastic k = 4 (24,576 tets), Maxwell and GLM-Maxwell k = 3 (196,608 tets) at full size with
    split-BF16 condensation products and FP64 refinement: within 1e-10 of the FP64 path per field
    (the FP64 path is checked against the oracle above), residual at or below refine_tol."""
    _need_gpu()
    import bench
    _T0[0] = time.time()
    glm = cfg == "glm"
    cfg = 5 if glm else cfg
    p = make_problem(cfg)
    if glm:
        p.physics = "maxwell_glm"
    print(f"case fullsize bf16 cfg={cfg} {p.physics} n_elem={p.n_elem}", flush=True)
    a = 1.0 / (GAMMA * p.dt)
    s = _solver(p, "fp64", krylov_tol=1e-12, krylov_maxit=4000, precond=bench.STAGE_PRECOND)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    f = random_vector(nl, cfg, 11)[:, None]
    from oracle import hdg as ohdg
    d = ohdg.make_discretisation(p)
    lb = (random_vector(nt, cfg, 12) * ohdg.boundary_trace_mask(d))[:, None]
    u, lam, _ = _stage(s, a, f, lb)
    s.close()
    sb = _solver(p, "mixed_bf16", krylov_tol=1e-12, krylov_maxit=4000, refine_tol=1e-11,
                 precond=bench.STAGE_PRECOND)
    ub, lamb, _ = _stage(sb, a, f, lb)
    res = sb.last_residual()
    _step(f"bf16 stage done ({sb.query('last_refine')} corrections, residual {res[0]:.2e})")
    sb.close()
    assert np.all(res <= 1e-11)
    groups = {"elastic": [list(range(6)), [6, 7, 8]], "maxwell": [[0, 1, 2], [3, 4, 5]],
              "maxwell_glm": [[0, 1, 2], [3, 4, 5], [6]]}[p.physics]
    m = len(sum(groups, []))
    X = p.xyz[p.elem_vert]
    dj = np.abs(np.linalg.det(np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))))[:, None, None]
    uf, ubf = u[:, 0].reshape(p.n_elem, m, -1), ub[:, 0].reshape(p.n_elem, m, -1)
    for g in groups:
        num = np.sqrt(np.sum(dj * (ubf[:, g] - uf[:, g]) ** 2))
        den = np.sqrt(np.sum(dj * uf[:, g] ** 2))
        assert num <= 1e-10 * den, (g, num / den)
    assert np.linalg.norm(lamb - lam) <= 1e-10 * np.linalg.norm(lam)
