"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on the same
seeded inputs.

Tolerances (relative, per field, L2(Omega) norm = |J|-weighted coefficient norm):
  FP64 mode              1e-12 (stage solution), 1e-11 element-wise (K_e, r_e, Z, z)
  mixed FP32 + refinement 1e-10 (after refinement; the FP32 factors alone give ~1e-6)
"""
import sys

import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle():
    from oracle import hdg as ohdg
    return ohdg


def _solver(p, precision="fp64", **kw):
    from paper_1807_00086_amd import Solver
    return Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=int(p.degree[0]),
                  precision=precision, nrhs=p.nrhs, **kw)


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _rel_field_errors(ohdg, d, u_gpu, u_ref):
    out = []
    groups = {"acoustic": [list(range(d.dim)), [d.dim]], "elastic": [list(range(6)), [6, 7, 8]],
              "maxwell": [[0, 1, 2], [3, 4, 5]], "maxwell_glm": [[0, 1, 2], [3, 4, 5], [6]]}[d.physics]
    for g in groups:
        num = ohdg.l2_norm_fields(d, u_gpu - u_ref, g)
        den = ohdg.l2_norm_fields(d, u_ref, g)
        out.append(num / max(den, 1e-300))
    return out


def _schur_rows(d):
    """(count, first row) of the densely factored block inside an element's local vector."""
    from oracle.polynomials import dim_p
    N = dim_p(int(d.degree[0]), d.dim)
    return {"acoustic": (N, d.dim * N), "elastic": (3 * N, 6 * N), "maxwell": (3 * N, 3 * N),
            "maxwell_glm": (4 * N, 3 * N)}[d.physics]


def _gpu_stage(s, a, f, lb):
    fd, lbd = _dev(f), _dev(lb)
    s.condense(a, fd, lbd)
    lam = torch.zeros_like(lbd)
    it, rr = s.trace_solve(lam)
    u = torch.zeros_like(fd)
    s.recover(lam, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), lam.cpu().numpy(), it, rr


CASES = [
    (1, dict()),                     # 2D acoustic workload itself: 8x8 -> 128 triangles, k=2
    (1, dict(n=5, k=3)),
    (1, dict(n=3, k=1)),
    (2, dict(n=2, k=1)),
    (2, dict(n=2, k=2)),
    (2, dict(n=3, k=3)),             # 162 tets: several workgroup waves, ragged
    (2, dict(n=2, k=4)),
    (3, dict(n=1, k=1)),             # elastic (velocity + symmetric stress)
    (3, dict(n=2, k=2)),
    (3, dict(n=1, k=3)),
    (3, dict(n=1, k=4)),             # workload degree; Schur right-hand sides in global scratch
    (5, dict(n=2, k=1)),             # Maxwell (E, H)
    (5, dict(n=2, k=2)),
    (5, dict(n=2, k=3)),             # workload degree
]


@pytest.mark.parametrize("cfg,kw", CASES)
def test_stage_parity_fp64(cfg, kw):
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(cfg, **kw)
    print(f"case cfg={cfg} {kw} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    f = random_vector(d.loc_off[-1], cfg, 1)
    lb = random_vector(d.tr_off[-1], cfg, 2) * ohdg.boundary_trace_mask(d)
    u_ref, lam_ref, cond = ohdg.solve_stage(d, a, f, lb)
    s = _solver(p)
    u, lam, it, rr = _gpu_stage(s, a, f, lb)
    assert rr <= 1e-13
    errs = _rel_field_errors(ohdg, d, u, u_ref)
    assert max(errs) <= 1e-12, errs
    assert np.linalg.norm(lam - lam_ref) <= 1e-12 * np.linalg.norm(lam_ref)
    # element-wise quantities of the condensation
    t = cond.Ke[0].shape[0]
    ne = p.n_elem
    ns, r0 = _schur_rows(d)
    Ke = s.element_data("K", 0, ne, t * t).reshape(ne, t, t)
    re = s.element_data("r", 0, ne, t).reshape(ne, t)
    Z = s.element_data("Z", 0, ne, ns * t).reshape(ne, ns, t)
    z = s.element_data("z", 0, ne, ns).reshape(ne, ns)
    for e in range(0, ne, max(1, ne // 17)):
        sc = np.abs(cond.Ke[e]).max()
        assert np.abs(Ke[e] - cond.Ke[e]).max() <= 1e-11 * sc
        assert np.abs(re[e] - cond.re[e][:, 0]).max() <= 1e-11 * max(np.abs(cond.re[e]).max(), 1e-300)
        Zr, zr = cond.Z[e][r0:r0 + ns], cond.z[e][r0:r0 + ns, 0]
        assert np.abs(Z[e] - Zr).max() <= 1e-11 * np.abs(Zr).max()
        assert np.abs(z[e] - zr).max() <= 1e-11 * np.abs(zr).max()
    s.close()


MIXED_CASES = [
    (1, dict()),
    (1, dict(n=4, k=4)),
    (2, dict(n=2, k=2)),
    (2, dict(n=3, k=3)),
    (3, dict(n=1, k=2)),
    (3, dict(n=1, k=4)),
    (5, dict(n=2, k=2)),
    (5, dict(n=2, k=3)),
]


@pytest.mark.parametrize("cfg,kw", MIXED_CASES)
def test_stage_parity_mixed(cfg, kw):
    """FP32 condensation + FP64 refinement reaches the FP64 oracle to 1e-10 per field."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(cfg, **kw)
    print(f"case mixed cfg={cfg} {kw} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    f = random_vector(d.loc_off[-1], cfg, 1)
    lb = random_vector(d.tr_off[-1], cfg, 2) * ohdg.boundary_trace_mask(d)
    u_ref, lam_ref, cond = ohdg.solve_stage(d, a, f, lb)
    s = _solver(p, precision="mixed_fp32", krylov_tol=1e-9, refine_tol=1e-12)
    u, lam, it, rr = _gpu_stage(s, a, f, lb)
    nref = s.query("last_refine")
    errs = _rel_field_errors(ohdg, d, u, u_ref)
    assert 1 <= nref <= 6
    assert max(errs) <= 1e-10, (errs, nref)
    assert np.all(s.last_residual() <= 1e-12), s.last_residual()
    assert np.linalg.norm(lam - lam_ref) <= 1e-10 * np.linalg.norm(lam_ref)
    # the FP32 Schur complements themselves are only single-precision accurate
    t = cond.Ke[0].shape[0]
    Ke = s.element_data("K", 0, 1, t * t).reshape(t, t)
    rel = np.abs(Ke - cond.Ke[0]).max() / np.abs(cond.Ke[0]).max()
    assert 1e-9 < rel < 1e-5
    # a second recover without a new condensation is a call-order error
    from paper_1807_00086_amd import HDGError
    with pytest.raises(HDGError) as ei:
        s.recover(_dev(lam), _dev(u))
    assert ei.value.code == 7
    s.close()


@pytest.mark.parametrize("cfg,kw", [(2, dict(n=3, k=3)), (2, dict(n=4, k=3)), (1, dict())])
def test_stage_parity_mixed_bench_settings(cfg, kw):
    """The mixed-precision path exactly as the benchmark runs it (its trace preconditioner, the
    first trace solve to its krylov_tol, the refinement stopping on the FP64 residual at its
    refine_tol) matches the FP64 oracle to 1e-10 per field, and the reported residual meets
    refine_tol."""
    _need_gpu()
    import bench
    ohdg = _oracle()
    p = make_problem(cfg, **kw)
    print(f"case mixed bench settings cfg={cfg} {kw} n_elem={p.n_elem} {bench.MIXED_OPTS}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    f = random_vector(d.loc_off[-1], cfg, 5)
    lb = random_vector(d.tr_off[-1], cfg, 6) * ohdg.boundary_trace_mask(d)
    u_ref, lam_ref, _ = ohdg.solve_stage(d, a, f, lb)
    s = _solver(p, precision="mixed_fp32", precond=bench.STAGE_PRECOND, **bench.MIXED_OPTS)
    u, lam, it, rr = _gpu_stage(s, a, f, lb)
    errs = _rel_field_errors(ohdg, d, u, u_ref)
    res = s.last_residual()
    print(f"  corrections {s.query('last_refine')}, residual {res[0]:.2e}, errors {errs}", flush=True)
    assert np.all(res <= bench.MIXED_OPTS["refine_tol"]), res
    assert max(errs) <= 1e-10, errs
    assert np.linalg.norm(lam - lam_ref) <= 1e-10 * np.linalg.norm(lam_ref)
    s.close()


def test_full_size_acoustic3d_mixed_equals_fp64():
    """Full 82,944-element workload: the refined mixed solution equals the FP64 path
    (itself oracle-checked above) to 1e-10 per field."""
    _need_gpu()
    p = make_problem(2)
    a = 1.0 / (0.43586652150845899 * p.dt)
    s64 = _solver(p)
    nl, nt = s64.query("n_local_dofs"), s64.query("n_trace_dofs")
    f = random_vector(nl, 2, 11)
    lb = random_vector(nt, 2, 12)
    # only the boundary-face entries of lam_bnd are read by the library
    u64, l64, _, _ = _gpu_stage(s64, a, f, lb)
    s64.close()
    s32 = _solver(p, precision="mixed_fp32", krylov_tol=1e-8, refine_tol=1e-12)
    u32, l32, _, _ = _gpu_stage(s32, a, f, lb)
    assert s32.query("last_refine") >= 1
    N = 20
    ue, ue32 = u64.reshape(p.n_elem, 4, N), u32.reshape(p.n_elem, 4, N)
    for comps in ([0, 1, 2], [3]):
        num = np.sqrt(np.sum(np.abs(_detJ(p))[:, None, None] * (ue32[:, comps] - ue[:, comps]) ** 2))
        den = np.sqrt(np.sum(np.abs(_detJ(p))[:, None, None] * ue[:, comps] ** 2))
        assert num / den <= 1e-10, (comps, num / den)
    assert np.linalg.norm(l32 - l64) <= 1e-10 * np.linalg.norm(l64)
    s32.close()


def _detJ(p):
    X = p.xyz[p.elem_vert]
    return np.linalg.det(np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1)))


def test_stage_parity_repeatable_bitwise():
    """Owner-computes assembly and fixed reduction order: two runs give identical bits."""
    _need_gpu()
    p = make_problem(2, n=3, k=2)
    s = _solver(p)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    f = random_vector(nl, 2, 1)
    lb = random_vector(nt, 2, 2)
    u1, l1, _, _ = _gpu_stage(s, 50.0, f, lb)
    u2, l2, _, _ = _gpu_stage(s, 50.0, f, lb)
    assert np.array_equal(u1, u2) and np.array_equal(l1, l2)


def test_full_size_acoustic3d_sampled():
    """The 82,944-element acoustic workload at full size, as the benchmark runs it: sampled
    element-level parity against the oracle, and the local equations A u + B lam = f of
    sampled elements hold for the recovered fields."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(2)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    s = _solver(p)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    assert nl == d.loc_off[-1] and nt == d.tr_off[-1]
    f = random_vector(nl, 2, 11)
    lb = random_vector(nt, 2, 12)
    u, lam, it, rr = _gpu_stage(s, a, f, lb)
    assert rr <= 1e-13
    n, t = 80, 40
    rng = np.random.default_rng(5)
    sample = np.unique(np.concatenate([[0, 1, p.n_elem - 1], rng.integers(0, p.n_elem, 300)]))
    for e in sample:
        A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
        li, ti = d.elem_local_dofs(e), d.elem_trace_dofs(e)
        Ke_ref = Dm - Cm @ np.linalg.solve(A, B)
        Ke = s.element_data("K", int(e), 1, t * t).reshape(t, t)
        assert np.abs(Ke - Ke_ref).max() <= 1e-11 * np.abs(Ke_ref).max()
        res = A @ u[li] + B @ lam[ti] - f[li]
        assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(f[li])
    # trace equations on sampled interior faces: sum_K (C u + D lam) = 0
    bm = ohdg.boundary_trace_mask(d)
    faces = rng.integers(0, d.skel.n_faces, 200)
    for F in faces:
        if d.skel.is_boundary[F]:
            sl = slice(d.tr_off[F], d.tr_off[F + 1])
            assert np.allclose(lam[sl], lb[sl], rtol=0, atol=1e-14)
            continue
        acc = 0.0
        scale = 0.0
        for e in d.skel.face_elems[F]:
            A, B, Cm, Dm, _ = ohdg.element_system(d, int(e), a)
            li, ti = d.elem_local_dofs(e), d.elem_trace_dofs(e)
            f_loc = list(d.skel.elem_faces[e]).index(F)
            rows = slice(f_loc * 10, (f_loc + 1) * 10)
            acc = acc + (Cm @ u[li] + Dm @ lam[ti])[rows]
            scale = max(scale, np.abs(Cm[rows] @ u[li]).max())
        assert np.abs(acc).max() <= 1e-10 * scale
    s.close()


def test_dirk_step_parity_fp64():
    """Two DIRK(3,3) steps through hdg_step against the oracle's stage recursion."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(2, n=2, k=2)
    d = ohdg.make_discretisation(p)
    u0 = random_vector(d.loc_off[-1], 2, 21)
    bm = ohdg.boundary_trace_mask(d)
    _, _, c = ohdg.dirk33()
    dt = 0.01
    lbs = {}
    for n in range(2):
        for i in range(3):
            lbs[round(n * dt + c[i] * dt, 12)] = random_vector(d.tr_off[-1], 2, 100 + 3 * n + i) * bm
    u_ref = u0.copy()
    for n in range(2):
        u_ref = ohdg.dirk_step(d, u_ref, n * dt, dt, lambda t: lbs[round(t, 12)])
    s = _solver(p)
    u = _dev(u0)
    lam = torch.zeros(d.tr_off[-1], dtype=torch.float64, device="cuda")
    for n in range(2):
        stages = np.stack([lbs[round(n * dt + c[i] * dt, 12)] for i in range(3)])
        s.step(n * dt, dt, "dirk33", u, lam, _dev(stages))
    torch.cuda.synchronize()
    errs = _rel_field_errors(ohdg, d, u.cpu().numpy(), u_ref)
    assert max(errs) <= 1e-12, errs
    s.close()


def test_apply_mass_and_projections():
    """Stage-glue mass application and the projection helpers against the oracle (a
    polynomial field, integrated exactly by both quadrature rules)."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(2, n=2, k=3)
    d = ohdg.make_discretisation(p)
    s = _solver(p)
    u = random_vector(d.loc_off[-1], 2, 31)
    f = torch.zeros(d.loc_off[-1], dtype=torch.float64, device="cuda")
    s.apply_mass(7.0, _dev(u), f)
    torch.cuda.synchronize()
    ref = ohdg.apply_mass(d, u, 7.0)
    assert np.abs(f.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()

    def poly(x, t=0.0):
        return np.stack([x[:, 0] ** 2, x[:, 1] * x[:, 2], x[:, 0] ** 3 - x[:, 2], 1 + x[:, 0] * x[:, 1]], 1)
    up = s.project_volume(poly(s.volume_points()))
    assert np.abs(up - ohdg.project_volume(d, poly)).max() <= 1e-12
    bp = s.boundary_points()
    lam = s.project_boundary(poly(bp)[:, 3])
    lref = ohdg.project_boundary(d, lambda x, t: poly(x)[:, 3])
    assert np.abs(lam - lref).max() <= 1e-12
    s.close()


def test_singular_pivot_reported():
    """Local blocks that cannot be factored are reported as HDG_E_SINGULAR by the next
    synchronising call (forced from the host with an infinite-impedance material, which
    removes the mass and stabilisation terms from the Schur block; no device fault)."""
    _need_gpu()
    from paper_1807_00086_amd import HDGError
    p = make_problem(2, n=1, k=2)
    p.elem_par[:, 1] = 1e300
    s = _solver(p)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    s.condense(1.0, _dev(np.ones(nl)), _dev(np.zeros(nt)))
    lam = torch.zeros(nt, dtype=torch.float64, device="cuda")
    with pytest.raises(HDGError) as ei:
        s.trace_solve(lam)
    assert ei.value.code == 5
    s.close()


def test_nonfinite_rhs_reports_noconv():
    _need_gpu()
    from paper_1807_00086_amd import HDGError
    p = make_problem(2, n=1, k=1)
    s = _solver(p)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    s.condense(1.0, _dev(np.full(nl, np.nan)), _dev(np.zeros(nt)))
    lam = torch.zeros(nt, dtype=torch.float64, device="cuda")
    with pytest.raises(HDGError) as ei:
        s.trace_solve(lam)
    assert ei.value.code == 6
    s.close()


GLM_CASES = [(dict(n=2, k=1), "fp64"), (dict(n=2, k=2), "fp64"), (dict(n=2, k=3), "fp64"),
             (dict(n=2, k=1), "mixed_fp32"), (dict(n=2, k=2), "mixed_fp32"), (dict(n=2, k=3), "mixed_fp32")]


@pytest.mark.parametrize("kw,prec", GLM_CASES)
def test_stage_parity_glm_maxwell(kw, prec):
    """GLM-Maxwell (section 5.2 with the multiplier phi of section 5.1.2, eliminated locally
    through the signed factorisation of the Schur block): H, E, phi and the trace against the
    oracle's (dmax1)-(dmax3) system; FP64 also the element Schur complements and local solves."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(5, **kw)
    p.physics = "maxwell_glm"
    print(f"case glm {kw} {prec} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    f = random_vector(d.loc_off[-1], 5, 7)
    lb = random_vector(d.tr_off[-1], 5, 8) * ohdg.boundary_trace_mask(d)
    u_ref, lam_ref, cond = ohdg.solve_stage(d, a, f, lb)
    kws = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    s = _solver(p, precision=prec, **kws)
    assert s.query("m_local") == 7
    u, lam, it, rr = _gpu_stage(s, a, f, lb)
    tol = 1e-12 if prec == "fp64" else 1e-10
    errs = _rel_field_errors(ohdg, d, u, u_ref)
    assert max(errs) <= tol, errs
    assert np.linalg.norm(lam - lam_ref) <= tol * np.linalg.norm(lam_ref)
    if prec == "fp64":
        t = cond.Ke[0].shape[0]
        ne = p.n_elem
        ns, r0 = _schur_rows(d)
        Ke = s.element_data("K", 0, ne, t * t).reshape(ne, t, t)
        Z = s.element_data("Z", 0, ne, ns * t).reshape(ne, ns, t)
        z = s.element_data("z", 0, ne, ns).reshape(ne, ns)
        for e in range(0, ne, max(1, ne // 11)):
            assert np.abs(Ke[e] - cond.Ke[e]).max() <= 1e-11 * np.abs(cond.Ke[e]).max()
            Zr, zr = cond.Z[e][r0:r0 + ns], cond.z[e][r0:r0 + ns, 0]
            assert np.abs(Z[e] - Zr).max() <= 1e-11 * np.abs(Zr).max()
            assert np.abs(z[e] - zr).max() <= 1e-11 * np.abs(zr).max()
    else:
        assert np.all(s.last_residual() <= 1e-12)
    s.close()


BF16_CASES = [(3, dict(n=1, k=2), "elastic"), (3, dict(n=1, k=3), "elastic"), (3, dict(n=1, k=4), "elastic"),
              (5, dict(n=2, k=2), "maxwell"), (5, dict(n=2, k=3), "maxwell"), (5, dict(n=2, k=2), "maxwell_glm")]


@pytest.mark.parametrize("cfg,kw,phys", BF16_CASES)
def test_stage_parity_mixed_bf16(cfg, kw, phys):
    """Split-BF16 matrix-core products in the condensation + FP64 refinement: the refined stage
    reaches the FP64 oracle to 1e-10 per field, while the BF16 Schur complements themselves are
    visibly less accurate than the FP32 ones (so the BF16 products are the ones that ran)."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(cfg, **kw)
    p.physics = phys
    print(f"case bf16 {phys} {kw} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    f = random_vector(d.loc_off[-1], cfg, 9)
    lb = random_vector(d.tr_off[-1], cfg, 10) * ohdg.boundary_trace_mask(d)
    u_ref, lam_ref, cond = ohdg.solve_stage(d, a, f, lb)
    s = _solver(p, precision="mixed_bf16", krylov_tol=1e-9, refine_tol=1e-12)
    u, lam, it, rr = _gpu_stage(s, a, f, lb)
    errs = _rel_field_errors(ohdg, d, u, u_ref)
    print(f"  corrections {s.query('last_refine')}, residual {s.last_residual()[0]:.2e}, errors {errs}", flush=True)
    assert max(errs) <= 1e-10, errs
    assert np.linalg.norm(lam - lam_ref) <= 1e-10 * np.linalg.norm(lam_ref)
    assert np.all(s.last_residual() <= 1e-12)
    t = cond.Ke[0].shape[0]
    Ke = s.element_data("K", 0, 1, t * t).reshape(t, t)
    rel = np.abs(Ke - cond.Ke[0]).max() / np.abs(cond.Ke[0]).max()
    assert 1e-7 < rel < 1e-2, rel
    s.close()
