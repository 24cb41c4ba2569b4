"""The multicolour block SSOR preconditioner of the trace CG (options.precond = ssor; the
symmetric counterpart, for the symmetric definite trace system, of the block incomplete
factorisation the paper uses in section 2.4.2).  The preconditioner changes the iterates, not
the solution: every stage must match the oracle to the usual tolerances (FP64 1e-12, mixed
1e-10 relative per field) with the trace solve converged to krylov_tol on the true residual, in
fewer CG iterations than block Jacobi."""
import numpy as np
import pytest

from synth import make_problem, random_vector, tag_box_faces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GAMMA = 0.43586652150845899


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _groups(physics):
    return {"acoustic": [[0, 1, 2], [3]], "elastic": [list(range(6)), [6, 7, 8]],
            "maxwell": [[0, 1, 2], [3, 4, 5]], "maxwell_glm": [[0, 1, 2], [3, 4, 5], [6]]}[physics]


CASES = [
    (2, dict(n=3, k=2), "acoustic", "fp64", False),      # face blocks of 6
    (2, dict(n=3, k=3), "acoustic", "fp64", False),      # 10: the benchmark degree
    (2, dict(n=3, k=3), "acoustic", "mixed_fp32", False),
    (2, dict(n=2, k=3), "acoustic", "fp64", True),       # with Neumann faces
    (3, dict(n=1, k=4), "elastic", "fp64", False),       # 45
    (5, dict(n=2, k=3), "maxwell", "fp64", False),       # 20
    (5, dict(n=2, k=3), "maxwell_glm", "fp64", False),
    (3, dict(n=1, k=4), "elastic", "mixed_bf16", False),   # split-BF16 products, symmetric K_e
]


@pytest.mark.parametrize("cfg,kw,phys,prec,neumann", CASES)
def test_ssor_stage_parity_and_iterations(cfg, kw, phys, prec, neumann):
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    p = make_problem(cfg, **kw)
    p.physics = phys
    if neumann:
        tag_box_faces(p, [(0, 0.0), (2, 1.0)])
    print(f"case ssor {phys} {kw} {prec} neumann={neumann} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    mask = ohdg.boundary_trace_mask(d) | ohdg.neumann_trace_mask(d)
    f = random_vector(d.loc_off[-1], cfg, 81)
    lb = random_vector(d.tr_off[-1], cfg, 82) * mask
    u_ref, lam_ref, _ = ohdg.solve_stage(d, a, f, lb)
    opts = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    res = {}
    for pc in ("jacobi", "ssor"):
        s = Solver(p.xyz, p.elem_vert, phys, p.elem_par, k=kw["k"], precision=prec, precond=pc,
                   bface_tag=p.bface_tag, **opts)
        if pc == "ssor":
            assert 1 <= s.query("n_colors") <= 7
        fd = torch.as_tensor(f, device="cuda")
        lbd = torch.as_tensor(lb, device="cuda")
        s.condense(a, fd, lbd)
        lam = torch.zeros_like(lbd)
        it, rr = s.trace_solve(lam)
        u = torch.zeros_like(fd)
        s.recover(lam, u)
        torch.cuda.synchronize()
        res[pc] = (u.cpu().numpy(), lam.cpu().numpy(), it, rr)
        s.close()
    u, lam, it, rr = res["ssor"]
    assert rr <= opts["krylov_tol"], rr
    assert it < res["jacobi"][2], (it, res["jacobi"][2])
    tol = 1e-12 if prec == "fp64" else 1e-10
    for g in _groups(phys):
        num = ohdg.l2_norm_fields(d, u - u_ref, g)
        den = ohdg.l2_norm_fields(d, u_ref, g)
        assert num <= tol * den, (g, num / den)
    assert np.linalg.norm(lam - lam_ref) <= tol * np.linalg.norm(lam_ref)
    print(f"iterations jacobi {res['jacobi'][2]} ssor {it}", flush=True)


@pytest.mark.parametrize("cfg,kw,phys,t", [(3, dict(n=1, k=4), "elastic", 180), (5, dict(n=1, k=3), "maxwell", 80)])
def test_element_matrices_exactly_symmetric_in_every_precision(cfg, kw, phys, t):
    """Eisenstat's form takes the scaled diagonal blocks as the identity, so the assembled K must
    be symmetric to the last bit: K_e is, in FP64, mixed FP32 and mixed BF16 (where the two
    triangles of a diagonal tile would round differently; the tile's upper triangle is mirrored)."""
    _need_gpu()
    from paper_1807_00086_amd import Solver
    p = make_problem(cfg, **kw)
    p.physics = phys
    a = 1.0 / (GAMMA * p.dt)
    for prec in ("fp64", "mixed_fp32", "mixed_bf16"):
        s = Solver(p.xyz, p.elem_vert, phys, p.elem_par, k=kw["k"], precision=prec)
        nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
        s.condense(a, torch.as_tensor(random_vector(nl, cfg, 89), device="cuda"),
                   torch.zeros(nt, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        for e in (0, p.n_elem // 2, p.n_elem - 1):
            K = s.element_data("K", e, 1, t * t).reshape(t, t)
            assert np.array_equal(K, K.T), (prec, e)
        s.close()


def test_ssor_variable_degree_single_rhs():
    """Acoustics of variable degree (k_e in 1..5, faces padded to the degree-5 block of 21 with
    identity rows) with one right-hand side: the SSOR CG on the padded system matches the oracle
    (FP64 1e-12 per field), the padding stays zero, and it takes fewer iterations than block
    Jacobi."""
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    from test_gpu_pvar import _pad, _unpad
    p = make_problem(4, nxyz=(2, 2, 1))
    p.nrhs = 1
    print(f"case ssor variable degree n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    f = random_vector(d.loc_off[-1], 4, 85)[:, None]
    lb = (random_vector(d.tr_off[-1], 4, 86) * ohdg.boundary_trace_mask(d))[:, None]
    u_ref, lam_ref, _ = ohdg.solve_stage(d, a, f, lb)
    res = {}
    for pc in ("jacobi", "ssor"):
        s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=None, degree=p.degree, precision="fp64",
                   precond=pc, krylov_tol=1e-13)
        fd = torch.as_tensor(f, device="cuda")
        lbd = torch.as_tensor(_pad(d, lb), device="cuda")
        s.condense(a, fd, lbd)
        lam = torch.zeros_like(lbd)
        it, rr = s.trace_solve(lam)
        u = torch.zeros_like(fd)
        s.recover(lam, u)
        torch.cuda.synchronize()
        res[pc] = (u.cpu().numpy(), lam.cpu().numpy(), it, rr, s.query("n_colors"))
        s.close()
    u, lam_p, it, rr, nc = res["ssor"]
    assert nc > 0 and rr <= 1e-13, (nc, rr)
    assert it < res["jacobi"][2], (it, res["jacobi"][2])
    lam, pad_max = _unpad(d, lam_p)
    assert pad_max == 0.0
    for g in _groups("acoustic"):
        num = ohdg.l2_norm_fields(d, u[:, 0] - u_ref[:, 0], g)
        den = ohdg.l2_norm_fields(d, u_ref[:, 0], g)
        assert num <= 1e-12 * den, (g, num / den)
    assert np.linalg.norm(lam - lam_ref) <= 1e-12 * np.linalg.norm(lam_ref)
    print(f"iterations jacobi {res['jacobi'][2]} ssor {it}", flush=True)


SSOR32_CASES = [
    (2, dict(n=2, k=2), "fp64", False),           # face blocks of 6
    (2, dict(n=2, k=3), "fp64", False),           # 10
    (2, dict(n=2, k=3), "mixed_fp32", False),     # correction solves with SSOR too
    (2, dict(n=2, k=3), "fp64", True),            # with Neumann faces
    (4, dict(nxyz=(2, 2, 1)), "fp64", False),     # variable degree: padded blocks of 21
]


@pytest.mark.parametrize("cfg,kw,prec,neumann", SSOR32_CASES)
def test_ssor_32_rhs_parity_and_iterations(cfg, kw, prec, neumann):
    """32 right-hand sides: the sweeps run the face blocks on the FP64 matrix cores (one face
    per wavefront, the 32 columns as the MFMA's N dimension) and the CG keeps per-column
    scalars; every column matches the oracle (FP64 1e-12, mixed 1e-10 relative per field) with
    the true residual of every column at krylov_tol, in fewer iterations than block Jacobi."""
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    from test_gpu_pvar import _pad, _unpad
    p = make_problem(cfg, **kw)
    if neumann:
        tag_box_faces(p, [(0, 0.0), (2, 1.0)])
    R = 32
    var = p.uniform_k is None
    print(f"case ssor 32 rhs cfg={cfg} {kw} {prec} neumann={neumann} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    mask = ohdg.boundary_trace_mask(d) | ohdg.neumann_trace_mask(d)
    F = random_vector(d.loc_off[-1] * R, cfg, 87).reshape(-1, R)
    LB = random_vector(d.tr_off[-1] * R, cfg, 88).reshape(-1, R) * mask[:, None]
    u_ref, lam_ref, _ = ohdg.solve_stage(d, a, F, LB)
    opts = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    res = {}
    for pc in ("jacobi", "ssor"):
        s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=p.uniform_k, degree=p.degree if var else None,
                   precision=prec, nrhs=R, precond=pc, bface_tag=p.bface_tag, **opts)
        fd = torch.as_tensor(np.ascontiguousarray(F), device="cuda")
        lbd = torch.as_tensor(np.ascontiguousarray(_pad(d, LB) if var else LB), device="cuda")
        s.condense(a, fd, lbd)
        lam = torch.zeros_like(lbd)
        it, rr = s.trace_solve(lam)
        u = torch.zeros_like(fd)
        s.recover(lam, u)
        torch.cuda.synchronize()
        res[pc] = (u.cpu().numpy(), lam.cpu().numpy(), it, rr)
        s.close()
    u, lam, it, rr = res["ssor"]
    assert rr <= opts["krylov_tol"], rr
    assert it < res["jacobi"][2], (it, res["jacobi"][2])
    if var:
        lam, pad_max = _unpad(d, lam)
        assert pad_max == 0.0
    tol = 1e-12 if prec == "fp64" else 1e-10
    for q in range(R):
        for g in _groups(p.physics):
            num = ohdg.l2_norm_fields(d, u[:, q] - u_ref[:, q], g)
            den = ohdg.l2_norm_fields(d, u_ref[:, q], g)
            assert num <= tol * den, (q, g, num / den)
        assert np.linalg.norm(lam[:, q] - lam_ref[:, q]) <= tol * np.linalg.norm(lam_ref[:, q]), q
    print(f"iterations jacobi {res['jacobi'][2]} ssor {it}", flush=True)


@pytest.mark.parametrize("R", [1, 32])
def test_ssor_iteration_limit_energy_decreases(R):
    """Stopped at the iteration limit m (HDG_E_NOCONV), the returned trace is the m-th CG iterate:
    its error in the energy norm of K (|e^T K e|, which CG minimises over a growing Krylov space) strictly
    decreases from m = 2 to 3 to 4 in every column.  With 32 columns the solution update of the
    last iteration is applied on its own at the limit (otherwise it rides on the next direction
    update), so a lost update would repeat the previous iterate."""
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import HDGError, Solver
    p = make_problem(2, n=2, k=3)
    print(f"case ssor iteration limit R={R} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    mask = ohdg.boundary_trace_mask(d)
    F = random_vector(d.loc_off[-1] * R, 2, 91).reshape(-1, R)
    LB = random_vector(d.tr_off[-1] * R, 2, 92).reshape(-1, R) * mask[:, None]
    cond = ohdg.condense(d, a, F)
    lam_ref = ohdg.trace_solve(d, cond, LB)
    K = cond.K.tocsr()
    energies = []
    for m in (2, 3, 4):
        s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=3, precision="fp64", nrhs=R, precond="ssor",
                   krylov_tol=1e-30, krylov_maxit=m)
        s.condense(a, torch.as_tensor(np.ascontiguousarray(F), device="cuda"),
                   torch.as_tensor(np.ascontiguousarray(LB), device="cuda"))
        lam = torch.zeros(d.tr_off[-1] * R, dtype=torch.float64, device="cuda")
        with pytest.raises(HDGError):
            s.trace_solve(lam)
        torch.cuda.synchronize()
        e = lam.cpu().numpy().reshape(-1, R) - lam_ref
        assert np.all(e[mask] == 0.0)   # Dirichlet values are set, not iterated
        energies.append(np.einsum("ir,ir->r", e, K @ e))
        s.close()
    # K is definite with the sign of its physics (negative for acoustics): compare |e^T K e|
    sgn = np.sign(energies[0][0])
    E2, E3, E4 = (sgn * E for E in energies)
    assert np.all(E2 > 0.0)
    assert np.all(E3 < E2) and np.all(E4 < E3), (E2, E3, E4)
    print(f"energy error m=2..4, worst ratio {np.max(E3 / E2):.3f} {np.max(E4 / E3):.3f}", flush=True)
