"""GPU parity with Neumann boundary faces (mesh.bface_tag): the faces on x = 0 and z = 1 carry
a Neumann condition, the other four faces of the box a Dirichlet one.  A Neumann face keeps its
element's flux rows in the trace system and adds the tested flux datum <g_N, mu>_F to their
right-hand side (section 4.1.2, the Gamma_N part of the trace equation).  Compared with the CPU
FP64 oracle (itself pinned by polynomial reproduction with Neumann faces) on the same seeded
data: random local right-hand sides, random Dirichlet values and random Neumann data.

Tolerances as for the Dirichlet-only stages: FP64 1e-12 relative per field, mixed precision
with FP64 refinement 1e-10 (and the reported FP64 residual at or below refine_tol).
"""
import numpy as np
import pytest

from synth import make_problem, random_vector, tag_box_faces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PLANES = [(0, 0.0), (2, 1.0)]
GAMMA = 0.43586652150845899


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _field_groups(physics):
    return {"acoustic": [[0, 1, 2], [3]], "elastic": [list(range(6)), [6, 7, 8]],
            "maxwell": [[0, 1, 2], [3, 4, 5]], "maxwell_glm": [[0, 1, 2], [3, 4, 5], [6]]}[physics]


def _problem(cfg, kw):
    if cfg == "glm":
        p = make_problem(5, **kw)
        p.physics = "maxwell_glm"
        cfg = 5
    else:
        p = make_problem(cfg, **kw)
    tag_box_faces(p, PLANES)
    return p, cfg


CASES = [
    (2, dict(n=2, k=2), 1, "fp64"),            # acoustic fast path
    (2, dict(n=2, k=3), 1, "mixed_fp32"),      # fused recovery and refinement
    (2, dict(n=2, k=2), 32, "fp64"),           # block-structured, 32 right-hand sides
    (2, dict(n=2, k=2), 32, "mixed_fp32"),
    (3, dict(n=1, k=2), 1, "fp64"),            # elastic
    (3, dict(n=1, k=2), 1, "mixed_fp32"),
    (5, dict(n=2, k=2), 1, "fp64"),            # Maxwell
    ("glm", dict(n=2, k=1), 1, "mixed_fp32"),  # GLM-Maxwell
    (4, dict(nxyz=(2, 2, 1)), 1, "fp64"),      # acoustics of variable degree
]


@pytest.mark.parametrize("cfg,kw,R,prec", CASES)
def test_neumann_stage_parity(cfg, kw, R, prec):
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    p, cfgi = _problem(cfg, kw)
    print(f"case neumann {p.physics} {kw} R={R} {prec} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    assert d.neumann.sum() > 0
    a = 1.0 / (GAMMA * p.dt)
    nl, nt = d.loc_off[-1], d.tr_off[-1]
    mask = ohdg.boundary_trace_mask(d) | ohdg.neumann_trace_mask(d)
    F = random_vector(nl * R, cfgi, 71).reshape(nl, R)
    LB = random_vector(nt * R, cfgi, 72).reshape(nt, R) * mask[:, None]
    u_ref, lam_ref, _ = ohdg.solve_stage(d, a, F, LB)
    mixed = prec != "fp64"
    kw_s = dict(krylov_tol=1e-9, refine_tol=1e-12) if mixed else dict(krylov_tol=1e-13)
    uk = p.uniform_k
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=uk, degree=None if uk else p.degree,
               precision=prec, nrhs=R, bface_tag=p.bface_tag, **kw_s)
    var = uk is None
    LBl = LB
    if var:
        from test_gpu_pvar import _pad
        LBl = _pad(d, LB)
    fd, lbd = _dev(F), _dev(LBl)
    s.condense(a, fd, lbd)
    lam = torch.zeros_like(lbd)
    s.trace_solve(lam)
    u = torch.zeros_like(fd)
    s.recover(lam, u)
    torch.cuda.synchronize()
    u, lam = u.cpu().numpy(), lam.cpu().numpy()
    if var:
        from test_gpu_pvar import _unpad
        lam = _unpad(d, lam)[0]
    if mixed:
        assert np.all(s.last_residual() <= 1e-12), s.last_residual()
    s.close()
    tol = 1e-10 if mixed else 1e-12
    for q in range(R):
        for g in _field_groups(p.physics):
            num = ohdg.l2_norm_fields(d, u[:, q] - u_ref[:, q], g)
            den = ohdg.l2_norm_fields(d, u_ref[:, q], g)
            assert num <= tol * den, (q, g, num / den)
        assert np.linalg.norm(lam[:, q] - lam_ref[:, q]) <= tol * np.linalg.norm(lam_ref[:, q])


def test_neumann_project_boundary_matches_oracle():
    """hdg_project_boundary on a mesh with Neumann faces: the L2 projection of the trace on
    Dirichlet faces, the tested flux on Neumann faces (polynomial data, exact quadrature)."""
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    p, _ = _problem(2, dict(n=2, k=2))
    d = ohdg.make_discretisation(p)
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=2, bface_tag=p.bface_tag)

    def pres(x):
        return 1.0 + x[:, 0] * x[:, 1] - x[:, 2] ** 2

    def vel(x):
        return np.stack([x[:, 1] ** 2, x[:, 0] - x[:, 2], x[:, 0] * x[:, 2]], 1)

    def normal(x):
        n = np.zeros_like(x)
        n[np.abs(x[:, 0]) < 1e-12, 0] = -1.0
        n[np.abs(x[:, 2] - 1.0) < 1e-12, 2] = 1.0
        return n

    bp = s.boundary_points()
    nb = normal(bp)
    on_n = np.abs(nb).sum(1) > 0
    vals = np.where(on_n, np.sum(vel(bp) * nb, 1), pres(bp))
    lam = s.project_boundary(vals)
    s.close()
    ref = ohdg.project_boundary(d, lambda x, t: pres(x)) + ohdg.neumann_load(
        d, lambda x, n, t: np.sum(vel(x) * n, 1))
    assert np.abs(lam - ref).max() <= 1e-12 * np.abs(ref).max()
