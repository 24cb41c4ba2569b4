"""GPU parity of the cached-factor path: hdg_condense_rhs (a new right-hand side condensed with
the factors of an earlier hdg_condense at the same stage coefficient) and hdg_step with
cache_factors, against the CPU FP64 oracle on the same seeded inputs.

Tolerances as for the fresh condensation: FP64 1e-12 per field (1e-11 element-wise r_e, z),
mixed FP32 + refinement 1e-10.
"""
import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GAMMA = 0.43586652150845899


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle():
    from oracle import hdg as ohdg
    return ohdg


def _solver(p, precision="fp64", **kw):
    from paper_1807_00086_amd import Solver
    uk = p.uniform_k
    return Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=uk, degree=None if uk else p.degree,
                  precision=precision, nrhs=1, **kw)


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _rel_errors(ohdg, d, u_gpu, u_ref):
    g = {"acoustic": [list(range(d.dim)), [d.dim]], "elastic": [list(range(6)), [6, 7, 8]],
         "maxwell": [[0, 1, 2], [3, 4, 5]], "maxwell_glm": [[0, 1, 2], [3, 4, 5], [6]]}[d.physics]
    return [ohdg.l2_norm_fields(d, u_gpu - u_ref, gi) / ohdg.l2_norm_fields(d, u_ref, gi) for gi in g]


CASES = [
    (1, dict()),                    # 2D, k = 2
    (2, dict(n=2, k=1)),
    (2, dict(n=2, k=2)),
    (2, dict(n=3, k=3)),            # workload degree, 162 tets
    (2, dict(n=2, k=4)),
    # block-structured kernels: the kept Schur factor, Z and K_e, the right-hand side condensed
    # by the refinement's pass at u = 0, lam = 0
    (3, dict(n=1, k=2)),            # elastic
    (3, dict(n=1, k=4)),
    (5, dict(n=2, k=2)),            # Maxwell
    ("glm", dict(n=2, k=2)),        # GLM-Maxwell
    (4, dict(nxyz=(2, 2, 1))),      # acoustics of variable degree, one right-hand side
]


def _problem(cfg, kw):
    if cfg == "glm":
        p = make_problem(5, **kw)
        p.physics = "maxwell_glm"
        return p, 5
    p = make_problem(cfg, **kw)
    p.nrhs = 1
    return p, cfg


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
@pytest.mark.parametrize("cfg,kw", CASES)
def test_condense_rhs_parity(cfg, kw, precision):
    """Factor with one right-hand side, condense a second one with the kept factors, solve and
    recover: the stage solution of the second right-hand side, as the oracle computes it."""
    _need_gpu()
    ohdg = _oracle()
    p, cfg = _problem(cfg, kw)
    print(f"case cached {precision} cfg={cfg} {p.physics} {kw} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (GAMMA * p.dt)
    bm = ohdg.boundary_trace_mask(d)
    f1, lb1 = random_vector(d.loc_off[-1], cfg, 31), random_vector(d.tr_off[-1], cfg, 32) * bm
    f2, lb2 = random_vector(d.loc_off[-1], cfg, 33), random_vector(d.tr_off[-1], cfg, 34) * bm
    u_ref, lam_ref, cond = ohdg.solve_stage(d, a, f2, lb2)
    mixed = precision == "mixed_fp32"
    kw_s = dict(krylov_tol=1e-9, refine_tol=1e-12) if mixed else {}
    s = _solver(p, precision, cache_factors=True, **kw_s)
    var = p.uniform_k is None     # variable degree: trace vectors padded to the degree-5 face space
    if var:
        from test_gpu_pvar import _pad, _unpad
        lb1, lb2 = _pad(d, lb1[:, None])[:, 0], _pad(d, lb2[:, None])[:, 0]
    s.condense(a, _dev(f1), _dev(lb1))
    f2d, lb2d = _dev(f2), _dev(lb2)
    s.condense_rhs(a, f2d, lb2d)
    lam = torch.zeros_like(lb2d)
    it, rr = s.trace_solve(lam)
    u = torch.zeros_like(f2d)
    s.recover(lam, u)
    torch.cuda.synchronize()
    u, lam = u.cpu().numpy(), lam.cpu().numpy()
    if var:
        lam = _unpad(d, lam[:, None])[0][:, 0]
    errs = _rel_errors(ohdg, d, u, u_ref)
    tol = 1e-10 if mixed else 1e-12
    assert max(errs) <= tol, errs
    assert np.linalg.norm(lam - lam_ref) <= tol * np.linalg.norm(lam_ref)
    if not mixed and p.physics == "acoustic" and p.uniform_k:
        # element-wise right-hand side quantities of the condensation
        t = cond.Ke[0].shape[0]
        ne = p.n_elem
        from oracle.polynomials import dim_p
        N = dim_p(int(d.degree[0]), d.dim)
        re = s.element_data("r", 0, ne, t).reshape(ne, t)
        z = s.element_data("z", 0, ne, N).reshape(ne, N)
        for e in range(0, ne, max(1, ne // 13)):
            assert np.abs(re[e] - cond.re[e][:, 0]).max() <= 1e-11 * np.abs(cond.re[e]).max()
            zr = cond.z[e][d.dim * N:, 0]
            assert np.abs(z[e] - zr).max() <= 1e-11 * np.abs(zr).max()
    s.close()


def test_dirk_step_cached_fp64():
    """Two DIRK(3,3) steps with cache_factors: the first stage factors, the other five only
    condense their right-hand sides; same result as the oracle's stage recursion."""
    _need_gpu()
    ohdg = _oracle()
    p = make_problem(2, n=2, k=2)
    d = ohdg.make_discretisation(p)
    u0 = random_vector(d.loc_off[-1], 2, 41)
    bm = ohdg.boundary_trace_mask(d)
    _, _, c = ohdg.dirk33()
    dt = 0.01
    lbs = {}
    for n in range(2):
        for i in range(3):
            lbs[round(n * dt + c[i] * dt, 12)] = random_vector(d.tr_off[-1], 2, 200 + 3 * n + i) * bm
    u_ref = u0.copy()
    for n in range(2):
        u_ref = ohdg.dirk_step(d, u_ref, n * dt, dt, lambda t: lbs[round(t, 12)])
    s = _solver(p, cache_factors=True)
    u = _dev(u0)
    lam = torch.zeros(d.tr_off[-1], dtype=torch.float64, device="cuda")
    for n in range(2):
        stages = np.stack([lbs[round(n * dt + c[i] * dt, 12)] for i in range(3)])
        s.step(n * dt, dt, "dirk33", u, lam, _dev(stages))
    torch.cuda.synchronize()
    errs = _rel_errors(ohdg, d, u.cpu().numpy(), u_ref)
    assert max(errs) <= 1e-12, errs
    s.close()


def test_condense_rhs_call_order_errors():
    """HDG_E_STATE (7) without kept factors at this stage coefficient, HDG_E_UNSUPPORTED (8)
    with 32 right-hand sides; both before any device work."""
    _need_gpu()
    from paper_1807_00086_amd import HDGError
    p = make_problem(2, n=1, k=2)
    s = _solver(p, cache_factors=True)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    f, lb = _dev(np.ones(nl)), _dev(np.zeros(nt))
    with pytest.raises(HDGError) as ei:
        s.condense_rhs(1.0, f, lb)          # nothing factored yet
    assert ei.value.code == 7
    s.condense(1.0, f, lb)
    with pytest.raises(HDGError) as ei:
        s.condense_rhs(2.0, f, lb)          # another stage coefficient
    assert ei.value.code == 7
    s.condense_rhs(1.0, f, lb)
    s.close()
    s = _solver(p)                           # FP64 without cache_factors keeps no factors
    s.condense(1.0, f, lb)
    with pytest.raises(HDGError) as ei:
        s.condense_rhs(1.0, f, lb)
    assert ei.value.code == 7
    s.close()
    from paper_1807_00086_amd import Solver   # 32 right-hand sides: no right-hand-side path
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=2, nrhs=32, cache_factors=True)
    nl, nt = s.query("n_local_dofs") * 32, s.query("n_trace_dofs") * 32
    f, lb = _dev(np.ones(nl)), _dev(np.zeros(nt))
    s.condense(1.0, f, lb)
    with pytest.raises(HDGError) as ei:
        s.condense_rhs(1.0, f, lb)
    assert ei.value.code == 8
    s.close()


@pytest.mark.parametrize("cfg,kw", [(3, dict(n=1, k=2)), ("glm", dict(n=2, k=1))])
@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_dirk_step_cached_block_structured(cfg, kw, precision):
    """Two DIRK(3,3) steps with cache_factors on the block-structured path (elastic and
    GLM-Maxwell): one factorisation per step size, five right-hand-side condensations; same
    result as the oracle's stage recursion."""
    _need_gpu()
    ohdg = _oracle()
    p, cfgi = _problem(cfg, kw)
    print(f"case cached dirk {precision} {p.physics} {kw} n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    u0 = random_vector(d.loc_off[-1], cfgi, 51)
    bm = ohdg.boundary_trace_mask(d)
    _, _, c = ohdg.dirk33()
    dt = 0.01
    lbs = {}
    for n in range(2):
        for i in range(3):
            lbs[round(n * dt + c[i] * dt, 12)] = random_vector(d.tr_off[-1], cfgi, 300 + 3 * n + i) * bm
    u_ref = u0.copy()
    for n in range(2):
        u_ref = ohdg.dirk_step(d, u_ref, n * dt, dt, lambda t: lbs[round(t, 12)])
    mixed = precision == "mixed_fp32"
    kw_s = dict(krylov_tol=1e-9, refine_tol=1e-12) if mixed else {}
    s = _solver(p, precision, cache_factors=True, **kw_s)
    u = _dev(u0)
    lam = torch.zeros(d.tr_off[-1], dtype=torch.float64, device="cuda")
    for n in range(2):
        stages = np.stack([lbs[round(n * dt + c[i] * dt, 12)] for i in range(3)])
        s.step(n * dt, dt, "dirk33", u, lam, _dev(stages))
    torch.cuda.synchronize()
    errs = _rel_errors(ohdg, d, u.cpu().numpy(), u_ref)
    assert max(errs) <= (1e-10 if mixed else 1e-12), errs
    s.close()
