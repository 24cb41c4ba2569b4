"""Independence of the right-hand-side columns in the 32-column path.

The trace CG keeps its scalars (r.z, p.q, the residual norm) per column, and several of its
reductions are fused into other kernels; a mix-up between columns, or a zero denominator not
guarded, would show here.  Column j of the 32-column stage is the one-column stage scaled by
s_j, with s_0 = 0 (an all-zero column must come back exactly zero) and s_1..s_31 spanning
sixteen orders of magnitude.  Tolerances: relative 1e-10 per column against the one-column
solve (both paths converge each column to its own relative tolerance).

The mixed-precision refinement stops on the FP64 residual of every column separately: columns of
independent content whose sizes span sixteen decades must each reach the oracle's solution to
1e-10 and report a residual at or below refine_tol.
"""
import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _stage(s, a, f, lb):
    fd = torch.as_tensor(np.ascontiguousarray(f), device="cuda")
    lbd = torch.as_tensor(np.ascontiguousarray(lb), device="cuda")
    s.condense(a, fd, lbd)
    lam = torch.zeros_like(lbd)
    s.trace_solve(lam)
    u = torch.zeros_like(fd)
    s.recover(lam, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), lam.cpu().numpy()


def _rel(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_32_columns_scaled_and_zero(prec):
    _need_gpu()
    from paper_1807_00086_amd import Solver
    p = make_problem(2, n=2, k=2)
    print(f"case columns {prec} n_elem={p.n_elem}", flush=True)
    a = 1.0 / (0.43586652150845899 * p.dt)
    kw = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    s1 = Solver(p.xyz, p.elem_vert, "acoustic", p.elem_par, k=2, precision=prec, nrhs=1, **kw)
    nl, nt = s1.query("n_local_dofs"), s1.query("n_trace_dofs")
    f = random_vector(nl, 2, 41)
    u1, lam1 = _stage(s1, a, f[:, None], np.zeros((nt, 1)))
    s1.close()
    scale = np.concatenate([[0.0], 10.0 ** np.linspace(-8, 8, 31)])
    s32 = Solver(p.xyz, p.elem_vert, "acoustic", p.elem_par, k=2, precision=prec, nrhs=32, **kw)
    u32, lam32 = _stage(s32, a, f[:, None] * scale[None, :], np.zeros((nt, 32)))
    s32.close()
    assert np.all(u32[:, 0] == 0.0) and np.all(lam32[:, 0] == 0.0)
    tol = 1e-10
    for j in range(1, 32):
        assert _rel(u32[:, j] / scale[j], u1[:, 0]) <= tol, (j, _rel(u32[:, j] / scale[j], u1[:, 0]))
        assert _rel(lam32[:, j] / scale[j], lam1[:, 0]) <= tol, j


def test_32_columns_mixed_independent_content_per_column_residual():
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    p = make_problem(2, n=2, k=2)
    print(f"case columns mixed independent n_elem={p.n_elem}", flush=True)
    d = ohdg.make_discretisation(p)
    a = 1.0 / (0.43586652150845899 * p.dt)
    nl, nt = d.loc_off[-1], d.tr_off[-1]
    scale = 10.0 ** np.linspace(-8, 8, 32)
    F = random_vector(nl * 32, 2, 43).reshape(nl, 32) * scale[None, :]
    LB = random_vector(nt * 32, 2, 44).reshape(nt, 32) * scale[None, :] * ohdg.boundary_trace_mask(d)[:, None]
    u_ref, lam_ref, _ = ohdg.solve_stage(d, a, F, LB)
    tol_res = 1e-12
    s = Solver(p.xyz, p.elem_vert, "acoustic", p.elem_par, k=2, precision="mixed_fp32", nrhs=32,
               krylov_tol=1e-9, refine_tol=tol_res)
    u, lam = _stage(s, a, F, LB)
    res = s.last_residual()
    s.close()
    assert res.shape == (32,) and np.all(res <= tol_res), res
    for j in range(32):
        assert _rel(u[:, j], u_ref[:, j]) <= 1e-10, (j, _rel(u[:, j], u_ref[:, j]))
        assert _rel(lam[:, j], lam_ref[:, j]) <= 1e-10, j
