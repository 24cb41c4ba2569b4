"""The trace solve that allocates nothing (hdg_trace_solve_static) against hdg_trace_solve.

Both run the same conjugate-gradient kernels in the same order; the static variant only keeps its
work vectors and partial sums in the library's file-scope device array.  Two calls in a row on
contexts of decreasing size (the second reuses the array the first left behind), FP64 and mixed
precision (FP32 matrix copy in the products): iteration counts equal and the solutions equal to
the last bit.  A system larger than the array is refused with HDG_E_ARG before any device work.
"""
import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _condensed(p, prec, seed, precond="jacobi"):
    from paper_1807_00086_amd import Solver
    kw = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=int(p.degree[0]), precision=prec, precond=precond,
               **kw)
    nl, nt = s.query("n_local_dofs"), s.query("n_trace_dofs")
    fd = torch.as_tensor(random_vector(nl, p.cfg_id, seed), device="cuda")
    lbd = torch.as_tensor(random_vector(nt, p.cfg_id, seed + 1), device="cuda")
    s.condense(1.0 / (0.43586652150845899 * p.dt), fd, lbd)
    return s, fd, lbd


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_trace_solve_static_equals_trace_solve_two_calls(prec):
    _need_gpu()
    for case, (cfg, kw) in enumerate([(2, dict(n=6, k=3)), (2, dict(n=2, k=2))]):   # second smaller
        p = make_problem(cfg, **kw)
        print(f"case no-alloc {prec} call {case + 1} n_elem={p.n_elem}", flush=True)
        s, fd, lbd = _condensed(p, prec, 60 + case)
        lam_ref = torch.zeros_like(lbd)
        it_ref, rr_ref = s.trace_solve(lam_ref)
        lam = torch.zeros_like(lbd)
        it, rr = s.trace_solve_static(lam)
        torch.cuda.synchronize()
        assert it == it_ref and rr == rr_ref, (it, it_ref, rr, rr_ref)
        assert torch.equal(lam, lam_ref)
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_trace_solve_static_in_an_ssor_context(prec):
    """A context configured for block SSOR skips the block-Jacobi inverses (and the FP32 copy of
    K) at condensation; the static solve, which runs block Jacobi, forms them itself and equals a
    block-Jacobi context's hdg_trace_solve on the same system to the last bit."""
    _need_gpu()
    p = make_problem(2, n=3, k=3)
    print(f"case no-alloc in an ssor context {prec} n_elem={p.n_elem}", flush=True)
    sj, _, lbd = _condensed(p, prec, 70)
    lam_ref = torch.zeros_like(lbd)
    it_ref, rr_ref = sj.trace_solve(lam_ref)
    ss, _, _ = _condensed(p, prec, 70, precond="ssor")
    assert ss.query("n_colors") > 0
    lam = torch.zeros_like(lbd)
    it, rr = ss.trace_solve_static(lam)
    torch.cuda.synchronize()
    assert it == it_ref and rr == rr_ref, (it, it_ref, rr, rr_ref)
    assert torch.equal(lam, lam_ref)
    sj.close()
    ss.close()


def test_trace_solve_static_rejects_a_system_beyond_its_scratch():
    _need_gpu()
    from paper_1807_00086_amd import HDGError, Solver
    p = make_problem(2, n=12, k=3)   # 21,600 faces x 10 modes x 32 columns: 4 vectors = 221 MB
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=3, nrhs=32)
    lam = torch.zeros(s.query("n_trace_dofs") * 32, dtype=torch.float64, device="cuda")
    with pytest.raises(HDGError) as ei:
        s.trace_solve_static(lam)
    assert ei.value.code == 1 and "static" in str(ei.value)
    s.close()
