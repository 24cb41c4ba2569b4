"""Device workspaces from the caller's allocator (options.dev_alloc / dev_free), here torch's
caching allocator through the binding's TorchAllocator: the stage results are bit-identical
to those of a context that allocates with hipMalloc (same kernels on the same data), torch
accounts for the workspaces while the context lives, and every block comes back at
hdg_destroy."""
import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(s, a, f, lb):
    fd = torch.as_tensor(f, device="cuda")
    lbd = torch.as_tensor(lb, device="cuda")
    s.condense(a, fd, lbd)
    lam = torch.zeros_like(lbd)
    s.trace_solve(lam)
    u = torch.zeros_like(fd)
    s.recover(lam, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), lam.cpu().numpy()


@pytest.mark.parametrize("cfg,kw,prec", [(2, dict(n=2, k=3), "fp64"), (2, dict(n=2, k=3), "mixed_fp32"),
                                         (3, dict(n=1, k=2), "mixed_fp32")])
def test_torch_allocator_matches_hipmalloc(cfg, kw, prec):
    _need_gpu()
    from oracle import hdg as ohdg
    from paper_1807_00086_amd import Solver
    from paper_1807_00086_amd.hdg import TorchAllocator
    p = make_problem(cfg, **kw)
    print(f"case allocator {p.physics} {kw} {prec}", flush=True)
    d = ohdg.make_discretisation(p)
    f = random_vector(d.loc_off[-1], cfg, 91)
    lb = random_vector(d.tr_off[-1], cfg, 92) * ohdg.boundary_trace_mask(d)
    a = 1.0 / (0.43586652150845899 * p.dt)
    opts = dict(krylov_tol=1e-9, refine_tol=1e-12) if prec != "fp64" else {}
    ref = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=p.uniform_k, precision=prec, **opts)
    u0, l0 = _run(ref, a, f, lb)
    ref.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    al = TorchAllocator()
    s = Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=p.uniform_k, precision=prec, allocator=al, **opts)
    assert al.nbytes > 0 and len(al.blocks) > 10
    assert torch.cuda.memory_allocated() - before >= al.nbytes
    assert all(ptr % 256 == 0 for ptr in al.blocks)
    u1, l1 = _run(s, a, f, lb)
    assert np.array_equal(u0, u1) and np.array_equal(l0, l1)
    s.close()
    assert al.blocks == {}
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
