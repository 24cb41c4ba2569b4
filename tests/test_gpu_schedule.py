"""Launch schedules of the block-structured condensation: the autotuner, its table file, and
the hipGraph that runs the degree classes of a variable-degree mesh as one launch.

A schedule only moves element buffers between LDS and per-workgroup global scratch (and the
reference tables between LDS and the caches) and sets how many wavefronts share an element's
tile work (four or eight), and the graph only changes how the class kernels are launched, so
every variant must give the default's result (relative 1e-13 here; in practice bitwise) and
stay within the oracle tolerances (FP64 1e-12, mixed FP32 + FP64 refinement 1e-10, relative L2
per field).
"""
import numpy as np
import pytest

from synth import make_problem, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BS = 21   # face space of degree 5: trace padding on meshes of variable degree


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(p, prec, **kw):
    from paper_1807_00086_amd import Solver
    uk = p.uniform_k
    return Solver(p.xyz, p.elem_vert, p.physics, p.elem_par, k=uk, degree=None if uk else p.degree,
                  precision=prec, nrhs=p.nrhs, **kw)


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


def _inputs(p, s, seed):
    """Seeded stage right-hand side and boundary data in the library's layouts."""
    nl, nt, R = s.query("n_local_dofs"), s.query("n_trace_dofs"), p.nrhs
    f = random_vector(nl * R, 90 + seed, 1).reshape(-1, R)
    return f, np.zeros((nt, R))


def _rel(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def _oracle_check(p, a, f, u, prec):
    """Stage solution of the oracle on the same inputs (homogeneous Dirichlet data)."""
    from oracle import hdg as ohdg
    d = ohdg.make_discretisation(p)
    assert d.loc_off[-1] * p.nrhs == f.size
    u_ref, _, _ = ohdg.solve_stage(d, a, f, np.zeros((d.tr_off[-1], p.nrhs)))
    tol = 1e-12 if prec == "fp64" else 1e-10
    assert _rel(u, u_ref) <= tol, _rel(u, u_ref)


TUNE_CASES = [
    (3, dict(n=1, k=4), "fp64"),         # elastic k = 4: Schur block in LDS (one group per CU) or not
    (3, dict(n=1, k=4), "mixed_fp32"),
    (5, dict(n=2, k=3), "fp64"),         # Maxwell k = 3
    (4, dict(nxyz=(2, 2, 2)), "fp64"),   # variable degree, 32 right-hand sides
    (4, dict(nxyz=(2, 2, 2)), "mixed_fp32"),
]


@pytest.mark.parametrize("cfg,kw,prec", TUNE_CASES)
def test_autotuned_schedules_match_default(cfg, kw, prec, tmp_path):
    _need_gpu()
    p = make_problem(cfg, **kw)
    print(f"case autotune cfg={cfg} {kw} {prec} n_elem={p.n_elem}", flush=True)
    a = 1.0 / p.dt
    opts = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    table = tmp_path / "tune.txt"
    s0 = _solver(p, prec, **opts)
    f, lb = _inputs(p, s0, cfg)
    u0, lam0 = _stage(s0, a, f, lb)
    sch0 = s0.schedules()
    s0.close()
    assert sch0 and set(sch0.values()) == {0}

    s1 = _solver(p, prec, autotune=True, autotune_table=str(table), **opts)
    u1, lam1 = _stage(s1, a, f, lb)
    sch1 = s1.schedules()
    u1b, _ = _stage(s1, a, f, lb)          # second stage: the tuned schedules, no timing
    s1.close()
    assert set(sch1) == set(sch0)
    assert all(v in (0, 1, 2, 3, 4) for v in sch1.values())
    assert _rel(u1, u0) <= 1e-13 and _rel(lam1, lam0) <= 1e-13
    assert _rel(u1b, u0) <= 1e-13
    if p.uniform_k:
        _oracle_check(p, a, f, u1, prec)
    if cfg == 3 and prec == "fp64":
        assert table.exists() and any(not ln.startswith("#") for ln in table.read_text().splitlines())

    # a new context reads the table instead of timing again
    if table.exists():
        s2 = _solver(p, prec, autotune_table=str(table), **opts)
        u2, _ = _stage(s2, a, f, lb)
        assert s2.schedules() == sch1
        s2.close()
        assert _rel(u2, u0) <= 1e-13


@pytest.mark.parametrize("prec,autotune", [("fp64", False), ("mixed_fp32", False), ("fp64", True)])
def test_graph_replays_match_eager(prec, autotune):
    """Capture, replay, re-capture for a new right-hand side, replay again; an eager context
    runs the same stages in between, and every replay is compared with it."""
    _need_gpu()
    p = make_problem(4, nxyz=(2, 2, 2))
    print(f"case graph {prec} autotune={autotune} n_elem={p.n_elem} degrees={np.bincount(p.degree)}", flush=True)
    assert len(set(p.degree.tolist())) > 2
    a = 1.0 / p.dt
    opts = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    se = _solver(p, prec, **opts)
    sg = _solver(p, prec, use_graph=True, autotune=autotune, **opts)
    f1, lb = _inputs(p, se, 1)
    f2, _ = _inputs(p, se, 2)
    fd1 = torch.as_tensor(f1, device="cuda")
    fd2 = torch.as_tensor(f2, device="cuda")
    lbd = torch.as_tensor(lb, device="cuda")
    for rnd, fd in enumerate([fd1, fd1, fd2, fd2, fd1]):
        res = []
        for s in (se, sg):
            s.condense(a, fd, lbd)
            lam = torch.zeros_like(lbd)
            s.trace_solve(lam)
            u = torch.zeros_like(fd)
            s.recover(lam, u)
            torch.cuda.synchronize()
            res.append((u.cpu().numpy(), lam.cpu().numpy()))
        (ue, le), (ug, lg) = res
        assert _rel(ug, ue) <= 1e-13, (rnd, _rel(ug, ue))
        assert _rel(lg, le) <= 1e-13, (rnd, _rel(lg, le))
    se.close()
    sg.close()


def test_tune_table_entries_validated(tmp_path):
    """The table parser skips comments, malformed lines and other devices, and a schedule that is
    not built for a class (Maxwell k = 3 FP32 fits the 75 KB rule whole, so schedule 1 does not
    exist for it) falls back to the default; a built one (schedule 2) is taken as read."""
    _need_gpu()
    dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    p = make_problem(5, n=2, k=3)
    print(f"case tune table device={dev} n_elem={p.n_elem}", flush=True)
    a = 1.0 / p.dt
    opts = dict(krylov_tol=1e-9, refine_tol=1e-12)
    s0 = _solver(p, "mixed_fp32", **opts)
    f, lb = _inputs(p, s0, 5)
    u0, _ = _stage(s0, a, f, lb)
    s0.close()
    for sched, expect in ((1, 0), (2, 2)):
        table = tmp_path / f"tune{sched}.txt"
        table.write_text("# comment line\n"
                         "not a table line\n"
                         f"otherdevice 2 3 3 1 1 2 0 0 0\n"
                         f"{dev} 2 3 3 1 1 {sched} 1.0 1.0 1.0\n")
        s1 = _solver(p, "mixed_fp32", autotune_table=str(table), **opts)
        u1, _ = _stage(s1, a, f, lb)
        assert s1.schedules() == {3: expect}, (sched, s1.schedules())
        s1.close()
        assert _rel(u1, u0) <= 1e-13


def test_tune_table_unwritable_path_is_harmless(tmp_path):
    """A table path that cannot be read or written (a missing directory) leaves tuning and the
    results unaffected: the library times the schedules and simply keeps no file."""
    _need_gpu()
    p = make_problem(3, n=1, k=4)
    print(f"case tune table unwritable n_elem={p.n_elem}", flush=True)
    a = 1.0 / p.dt
    path = tmp_path / "missing_dir" / "tune.txt"
    s0 = _solver(p, "fp64", krylov_tol=1e-13)
    f, lb = _inputs(p, s0, 3)
    u0, _ = _stage(s0, a, f, lb)
    s0.close()
    s1 = _solver(p, "fp64", krylov_tol=1e-13, autotune=True, autotune_table=str(path))
    u1, _ = _stage(s1, a, f, lb)
    assert set(s1.schedules()) == {4}
    s1.close()
    assert not path.exists()
    assert _rel(u1, u0) <= 1e-13


WAVE8_CASES = [
    (3, dict(n=1, k=4), "fp64"),         # elastic k = 4: blocked factorisation of the 105-unknown Schur block
    (3, dict(n=1, k=2), "mixed_fp32"),   # elastic k = 2: register Cholesky beside the B~2 wavefronts
    (3, dict(n=1, k=4), "mixed_bf16"),
    (5, dict(n=2, k=3), "fp64"),         # Maxwell
    (5, dict(n=1, k=3), "maxwell_glm/fp64"),
    (4, dict(nxyz=(2, 2, 2)), "fp64"),   # variable degree, 32 right-hand sides: every class
]


@pytest.mark.parametrize("sched", [3, 4])
@pytest.mark.parametrize("cfg,kw,prec", WAVE8_CASES)
def test_eight_wavefront_schedule_matches_default(cfg, kw, prec, sched, tmp_path):
    """Schedules 3 and 4 (eight wavefronts per element workgroup, a whole CU's LDS; reference
    tables in LDS or through the caches) read from a tune table for every class: the same result
    as the default schedule (relative 1e-13) and the oracle's tolerance on uniform meshes."""
    _need_gpu()
    from paper_1807_00086_amd.hdg import PHYSICS, PRECISION
    phys = None
    if "/" in prec:
        phys, prec = prec.split("/")
    p = make_problem(cfg, **kw)
    if phys:
        p.physics = phys
    dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    print(f"case schedule {sched} cfg={cfg} {kw} {p.physics} {prec} n_elem={p.n_elem}", flush=True)
    a = 1.0 / p.dt
    opts = dict(krylov_tol=1e-13) if prec == "fp64" else dict(krylov_tol=1e-9, refine_tol=1e-12)
    s0 = _solver(p, prec, **opts)
    f, lb = _inputs(p, s0, cfg + 7)
    u0, lam0 = _stage(s0, a, f, lb)
    classes = sorted(s0.schedules())
    s0.close()
    kf = 5 if p.uniform_k is None else p.uniform_k
    table = tmp_path / "tune8.txt"
    table.write_text("".join(f"{dev} {PHYSICS[p.physics]} {k} {kf} {p.nrhs} {PRECISION[prec]} {sched} 1 1 1 1 1\n"
                             for k in classes))
    s3 = _solver(p, prec, autotune_table=str(table), **opts)
    u3, lam3 = _stage(s3, a, f, lb)
    assert s3.schedules() == {k: sched for k in classes}, s3.schedules()
    u3b, _ = _stage(s3, a, f, lb)
    s3.close()
    assert _rel(u3, u0) <= 1e-13 and _rel(lam3, lam0) <= 1e-13, (_rel(u3, u0), _rel(lam3, lam0))
    assert _rel(u3b, u0) <= 1e-13
    if p.uniform_k:
        _oracle_check(p, a, f, u3, prec)
