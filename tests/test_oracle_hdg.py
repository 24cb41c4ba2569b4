"""Pins of the oracle's HDG discretisation against what the paper and the mathematics fix:

* brute force: the condensed solve equals the solve of the whole uncondensed system
  (section 2.4.1: the elimination of the local unknowns is exact);
* structure: element Schur complements are symmetric and the assembled trace operator is
  definite (sign per physics);
* manufactured single-stage problems converge at O(h^{k+1}) in every field (the optimal
  rates reported in sections 4.3 and 5.4);
* exact plane waves stay exact up to O(h^{k+1}) + O(dt^3) under DIRK(3,3);
* energy is non-increasing with homogeneous data (energy identities of sections 4.2.3 and
  5.3 and their acoustic analogue);
* DIRK(3,3) order conditions and the stiffly-accurate update weights (section 2.3.2);
* face / trace-unknown counts (table eppMeshes).
"""
import os

import numpy as np
import pytest

from synth import make_problem
from oracle import hdg
from oracle.polynomials import dim_p

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_stage(p, seed=0, a=37.0):
    d = hdg.make_discretisation(p)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(d.loc_off[-1])
    lb = rng.standard_normal(d.tr_off[-1]) * hdg.boundary_trace_mask(d)
    return d, a, f, lb


@pytest.mark.parametrize("cfg,kw", [
    (1, dict(n=3)), (1, dict(n=2, k=4)), (2, dict(n=2, k=1)), (2, dict(n=1, k=3)),
    (3, dict(n=1, k=1)), (5, dict(n=1, k=2)), (4, dict(nxyz=(2, 1, 1))),
])
def test_condensed_equals_full_system(cfg, kw):
    d, a, f, lb = _rand_stage(make_problem(cfg, **kw))
    u, lam, cond = hdg.solve_stage(d, a, f, lb)
    uf, lf = hdg.solve_full(d, a, f, lb)
    assert np.linalg.norm(u - uf) <= 1e-12 * np.linalg.norm(uf)
    assert np.linalg.norm(lam - lf) <= 1e-12 * np.linalg.norm(lf)


@pytest.mark.parametrize("cfg,kw,sign", [
    (2, dict(n=2, k=2), -1.0), (3, dict(n=1, k=2), 1.0), (5, dict(n=2, k=1), 1.0),
    (1, dict(n=3, k=3), -1.0),
])
def test_schur_symmetric_and_definite(cfg, kw, sign):
    d, a, f, lb = _rand_stage(make_problem(cfg, **kw))
    cond = hdg.condense(d, a, f)
    for Ke in cond.Ke[:5]:
        assert np.abs(Ke - Ke.T).max() <= 1e-12 * np.abs(Ke).max()
        assert np.all(sign * np.linalg.eigvalsh(Ke) > 0)
    bm = hdg.boundary_trace_mask(d)
    K = cond.K.toarray()[~bm][:, ~bm]
    assert np.all(sign * np.linalg.eigvalsh(0.5 * (K + K.T)) > 0)


def test_local_block_lu_without_pivoting_exists():
    """Every leading principal minor of A_K is nonzero (LU without pivoting exists)."""
    for cfg, kw in [(2, dict(n=1, k=2)), (3, dict(n=1, k=1)), (5, dict(n=1, k=2))]:
        d, a, f, lb = _rand_stage(make_problem(cfg, **kw))
        A = hdg.element_system(d, 0, a)[0]
        # Gaussian elimination without pivoting: all pivots must be nonzero
        U = A.copy()
        n = U.shape[0]
        piv = []
        for j in range(n):
            piv.append(U[j, j])
            U[j + 1:, j:] -= np.outer(U[j + 1:, j] / U[j, j], U[j, j:])
        assert min(abs(np.asarray(piv))) > 1e-8 * max(abs(np.asarray(piv)))


# ----------------------------------------------------------------------------- manufactured
def _grad_fd(func, x, h=1e-3):
    """Fourth-order central differences of func(x) -> [q, m]; returns [q, m, d]."""
    out = []
    for r in range(x.shape[1]):
        e = np.zeros(x.shape[1])
        e[r] = h
        out.append((-func(x + 2 * e) + 8 * func(x + e) - 8 * func(x - e) + func(x - 2 * e)) / (12 * h))
    return np.stack(out, axis=-1)


def _acoustic_exact(dim):
    def fields(x):
        s = x @ np.array([1.0, 2.0, 3.0][:dim])
        p = np.sin(s)
        if dim == 2:
            v = np.stack([np.cos(2 * x[:, 0] - x[:, 1]), np.sin(x[:, 0] + 0.5 * x[:, 1])], 1)
        else:
            v = np.stack([np.cos(2 * x[:, 0] - x[:, 1]), np.sin(x[:, 0] + x[:, 2]),
                          np.cos(x[:, 1] - x[:, 2])], 1)
        return np.concatenate([v, p[:, None]], 1)
    return fields


def _manufactured(physics, dim, par, a):
    rho, c = (par[0], par[1]) if physics == "acoustic" else (None, None)
    if physics == "acoustic":
        U = _acoustic_exact(dim)

        def src(x, t=0.0):
            u = U(x)
            g = _grad_fd(U, x)
            sv = a * rho * u[:, :dim] + g[:, dim, :]
            sp = a / (rho * c * c) * u[:, dim] + sum(g[:, i, i] for i in range(dim))
            return np.concatenate([sv, sp[:, None]], 1)
        return U, src
    if physics == "maxwell":
        eps, mu, sig = par

        def U(x):
            H = np.stack([np.sin(x[:, 1] + x[:, 2]), np.cos(x[:, 0] - x[:, 2]), np.sin(2 * x[:, 0] + x[:, 1])], 1)
            E = np.stack([np.cos(x[:, 1] - 2 * x[:, 2]), np.sin(x[:, 0] + x[:, 2]), np.cos(x[:, 0] + x[:, 1])], 1)
            return np.concatenate([H, E], 1)

        def curl(g, off):
            return np.stack([g[:, off + 2, 1] - g[:, off + 1, 2], g[:, off + 0, 2] - g[:, off + 2, 0],
                             g[:, off + 1, 0] - g[:, off + 0, 1]], 1)

        def src(x, t=0.0):
            u = U(x)
            g = _grad_fd(U, x)
            sH = a * mu * u[:, :3] + curl(g, 3)
            sE = (a * eps + sig) * u[:, 3:] - curl(g, 0)
            return np.concatenate([sH, sE], 1)
        return U, src
    if physics == "elastic":
        rho, lam, mu = par
        pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]

        def U(x):
            s = np.stack([np.sin(x[:, 0] + x[:, 1]), np.cos(x[:, 1] - x[:, 2]), np.sin(x[:, 2] + 2 * x[:, 0]),
                          np.cos(x[:, 0] + x[:, 2]), np.sin(x[:, 1] - x[:, 0]), np.cos(2 * x[:, 1] + x[:, 2])], 1)
            v = np.stack([np.cos(2 * x[:, 0] - x[:, 1]), np.sin(x[:, 0] + x[:, 2]), np.cos(x[:, 1] - x[:, 2])], 1)
            return np.concatenate([s, v], 1)

        def src(x, t=0.0):
            u = U(x)
            g = _grad_fd(U, x)
            sig = np.zeros((x.shape[0], 3, 3))
            for al, (i, j) in enumerate(pairs):
                sig[:, i, j] = sig[:, j, i] = u[:, al]
            tr = np.trace(sig, axis1=1, axis2=2)
            comp = (sig - (lam / (3 * lam + 2 * mu)) * tr[:, None, None] * np.eye(3)) / (2 * mu)
            gv = g[:, 6:9, :]
            symg = 0.5 * (gv + np.transpose(gv, (0, 2, 1)))
            ss = a * comp - symg
            s6 = np.stack([ss[:, i, j] for (i, j) in pairs], 1)
            divs = np.zeros((x.shape[0], 3))
            for al, (i, j) in enumerate(pairs):
                divs[:, i] += g[:, al, j]
                if i != j:
                    divs[:, j] += g[:, al, i]
            sv = a * rho * u[:, 6:9] - divs
            return np.concatenate([s6, sv], 1)
        return U, src
    raise ValueError(physics)


def _manufactured_errors(cfg, ns, k, a=5.0, comps_groups=None):
    errs = []
    for n in ns:
        p = make_problem(cfg, n=n, k=k)
        # homogeneous material so that the manufactured source is element-independent
        p.elem_par[:] = {"acoustic": [1.3, 0.8], "maxwell": [1.2, 0.9, 0.05],
                         "elastic": [1.1, 1.7, 0.9]}[p.physics]
        d = hdg.make_discretisation(p)
        U, src = _manufactured(p.physics, p.dim, p.elem_par[0], a)
        f = hdg.load_vector(d, src)
        lb = hdg.project_boundary(d, lambda x, t: U(x)[:, {"acoustic": [p.dim], "maxwell": [3, 4, 5],
                                                            "elastic": [6, 7, 8]}[p.physics]]
                                  if p.physics != "acoustic" else U(x)[:, p.dim])
        u, lam, _ = hdg.solve_stage(d, a, f, lb)
        errs.append([hdg.l2_error_fields(d, u, lambda x, t: U(x), 0.0, g) for g in comps_groups])
    errs = np.asarray(errs)
    rates = np.log(errs[:-1] / errs[1:]) / np.log(np.asarray(ns[1:]) / np.asarray(ns[:-1]))[:, None]
    return errs, rates


@pytest.mark.parametrize("k", [1, 2])
def test_manufactured_acoustic2d_rates(k):
    errs, rates = _manufactured_errors(1, [4, 8], k, comps_groups=[[0, 1], [2]])
    assert np.all(rates > k + 1 - 0.3), (errs, rates)


# On the coarse jittered 3D meshes affordable here the flux-like fields are still
# pre-asymptotic (measured 1.5 -> 1.7 -> 1.9 for k=1 on n = 2, 3, 4, 6), so the 3D bars are
# looser than k+1; a dropped term or a wrong sign gives rates of 1 or below.
def test_manufactured_acoustic3d_rates():
    errs, rates = _manufactured_errors(2, [2, 4], 2, comps_groups=[[0, 1, 2], [3]])
    assert np.all(rates > 2.3), (errs, rates)
    assert rates[0, 1] > 2.6, (errs, rates)


def test_manufactured_maxwell_rates():
    errs, rates = _manufactured_errors(5, [2, 4], 1, comps_groups=[[0, 1, 2], [3, 4, 5]])
    assert np.all(rates > 1.5), (errs, rates)


def test_manufactured_elastic_rates():
    errs, rates = _manufactured_errors(3, [2, 4], 1, comps_groups=[list(range(6)), [6, 7, 8]])
    assert np.all(rates > 1.5), (errs, rates)


# ----------------------------------------------------------------------------- time stepping
def test_dirk33_order_conditions_and_gamma():
    A, b, c = hdg.dirk33()
    g = float(open(os.path.join(GOLDEN, "dirk33_alexander.txt")).read().split("gamma")[-1].split()[0])
    assert abs(A[0, 0] - g) < 1e-15
    assert abs(b.sum() - 1) < 1e-14
    assert abs(b @ c - 0.5) < 1e-14
    assert abs(b @ c ** 2 - 1 / 3) < 1e-14
    assert abs(b @ A @ c - 1 / 6) < 1e-14
    Dm = np.linalg.inv(A)
    e = b @ Dm
    np.testing.assert_allclose(e, [0, 0, 1], atol=1e-13)
    assert abs(1 - np.sum(b @ Dm)) < 1e-13
    # L-stability: R(z) = 1 + z b (I - zA)^{-1} 1 -> 0 as z -> -inf
    z = -1e8
    R = 1 + z * b @ np.linalg.solve(np.eye(3) - z * A, np.ones(3))
    assert abs(R) < 1e-6


def _plane_wave_2d(x, t):
    p = np.sin(2 * np.pi * (x[:, 0] - t))
    return np.stack([p, np.zeros_like(p), p], 1)


def test_plane_wave_2d_dirk_temporal_order():
    """Same mesh, shrinking dt: the discrete solution converges at third order in time to
    the fine-dt discrete solution (DIRK(3,3))."""
    p = make_problem(1, n=3, k=2)
    d = hdg.make_discretisation(p)
    u0 = hdg.project_volume(d, _plane_wave_2d, 0.0)

    def bnd(t):
        return hdg.project_boundary(d, lambda x, tt: _plane_wave_2d(x, tt)[:, 2], t)

    T = 0.12

    def run(nsteps):
        u = u0.copy()
        dt = T / nsteps
        for s in range(nsteps):
            u = hdg.dirk_step(d, u, s * dt, dt, bnd)
        return u

    ref = run(48)
    e = [np.linalg.norm(run(n) - ref) for n in (3, 6)]
    rate = np.log2(e[0] / e[1])
    assert rate > 2.6, (e, rate)


def test_plane_wave_acoustic2d_workload_error():
    """The 2D acoustic workload (one backward-Euler step, dt = 0.01, from the exact plane
    wave): the error stays at the size of one step's local truncation error."""
    p = make_problem(1)
    d = hdg.make_discretisation(p)
    u0 = hdg.project_volume(d, _plane_wave_2d, 0.0)
    bnd = lambda t: hdg.project_boundary(d, lambda x, tt: _plane_wave_2d(x, tt)[:, 2], t)
    u1 = hdg.dirk_step(d, u0, 0.0, 0.01, bnd, scheme="be")
    err = hdg.l2_error_fields(d, u1, _plane_wave_2d, 0.01, [0, 1, 2])
    ref = hdg.l2_norm_fields(d, u1, [0, 1, 2])
    assert err / ref < 3e-2


@pytest.mark.parametrize("cfg,kw", [(1, dict(n=3, k=2)), (2, dict(n=1, k=2)), (3, dict(n=1, k=1)),
                                    (5, dict(n=1, k=2))])
def test_energy_non_increasing(cfg, kw):
    p = make_problem(cfg, **kw)
    d = hdg.make_discretisation(p)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(d.loc_off[-1])
    zero = np.zeros(d.tr_off[-1])
    E0 = hdg.energy(d, u)
    for s in range(3):
        u = hdg.dirk_step(d, u, s * 0.05, 0.05, lambda t: zero)
        E1 = hdg.energy(d, u)
        assert E1 <= E0 * (1 + 1e-13)
        E0 = E1


# ----------------------------------------------------------------------------- counting
def test_face_counts_match_closed_forms():
    for n in (1, 2, 3):
        p = make_problem(2, n=n, k=1)
        d = hdg.make_discretisation(p)
        assert d.skel.n_faces == 12 * n ** 3 + 6 * n ** 2
        assert int(d.skel.is_boundary.sum()) == 12 * n ** 2
    p = make_problem(4, nxyz=(2, 3, 2), k=1)
    d = hdg.make_discretisation(p)
    nx, ny, nz = 2, 3, 2
    V = nx * ny * nz
    box_faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    assert d.skel.n_faces == 4 * V + 2 * box_faces
    assert np.all(d.skel.face_elems[:, 0] >= 0)


def test_eppler_table_trace_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "eppler_meshes.txt")) if not l.startswith("#")]
    for mesh, k, ne, nglob, m in rows:
        nf = dim_p(int(k), 2)
        assert int(nglob) % nf == 0
        faces = int(nglob) // nf
        # each tetrahedron has 4 faces, interior faces are shared: 2 N_e < faces < 4 N_e
        assert 2 * int(ne) < faces < 4 * int(ne)
