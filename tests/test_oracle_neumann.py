"""Pins of the oracle's Neumann boundary faces (section 4.1.2: the trace equation's Gamma_N
part <flux_hat - g_N, mu>_F = 0, for acoustics the prescribed normal velocity, for elasticity
the traction, for Maxwell n x H).

Polynomial reproduction: when the exact solution of a stage problem lies in the discrete
spaces (fields of degree <= k, their traces in the face spaces), the HDG stage solution is its
L2 projection, because the exact fields satisfy every discrete equation (the stabilisation
terms vanish since u - u_hat = 0 on every face) and the discrete problem has one solution.  The
data are computed from the fields alone: the source from the strong form of each equation, the
Dirichlet values by L2 projection, the Neumann data as the flux of the exact fields tested on
the face.  A wrong sign of the Neumann datum, a dropped datum, a Neumann face handled as a
Dirichlet one, or a wrong normal fails the 1e-9 bound by orders of magnitude (the planted
variants below show it).
"""
import itertools

import numpy as np
import pytest

from oracle import hdg
from synth import make_problem, tag_box_faces

A_STAGE = 3.0


class Poly:
    """Random polynomial of total degree <= k in dim variables, with its exact gradient."""

    def __init__(self, dim, k, rng):
        self.exps = [e for e in itertools.product(range(k + 1), repeat=dim) if sum(e) <= k]
        self.c = rng.standard_normal(len(self.exps))

    def __call__(self, x):
        out = np.zeros(x.shape[0])
        for c, e in zip(self.c, self.exps):
            out += c * np.prod(x ** np.asarray(e), axis=1)
        return out

    def grad(self, x):
        g = np.zeros(x.shape)
        for c, e in zip(self.c, self.exps):
            for r in range(x.shape[1]):
                if e[r] == 0:
                    continue
                ee = np.asarray(e)
                ee[r] -= 1
                g[:, r] += c * e[r] * np.prod(x ** ee, axis=1)
        return g


def _fields(physics, k, par, rng):
    """(U(x) -> [q, m], source(x) -> [q, m], dirichlet(x) -> values, flux(x, n) -> values)."""
    if physics == "acoustic":
        rho, c = par[0], par[1]
        P = [Poly(3, k, rng) for _ in range(4)]          # v1, v2, v3, p

        def U(x):
            return np.stack([q(x) for q in P], 1)

        def src(x, t=0.0):
            gp = P[3].grad(x)
            div = sum(P[i].grad(x)[:, i] for i in range(3))
            sv = A_STAGE * rho * U(x)[:, :3] + gp
            sp = A_STAGE / (rho * c * c) * P[3](x) + div
            return np.concatenate([sv, sp[:, None]], 1)
        return U, src, (lambda x, t: P[3](x)), (lambda x, n, t: np.sum(U(x)[:, :3] * n, axis=1))
    if physics == "elastic":
        rho, lam, mu = par
        pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
        P = [Poly(3, k, rng) for _ in range(9)]          # sigma (Voigt order above), v

        def U(x):
            return np.stack([q(x) for q in P], 1)

        def sig(x):
            u = U(x)
            s = np.zeros((x.shape[0], 3, 3))
            for al, (i, j) in enumerate(pairs):
                s[:, i, j] = s[:, j, i] = u[:, al]
            return s

        def src(x, t=0.0):
            s = sig(x)
            tr = np.trace(s, axis1=1, axis2=2)
            comp = (s - (lam / (3 * lam + 2 * mu)) * tr[:, None, None] * np.eye(3)) / (2 * mu)
            gv = np.stack([P[6 + i].grad(x) for i in range(3)], 1)    # [q, i, j] = d v_i / d x_j
            symg = 0.5 * (gv + np.transpose(gv, (0, 2, 1)))
            ss = A_STAGE * comp - symg
            divs = np.zeros((x.shape[0], 3))
            for al, (i, j) in enumerate(pairs):
                g = P[al].grad(x)
                divs[:, i] += g[:, j]
                if i != j:
                    divs[:, j] += g[:, i]
            sv = A_STAGE * rho * U(x)[:, 6:9] - divs
            return np.concatenate([np.stack([ss[:, i, j] for (i, j) in pairs], 1), sv], 1)
        return U, src, (lambda x, t: U(x)[:, 6:9]), (lambda x, n, t: np.einsum("qij,qj->qi", sig(x), n))
    eps, mu, sc = par                                    # maxwell
    P = [Poly(3, k, rng) for _ in range(6)]              # H, E

    def U(x):
        return np.stack([q(x) for q in P], 1)

    def curl(off, x):
        g = [P[off + i].grad(x) for i in range(3)]
        return np.stack([g[2][:, 1] - g[1][:, 2], g[0][:, 2] - g[2][:, 0], g[1][:, 0] - g[0][:, 1]], 1)

    def src(x, t=0.0):
        u = U(x)
        return np.concatenate([A_STAGE * mu * u[:, :3] + curl(3, x),
                               (A_STAGE * eps + sc) * u[:, 3:] - curl(0, x)], 1)
    return U, src, (lambda x, t: U(x)[:, 3:6]), (lambda x, n, t: np.cross(n, U(x)[:, :3]))


def _case(cfg, k, planes, seed=0):
    p = make_problem(cfg, n=2, k=k)
    p.elem_par[:] = {"acoustic": [1.3, 0.8], "elastic": [1.1, 1.7, 0.9], "maxwell": [1.2, 0.9, 0.05]}[p.physics]
    tag_box_faces(p, planes)
    d = hdg.make_discretisation(p)
    U, src, dir_f, flux_f = _fields(p.physics, k, p.elem_par[0], np.random.default_rng(seed))
    f = hdg.load_vector(d, src)
    lb = hdg.project_boundary(d, dir_f) + hdg.neumann_load(d, flux_f)
    return p, d, U, f, lb, flux_f


def _reproduction_error(d, U, f, lb):
    u, lam, _ = hdg.solve_stage(d, A_STAGE, f, lb)
    ref = hdg.project_volume(d, lambda x, t: U(x))
    return float(np.abs(u - ref).max() / np.abs(ref).max())


MIXED = [(0, 0.0), (2, 1.0)]          # x = 0 and z = 1 Neumann, the other four faces Dirichlet
ALL = [(a, v) for a in range(3) for v in (0.0, 1.0)]


@pytest.mark.parametrize("cfg,k,planes", [(2, 2, MIXED), (2, 1, ALL), (3, 2, MIXED), (5, 2, MIXED)])
def test_neumann_polynomial_reproduction(cfg, k, planes):
    p, d, U, f, lb, _ = _case(cfg, k, planes)
    assert d.neumann.sum() > 0 and (d.skel.is_boundary & ~d.neumann).sum() == (0 if planes is ALL else
                                                                             d.skel.is_boundary.sum() - d.neumann.sum())
    err = _reproduction_error(d, U, f, lb)
    assert err <= 1e-9, err


def test_neumann_pin_detects_planted_mistakes():
    p, d, U, f, lb, flux_f = _case(2, 2, MIXED)
    nm = hdg.neumann_trace_mask(d)
    assert _reproduction_error(d, U, f, lb) <= 1e-9
    flipped = lb.copy()
    flipped[nm] *= -1.0                                   # wrong sign of the datum
    assert _reproduction_error(d, U, f, flipped) > 1e-3
    dropped = lb.copy()
    dropped[nm] = 0.0                                     # datum dropped
    assert _reproduction_error(d, U, f, dropped) > 1e-3
    inward = hdg.project_boundary(d, lambda x, t: U(x)[:, 3]) + hdg.neumann_load(
        d, lambda x, n, t: flux_f(x, -n, t))              # inward normal
    assert _reproduction_error(d, U, f, inward) > 1e-3


@pytest.mark.parametrize("cfg,k", [(2, 2), (3, 1), (5, 1)])
def test_neumann_condensed_equals_full_system(cfg, k):
    """Random local and boundary data with Neumann faces: condensation + trace solve +
    recovery equals the direct solve of the whole uncondensed system."""
    p = make_problem(cfg, n=2, k=k)
    tag_box_faces(p, MIXED)
    d = hdg.make_discretisation(p)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(d.loc_off[-1])
    lb = rng.standard_normal(d.tr_off[-1]) * (hdg.boundary_trace_mask(d) | hdg.neumann_trace_mask(d))
    u, lam, _ = hdg.solve_stage(d, 2.0, f, lb)
    uf, lf = hdg.solve_full(d, 2.0, f, lb)
    assert np.abs(u - uf).max() <= 1e-10 * np.abs(uf).max()
    assert np.abs(lam - lf).max() <= 1e-10 * np.abs(lf).max()


def test_bface_tag_validation():
    p = make_problem(2, n=1, k=1)
    tag = np.zeros(p.elem_vert.shape, dtype=np.int8)
    tag[:] = 1                                            # tags interior faces too
    p.bface_tag = tag
    with pytest.raises(ValueError):
        hdg.make_discretisation(p)
    p.bface_tag = np.full(p.elem_vert.shape, 2, dtype=np.int8)
    with pytest.raises(ValueError):
        hdg.make_discretisation(p)
