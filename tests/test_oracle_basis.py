"""Pins of the oracle's polynomial machinery against closed forms and library routines.

These fix the bases and quadrature of section 2.2 (P_k on the reference simplex and face)
independently of the oracle's own formulas.
"""
from math import factorial

import numpy as np
import pytest
import scipy.special as sps

from oracle import polynomials as P


@pytest.mark.parametrize("n,a,b", [(0, 0, 0), (3, 0, 0), (4, 3, 0), (5, 8, 0), (2, 1, 2)])
def test_jacobi_matches_scipy(n, a, b):
    x = np.linspace(-1, 1, 17)
    np.testing.assert_allclose(P.jacobi(n, a, b, x), sps.eval_jacobi(n, a, b, x), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,a,b", [(0, 0, 0), (4, 0, 0), (3, 5, 0), (5, 12, 0)])
def test_jacobi_norm_closed_form(n, a, b):
    x, w = sps.roots_jacobi(20, a, b)          # library Gauss-Jacobi rule
    val = np.sum(w * sps.eval_jacobi(n, a, b, x) ** 2)
    assert abs(val - P.jacobi_norm2(n, a, b)) < 1e-12 * val


def _monomial_integral(exps):
    """int over the unit simplex of x^a y^b z^c = a! b! c! / (a+b+c+d)!"""
    d = len(exps)
    num = np.prod([factorial(e) for e in exps])
    return num / factorial(sum(exps) + d)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_quadrature_exact_on_monomials(d):
    deg = 9
    pts, w = P.rule_for_degree(d, deg)
    import itertools
    for exps in itertools.product(range(deg + 1), repeat=d):
        if sum(exps) > deg:
            continue
        val = np.sum(w * np.prod(pts ** np.asarray(exps)[None, :], axis=1))
        assert abs(val - _monomial_integral(exps)) < 1e-14


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_pkd_orthonormal(d, k):
    pts, w = P.rule_for_degree(d, 2 * k + 2)
    V = P.pkd_eval(k, pts)
    assert V.shape[1] == P.dim_p(k, d)
    G = V.T @ (w[:, None] * V)
    np.testing.assert_allclose(G, np.eye(V.shape[1]), atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("k", [1, 4])
def test_pkd_spans_pk(d, k):
    """Every monomial of degree <= k is reproduced exactly by its projection."""
    import itertools
    pts, w = P.rule_for_degree(d, 2 * k + 2)
    V = P.pkd_eval(k, pts)
    for exps in itertools.product(range(k + 1), repeat=d):
        if sum(exps) > k:
            continue
        mono = np.prod(pts ** np.asarray(exps)[None, :], axis=1)
        coef = V.T @ (w * mono)
        np.testing.assert_allclose(V @ coef, mono, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("k", [1, 3])
def test_pkd_gradient_divergence_theorem(d, k):
    """int_T d_r(phi_i phi_j) = int_dT phi_i phi_j n_r: pins the reference gradients."""
    pts, w = P.rule_for_degree(d, 2 * k + 2)
    V = P.pkd_eval(k, pts)
    G = P.pkd_grad(k, pts)
    lhs = np.einsum("q,qir,qj->rij", w, G, V)
    lhs = lhs + np.transpose(lhs, (0, 2, 1))
    # faces of the reference simplex: x_r = 0 for each r (normal -e_r) and the slanted face
    rhs = np.zeros_like(lhs)
    fpts, fw = P.rule_for_degree(d - 1, 2 * k + 2)
    verts = np.vstack([np.zeros(d), np.eye(d)])
    faces = [[v for v in range(d + 1) if v != f] for f in range(d + 1)]
    for fv in faces:
        X = verts[fv]
        T = (X[1:] - X[0]).T
        y = X[0] + fpts @ T.T
        if d == 2:
            meas = np.linalg.norm(T[:, 0])
            nrm = np.array([T[1, 0], -T[0, 0]])
        else:
            cr = np.cross(T[:, 0], T[:, 1])
            meas = np.linalg.norm(cr)
            nrm = cr
        nrm = nrm / np.linalg.norm(nrm)
        if np.dot(nrm, y.mean(0) - verts.mean(0)) < 0:
            nrm = -nrm
        Vf = P.pkd_eval(k, y)
        rhs += np.einsum("q,qi,qj,r->rij", fw * meas, Vf, Vf, nrm)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)


def test_pkd_gradient_vs_finite_difference():
    pts = np.array([[0.2, 0.3, 0.1], [0.1, 0.1, 0.6]])
    G = P.pkd_grad(3, pts)
    h = 1e-6
    for r in range(3):
        e = np.zeros(3)
        e[r] = h
        fd = (P.pkd_eval(3, pts + e) - P.pkd_eval(3, pts - e)) / (2 * h)
        np.testing.assert_allclose(G[..., r], fd, atol=1e-7)
