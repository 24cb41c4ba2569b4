"""Orthonormal polynomial bases on the reference simplices and quadrature rules (oracle).

Section 2.2 of the paper builds every volume space on P_k of the reference element and
every trace space on P_k of the reference face.  The method does not fix a basis; both
the oracle and the HIP library use the orthonormal Proriol-Koornwinder-Dubiner (PKD)
basis, here written out independently:

  reference segment    [0,1]
  reference triangle   vertices (0,0), (1,0), (0,1)
  reference tetrahedron vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1)

Ordering (hierarchical by total degree s):
  segment      i = 0..k
  triangle     for s in 0..k: for i in 0..s: j = s-i
  tetrahedron  for s in 0..k: for i in 0..s: for j in 0..s-i: l = s-i-j

Each function is normalised so that its square integrates to one over the reference
simplex (Lebesgue measure in the reference coordinates).

Jacobi polynomials are evaluated from their explicit finite-sum formula (valid for complex
arguments), and gradients are taken by the complex-step derivative
f'(x) = Im f(x + i h) / h with h = 1e-30, which is exact to rounding for polynomials.

Quadrature: collapsed (Duffy) tensor products of Gauss-Legendre rules on [0,1].
"""
from __future__ import annotations

from functools import lru_cache
from math import comb, gamma, sqrt

import numpy as np

CSTEP = 1e-30


# ----------------------------------------------------------------------------- Jacobi
def jacobi(n: int, a: int, b: int, x):
    """P_n^{(a,b)}(x) = sum_s C(n+a, n-s) C(n+b, s) ((x-1)/2)^s ((x+1)/2)^(n-s)."""
    x = np.asarray(x)
    xm = (x - 1.0) / 2.0
    xp = (x + 1.0) / 2.0
    out = np.zeros_like(x, dtype=np.result_type(x, np.float64))
    for s in range(n + 1):
        out = out + comb(n + a, n - s) * comb(n + b, s) * xm ** s * xp ** (n - s)
    return out


def jacobi_norm2(n: int, a: int, b: int) -> float:
    """int_{-1}^{1} (1-x)^a (1+x)^b P_n^{(a,b)}(x)^2 dx (closed form)."""
    return (2.0 ** (a + b + 1) / (2 * n + a + b + 1)
            * gamma(n + a + 1) * gamma(n + b + 1) / (gamma(n + a + b + 1) * gamma(n + 1)))


def jacobi_on(n: int, a: int, b: int, x):
    """Orthonormal Jacobi polynomial w.r.t. the weight (1-x)^a (1+x)^b on [-1,1]."""
    return jacobi(n, a, b, x) / sqrt(jacobi_norm2(n, a, b))


# ----------------------------------------------------------------------------- indices
def dim_p(k: int, d: int) -> int:
    """dim P_k on a d-simplex."""
    return comb(k + d, d)


def multi_indices(k: int, d: int):
    if d == 1:
        return [(i,) for i in range(k + 1)]
    if d == 2:
        return [(i, s - i) for s in range(k + 1) for i in range(s + 1)]
    if d == 3:
        return [(i, j, s - i - j) for s in range(k + 1) for i in range(s + 1)
                for j in range(s - i + 1)]
    raise ValueError(d)


# ----------------------------------------------------------------------------- PKD bases
def _collapsed(xi):
    """Map reference coordinates in [0,1]-simplex to the collapsed coordinates (a,b,c)
    in [-1,1] of the standard [-1,1]-simplex."""
    d = xi.shape[-1]
    r = 2.0 * xi - 1.0
    if d == 1:
        return (r[..., 0],)
    if d == 2:
        rr, ss = r[..., 0], r[..., 1]
        den = 1.0 - ss
        a = np.where(np.abs(den) > 1e-14, 2.0 * (1.0 + rr) / np.where(np.abs(den) > 1e-14, den, 1.0) - 1.0, -1.0)
        return a, ss
    rr, ss, tt = r[..., 0], r[..., 1], r[..., 2]
    den1 = -ss - tt
    den2 = 1.0 - tt
    ok1 = np.abs(den1) > 1e-14
    ok2 = np.abs(den2) > 1e-14
    a = np.where(ok1, 2.0 * (1.0 + rr) / np.where(ok1, den1, 1.0) - 1.0, -1.0)
    b = np.where(ok2, 2.0 * (1.0 + ss) / np.where(ok2, den2, 1.0) - 1.0, -1.0)
    return a, b, tt


def pkd_eval(k: int, xi):
    """Values of the orthonormal PKD basis of P_k at points xi[..., d] of the [0,1]-simplex.

    Returns array [..., N].  Works for complex xi (used for complex-step gradients).
    """
    xi = np.asarray(xi)
    d = xi.shape[-1]
    co = _collapsed(xi)
    cols = []
    if d == 1:
        (a,) = co
        for (i,) in multi_indices(k, 1):
            cols.append(sqrt(2.0) * jacobi_on(i, 0, 0, a))
    elif d == 2:
        a, b = co
        for i, j in multi_indices(k, 2):
            cols.append(2.0 * sqrt(2.0) * jacobi_on(i, 0, 0, a)
                        * jacobi_on(j, 2 * i + 1, 0, b) * (1.0 - b) ** i)
    else:
        a, b, c = co
        for i, j, l in multi_indices(k, 3):
            cols.append(8.0 * jacobi_on(i, 0, 0, a) * jacobi_on(j, 2 * i + 1, 0, b)
                        * (1.0 - b) ** i * jacobi_on(l, 2 * i + 2 * j + 2, 0, c)
                        * (1.0 - c) ** (i + j))
    return np.stack(cols, axis=-1)


def pkd_grad(k: int, xi):
    """Reference gradient of the PKD basis: array [..., N, d] (complex-step derivative)."""
    xi = np.asarray(xi, dtype=np.float64)
    d = xi.shape[-1]
    out = []
    for r in range(d):
        pert = xi.astype(np.complex128)
        pert[..., r] += 1j * CSTEP
        out.append(np.imag(pkd_eval(k, pert)) / CSTEP)
    return np.stack(out, axis=-1)


# ----------------------------------------------------------------------------- quadrature
@lru_cache(maxsize=None)
def gauss01(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return (x + 1.0) / 2.0, w / 2.0


@lru_cache(maxsize=None)
def simplex_rule(d: int, q: int):
    """Collapsed Gauss rule on the [0,1]-simplex with q points per direction.

    Exact for polynomials of total degree <= 2q-1-(d-1).
    """
    x, w = gauss01(q)
    if d == 1:
        return x[:, None].copy(), w.copy()
    if d == 2:
        U, V = np.meshgrid(x, x, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        pts = np.stack([U, (1 - U) * V], axis=-1).reshape(-1, 2)
        wts = (WU * WV * (1 - U)).ravel()
        return pts, wts
    U, V, W = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([U, (1 - U) * V, (1 - U) * (1 - V) * W], axis=-1).reshape(-1, 3)
    wts = (WU * WV * WW * (1 - U) ** 2 * (1 - V)).ravel()
    return pts, wts


def rule_for_degree(d: int, deg: int):
    q = max(1, (deg + d + 1) // 2 + 1)
    return simplex_rule(d, q)
