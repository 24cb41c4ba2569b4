"""Local post-processing of the acoustic pressure (oracle).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to pin the oracle's acoustic local solver.

The introduction of the paper points out that HDG methods admit a superconvergent
approximation computed by a local, element-by-element post-processing step, and section
3.1.3 describes one (for the velocity of incompressible flow) that gains one order: k+2 for
k >= 1.  The paper gives no post-processing for acoustics.  The reading taken here uses the
velocity row of one implicit stage, a rho v + grad p = F_v (F_v: the velocity right-hand side
of the stage, a rho v* plus any source), which fixes grad p from the velocity; on each element
K the post-processed pressure p* in P_{k+1}(K) solves the Neumann problem

    (grad p*, grad w)_K = (F_v - a rho v_h, grad w)_K   for all w in P_{k+1}(K),
    (p*, 1)_K = (p_h, 1)_K,

the scalar analogue of the post-processing of Cockburn, Gopalakrishnan and Lazarov for
hybridised diffusion.  ||p - p*|| = O(h^{k+2}) then pins the whole acoustic local solver
(flux, stabilisation and signs): a wrong term leaves p_h, or its element means, only O(h^{k+1})
accurate and the gain disappears.
"""
from __future__ import annotations

import numpy as np

from .mesh import element_map
from .polynomials import dim_p, pkd_eval, pkd_grad, rule_for_degree


def postprocess_pressure(disc, u, a: float, src_v):
    """Return the coefficients of p* in the orthonormal basis of P_{k_K + 1}(K) for every
    element K (a list of arrays).  ``u``: the stage solution (acoustic layout [v_1..v_d, p]),
    ``src_v(x) -> [q, d]``: the velocity right-hand side F_v of the stage as a function."""
    assert disc.physics == "acoustic"
    dim = disc.dim
    out = []
    for e in range(disc.n_elem):
        k = int(disc.degree[e])
        N, Np = dim_p(k, dim), dim_p(k + 1, dim)
        rho = disc.elem_par[e][0]
        X0, J, det, Jinv = element_map(disc.xyz, disc.elem_vert, e)
        xi, w = rule_for_degree(dim, 2 * (k + 1) + 6)
        xq = X0 + xi @ J.T
        wq = w * abs(det)
        phi_k = pkd_eval(k, xi)                           # [q, N]
        phi_p = pkd_eval(k + 1, xi)                       # [q, Np]
        gphi_p = pkd_grad(k + 1, xi) @ Jinv               # [q, Np, d]
        ue = u[disc.loc_off[e]:disc.loc_off[e + 1]].reshape(dim + 1, N)
        vh = phi_k @ ue[:dim].T                           # [q, d]
        ph = phi_k @ ue[dim]                              # [q]
        g = np.atleast_2d(src_v(xq)) - a * rho * vh       # approximation of grad p
        S = np.einsum("q,qis,qjs->ij", wq, gphi_p, gphi_p)
        rhs = np.einsum("q,qis,qs->i", wq, gphi_p, g)
        # the constant is in the kernel of S: replace the first row by the mean condition
        S[0, :] = np.einsum("q,qj->j", wq, phi_p)
        rhs[0] = float(np.sum(wq * ph))
        out.append(np.linalg.solve(S, rhs))
    return out


def postprocessed_error(disc, pstar, p_exact):
    """||p* - p_exact||_{L2(Omega)} by quadrature (p_exact(x) -> [q])."""
    dim = disc.dim
    tot = 0.0
    for e in range(disc.n_elem):
        k = int(disc.degree[e])
        X0, J, det, _ = element_map(disc.xyz, disc.elem_vert, e)
        xi, w = rule_for_degree(dim, 2 * (k + 1) + 6)
        xq = X0 + xi @ J.T
        vals = pkd_eval(k + 1, xi) @ pstar[e]
        tot += float(np.sum(w * abs(det) * (vals - p_exact(xq)) ** 2))
    return np.sqrt(tot)
