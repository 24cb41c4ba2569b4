"""Local HDG matrices of one element, built by quadrature in physical coordinates (oracle).

Every physics is written in the linear stage form of one implicit step (section 2.3;
Newton linearisation of section 2.4.1, exact for these linear problems):

    A u + B lam = f          (local equations of element K, test functions in V_h^k)
    C u + D lam = g          (the element's contribution to the trace equations)

with A = a*Mw + L, where Mw is the time-derivative weight ("mass") of the DAE
M du/dt + f(u, v, t) = 0 and a = d_ii / dt the stage coefficient.

Unknown ordering inside an element: component-major, then basis index.  The leading
components are the "flux-like" fields whose weight block is block-diagonal:
  acoustic  u = [v_1..v_d, p],            trace lam = p_hat (1 component)
  elastic   u = [s11,s22,s33,s23,s13,s12, v_1,v_2,v_3],  trace lam = v_hat (3 comps)
  maxwell   u = [H_1,H_2,H_3, E_1,E_2,E_3], trace lam = tangential E_hat in the face
            frame (t1, t2) (2 comps)
Trace ordering inside an element: local face 0..d, then component, then face basis index.

Formulations
  acoustic  (derived from the general recipe of the introduction: local Galerkin
            projection, numerical flux v_hat.n = v.n + tau (p - p_hat), jump condition;
            tau = 1/(rho c), the impedance choice of section 4.1.3):
              (a rho v, w) - (p, div w) + <p_hat, w.n> = (a rho v*, w)
              (a/(rho c^2) p, q) + (div v, q) + <tau (p - p_hat), q> = (a/(rho c^2) p*, q) + (s, q)
              sum_K <v.n + tau (p - p_hat), mu>_F = 0
  elastic   velocity / symmetric-stress form of section 4.1.2 (equivalent to the
            velocity / deformation-gradient form for element-wise constant Lame
            coefficients), stress flux sigma_hat n = sigma n - S (v - v_hat), S = 2 rho c_s I
            (the value used in section 4.3); the face term of the momentum equation
            enters with the sign for which the energy identity of section 4.2.3 holds:
              (a A sigma, tau) + (v, div tau) - <v_hat, tau n> = (a A sigma*, tau)
              (a rho v, w) + (sigma, grad w) - <sigma n - S (v - v_hat), w> = (a rho v*, w)
              sum_K <sigma n - S (v - v_hat), mu>_F = 0
            A sigma = (sigma - lambda/(3 lambda + 2 mu) tr(sigma) I) / (2 mu).
  maxwell   section 5.2 without the GLM multiplier, J = sigma_c E (Ohmic), tau = 2:
              (a mu H, w) + (E, curl w) + <E_hat^t, w x n> = (a mu H*, w)
              ((a eps + sigma_c) E, v) - (H, curl v) - <H_hat^t, v x n> = (a eps E*, v)
              H_hat^t = H^t - tau (E - E_hat^t) x n
              sum_K <n x H_hat^t, mu>_F = 0
  maxwell_glm  section 5.2 with the generalised Lagrange multiplier phi of section 5.1.2
            (u = [H_1,H_2,H_3, E_1,E_2,E_3, phi]; equations (dmax1)-(dmax3) in stage form,
            phi_hat = 0 on every face as in (dmax1), alpha_1 = alpha_2 = alpha_3 = 1, the only
            values the paper runs in section 5.4; no charge density):
              the two maxwell rows above, the E row also carrying - (phi, div v), and
              ((a/alpha_1^2 + 1/alpha_2^2) phi, psi) + (1/alpha_3^2) <phi, psi>_dK
                + (div E, psi) = (a/alpha_1^2 phi*, psi)
            the trace equation is that of maxwell (phi does not enter it).
  elastic_fv  the velocity / deformation-gradient form of section 4.1.2 exactly as the paper
            writes it (u = [F_11,F_12,F_13,F_21,..,F_33, v_1,v_2,v_3], F row-major), used only
            to pin the elastic form above (they must give the same v, v_hat and
            sigma(F_h) = sigma_h):
              (a F, G) + (v, div G) - <v_hat, G n> = (a F*, G)
              (a rho v, w) + (sigma(F), grad w) - <sigma(F) n - S (v - v_hat), w> = (a rho v*, w)
              sum_K <sigma(F) n - S (v - v_hat), mu>_F = 0
            sigma(F) = mu (F + F^T) + lambda tr(F) I.  The law of section 4.1.1 adds the constant
            (-lambda d - 2 mu) I; a constant tensor c I drops out of the last two lines
            ((c I, grad w)_K = <c n, w>_dK), so F may be measured from the identity.
"""
from __future__ import annotations

import numpy as np

from .mesh import element_map, face_map, face_measure_and_normal, face_frame
from .polynomials import pkd_eval, pkd_grad, rule_for_degree, dim_p

# symmetric-tensor basis for the 6-component stress: sigma = sum_a s_a E_a
SYM_BASIS = np.zeros((6, 3, 3))
for _a, (_i, _j) in enumerate([(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]):
    SYM_BASIS[_a, _i, _j] = 1.0
    SYM_BASIS[_a, _j, _i] = 1.0

LEVI = np.zeros((3, 3, 3))
LEVI[0, 1, 2] = LEVI[1, 2, 0] = LEVI[2, 0, 1] = 1.0
LEVI[0, 2, 1] = LEVI[2, 1, 0] = LEVI[1, 0, 2] = -1.0

N_COMP = {"acoustic": None, "elastic": 9, "maxwell": 6, "maxwell_glm": 7, "elastic_fv": 12}
N_TRACE_COMP = {"acoustic": 1, "elastic": 3, "maxwell": 2, "maxwell_glm": 2, "elastic_fv": 3}

# GLM coefficients alpha_1, alpha_2, alpha_3 of (dmax3) (section 5.4 runs all three at 1)
GLM_ALPHA = (1.0, 1.0, 1.0)


def n_local_comp(physics: str, dim: int) -> int:
    return dim + 1 if physics == "acoustic" else N_COMP[physics]


def stabilisation(physics: str, par):
    """tau (acoustic, maxwell) or the scalar S of S = s I (elastic)."""
    if physics == "acoustic":
        rho, c = par[0], par[1]
        return 1.0 / (rho * c)
    if physics in ("elastic", "elastic_fv"):
        rho, mu = par[0], par[2]
        return 2.0 * rho * np.sqrt(mu / rho)
    return 2.0


class ElementQuad:
    """Volume and face quadrature data of one element in physical coordinates."""

    def __init__(self, xyz, elem_vert, skel, e, k, face_k):
        self.dim = dim = xyz.shape[1]
        self.k = k
        X0, J, det, Jinv = element_map(xyz, elem_vert, e)
        self.X0, self.J, self.det, self.Jinv = X0, J, det, Jinv
        xi, w = rule_for_degree(dim, 2 * k + 2)
        self.xq = X0 + xi @ J.T
        self.wq = w * abs(det)
        self.phi = pkd_eval(k, xi)                       # [q, N]
        self.gphi = pkd_grad(k, xi) @ Jinv               # [q, N, d] physical gradient
        self.N = self.phi.shape[1]
        cen = xyz[elem_vert[e]].mean(axis=0)
        self.faces = []
        for f in range(dim + 1):
            g = skel.elem_faces[e, f]
            fv = skel.faces[g]
            kf = face_k[f]
            st, wf = rule_for_degree(dim - 1, kf + k + 2)
            P0, T = face_map(xyz, fv)
            y = P0 + st @ T.T
            meas, nrm = face_measure_and_normal(xyz, fv, cen)
            jac = meas * (2.0 if dim == 3 else 1.0)
            xi_f = (y - X0) @ Jinv.T
            fd = dict(
                gid=g, kf=kf, y=y, w=wf * jac, n=nrm, meas=meas,
                phi=pkd_eval(k, xi_f),
                psi=pkd_eval(kf, st),
            )
            if dim == 3:
                fd["frame"] = face_frame(xyz, fv)
            self.faces.append(fd)

    # elementary integrals
    def mass(self):
        return np.einsum("q,qi,qj->ij", self.wq, self.phi, self.phi)

    def deriv(self):
        """Dx[s][i][j] = (phi_i, d phi_j / d x_s)_K."""
        return np.einsum("q,qi,qjs->sij", self.wq, self.phi, self.gphi)

    def face_vv(self, f):
        fd = self.faces[f]
        return np.einsum("q,qi,qj->ij", fd["w"], fd["phi"], fd["phi"])

    def face_vt(self, f):
        fd = self.faces[f]
        return np.einsum("q,qi,ql->il", fd["w"], fd["phi"], fd["psi"])

    def face_tt(self, f):
        fd = self.faces[f]
        return np.einsum("q,ql,qm->lm", fd["w"], fd["psi"], fd["psi"])


def local_system(physics, eq: ElementQuad, par, a):
    """Return (A, B, C, D, Mw) of one element (see module docstring)."""
    dim, N = eq.dim, eq.N
    M = eq.mass()
    Dx = eq.deriv()
    nf = dim + 1
    Ff = [eq.face_vv(f) for f in range(nf)]
    Gf = [eq.face_vt(f) for f in range(nf)]
    Hf = [eq.face_tt(f) for f in range(nf)]
    NF = [G.shape[1] for G in Gf]
    mt = 1 if physics == "acoustic" else N_TRACE_COMP[physics]
    toff = np.concatenate([[0], np.cumsum([mt * q for q in NF])])
    t = int(toff[-1])
    m = n_local_comp(physics, dim)
    n = m * N
    A = np.zeros((n, n))
    Mw = np.zeros((n, n))
    B = np.zeros((n, t))
    C = np.zeros((t, n))
    D = np.zeros((t, t))
    tau = stabilisation(physics, par)

    def blk(ci):
        return slice(ci * N, (ci + 1) * N)

    def tblk(f, c):
        return slice(toff[f] + c * NF[f], toff[f] + (c + 1) * NF[f])

    if physics == "acoustic":
        rho, c = par[0], par[1]
        P = dim  # index of the pressure component
        for x in range(dim):
            Mw[blk(x), blk(x)] = rho * M
            A[blk(x), blk(P)] = -Dx[x].T
            A[blk(P), blk(x)] = Dx[x]
        Mw[blk(P), blk(P)] = M / (rho * c * c)
        L_pp = tau * sum(Ff)
        A += a * Mw
        A[blk(P), blk(P)] += L_pp
        for f in range(nf):
            nrm = eq.faces[f]["n"]
            for x in range(dim):
                B[blk(x), tblk(f, 0)] = nrm[x] * Gf[f]
                C[tblk(f, 0), blk(x)] = nrm[x] * Gf[f].T
            B[blk(P), tblk(f, 0)] = -tau * Gf[f]
            C[tblk(f, 0), blk(P)] = tau * Gf[f].T
            D[tblk(f, 0), tblk(f, 0)] = -tau * Hf[f]
        return A, B, C, D, Mw

    if physics == "elastic":
        rho, lam, mu = par
        S = tau
        E = SYM_BASIS
        trE = np.einsum("aii->a", E)
        comp = (np.einsum("aij,bij->ab", E, E) - lam / (3 * lam + 2 * mu) * np.outer(trE, trE)) / (2 * mu)
        for al in range(6):
            for be in range(6):
                Mw[blk(al), blk(be)] = comp[al, be] * M
            for x in range(3):
                # (v, div tau): tau = E_al phi_i, v = e_x phi_j
                A[blk(al), blk(6 + x)] = sum(E[al, x, b] * Dx[b].T for b in range(3))
                # (sigma, grad w) - <sigma n, w>: sigma = E_al phi_j, w = e_x phi_i
                A[blk(6 + x), blk(al)] = sum(
                    E[al, x, b] * (Dx[b].T - sum(eq.faces[f]["n"][b] * Ff[f] for f in range(nf)))
                    for b in range(3))
        for x in range(3):
            Mw[blk(6 + x), blk(6 + x)] = rho * M
        A += a * Mw
        for x in range(3):
            A[blk(6 + x), blk(6 + x)] += S * sum(Ff)
        for f in range(nf):
            nrm = eq.faces[f]["n"]
            for y in range(3):
                for al in range(6):
                    En = E[al, y, :] @ nrm
                    B[blk(al), tblk(f, y)] = -En * Gf[f]
                    C[tblk(f, y), blk(al)] = En * Gf[f].T
                B[blk(6 + y), tblk(f, y)] = -S * Gf[f]
                C[tblk(f, y), blk(6 + y)] = -S * Gf[f].T
                D[tblk(f, y), tblk(f, y)] = S * Hf[f]
        return A, B, C, D, Mw

    if physics in ("maxwell", "maxwell_glm"):
        eps, mu, sig = par[0], par[1], par[2]
        for x in range(3):
            Mw[blk(x), blk(x)] = mu * M
            Mw[blk(3 + x), blk(3 + x)] = eps * M
            for y in range(3):
                # (E, curl w): w = e_x phi_i, E = e_y phi_j
                A[blk(x), blk(3 + y)] = sum(LEVI[y, s, x] * Dx[s].T for s in range(3))
                # -(H, curl v) - <H, v x n>: v = e_x phi_i, H = e_y phi_j
                A[blk(3 + x), blk(y)] = -sum(LEVI[y, s, x] * Dx[s].T for s in range(3)) - sum(
                    (LEVI[y, x, :] @ eq.faces[f]["n"]) * Ff[f] for f in range(nf))
                A[blk(3 + x), blk(3 + y)] = tau * sum(
                    ((1.0 if x == y else 0.0) - eq.faces[f]["n"][x] * eq.faces[f]["n"][y]) * Ff[f]
                    for f in range(nf))
            A[blk(3 + x), blk(3 + x)] += sig * M
        A += a * Mw
        for f in range(nf):
            nrm = eq.faces[f]["n"]
            t1, t2 = eq.faces[f]["frame"]
            for ci, tc in enumerate((t1, t2)):
                for x in range(3):
                    ex = np.eye(3)[x]
                    B[blk(x), tblk(f, ci)] = (tc @ np.cross(ex, nrm)) * Gf[f]
                    B[blk(3 + x), tblk(f, ci)] = -tau * tc[x] * Gf[f]
                    C[tblk(f, ci), blk(x)] = (tc @ np.cross(nrm, ex)) * Gf[f].T
                    C[tblk(f, ci), blk(3 + x)] = -tau * tc[x] * Gf[f].T
                D[tblk(f, ci), tblk(f, ci)] = tau * Hf[f]
        if physics == "maxwell_glm":
            a1, a2, a3 = GLM_ALPHA
            PH = 6
            Mw[blk(PH), blk(PH)] = M / a1 ** 2
            A[blk(PH), blk(PH)] = (a / a1 ** 2 + 1.0 / a2 ** 2) * M + sum(Ff) / a3 ** 2
            for x in range(3):
                # - (phi, div v): v = e_x phi_i, phi = phi_j
                A[blk(3 + x), blk(PH)] = -Dx[x].T
                # (div E, psi): E = e_x phi_j, psi = phi_i
                A[blk(PH), blk(3 + x)] = Dx[x]
        return A, B, C, D, Mw

    if physics == "elastic_fv":
        rho, lam, mu = par
        S = tau
        iF = lambda i, j: 3 * i + j
        V = 9

        def stress_coef(x, j, a_, b_):
            """d sigma_xj / d F_ab for sigma(F) = mu (F + F^T) + lambda tr(F) I."""
            return (mu * ((a_ == x) * (b_ == j) + (a_ == j) * (b_ == x))
                    + lam * (x == j) * (a_ == b_))

        for i in range(3):
            for j in range(3):
                Mw[blk(iF(i, j)), blk(iF(i, j))] = M
                # (v, div G): G = e_i e_j^T phi_m, div G = e_i d_j phi_m
                A[blk(iF(i, j)), blk(V + i)] = Dx[j].T
        for x in range(3):
            Mw[blk(V + x), blk(V + x)] = rho * M
            for a_ in range(3):
                for b_ in range(3):
                    # (sigma(F), grad w) - <sigma(F) n, w>: w = e_x phi_m, F = e_a e_b^T phi_n
                    A[blk(V + x), blk(iF(a_, b_))] = sum(
                        stress_coef(x, j, a_, b_) * (Dx[j].T - sum(eq.faces[f]["n"][j] * Ff[f] for f in range(nf)))
                        for j in range(3))
        A += a * Mw
        for x in range(3):
            A[blk(V + x), blk(V + x)] += S * sum(Ff)
        for f in range(nf):
            nrm = eq.faces[f]["n"]
            for i in range(3):
                for j in range(3):
                    # - <v_hat, G n>
                    B[blk(iF(i, j)), tblk(f, i)] = -nrm[j] * Gf[f]
            for y in range(3):
                for a_ in range(3):
                    for b_ in range(3):
                        sn = sum(stress_coef(y, j, a_, b_) * nrm[j] for j in range(3))
                        C[tblk(f, y), blk(iF(a_, b_))] = sn * Gf[f].T
                B[blk(V + y), tblk(f, y)] = -S * Gf[f]
                C[tblk(f, y), blk(V + y)] = -S * Gf[f].T
                D[tblk(f, y), tblk(f, y)] = S * Hf[f]
        return A, B, C, D, Mw

    raise ValueError(physics)


def local_sizes(physics, dim, k, face_k):
    N = dim_p(k, dim)
    m = n_local_comp(physics, dim)
    mt = N_TRACE_COMP[physics]
    return m * N, sum(mt * dim_p(q, dim - 1) for q in face_k)
