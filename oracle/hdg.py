"""Static condensation, trace solve, recovery and time stepping (oracle).

Section 2.4.1: with the local block A block-diagonal over elements, the local unknowns
are eliminated element by element, leaving the global trace system

    K lam = r,   K = sum_K P_K^T (D_K - C_K A_K^{-1} B_K) P_K,
                 r = sum_K P_K^T (g_K - C_K A_K^{-1} f_K),

and afterwards u_K = A_K^{-1} (f_K - B_K lam_K) (the first block row).  The system is
written in the linear form A u + B lam = f (so the right-hand side carries the sign of
f directly; see the module docstring of ``physics``).

Dirichlet faces carry the L2 projection of the boundary data onto the face space
(the trace equations of sections 4.1.2 and 5.2 replace the jump condition there by
<lam - g_D, mu>_F = 0); their values are moved to the right-hand side.  Neumann faces
(section 4.1.2, the Gamma_N part of the trace equation: <flux_hat - g_N, mu>_F = 0) keep
the one-sided flux row of their element and carry the tested datum <g_N, mu>_F on the
right-hand side of that row.  The boundary vector lam_bnd of the solvers holds both: the
projected Dirichlet values on Dirichlet faces and the tested fluxes on Neumann faces.

Time stepping: DIRK stages written as in section 2.3.2,
    sum_j d_ij M (U_j - u^n) + dt f(U_i, V_i, t_n + c_i dt) = 0,
i.e. a M U_i + L U_i = a M u*_i + s with a = d_ii/dt and
u*_i = u^n - (1/d_ii) sum_{j<i} d_ij (U_j - u^n); then
u^{n+1} = (1 - sum_i b_i sum_j d_ij) u^n + sum_j e_j U_j,  e_j = sum_i b_i d_ij.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import build_skeleton, face_map, face_frame, face_measure_and_normal
from .physics import ElementQuad, local_system, n_local_comp, N_TRACE_COMP, stabilisation
from .polynomials import dim_p, pkd_eval, rule_for_degree


# ----------------------------------------------------------------------------- DIRK(3,3)
def dirk33():
    """Alexander's 3-stage, third-order, L-stable, stiffly accurate SDIRK (the DIRK(3,3)
    scheme the paper uses throughout).  gamma is the root in (1/6, 1/2) of
    x^3 - 3x^2 + 3x/2 - 1/6 = 0."""
    roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    g = float(min((r.real for r in roots if abs(r.imag) < 1e-12 and 1 / 6 < r.real < 0.5)))
    b1 = -1.5 * g * g + 4.0 * g - 0.25
    b2 = 1.5 * g * g - 5.0 * g + 1.25
    A = np.array([[g, 0.0, 0.0], [(1 - g) / 2, g, 0.0], [b1, b2, g]])
    b = np.array([b1, b2, g])
    c = A.sum(axis=1)
    return A, b, c


def backward_euler():
    return np.array([[1.0]]), np.array([1.0]), np.array([1.0])


# ----------------------------------------------------------------------------- discretisation
@dataclass
class Discretisation:
    physics: str
    dim: int
    xyz: np.ndarray
    elem_vert: np.ndarray
    elem_par: np.ndarray
    degree: np.ndarray
    skel: object = None
    face_k: np.ndarray = None          # [n_faces]
    elem_face_k: np.ndarray = None     # [n_elem, dim+1]
    loc_off: np.ndarray = None         # [n_elem+1] local dof offsets
    tr_off: np.ndarray = None          # [n_faces+1] trace dof offsets
    neumann: np.ndarray = None         # [n_faces] bool: boundary face with a Neumann condition
    quad: dict = field(default_factory=dict)

    @property
    def n_elem(self):
        return self.elem_vert.shape[0]

    @property
    def m_local(self):
        return n_local_comp(self.physics, self.dim)

    @property
    def m_trace(self):
        return N_TRACE_COMP[self.physics]

    def elem_quad(self, e) -> ElementQuad:
        q = self.quad.get(e)
        if q is None:
            q = ElementQuad(self.xyz, self.elem_vert, self.skel, e, int(self.degree[e]),
                            [int(x) for x in self.elem_face_k[e]])
            self.quad[e] = q
        return q

    def elem_trace_dofs(self, e):
        idx = []
        for f in range(self.dim + 1):
            g = self.skel.elem_faces[e, f]
            idx.extend(range(self.tr_off[g], self.tr_off[g + 1]))
        return np.asarray(idx, dtype=np.int64)

    def elem_local_dofs(self, e):
        return np.arange(self.loc_off[e], self.loc_off[e + 1])


def make_discretisation(problem) -> Discretisation:
    """Skeleton, face degrees (k_F = max of the neighbours' degrees) and dof offsets.
    problem.bface_tag (optional, [n_elem, dim+1], the local face opposite vertex f): 1 marks a
    Neumann boundary face, 0 a Dirichlet one; interior faces must carry 0."""
    skel = build_skeleton(problem.elem_vert)
    deg = np.asarray(problem.degree, dtype=np.int64)
    fk = np.zeros(skel.n_faces, dtype=np.int64)
    for s in range(2):
        e = skel.face_elems[:, s]
        ok = e >= 0
        fk[ok] = np.maximum(fk[ok], deg[e[ok]])
    dim = problem.dim
    d = Discretisation(problem.physics, dim, problem.xyz, problem.elem_vert,
                       np.asarray(problem.elem_par, dtype=np.float64), deg, skel)
    d.face_k = fk
    d.elem_face_k = fk[skel.elem_faces]
    nloc = np.array([d.m_local * dim_p(int(k), dim) for k in deg])
    d.loc_off = np.concatenate([[0], np.cumsum(nloc)])
    ntr = np.array([d.m_trace * dim_p(int(k), dim - 1) for k in fk])
    d.tr_off = np.concatenate([[0], np.cumsum(ntr)])
    d.neumann = np.zeros(skel.n_faces, dtype=bool)
    tag = getattr(problem, "bface_tag", None)
    if tag is not None:
        tag = np.asarray(tag)
        if tag.shape != skel.elem_faces.shape or not np.isin(tag, (0, 1)).all():
            raise ValueError("bface_tag: [n_elem, dim+1] of 0 (Dirichlet) or 1 (Neumann)")
        faces = skel.elem_faces[tag == 1]
        if (~skel.is_boundary[faces]).any():
            raise ValueError("bface_tag: Neumann tag on an interior face")
        d.neumann[faces] = True
    return d


def element_system(disc: Discretisation, e: int, a: float):
    return local_system(disc.physics, disc.elem_quad(e), disc.elem_par[e], a)


# ----------------------------------------------------------------------------- projections
def project_volume(disc: Discretisation, func, t=0.0):
    """Element-wise L2 projection of func(x, t) -> [q, m] onto V_h^k (coefficients in the
    orthonormal basis: u_i = (func, phi_i)_K / |K-map det|)."""
    out = np.zeros(disc.loc_off[-1])
    for e in range(disc.n_elem):
        q = disc.elem_quad(e)
        vals = np.atleast_2d(func(q.xq, t))
        if vals.shape[0] != q.xq.shape[0]:
            vals = vals.T
        coef = np.einsum("q,qi,qc->ci", q.wq, q.phi, vals) / abs(q.det)
        out[disc.loc_off[e]:disc.loc_off[e + 1]] = coef.ravel()
    return out


def load_vector(disc: Discretisation, func, t=0.0):
    """Tested source (s, w)_K for every basis test function w of every component.
    func(x, t) -> [q, m] in the component order of ``physics``; for the elastic stress the
    six entries are the physical components s11, s22, s33, s23, s13, s12 and the test
    tensor of an off-diagonal component is E_ab + E_ba (weight 2)."""
    m = disc.m_local
    wc = np.ones(m)
    if disc.physics == "elastic":
        wc[3:6] = 2.0
    out = np.zeros(disc.loc_off[-1])
    for e in range(disc.n_elem):
        q = disc.elem_quad(e)
        vals = np.atleast_2d(func(q.xq, t))
        if vals.shape[0] != q.xq.shape[0]:
            vals = vals.T
        coef = np.einsum("q,qi,qc->ci", q.wq, q.phi, vals) * wc[:, None]
        out[disc.loc_off[e]:disc.loc_off[e + 1]] = coef.ravel()
    return out


def face_quadrature(disc, g, deg):
    fv = disc.skel.faces[g]
    st, w = rule_for_degree(disc.dim - 1, deg)
    P0, T = face_map(disc.xyz, fv)
    y = P0 + st @ T.T
    if disc.dim == 3:
        jac = np.linalg.norm(np.cross(T[:, 0], T[:, 1]))
    else:
        jac = np.linalg.norm(T[:, 0])
    return st, y, w * jac


def project_boundary(disc: Discretisation, func, t=0.0):
    """L2 projection of Dirichlet data onto the trace space of every Dirichlet boundary face.
    Maxwell: func returns the full field; its tangential part in the face frame is used.
    Returns a full-length trace vector (zeros on interior and Neumann faces)."""
    lam = np.zeros(disc.tr_off[-1])
    for g in np.nonzero(disc.skel.is_boundary & ~disc.neumann)[0]:
        kf = int(disc.face_k[g])
        st, y, w = face_quadrature(disc, g, 2 * kf + 6)
        psi = pkd_eval(kf, st)
        vals = np.atleast_2d(func(y, t))
        if vals.shape[0] != y.shape[0]:
            vals = vals.T
        if disc.physics in ("maxwell", "maxwell_glm"):
            t1, t2 = face_frame(disc.xyz, disc.skel.faces[g])
            vals = np.stack([vals @ t1, vals @ t2], axis=1)
        Hm = np.einsum("q,ql,qm->lm", w, psi, psi)
        rhs = np.einsum("q,ql,qc->cl", w, psi, vals)
        coef = np.linalg.solve(Hm, rhs.T).T
        lam[disc.tr_off[g]:disc.tr_off[g + 1]] = coef.ravel()
    return lam


def neumann_load(disc: Discretisation, func, t=0.0):
    """Tested Neumann data <g_N, mu_l>_F on every Neumann face (zeros elsewhere), the
    right-hand side of the face's flux row (section 4.1.2, Gamma_N part of the trace
    equation).  func(x, n, t) -> the prescribed flux at the points x with n the outward unit
    normal: acoustic v.n (scalar), elastic the traction sigma n (3), Maxwell n x H (3; its
    components along the face frame t1, t2 are tested)."""
    out = np.zeros(disc.tr_off[-1])
    for g in np.nonzero(disc.neumann)[0]:
        kf = int(disc.face_k[g])
        st, y, w = face_quadrature(disc, g, 2 * kf + 6)
        psi = pkd_eval(kf, st)
        e = int(disc.skel.face_elems[g, 0])
        cen = disc.xyz[disc.elem_vert[e]].mean(axis=0)
        _, nrm = face_measure_and_normal(disc.xyz, disc.skel.faces[g], cen)
        vals = np.asarray(func(y, np.broadcast_to(nrm, y.shape), t), dtype=np.float64)
        vals = vals.reshape(y.shape[0], -1)
        if disc.physics in ("maxwell", "maxwell_glm"):
            t1, t2 = face_frame(disc.xyz, disc.skel.faces[g])
            vals = np.stack([vals @ t1, vals @ t2], axis=1)
        out[disc.tr_off[g]:disc.tr_off[g + 1]] = np.einsum("q,ql,qc->cl", w, psi, vals).ravel()
    return out


def point_source_rhs(disc: Discretisation, points):
    """Right-hand side columns for unit point sources in the pressure equation:
    column s holds phi_i(x_s) in the pressure block of the element containing x_s."""
    assert disc.physics == "acoustic"
    F = np.zeros((disc.loc_off[-1], len(points)))
    X = disc.xyz[disc.elem_vert]          # [ne, d+1, d]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    Jinv = np.linalg.inv(J)
    for s, x in enumerate(points):
        xi = np.einsum("eij,ej->ei", Jinv, x[None, :] - X[:, 0, :])
        bary = np.concatenate([1 - xi.sum(1, keepdims=True), xi], axis=1)
        inside = np.nonzero(np.all(bary >= -1e-12, axis=1))[0]
        e = int(inside[0])
        k = int(disc.degree[e])
        N = dim_p(k, disc.dim)
        phi = pkd_eval(k, xi[e][None, :])[0]
        p0 = disc.loc_off[e] + disc.dim * N
        F[p0:p0 + N, s] = phi
    return F


# ----------------------------------------------------------------------------- condensation
@dataclass
class Condensed:
    K: sp.csr_matrix
    r: np.ndarray
    Z: list
    z: list
    Ke: list
    re: list


def condense(disc: Discretisation, a: float, f_loc, g_tr=None):
    """Per-element local solves and Schur complements, assembled into the global trace
    system (no Dirichlet elimination yet).  f_loc: [n_loc] or [n_loc, r]."""
    f_loc = np.asarray(f_loc)
    vec = f_loc.ndim == 1
    F = f_loc[:, None] if vec else f_loc
    nr = F.shape[1]
    ntr = disc.tr_off[-1]
    rows, cols, vals = [], [], []
    r = np.zeros((ntr, nr))
    Zs, zs, Kes, res = [], [], [], []
    for e in range(disc.n_elem):
        A, B, C, D, _ = element_system(disc, e, a)
        li = disc.elem_local_dofs(e)
        ti = disc.elem_trace_dofs(e)
        fe = F[li]
        ge = np.zeros((len(ti), nr)) if g_tr is None else np.asarray(g_tr).reshape(ntr, nr)[ti]
        Z = np.linalg.solve(A, B)
        z = np.linalg.solve(A, fe)
        Ke = D - C @ Z
        re = ge - C @ z
        Zs.append(Z)
        zs.append(z)
        Kes.append(Ke)
        res.append(re)
        rr, cc = np.meshgrid(ti, ti, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(Ke.ravel())
        r[ti] += re
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ntr, ntr))
    return Condensed(K, r[:, 0] if vec else r, Zs, zs, Kes, res)


def boundary_trace_mask(disc: Discretisation):
    """Trace dofs of the Dirichlet faces (the rows that become lam = lam_D)."""
    mask = np.zeros(disc.tr_off[-1], dtype=bool)
    for g in np.nonzero(disc.skel.is_boundary & ~disc.neumann)[0]:
        mask[disc.tr_off[g]:disc.tr_off[g + 1]] = True
    return mask


def neumann_trace_mask(disc: Discretisation):
    """Trace dofs of the Neumann faces (flux rows with the tested datum on the right)."""
    mask = np.zeros(disc.tr_off[-1], dtype=bool)
    for g in np.nonzero(disc.neumann)[0]:
        mask[disc.tr_off[g]:disc.tr_off[g + 1]] = True
    return mask


def trace_solve(disc: Discretisation, cond: Condensed, lam_bnd):
    """Solve K lam = r on the trace dofs of interior and Neumann faces with the Dirichlet
    values lam_bnd fixed on Dirichlet faces (sparse LU); the Neumann rows add lam_bnd (the
    tested flux data) to r."""
    bm = boundary_trace_mask(disc)
    im = ~bm
    r = cond.r
    vec = r.ndim == 1
    R = r[:, None] if vec else r
    LB = np.asarray(lam_bnd).reshape(R.shape[0], -1)
    if LB.shape[1] != R.shape[1]:
        LB = np.repeat(LB, R.shape[1], axis=1)
    nm = neumann_trace_mask(disc)
    R = R.copy()
    R[nm] += LB[nm]
    K = cond.K.tocsr()
    Kii = K[im][:, im].tocsc()
    Kib = K[im][:, bm]
    rhs = R[im] - Kib @ LB[bm]
    lu = spla.splu(Kii)
    lam = np.array(LB, dtype=np.float64)
    lam[im] = lu.solve(rhs)
    return lam[:, 0] if vec else lam


def recover(disc: Discretisation, cond: Condensed, lam):
    """u_K = z_K - Z_K lam_K."""
    vec = np.asarray(lam).ndim == 1
    L = np.asarray(lam)[:, None] if vec else np.asarray(lam)
    u = np.zeros((disc.loc_off[-1], L.shape[1]))
    for e in range(disc.n_elem):
        ti = disc.elem_trace_dofs(e)
        u[disc.elem_local_dofs(e)] = cond.z[e] - cond.Z[e] @ L[ti]
    return u[:, 0] if vec else u


def solve_stage(disc: Discretisation, a: float, f_loc, lam_bnd):
    """One implicit stage through condensation: returns (u, lam, condensed data)."""
    cond = condense(disc, a, f_loc)
    lam = trace_solve(disc, cond, lam_bnd)
    u = recover(disc, cond, lam)
    return u, lam, cond


def solve_full(disc: Discretisation, a: float, f_loc, lam_bnd):
    """Brute force: assemble the whole uncondensed system [A B; C D] (local and trace
    unknowns together) and solve it directly."""
    nl, nt = disc.loc_off[-1], disc.tr_off[-1]
    bm = boundary_trace_mask(disc)
    rows, cols, vals = [], [], []

    def add(r0, c0, Mblk):
        rr, cc = np.meshgrid(r0, c0, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(Mblk.ravel())

    for e in range(disc.n_elem):
        A, B, C, D, _ = element_system(disc, e, a)
        li = disc.elem_local_dofs(e)
        ti = disc.elem_trace_dofs(e)
        add(li, li, A)
        add(li, nl + ti, B)
        keep = ~bm[ti]
        add(nl + ti[keep], li, C[keep])
        add(nl + ti[keep], nl + ti, D[keep])
    bidx = np.nonzero(bm)[0]
    rows.append(nl + bidx)          # Dirichlet rows: lam = projected boundary data
    cols.append(nl + bidx)
    vals.append(np.ones(len(bidx)))
    Mglob = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nl + nt, nl + nt))
    rhs = np.zeros(nl + nt)
    rhs[:nl] = f_loc
    rhs[nl:][bm] = np.asarray(lam_bnd)[bm]
    nm = neumann_trace_mask(disc)
    rhs[nl:][nm] = np.asarray(lam_bnd)[nm]     # tested Neumann flux data
    sol = spla.spsolve(Mglob.tocsc(), rhs)
    return sol[:nl], sol[nl:]


# ----------------------------------------------------------------------------- operators
def apply_mass(disc: Discretisation, u, a=1.0):
    """a * Mw u, element by element."""
    out = np.zeros_like(u)
    for e in range(disc.n_elem):
        _, _, _, _, Mw = element_system(disc, e, 0.0)
        li = disc.elem_local_dofs(e)
        out[li] = a * (Mw @ u[li])
    return out


def energy(disc: Discretisation, u):
    """Discrete energy 1/2 (u, Mw u)."""
    return 0.5 * float(u @ apply_mass(disc, u))


def l2_norm_fields(disc: Discretisation, u, comps):
    """sqrt(sum_K |det| sum_{c in comps} sum_i u_{c,i}^2)  (orthonormal basis, affine
    elements: the L2(Omega) norm of the listed components)."""
    tot = 0.0
    for e in range(disc.n_elem):
        k = int(disc.degree[e])
        N = dim_p(k, disc.dim)
        q = disc.elem_quad(e)
        ue = u[disc.loc_off[e]:disc.loc_off[e + 1]].reshape(-1, N)
        tot += abs(q.det) * float(np.sum(ue[list(comps)] ** 2))
    return np.sqrt(tot)


def l2_error_fields(disc: Discretisation, u, func, t, comps):
    """|| u_h - func(., t) ||_{L2(Omega)} over the listed components, by quadrature."""
    tot = 0.0
    for e in range(disc.n_elem):
        k = int(disc.degree[e])
        N = dim_p(k, disc.dim)
        q = disc.elem_quad(e)
        ue = u[disc.loc_off[e]:disc.loc_off[e + 1]].reshape(-1, N)
        uh = q.phi @ ue.T
        ex = np.atleast_2d(func(q.xq, t))
        if ex.shape[0] != q.xq.shape[0]:
            ex = ex.T
        diff = (uh - ex)[:, list(comps)]
        tot += float(np.sum(q.wq[:, None] * diff ** 2))
    return np.sqrt(tot)


def dirk_step(disc: Discretisation, u, t, dt, bnd_func, scheme="dirk33", src=None):
    """Advance u^n -> u^{n+1}.  bnd_func(t) returns the projected boundary trace vector at
    time t; src(t) an optional local source vector (already tested against the basis)."""
    Ark, b, c = dirk33() if scheme == "dirk33" else backward_euler()
    s = len(b)
    Dm = np.linalg.inv(Ark)
    U = []
    for i in range(s):
        a = Dm[i, i] / dt
        ustar = u.copy()
        for j in range(i):
            ustar -= (Dm[i, j] / Dm[i, i]) * (U[j] - u)
        f = apply_mass(disc, ustar, a)
        if src is not None:
            f = f + src(t + c[i] * dt)
        Ui, _, _ = solve_stage(disc, a, f, bnd_func(t + c[i] * dt))
        U.append(Ui)
    e = b @ Dm
    unew = (1.0 - float(np.sum(b @ Dm))) * u
    for j in range(s):
        unew = unew + e[j] * U[j]
    return unew
