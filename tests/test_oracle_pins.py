"""Further pins of the oracle against what the paper and the mathematics fix.

* P6: the velocity / symmetric-stress elastic form the oracle (and the library) use equals
  the velocity / deformation-gradient form the paper writes in section 4.1.2, element by
  element and on the trace, for element-wise constant Lame coefficients.
* P7: the local post-processing of the acoustic pressure gains one order (k+2), the
  superconvergence the introduction and section 3.1.3 describe.
* The acoustic stabilisation tau = 1/(rho c) makes the numerical trace the exact solution of
  the acoustic Riemann problem (a textbook result obtained here from the two characteristic
  relations); the elastic S and the Maxwell tau equal the values of the paper's experiments.
* Point sources: the right-hand side columns reproduce point values of polynomials.
* The L2 field norm equals its closed form and the quadrature of the same field.
* GLM-Maxwell (section 5.1.2, equations (dmax1)-(dmax3)): condensation exact, Schur blocks
  symmetric definite, energy non-increasing, optimal rates for H, E and phi.
* Rates at the benchmark degree (3D acoustics k = 3) and on the paper's cavity fields
  (section 5.4, eps_r = 2, mu_r = 1, omega = 1, tau = 2) at k = 1, 2.
* Table eppMeshes: boundary face counts implied by the printed trace-unknown counts.
"""
import os

import numpy as np
import pytest

from synth import make_problem
from oracle import hdg
from oracle import physics as ophys
from oracle.polynomials import dim_p, pkd_eval, rule_for_degree
from oracle.postprocess import postprocess_pressure, postprocessed_error
from test_oracle_hdg import _grad_fd, _manufactured, _manufactured_errors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rates(errs, ns):
    errs = np.asarray(errs)
    return np.log(errs[:-1] / errs[1:]) / np.log(np.asarray(ns[1:], float) / np.asarray(ns[:-1], float))[
        (slice(None),) + (None,) * (errs.ndim - 1)]


# ----------------------------------------------------------------------------- P6
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


@pytest.mark.parametrize("k", [1, 2])
def test_elastic_stress_form_equals_paper_deformation_gradient_form(k):
    """Section 4.1.2 states the HDG scheme for (F, v, v_hat); the oracle's elastic physics uses
    (sigma_sym, v, v_hat).  For element-wise constant Lame coefficients both must give the same
    v_h and v_hat_h, and sigma(F_h) must equal sigma_h, for any stage right-hand side whose
    stress part is sigma(F*)."""
    p = make_problem(3, n=1, k=k)
    ds = hdg.make_discretisation(p)
    p.physics = "elastic_fv"
    df = hdg.make_discretisation(p)
    a = 41.0
    N = dim_p(k, 3)
    rng = np.random.default_rng(11)
    ne = p.n_elem
    Fs = rng.standard_normal((ne, 3, 3, N))
    vs = rng.standard_normal((ne, 3, N))
    body = rng.standard_normal((ne, 3, N))
    lb = rng.standard_normal(ds.tr_off[-1]) * hdg.boundary_trace_mask(ds)
    ff = np.zeros(df.loc_off[-1])
    fs = np.zeros(ds.loc_off[-1])
    sig_of = []
    for e in range(ne):
        rho, lam, mu = p.elem_par[e]

        def sigma(F, mu=mu, lam=lam):   # linear law of section 4.1.1 coefficient-wise
            return mu * (F + np.swapaxes(F, 0, 1)) + lam * np.trace(F)[None, None] * np.eye(3)[:, :, None]
        sig_of.append(sigma)
        ustar_f = np.concatenate([Fs[e].reshape(9 * N), vs[e].reshape(3 * N)])
        S = sigma(Fs[e])
        ustar_s = np.concatenate([np.stack([S[i, j] for (i, j) in PAIRS]).reshape(6 * N), vs[e].reshape(3 * N)])
        Mwf = hdg.element_system(df, e, 0.0)[4]
        Mws = hdg.element_system(ds, e, 0.0)[4]
        bf = np.zeros(12 * N)
        bf[9 * N:] = body[e].ravel()
        bs_ = np.zeros(9 * N)
        bs_[6 * N:] = body[e].ravel()
        ff[df.loc_off[e]:df.loc_off[e + 1]] = a * Mwf @ ustar_f + bf
        fs[ds.loc_off[e]:ds.loc_off[e + 1]] = a * Mws @ ustar_s + bs_
    uf, lf, _ = hdg.solve_stage(df, a, ff, lb)
    us, ls, _ = hdg.solve_stage(ds, a, fs, lb)
    assert np.linalg.norm(lf - ls) <= 1e-12 * np.linalg.norm(ls)
    uf = uf.reshape(ne, 12, N)
    us = us.reshape(ne, 9, N)
    assert np.linalg.norm(uf[:, 9:] - us[:, 6:]) <= 1e-12 * np.linalg.norm(us[:, 6:])
    sig_f = np.stack([np.stack([sig_of[e](uf[e, :9].reshape(3, 3, N))[i, j] for (i, j) in PAIRS]) for e in range(ne)])
    assert np.linalg.norm(sig_f - us[:, :6]) <= 1e-12 * np.linalg.norm(us[:, :6])
    # the skew part of F_h is not determined by sigma: the two forms differ in F, not in sigma
    skew = uf[:, :9].reshape(ne, 3, 3, N)
    assert np.linalg.norm(skew - np.swapaxes(skew, 1, 2)) > 1e-3 * np.linalg.norm(skew)


def test_paper_stress_law_constant_part_drops_out():
    """The law of section 4.1.1 is affine in F; its constant part c I contributes
    (c I, grad w)_K - <c I n, w>_dK = 0 to the momentum row, so the (F, v) system above may
    measure F from the identity.  Checked by quadrature on a jittered element."""
    p = make_problem(3, n=1, k=3)
    d = hdg.make_discretisation(p)
    q = d.elem_quad(2)
    vol = np.einsum("q,qis->is", q.wq, q.gphi)                # (I, grad(e_s phi_i))_K row-wise
    face = sum(np.einsum("q,qi->i", fd["w"], fd["phi"])[:, None] * fd["n"][None, :] for fd in q.faces)
    assert np.abs(vol - face).max() <= 1e-13 * np.abs(vol).max()


# ----------------------------------------------------------------------------- P7
@pytest.mark.parametrize("k,ns", [(1, [8, 16]), (2, [8, 16]), (3, [4, 8])])
def test_postprocessed_pressure_superconverges(k, ns):
    """2D manufactured single stage: p_h converges at k+1 and the post-processed p* at k+2."""
    ep, eh = [], []
    a = 5.0
    for n in ns:
        p = make_problem(1, n=n, k=k)
        p.elem_par[:] = [1.3, 0.8]
        d = hdg.make_discretisation(p)
        U, src = _manufactured("acoustic", 2, p.elem_par[0], a)
        f = hdg.load_vector(d, src)
        lb = hdg.project_boundary(d, lambda x, t: U(x)[:, 2])
        u, _, _ = hdg.solve_stage(d, a, f, lb)
        ps = postprocess_pressure(d, u, a, lambda x: src(x)[:, :2])
        ep.append(postprocessed_error(d, ps, lambda x: U(x)[:, 2]))
        eh.append(hdg.l2_error_fields(d, u, lambda x, t: U(x), 0.0, [2]))
    rp, rh = _rates(ep, ns)[0], _rates(eh, ns)[0]
    assert rp > k + 2 - 0.25, (ep, rp)
    assert abs(rh - (k + 1)) < 0.25, (eh, rh)
    assert ep[-1] < 0.25 * eh[-1]


# ----------------------------------------------------------------------------- stabilisation
def _two_triangle_trace():
    """Numerical trace on the shared face of two triangles holding constant states."""
    p = make_problem(1, n=1, k=2)
    p.elem_par = np.array([[1.3, 0.7], [0.8, 1.9]])
    d = hdg.make_discretisation(p)
    states = [(0.9, np.array([0.3, -0.2])), (-0.4, np.array([-0.5, 0.6]))]
    g = int(np.nonzero(~d.skel.is_boundary)[0][0])
    rhs, Dsum, nrm0 = 0.0, 0.0, None
    for e in range(2):
        A, B, C, D, _ = hdg.element_system(d, e, 7.0)
        q = d.elem_quad(e)
        c0 = np.einsum("q,qi->i", q.wq, q.phi) / abs(q.det)    # coefficients of the constant 1
        pe, ve = states[e]
        ue = np.concatenate([ve[0] * c0, ve[1] * c0, pe * c0])
        f = int(np.nonzero(d.skel.elem_faces[e] == g)[0][0])
        nf = dim_p(int(d.face_k[g]), 1)
        rows = slice(f * nf, (f + 1) * nf)
        rhs = rhs + C[rows] @ ue
        Dsum = Dsum + D[rows, rows]
        if e == 0:
            nrm0 = q.faces[f]["n"]
    lam = np.linalg.solve(Dsum, -rhs)
    st, _ = rule_for_degree(1, 6)
    vals = pkd_eval(int(d.face_k[g]), st) @ lam
    # exact Riemann state: the characteristic p + Z u_n leaves element 0 (normal n0), p - Z u_n
    # leaves element 1; Z = rho c
    Z0, Z1 = 1.3 * 0.7, 0.8 * 1.9
    (p0, v0), (p1, v1) = states
    M = np.array([[1.0, Z0], [1.0, -Z1]])
    pstar, _ = np.linalg.solve(M, [p0 + Z0 * (v0 @ nrm0), p1 - Z1 * (v1 @ nrm0)])
    return vals, pstar


def test_acoustic_trace_is_exact_riemann_state():
    vals, pstar = _two_triangle_trace()
    assert np.abs(vals - pstar).max() <= 1e-12 * abs(pstar)


def test_riemann_pin_detects_a_wrong_impedance(monkeypatch):
    """Planted mistake: tau = rho c instead of 1/(rho c) moves the trace off the Riemann state."""
    orig = ophys.stabilisation

    def wrong(physics, par):
        return par[0] * par[1] if physics == "acoustic" else orig(physics, par)
    monkeypatch.setattr(ophys, "stabilisation", wrong)
    vals, pstar = _two_triangle_trace()
    assert np.abs(vals - pstar).max() > 1e-2


def test_stabilisation_equals_paper_experiment_values():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "stabilisation_paper.txt")) if not l.startswith("#")]
    assert rows
    for phys, p0, p1, p2, val in rows:
        assert abs(ophys.stabilisation(phys, [float(p0), float(p1), float(p2)]) - float(val)) < 1e-14


# ----------------------------------------------------------------------------- helpers of hdg
@pytest.mark.parametrize("cfg,kw,deg", [(2, dict(n=2, k=3), 3), (4, dict(nxyz=(2, 2, 2)), 1)])
def test_point_source_columns_reproduce_point_values(cfg, kw, deg):
    """Column s of the point-source right-hand side holds phi_i(x_s) in the pressure block of
    the element containing x_s, so for any q in P_k, sum_i F_is (q, phi_i)_K / |J| = q(x_s)."""
    p = make_problem(cfg, **kw)
    d = hdg.make_discretisation(p)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.05, 0.95, size=(7, 3))
    F = hdg.point_source_rhs(d, pts)
    coef = rng.standard_normal((deg + 1,) * 3)

    def qpoly(x):
        return np.polynomial.polynomial.polyval3d(x[:, 0], x[:, 1], x[:, 2], coef * (
            np.add.outer(np.add.outer(np.arange(deg + 1), np.arange(deg + 1)), np.arange(deg + 1)) <= deg))
    cq = hdg.project_volume(d, lambda x, t: np.stack([0 * x[:, 0]] * 3 + [qpoly(x)], 1))
    got = F.T @ cq
    assert np.allclose(got, qpoly(pts), rtol=1e-11, atol=1e-11 * np.abs(qpoly(pts)).max())
    assert np.all(np.count_nonzero(F, axis=0) <= dim_p(max(int(x) for x in p.degree), 3))


def test_l2_norm_closed_form_and_quadrature():
    # the constant 1 on the (jittered) unit square and unit cube has norm 1
    for cfg, kw in [(1, dict(n=3, k=2)), (2, dict(n=2, k=2))]:
        p = make_problem(cfg, **kw)
        d = hdg.make_discretisation(p)
        m = d.m_local
        u = hdg.project_volume(d, lambda x, t: np.concatenate(
            [np.zeros((x.shape[0], m - 1)), np.ones((x.shape[0], 1))], 1))
        assert abs(hdg.l2_norm_fields(d, u, [m - 1]) - 1.0) < 1e-13
        assert hdg.l2_norm_fields(d, u, list(range(m - 1))) == 0.0
        # energy 1/2 (u, Mw u) of the pressure p = 1 is 1/2 int p^2 / (rho c^2)
        expect = 0.5 * sum(abs(np.linalg.det((p.xyz[ev[1:]] - p.xyz[ev[0]]).T)) / np.prod(range(1, d.dim + 1))
                           / (par[0] * par[1] ** 2) for ev, par in zip(p.elem_vert, p.elem_par))
        assert abs(hdg.energy(d, u) - expect) < 1e-13 * expect
    # random fields of variable degree: the coefficient norm equals the quadrature of the field
    p = make_problem(4, nxyz=(2, 2, 1))
    d = hdg.make_discretisation(p)
    u = np.random.default_rng(2).standard_normal(d.loc_off[-1])
    for comps in ([0, 1, 2], [3], [1, 3]):
        ref = hdg.l2_error_fields(d, u, lambda x, t: np.zeros((x.shape[0], 4)), 0.0, comps)
        assert abs(hdg.l2_norm_fields(d, u, comps) - ref) <= 1e-12 * ref


# ----------------------------------------------------------------------------- GLM-Maxwell
@pytest.mark.parametrize("k", [1, 2])
def test_glm_condensed_equals_full_and_schur_definite(k):
    p = make_problem(5, n=1, k=k)
    p.physics = "maxwell_glm"
    d = hdg.make_discretisation(p)
    rng = np.random.default_rng(k)
    f = rng.standard_normal(d.loc_off[-1])
    lb = rng.standard_normal(d.tr_off[-1]) * hdg.boundary_trace_mask(d)
    u, lam, cond = hdg.solve_stage(d, 29.0, f, lb)
    uf, lf = hdg.solve_full(d, 29.0, f, lb)
    assert np.linalg.norm(u - uf) <= 1e-12 * np.linalg.norm(uf)
    assert np.linalg.norm(lam - lf) <= 1e-12 * np.linalg.norm(lf)
    for Ke in cond.Ke[:4]:
        assert np.abs(Ke - Ke.T).max() <= 1e-12 * np.abs(Ke).max()
        assert np.all(np.linalg.eigvalsh(Ke) > 0)


def test_glm_energy_non_increasing():
    """Energy identity of section 5.3 with phi: 1/2 (eps E, E) + 1/2 (mu H, H) + 1/(2 alpha_1^2)
    (phi, phi) does not grow without sources and boundary data."""
    p = make_problem(5, n=1, k=2)
    p.physics = "maxwell_glm"
    d = hdg.make_discretisation(p)
    u = np.random.default_rng(3).standard_normal(d.loc_off[-1])
    zero = np.zeros(d.tr_off[-1])
    E0 = hdg.energy(d, u)
    for s in range(3):
        u = hdg.dirk_step(d, u, s * 0.05, 0.05, lambda t: zero)
        E1 = hdg.energy(d, u)
        assert E1 <= E0 * (1 + 1e-13)
        E0 = E1


def _cavity(x, t, omega=1.0):
    """Standing wave of the cavity experiment of section 5.4: [H_1,H_2,H_3, E_1,E_2,E_3]."""
    sx, sy, sz = (np.sin(omega * x[:, i]) for i in range(3))
    cx, cy, cz = (np.cos(omega * x[:, i]) for i in range(3))
    E = np.stack([sy * sz, sx * sz, sy * sx], 1) * np.sin(omega * t)
    H = np.stack([(cy * sx - cz * sx), (cz * sy - cx * sy), (cx * sz - cy * sz)], 1) * np.cos(omega * t)
    return np.concatenate([H, E], 1)


def _maxwell_stage_errors(physics, ns, k, a=8.0, t=0.7):
    """Single implicit stage whose exact solution is the cavity field at time t (eps = 2,
    mu = 1, sigma = 0, tau = 2): source s = a M u_ex + L u_ex from the strong form."""
    eps, mu = 2.0, 1.0
    errs = []
    for n in ns:
        p = make_problem(5, n=n, k=k)
        p.physics = physics
        p.elem_par[:] = [eps, mu, 0.0]
        d = hdg.make_discretisation(p)
        glm = physics == "maxwell_glm"

        def U(x):
            u = _cavity(x, t)
            return np.concatenate([u, np.zeros((x.shape[0], 1))], 1) if glm else u

        def src(x, tt=0.0):
            u = U(x)
            g = _grad_fd(U, x)

            def curl(off):
                return np.stack([g[:, off + 2, 1] - g[:, off + 1, 2], g[:, off + 0, 2] - g[:, off + 2, 0],
                                 g[:, off + 1, 0] - g[:, off + 0, 1]], 1)
            sH = a * mu * u[:, :3] + curl(3)
            sE = a * eps * u[:, 3:6] - curl(0)
            out = [sH, sE]
            if glm:
                out.append((g[:, 3, 0] + g[:, 4, 1] + g[:, 5, 2])[:, None])   # phi = 0: div E
            return np.concatenate(out, 1)
        f = hdg.load_vector(d, src)
        lb = hdg.project_boundary(d, lambda x, tt: U(x)[:, 3:6])
        u, _, _ = hdg.solve_stage(d, a, f, lb)
        groups = [[0, 1, 2], [3, 4, 5]] + ([[6]] if glm else [])
        errs.append([hdg.l2_error_fields(d, u, lambda x, tt: U(x), 0.0, gq) for gq in groups])
    return np.asarray(errs), _rates(errs, ns)


@pytest.mark.parametrize("k,bar", [(1, 1.7), (2, 2.35)])
def test_cavity_fields_optimal_rates(k, bar):
    """Tables tab1-tab2 report optimal L2 rates (about k+1) for H and E on the cavity; the same
    fields as a manufactured stage on the jittered Kuhn meshes."""
    errs, rates = _maxwell_stage_errors("maxwell", [2, 3, 4] if k == 1 else [2, 3], k)
    assert np.all(rates[-1] > bar), (errs, rates)


def test_glm_cavity_rates_include_phi():
    """Table tab4: phi_h converges at least at the optimal rate (the exact phi is zero)."""
    errs, rates = _maxwell_stage_errors("maxwell_glm", [2, 3, 4], 1)
    assert np.all(rates[-1, :2] > 1.7), (errs, rates)
    assert rates[-1, 2] > 1.7 and errs[-1, 2] < errs[-1, 1], (errs, rates)


# ----------------------------------------------------------------------------- rates
def test_manufactured_acoustic3d_k3_rates():
    """The benchmark degree: k = 3 in 3D, errors O(h^4) (pre-asymptotic on these meshes)."""
    errs, rates = _manufactured_errors(2, [2, 3, 4], 3, comps_groups=[[0, 1, 2], [3]])
    assert np.all(rates[-1] > 3.3), (errs, rates)


@pytest.mark.parametrize("cfg,k,ns,bar", [(5, 1, [2, 3, 4], 1.7), (3, 1, [2, 3, 4], 1.8),
                                          (3, 2, [2, 3], 2.7), (5, 2, [2, 3], 2.4)])
def test_manufactured_rates_tight(cfg, k, ns, bar):
    groups = {5: [[0, 1, 2], [3, 4, 5]], 3: [list(range(6)), [6, 7, 8]]}[cfg]
    errs, rates = _manufactured_errors(cfg, ns, k, comps_groups=groups)
    assert np.all(rates[-1] > bar), (errs, rates)


# ----------------------------------------------------------------------------- counting
def test_eppler_boundary_faces_from_printed_counts():
    """Each printed count / dim P_4(face) gives the faces F; with 4 faces per tetrahedron and
    interior faces shared, the boundary has 2F - 4 N_e faces: a positive even number (a closed
    triangulated surface has 3 F_b = 2 E_b) and a small fraction of the faces."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "eppler_meshes.txt")) if not l.startswith("#")]
    prev = 0
    for mesh, k, ne, nglob, m in rows:
        faces = int(nglob) // dim_p(int(k), 2)
        nb = 2 * faces - 4 * int(ne)
        assert nb > 0 and nb % 2 == 0 and nb < 0.05 * faces
        assert nb > prev          # uniform refinement grows the surface mesh too
        prev = nb
