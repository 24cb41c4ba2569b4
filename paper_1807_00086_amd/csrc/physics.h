// Local stage equations of each physics, as implemented by the condensation kernels.
//
// Every implicit stage (section 2.3.2 written as in section 2.4.1) is, per element K,
//     A u + B lam = f,     C u + D lam = g,      A = a Mw + L,
// with a = d_ii / dt, Mw the time-derivative weight of the DAE M du/dt + f(u,v,t) = 0 and
// lam the element's face traces.  The trace rows of all elements sharing a face add up to
// the jump condition of the numerical flux; on Dirichlet faces lam is prescribed.
//
// Acoustics (velocity v, pressure p, trace p_hat; numerical flux
// v_hat.n = v.n + tau (p - p_hat) with the impedance choice tau = 1/(rho c), following the
// dimensional argument of section 4.1.3):
//   (a rho v, w) - (p, div w) + <p_hat, w.n>          = (a rho v*, w)
//   (a/(rho c^2) p, q) + (div v, q) + <tau (p - p_hat), q> = (a/(rho c^2) p*, q) + (s, q)
//   sum_K <v.n + tau (p - p_hat), mu>_F = 0
// Elastodynamics (section 4.1.2 in velocity / symmetric-stress form, flux
// sigma_hat n = sigma n - S (v - v_hat), S = 2 rho c_s I as in section 4.3; face term with
// the sign for which the energy identity of section 4.2.3 holds):
//   (a Acomp sigma, tau) + (v, div tau) - <v_hat, tau n>             = (a Acomp sigma*, tau)
//   (a rho v, w) + (sigma, grad w) - <sigma n - S (v - v_hat), w>    = (a rho v*, w)
//   sum_K <sigma n - S (v - v_hat), mu>_F = 0
// Maxwell (section 5.2 without the GLM multiplier, Ohmic current J = sigma_c E, tau = 2):
//   (a mu H, w) + (E, curl w) + <E_hat^t, w x n>                          = (a mu H*, w)
//   ((a eps + sigma_c) E, v) - (H, curl v) - <H^t - tau (E - E_hat^t) x n, v x n> = (a eps E*, v)
//   sum_K <n x H_hat^t, mu>_F = 0
//
// Elimination order (LU without pivoting of A, flux-like block first).  The leading block of
// A couples no basis functions of different index (Mw is |J| times a small matrix over
// components, orthonormal basis), so its elimination is closed form and only the Schur block
//   S = A22 - A21 A11^{-1} A12
// is factored densely.  This is the same L and U that a dense no-pivot LU of A produces; the
// structural zeros of A11 are skipped.
#pragma once

namespace hdg {

__host__ __device__ constexpr int dimp(int k, int d) {
    return d == 1 ? k + 1 : (d == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6);
}

}  // namespace hdg
