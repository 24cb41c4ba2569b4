// Reference-element tables (host, FP64).  See reftab.h.
//
// Orthonormal Jacobi polynomials come from the classical three-term recurrence; Gauss-Jacobi
// nodes and weights from the Golub-Welsch eigenvalue problem of the Jacobi matrix (solved
// with cyclic Jacobi rotations); the PKD basis and its gradient from the collapsed-coordinate
// factorisation phi = c * A(x1, 1-x2-x3) * B(x2, 1-x3) * C(x3) with every factor polynomial.
#include "reftab.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace hdg {

int dim_p(int k, int d) {
    if (d == 0) return 1;
    if (d == 1) return k + 1;
    if (d == 2) return (k + 1) * (k + 2) / 2;
    return (k + 1) * (k + 2) * (k + 3) / 6;
}

// P_n^{(a,b)}(x), unnormalised, and its derivative.
static void jacobi_raw(int n, double a, double b, double x, double* p, double* dp) {
    auto eval = [&](int m, double aa, double bb) {
        if (m < 0) return 0.0;
        double p0 = 1.0;
        if (m == 0) return p0;
        double p1 = 0.5 * (aa - bb) + 0.5 * (aa + bb + 2.0) * x;
        for (int j = 2; j <= m; ++j) {
            double s = 2.0 * j + aa + bb;
            double c1 = 2.0 * j * (j + aa + bb) * (s - 2.0);
            double c2 = (s - 1.0) * (s * (s - 2.0) * x + aa * aa - bb * bb);
            double c3 = 2.0 * (j + aa - 1.0) * (j + bb - 1.0) * s;
            double p2 = (c2 * p1 - c3 * p0) / c1;
            p0 = p1;
            p1 = p2;
        }
        return p1;
    };
    *p = eval(n, a, b);
    if (dp) *dp = (n == 0) ? 0.0 : 0.5 * (n + a + b + 1.0) * eval(n - 1, a + 1.0, b + 1.0);
}

static double jacobi_norm(int n, double a, double b) {
    double lg = (a + b + 1.0) * std::log(2.0) - std::log(2.0 * n + a + b + 1.0) +
                std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) - std::lgamma(n + a + b + 1.0) -
                std::lgamma(n + 1.0);
    return std::sqrt(std::exp(lg));
}

// orthonormal w.r.t. (1-x)^a (1+x)^b on [-1,1]
static void jacobi_on(int n, double a, double b, double x, double* p, double* dp) {
    double s = 1.0 / jacobi_norm(n, a, b);
    jacobi_raw(n, a, b, x, p, dp);
    *p *= s;
    if (dp) *dp *= s;
}

static inline double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

void pkd_eval(int d, int k, const double* xi, double* val, double* grad) {
    int idx = 0;
    if (d == 1) {
        for (int i = 0; i <= k; ++i, ++idx) {
            double h, dh;
            jacobi_on(i, 0, 0, 2.0 * xi[0] - 1.0, &h, &dh);
            val[idx] = std::sqrt(2.0) * h;
            if (grad) grad[idx] = 2.0 * std::sqrt(2.0) * dh;
        }
        return;
    }
    if (d == 2) {
        const double x1 = xi[0], x2 = xi[1];
        const double w = 1.0 - x2;
        const double a = (w > 1e-14) ? 2.0 * x1 / w - 1.0 : -1.0;
        const double b = 2.0 * x2 - 1.0;
        for (int s = 0; s <= k; ++s)
            for (int i = 0; i <= s; ++i, ++idx) {
                int j = s - i;
                double h1, dh1, h2, dh2;
                jacobi_on(i, 0, 0, a, &h1, &dh1);
                jacobi_on(j, 2 * i + 1, 0, b, &h2, &dh2);
                double sc = 2.0 * std::sqrt(2.0) * ipow(2.0, i);
                double A = h1 * ipow(w, i);
                val[idx] = sc * A * h2;
                if (grad) {
                    double dA1 = (i > 0) ? 2.0 * dh1 * ipow(w, i - 1) : 0.0;
                    double dAw = (i > 0) ? ipow(w, i - 1) * (-(a + 1.0) * dh1 + i * h1) : 0.0;
                    grad[idx * 2 + 0] = sc * dA1 * h2;
                    grad[idx * 2 + 1] = sc * (-dAw * h2 + A * 2.0 * dh2);
                }
            }
        return;
    }
    const double x1 = xi[0], x2 = xi[1], x3 = xi[2];
    const double w = 1.0 - x2 - x3, v = 1.0 - x3;
    const double a = (w > 1e-14) ? 2.0 * x1 / w - 1.0 : -1.0;
    const double b = (v > 1e-14) ? 2.0 * x2 / v - 1.0 : -1.0;
    const double c = 2.0 * x3 - 1.0;
    for (int s = 0; s <= k; ++s)
        for (int i = 0; i <= s; ++i)
            for (int j = 0; j <= s - i; ++j, ++idx) {
                int l = s - i - j;
                double h1, dh1, h2, dh2, h3, dh3;
                jacobi_on(i, 0, 0, a, &h1, &dh1);
                jacobi_on(j, 2 * i + 1, 0, b, &h2, &dh2);
                jacobi_on(l, 2 * i + 2 * j + 2, 0, c, &h3, &dh3);
                double sc = 8.0 * ipow(2.0, 2 * i + j);
                double A = h1 * ipow(w, i), B = h2 * ipow(v, j), C = h3;
                val[idx] = sc * A * B * C;
                if (grad) {
                    double dA1 = (i > 0) ? 2.0 * dh1 * ipow(w, i - 1) : 0.0;
                    double dAw = (i > 0) ? ipow(w, i - 1) * (-(a + 1.0) * dh1 + i * h1) : 0.0;
                    double dB2 = (j > 0) ? 2.0 * dh2 * ipow(v, j - 1) : 0.0;
                    double dBv = (j > 0) ? ipow(v, j - 1) * (-(b + 1.0) * dh2 + j * h2) : 0.0;
                    double dC3 = 2.0 * dh3;
                    grad[idx * 3 + 0] = sc * dA1 * B * C;
                    grad[idx * 3 + 1] = sc * (-dAw * B * C + A * dB2 * C);
                    grad[idx * 3 + 2] = sc * (-dAw * B * C - A * dBv * C + A * B * dC3);
                }
            }
}

// symmetric eigenproblem by cyclic Jacobi rotations (small dense matrices only)
static void sym_eig(int n, std::vector<double>& Amat, std::vector<double>& V) {
    V.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += Amat[p * n + q] * Amat[p * n + q];
        if (off < 1e-32) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = Amat[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = Amat[p * n + p], aqq = Amat[q * n + q];
                double theta = 0.5 * (aqq - app) / apq;
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < n; ++r) {
                    double arp = Amat[r * n + p], arq = Amat[r * n + q];
                    Amat[r * n + p] = cs * arp - sn * arq;
                    Amat[r * n + q] = sn * arp + cs * arq;
                }
                for (int r = 0; r < n; ++r) {
                    double apr = Amat[p * n + r], aqr = Amat[q * n + r];
                    Amat[p * n + r] = cs * apr - sn * aqr;
                    Amat[q * n + r] = sn * apr + cs * aqr;
                }
                for (int r = 0; r < n; ++r) {
                    double vrp = V[r * n + p], vrq = V[r * n + q];
                    V[r * n + p] = cs * vrp - sn * vrq;
                    V[r * n + q] = sn * vrp + cs * vrq;
                }
            }
    }
}

// Gauss-Jacobi rule on [0,1] for the weight (1-u)^alpha (beta = 0), q points.
static void gauss_jacobi01(int q, double alpha, std::vector<double>& x, std::vector<double>& w) {
    const double be = 0.0, al = alpha;
    std::vector<double> T(q * q, 0.0);
    for (int n = 0; n < q; ++n) {
        double s = 2.0 * n + al + be;
        T[n * q + n] = (n == 0) ? (be - al) / (al + be + 2.0) : (be * be - al * al) / (s * (s + 2.0));
        if (n + 1 < q) {
            int m = n + 1;
            double sm = 2.0 * m + al + be;
            double num = 4.0 * m * (m + al) * (m + be) * (m + al + be);
            double den = sm * sm * (sm + 1.0) * (sm - 1.0);
            double off = std::sqrt(num / den);
            T[n * q + m] = T[m * q + n] = off;
        }
    }
    std::vector<double> V;
    sym_eig(q, T, V);
    double mu0 = std::exp((al + be + 1.0) * std::log(2.0) + std::lgamma(al + 1.0) + std::lgamma(be + 1.0) -
                          std::lgamma(al + be + 2.0));
    std::vector<std::pair<double, double>> nw(q);
    for (int i = 0; i < q; ++i) nw[i] = {T[i * q + i], mu0 * V[0 * q + i] * V[0 * q + i]};
    std::sort(nw.begin(), nw.end());
    x.resize(q);
    w.resize(q);
    for (int i = 0; i < q; ++i) {
        x[i] = 0.5 * (nw[i].first + 1.0);
        w[i] = nw[i].second / std::pow(2.0, al + 1.0);
    }
}

void simplex_quadrature(int d, int q, std::vector<double>& pts, std::vector<double>& wts) {
    pts.clear();
    wts.clear();
    if (d == 0) {
        wts.push_back(1.0);
        return;
    }
    std::vector<double> x0, w0, x1, w1, x2, w2;
    gauss_jacobi01(q, 0.0, x0, w0);
    if (d == 1) {
        for (int i = 0; i < q; ++i) {
            pts.push_back(x0[i]);
            wts.push_back(w0[i]);
        }
        return;
    }
    gauss_jacobi01(q, 1.0, x1, w1);
    if (d == 2) {
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                double u = x1[i], v = x0[j];
                pts.push_back(u);
                pts.push_back((1.0 - u) * v);
                wts.push_back(w1[i] * w0[j]);
            }
        return;
    }
    gauss_jacobi01(q, 2.0, x2, w2);
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int l = 0; l < q; ++l) {
                double u = x2[i], v = x1[j], t = x0[l];
                pts.push_back(u);
                pts.push_back((1.0 - u) * v);
                pts.push_back((1.0 - u) * (1.0 - v) * t);
                wts.push_back(w2[i] * w1[j] * w0[l]);
            }
}

int n_face_perms(int d) { return d == 3 ? 6 : (d == 2 ? 2 : 1); }

void face_perm(int d, int p, int* perm) {
    static const int P3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int P2[2][2] = {{0, 1}, {1, 0}};
    if (d == 3)
        for (int i = 0; i < 3; ++i) perm[i] = P3[p][i];
    else if (d == 2)
        for (int i = 0; i < 2; ++i) perm[i] = P2[p][i];
    else
        perm[0] = 0;
}

void local_face_vertices(int d, int f, int* lv) {
    int c = 0;
    for (int v = 0; v <= d; ++v)
        if (v != f) lv[c++] = v;
}

static void ref_vertex(int d, int v, double* x) {
    for (int r = 0; r < d; ++r) x[r] = 0.0;
    if (v > 0) x[v - 1] = 1.0;
}

// map reference-face coordinates s[d-1] to the element reference point for face f, perm p
static void face_point(int d, int f, int p, const double* s, double* xi) {
    int lv[3], perm[3];
    local_face_vertices(d, f, lv);
    face_perm(d, p, perm);
    double V[3][3];
    for (int m = 0; m < d; ++m) ref_vertex(d, lv[perm[m]], V[m]);
    for (int r = 0; r < d; ++r) {
        double x = V[0][r];
        for (int m = 1; m < d; ++m) x += (V[m][r] - V[0][r]) * s[m - 1];
        xi[r] = x;
    }
}

void build_ref_tables(int d, int k, RefTables& T) {
    T.d = d;
    T.k = k;
    T.N = dim_p(k, d);
    T.nf = d + 1;
    const int N = T.N;
    std::vector<double> pts, wts;
    simplex_quadrature(d, k + 2, pts, wts);
    const int nq = (int)wts.size();
    T.Sr.assign(d * N * N, 0.0);
    std::vector<double> val(N), grad(N * d);
    for (int q = 0; q < nq; ++q) {
        pkd_eval(d, k, &pts[q * d], val.data(), grad.data());
        for (int r = 0; r < d; ++r)
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) T.Sr[(r * N + i) * N + j] += wts[q] * val[i] * grad[j * d + r];
    }
    // face mass tables
    std::vector<double> fp, fw;
    simplex_quadrature(d - 1, k + 2, fp, fw);
    const int nfq = (int)fw.size();
    T.Mf.assign((d + 1) * N * N, 0.0);
    for (int f = 0; f <= d; ++f)
        for (int q = 0; q < nfq; ++q) {
            double xi[3];
            face_point(d, f, 0, &fp[q * (d - 1)], xi);
            pkd_eval(d, k, xi, val.data(), nullptr);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) T.Mf[(f * N + i) * N + j] += fw[q] * val[i] * val[j];
        }
    // all products Sr Ss^T
    T.Tfull.assign(d * d * N * N, 0.0);
    for (int r = 0; r < d; ++r)
        for (int s = 0; s < d; ++s)
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) {
                    double acc = 0.0;
                    for (int m = 0; m < N; ++m) acc += T.Sr[(r * N + i) * N + m] * T.Sr[(s * N + j) * N + m];
                    T.Tfull[((r * d + s) * N + i) * N + j] = acc;
                }
    // symmetric products Sr Ss^T
    int npair = d * (d + 1) / 2;
    T.Tsym.assign(npair * N * N, 0.0);
    int c = 0;
    for (int r = 0; r < d; ++r)
        for (int s = r; s < d; ++s, ++c)
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) {
                    double acc = 0.0;
                    for (int m = 0; m < N; ++m) {
                        acc += T.Sr[(r * N + i) * N + m] * T.Sr[(s * N + j) * N + m];
                        if (s != r) acc += T.Sr[(s * N + i) * N + m] * T.Sr[(r * N + j) * N + m];
                    }
                    T.Tsym[(c * N + i) * N + j] = acc;
                }
}

void build_face_tables(int d, int k, int kF, RefFaceTables& E) {
    E.d = d;
    E.k = k;
    E.kF = kF;
    E.N = dim_p(k, d);
    E.NF = dim_p(kF, d - 1);
    E.nperm = n_face_perms(d);
    const int N = E.N, NF = E.NF;
    std::vector<double> fp, fw;
    simplex_quadrature(d - 1, std::max(k, kF) + 2, fp, fw);
    const int nfq = (int)fw.size();
    E.E.assign((d + 1) * E.nperm * N * NF, 0.0);
    std::vector<double> val(N), psi(NF);
    for (int f = 0; f <= d; ++f)
        for (int p = 0; p < E.nperm; ++p)
            for (int q = 0; q < nfq; ++q) {
                double xi[3];
                face_point(d, f, p, &fp[q * (d - 1)], xi);
                pkd_eval(d, k, xi, val.data(), nullptr);
                pkd_eval(d - 1, kF, &fp[q * (d - 1)], psi.data(), nullptr);
                double* Eb = &E.E[((f * E.nperm + p) * N) * NF];
                for (int i = 0; i < N; ++i)
                    for (int l = 0; l < NF; ++l) Eb[i * NF + l] += fw[q] * val[i] * psi[l];
            }
}

}  // namespace hdg
