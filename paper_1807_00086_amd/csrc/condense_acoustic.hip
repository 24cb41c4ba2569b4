// Acoustic HDG condensation and recovery kernels for gfx950.
//
// Per element (unknowns u = [v_1..v_d, p], trace p_hat on the d+1 faces):
//   A = [[a rho |J| I,  -Q^T], [Q, a|J|/(rho c^2) I + tau sum_f s_f Mf_f]],
//   Q_x = |J| sum_r G_rx Sr_r  (Q_x[i][j] = (phi_i, d phi_j / d x_x)_K),
//   B = [[n_fx s_f E_f], [-tau s_f E_f]],  C = [[n_fx s_f E_f^T, tau s_f E_f^T]],
//   D = -tau s_f I on each face block,
// where G = J^{-1}, s_f the face measure over the reference-face measure, E_f the oriented
// volume-trace face table.  The velocity block is diagonal, so LU without pivoting reduces
// to the pressure Schur block
//   S = a|J|/(rho c^2) I + tau sum_f s_f Mf_f + (|J| / (a rho)) sum_{r,s} (G G^T)_rs Sr_r Sr_s^T,
// (the last sum uses the precomputed symmetric products), followed by
//   [Z_p | z_p] = S^{-1} [B~ | f~],  B~_f = -s_f (tau I + (1/(a rho)) sum_r beta_fr Sr_r) E_f,
//   beta_fr = sum_x G_rx n_fx,  f~ = f_p - (1/(a rho)) sum_r Sr_r (sum_x G_rx f_vx),
//   Z_v,x = (1/(a rho)) (n_fx s_f E_f / |J| + sum_r G_rx Sr_r^T Z_p)  (same for z_v),
//   K_e = D - C Z,  r_e = -C z.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "physics.h"

namespace hdg {

namespace {

constexpr int NT = 256;

template <int D, int K, int R, typename T>
struct AcDims {
    static constexpr int N = dimp(K, D);
    static constexpr int NF = dimp(K, D - 1);
    static constexpr int NFACE = D + 1;
    static constexpr int TT = NFACE * NF;          // trace unknowns per element
    static constexpr int C = TT + R;               // columns of [B~ | f~]
    static constexpr int NLOC = (D + 1) * N;       // local unknowns per element
    static constexpr int NPERM = (D == 3) ? 6 : 2;
    static constexpr int NPAIR = D * (D + 1) / 2;
    static constexpr int WSZ = NFACE * N * N;      // per-face W_f scratch
    static constexpr int YSZ = D * N * C;
    static constexpr int YW = (WSZ > YSZ) ? WSZ : YSZ;
};

template <int D, int K, int R, typename T>
__global__ __launch_bounds__(NT) void condense_acoustic_kernel(
    int64_t ne, double a_in, const double* __restrict__ geom, const int32_t* __restrict__ eperm,
    const T* __restrict__ Sr, const T* __restrict__ Mf, const T* __restrict__ Tsym,
    const T* __restrict__ Ef, const double* __restrict__ f_loc, T* __restrict__ Ke,
    T* __restrict__ re, T* __restrict__ Zt, T* __restrict__ zout, T* __restrict__ LUout,
    int* __restrict__ status) {
    using Dm = AcDims<D, K, R, T>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, TT = Dm::TT, C = Dm::C;
    constexpr int NLOC = Dm::NLOC, NPERM = Dm::NPERM, NPAIR = Dm::NPAIR;

    __shared__ T S[N * N];
    __shared__ T X[N * C];
    __shared__ T YW[Dm::YW];          // W_f (phase 1) then Y_r = Sr_r^T X (phase 3)
    __shared__ T P[N * C];
    __shared__ T El[NFACE * N * NF];  // oriented face tables of this element
    __shared__ T FV[D * N * R];       // velocity right-hand side
    __shared__ T GRv[D * N * R];      // sum_x G_rx f_vx
    __shared__ double geo[GEOM_STRIDE];

    const int tid = threadIdx.x;
    const T a = (T)a_in;

    for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
        // ------------------------------------------------------------------ load
        if (tid < GEOM_STRIDE) geo[tid] = geom[e * GEOM_STRIDE + tid];
        for (int idx = tid; idx < NFACE * N * NF; idx += NT) {
            int f = idx / (N * NF), rem = idx % (N * NF);
            int p = eperm[e * NFACE + f];
            El[idx] = Ef[(size_t)(f * NPERM + p) * N * NF + rem];
        }
        const double* fe = f_loc + (size_t)e * NLOC * R;
        for (int idx = tid; idx < D * N * R; idx += NT) FV[idx] = (T)fe[idx];
        for (int idx = tid; idx < N * R; idx += NT) {
            int i = idx / R, q = idx % R;
            X[i * C + TT + q] = (T)fe[D * N * R + idx];
        }
        __syncthreads();

        const T J = (T)geo[0];
        T G[D][D];
        for (int r = 0; r < D; ++r)
            for (int x = 0; x < D; ++x) G[r][x] = (T)geo[1 + r * D + x];
        T sf[NFACE], nf[NFACE][D];
        for (int f = 0; f < NFACE; ++f) {
            sf[f] = (T)geo[1 + D * D + f];
            for (int x = 0; x < D; ++x) nf[f][x] = (T)geo[1 + D * D + NFACE + f * D + x];
        }
        const T rho = (T)geo[GEO_PAR], cc = (T)geo[GEO_PAR + 1];
        const T tau = (T)geo[GEO_STAB];
        const T arho = a * rho;
        const T inv_arho = T(1) / arho;
        const T alpha_p = a * J / (rho * cc * cc);
        T gam[NPAIR];
        {
            int c = 0;
            for (int r = 0; r < D; ++r)
                for (int s = r; s < D; ++s, ++c) {
                    T g = 0;
                    for (int x = 0; x < D; ++x) g += G[r][x] * G[s][x];
                    gam[c] = g;
                }
        }
        T beta[NFACE][D];
        for (int f = 0; f < NFACE; ++f)
            for (int r = 0; r < D; ++r) {
                T b = 0;
                for (int x = 0; x < D; ++x) b += G[r][x] * nf[f][x];
                beta[f][r] = b;
            }

        // ------------------------------------------------------------------ phase 1: form
        const T cT = J * inv_arho;
        for (int idx = tid; idx < N * N; idx += NT) {
            int i = idx / N, j = idx % N;
            T s = (i == j) ? alpha_p : T(0);
            T fm = 0;
            for (int f = 0; f < NFACE; ++f) fm += sf[f] * Mf[f * N * N + idx];
            s += tau * fm;
            T tt = 0;
            for (int c = 0; c < NPAIR; ++c) tt += gam[c] * Tsym[c * N * N + idx];
            S[idx] = s + cT * tt;
        }
        // W_f = tau I + (1/(a rho)) sum_r beta_fr Sr_r
        for (int idx = tid; idx < NFACE * N * N; idx += NT) {
            int f = idx / (N * N), ij = idx % (N * N);
            T w = 0;
            for (int r = 0; r < D; ++r) w += beta[f][r] * Sr[r * N * N + ij];
            w *= inv_arho;
            if (ij / N == ij % N) w += tau;
            YW[idx] = w;
        }
        // g_r = sum_x G_rx f_vx
        for (int idx = tid; idx < D * N * R; idx += NT) {
            int r = idx / (N * R), iq = idx % (N * R);
            T g = 0;
            for (int x = 0; x < D; ++x) g += G[r][x] * FV[x * N * R + iq];
            GRv[idx] = g;
        }
        __syncthreads();
        // B~ columns and f~
        for (int idx = tid; idx < N * C; idx += NT) {
            int i = idx / C, c = idx % C;
            if (c < TT) {
                int f = c / NF, l = c % NF;
                const T* W = &YW[f * N * N + i * N];
                const T* E = &El[f * N * NF + l];
                T acc = 0;
                for (int j = 0; j < N; ++j) acc += W[j] * E[j * NF];
                X[idx] = -sf[f] * acc;
            } else {
                int q = c - TT;
                T acc = 0;
                for (int r = 0; r < D; ++r) {
                    const T* Srow = &Sr[r * N * N + i * N];
                    for (int j = 0; j < N; ++j) acc += Srow[j] * GRv[(r * N + j) * R + q];
                }
                X[idx] = X[idx] - inv_arho * acc;
            }
        }
        __syncthreads();

        // ------------------------------------------------------------------ phase 2: LU(S), solve
        // pivots below 64 N eps of the largest diagonal entry, or non-finite, are reported
        T dmax = 0;
        for (int i = 0; i < N; ++i) dmax = fmax(dmax, fabs(S[i * N + i]));
        const T ptol = T(64 * N) * (sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7)) * dmax;
        for (int j = 0; j < N; ++j) {
            const T piv = S[j * N + j];
            if (tid == 0 && !(fabs(piv) > ptol && piv - piv == T(0))) atomicOr(status, 1);
            const T ipiv = T(1) / piv;
            for (int i = j + 1 + tid; i < N; i += NT) S[i * N + j] *= ipiv;
            __syncthreads();
            const int m = N - j - 1;
            for (int idx = tid; idx < m * m; idx += NT) {
                int i = j + 1 + idx / m, c = j + 1 + idx % m;
                S[i * N + c] -= S[i * N + j] * S[j * N + c];
            }
            __syncthreads();
        }
        if (LUout) {
            for (int idx = tid; idx < N * N; idx += NT) LUout[(size_t)e * N * N + idx] = S[idx];
        }
        // forward (unit lower)
        for (int j = 0; j < N - 1; ++j) {
            const int m = N - j - 1;
            for (int idx = tid; idx < m * C; idx += NT) {
                int i = j + 1 + idx / C, c = idx % C;
                X[i * C + c] -= S[i * N + j] * X[j * C + c];
            }
            __syncthreads();
        }
        // backward
        for (int j = N - 1; j >= 0; --j) {
            if (tid < C) X[j * C + tid] /= S[j * N + j];
            __syncthreads();
            for (int idx = tid; idx < j * C; idx += NT) {
                int i = idx / C, c = idx % C;
                X[i * C + c] -= S[i * N + j] * X[j * C + c];
            }
            __syncthreads();
        }

        // ------------------------------------------------------------------ phase 3: Y_r = Sr_r^T X
        for (int idx = tid; idx < D * N * C; idx += NT) {
            int r = idx / (N * C), ic = idx % (N * C);
            int i = ic / C, c = ic % C;
            const T* Scol = &Sr[r * N * N + i];
            T acc = 0;
            for (int j = 0; j < N; ++j) acc += Scol[j * N] * X[j * C + c];
            YW[idx] = acc;
        }
        __syncthreads();

        // ------------------------------------------------------------------ phase 4: write Z, z
        const T invJ = T(1) / J;
        T* Zte = Zt + (size_t)e * TT * NLOC;
        for (int idx = tid; idx < TT * NLOC; idx += NT) {
            int c = idx / NLOC, row = idx % NLOC;
            int x = row / N, i = row % N;
            T v;
            if (x < D) {
                int f = c / NF, l = c % NF;
                T acc = nf[f][x] * sf[f] * El[f * N * NF + i * NF + l] * invJ;
                for (int r = 0; r < D; ++r) acc += G[r][x] * YW[(r * N + i) * C + c];
                v = inv_arho * acc;
            } else {
                v = X[i * C + c];
            }
            Zte[idx] = v;
        }
        T* ze = zout + (size_t)e * NLOC * R;
        for (int idx = tid; idx < NLOC * R; idx += NT) {
            int row = idx / R, q = idx % R;
            int x = row / N, i = row % N;
            T v;
            if (x < D) {
                T acc = FV[(x * N + i) * R + q] * invJ;
                for (int r = 0; r < D; ++r) acc += G[r][x] * YW[(r * N + i) * C + TT + q];
                v = inv_arho * acc;
            } else {
                v = X[i * C + TT + q];
            }
            ze[idx] = v;
        }

        // ------------------------------------------------------------------ phase 5: K_e, r_e
        T* Kee = Ke + (size_t)e * TT * TT;
        T* ree = re + (size_t)e * TT * R;
        for (int f = 0; f < NFACE; ++f) {
            // P = sum_x n_fx Z_v,x + tau Z_p  (and the same for the z columns)
            for (int idx = tid; idx < N * C; idx += NT) {
                int i = idx / C, c = idx % C;
                T acc = 0;
                if (c < TT) {
                    int g = c / NF, l = c % NF;
                    T nn = 0;
                    for (int x = 0; x < D; ++x) nn += nf[f][x] * nf[g][x];
                    acc = nn * sf[g] * El[g * N * NF + i * NF + l] * invJ;
                } else {
                    int q = c - TT;
                    for (int x = 0; x < D; ++x) acc += nf[f][x] * FV[(x * N + i) * R + q];
                    acc *= invJ;
                }
                for (int r = 0; r < D; ++r) acc += beta[f][r] * YW[(r * N + i) * C + c];
                P[idx] = inv_arho * acc + tau * X[idx];
            }
            __syncthreads();
            for (int idx = tid; idx < NF * C; idx += NT) {
                int l = idx / C, c = idx % C;
                T acc = 0;
                for (int i = 0; i < N; ++i) acc += El[f * N * NF + i * NF + l] * P[i * C + c];
                T v = -sf[f] * acc;
                if (c < TT) {
                    if (c == f * NF + l) v -= tau * sf[f];
                    Kee[(f * NF + l) * TT + c] = v;
                } else {
                    ree[(f * NF + l) * R + (c - TT)] = v;
                }
            }
            __syncthreads();
        }
    }
}

// u_e = z_e - Z_e lam_e ; Zt column-major per element
template <int R, typename T>
__global__ __launch_bounds__(NT) void recover_kernel(int64_t ne, int nloc, int tt, int nfe, int bs,
                                                     const int32_t* __restrict__ eface,
                                                     const T* __restrict__ Zt, const T* __restrict__ z,
                                                     const double* __restrict__ lam,
                                                     double* __restrict__ u, int epb) {
    extern __shared__ double lsh[];   // [epb][tt][R]
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    for (int idx = tid; idx < epb * tt * R; idx += NT) {
        int s = idx / (tt * R), rem = idx % (tt * R);
        int c = rem / R, q = rem % R;
        int64_t e = e0 + s;
        double v = 0.0;
        if (e < ne) {
            int f = c / bs, l = c % bs;
            int32_t F = eface[e * nfe + f];
            v = lam[((int64_t)F * bs + l) * R + q];
        }
        lsh[idx] = v;
    }
    __syncthreads();
    const int s = tid / nloc, row = tid % nloc;
    const int64_t e = e0 + s;
    if (s >= epb || e >= ne) return;
    const T* Ze = Zt + (size_t)e * tt * nloc;
    const double* le = lsh + s * tt * R;
    double acc[R];
    for (int q = 0; q < R; ++q) acc[q] = (double)z[((size_t)e * nloc + row) * R + q];
    for (int c = 0; c < tt; ++c) {
        double zz = (double)Ze[(size_t)c * nloc + row];
        for (int q = 0; q < R; ++q) acc[q] -= zz * le[c * R + q];
    }
    for (int q = 0; q < R; ++q) u[((size_t)e * nloc + row) * R + q] = acc[q];
}

template <int D, int K, int R, typename T>
int launch_ac(hdg_ctx* c, double a, const double* f_loc, const T* Sr, const T* Mf, const T* Tsym,
              const T* Ef) {
    int grid = (int)std::min<int64_t>(c->n_elem, 256 * 64);
    hipLaunchKernelGGL((condense_acoustic_kernel<D, K, R, T>), dim3(grid), dim3(NT), 0, c->stream,
                       c->n_elem, a, c->d_geom, c->d_eperm, Sr, Mf, Tsym, Ef, f_loc, (T*)c->d_Ke,
                       (T*)c->d_re, (T*)c->d_Zt, (T*)c->d_z,
                       c->precision == HDG_MIXED_FP32 ? (T*)c->d_LU : (T*)nullptr, c->d_status);
    return (int)hipGetLastError();
}

template <typename T>
int dispatch_ac(hdg_ctx* c, double a, const double* f_loc, const T* Sr, const T* Mf, const T* Tsym,
                const T* Ef) {
    const int D = c->dim, K = c->k, R = c->nrhs;
#define HDG_AC_CASE(DD, KK, RR)                                                     \
    if (D == DD && K == KK && R == RR)                                              \
        return launch_ac<DD, KK, RR, T>(c, a, f_loc, Sr, Mf, Tsym, Ef);
    HDG_AC_CASE(2, 1, 1) HDG_AC_CASE(2, 2, 1) HDG_AC_CASE(2, 3, 1) HDG_AC_CASE(2, 4, 1)
    HDG_AC_CASE(3, 1, 1) HDG_AC_CASE(3, 2, 1) HDG_AC_CASE(3, 3, 1) HDG_AC_CASE(3, 4, 1)
#undef HDG_AC_CASE
    return -1;
}

}  // namespace

int launch_condense_acoustic(hdg_ctx* c, double a, const double* f_loc) {
    if (c->precision == HDG_FP64)
        return dispatch_ac<double>(c, a, f_loc, c->tab.Sr, c->tab.Mf, c->tab.Tsym, c->tab.Ef);
    return dispatch_ac<float>(c, a, f_loc, c->tab.Sr32, c->tab.Mf32, c->tab.Tsym32, c->tab.Ef32);
}

int launch_recover(hdg_ctx* c, const double* lambda, double* u, bool) {
    const int nloc = c->n_loc, tt = c->n_tr, R = c->nrhs;
    int epb = std::max(1, NT / nloc);
    int64_t grid = (c->n_elem + epb - 1) / epb;
    size_t shm = (size_t)epb * tt * R * sizeof(double);
    if (R != 1) return -1;
    if (c->precision == HDG_FP64)
        hipLaunchKernelGGL((recover_kernel<1, double>), dim3((unsigned)grid), dim3(NT), shm, c->stream,
                           c->n_elem, nloc, tt, c->dim + 1, c->bs, c->d_eface, (const double*)c->d_Zt,
                           (const double*)c->d_z, lambda, u, epb);
    else
        hipLaunchKernelGGL((recover_kernel<1, float>), dim3((unsigned)grid), dim3(NT), shm, c->stream,
                           c->n_elem, nloc, tt, c->dim + 1, c->bs, c->d_eface, (const float*)c->d_Zt,
                           (const float*)c->d_z, lambda, u, epb);
    return (int)hipGetLastError();
}

}  // namespace hdg
