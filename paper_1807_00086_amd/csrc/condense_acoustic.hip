// Acoustic HDG condensation and recovery kernels for gfx950.
//
// Per element (unknowns u = [v_1..v_d, p], trace p_hat on the d+1 faces):
//   A = [[a rho |J| I,  -Q^T], [Q, a|J|/(rho c^2) I + tau sum_f s_f Mf_f]],
//   Q_x = |J| sum_r G_rx Sr_r  (Q_x[i][j] = (phi_i, d phi_j / d x_x)_K),
//   B = [[n_fx s_f E_f], [-tau s_f E_f]],  C = [[n_fx s_f E_f^T, tau s_f E_f^T]],
//   D = -tau s_f I on each face block,
// with G = J^{-1}, s_f the face measure over the reference-face measure, E_f the oriented
// volume-trace face table.  LU without pivoting of A, velocity block first: the velocity
// block is a rho |J| I, so its elimination is closed form and leaves the SPD pressure block
//   S  = a|J|/(rho c^2) I + tau sum_f s_f Mf_f + (|J|/(a rho)) sum_{r,s} (G G^T)_rs Sr_r Sr_s^T
//   B~ = [-s_f (tau I + (1/(a rho)) sum_r beta_fr Sr_r) E_f]_f,   beta_fr = sum_x G_rx n_fx
//   f~ = f_p - (1/(a rho)) sum_r Sr_r (sum_x G_rx f_vx).
// With S = L L^T (Cholesky), W = L^{-1} B~, w = L^{-1} f~:
//   K_e = D - (1/(a rho |J|)) B_v^T B_v + W^T W,      r_e = -(1/(a rho |J|)) B_v^T f_v + W^T w,
//   Z_p = L^{-T} W,  z_p = L^{-T} w   (pressure rows of Z = A^{-1} B and z = A^{-1} f),
// where (B_v^T B_v)_{fg} = s_f s_g (n_f . n_g) E_f^T E_g.  Recovery (first block row):
//   p = z_p - Z_p lam,   v_x = (f_vx - sum_f n_fx s_f E_f lam_f + Q_x^T p) / (a rho |J|).
//
// Execution: one element per wavefront, several wavefronts per workgroup sharing the
// reference tables in LDS; all intra-element synchronisation is wavefront-local.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "mfma.h"
#include "physics.h"

namespace hdg {

namespace {

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal of a pivot: hardware estimate refined by Newton steps (FP64: two steps from the
// half-precision estimate; FP32: the estimate is within one ulp already).
__device__ __forceinline__ double pivot_rcp(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float pivot_rcp(float p) { return __builtin_amdgcn_rcpf(p); }
// Square root of an inverse pivot: correctly rounded in FP64; in FP32 the hardware square root
// (within one ulp), as the FP32 factors are refined in FP64 anyway.
__device__ __forceinline__ double pivot_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float pivot_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename T>
__device__ __forceinline__ T eps_of() {
    return sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7);
}

template <int D, int K, int R>
struct AcDims {
    static constexpr int N = dimp(K, D);
    static constexpr int NF = dimp(K, D - 1);
    static constexpr int NFACE = D + 1;
    static constexpr int TT = NFACE * NF;          // trace unknowns per element
    static constexpr int C = TT + R;               // columns of [B~ | f~]
    static constexpr int NLOC = (D + 1) * N;       // local unknowns per element
    static constexpr int NPERM = (D == 3) ? 6 : 2;
    static constexpr int NPAIR = D * (D + 1) / 2;
};

// per-wavefront LDS scratch (SHE: the oriented face tables are read from the workgroup's copy
// of all orientations instead of being gathered per element)
template <int D, int K, int R, typename T, bool SHE>
struct AcScratch {
    using Dm = AcDims<D, K, R>;
    static constexpr int NST = (Dm::N * Dm::N > Dm::NFACE * Dm::N * R) ? Dm::N * Dm::N : Dm::NFACE * Dm::N * R;
    T Sb[NST];                                   // S; staging of G f_v and n.f_v
    T X[Dm::N * Dm::C];                          // [B~ | f~] -> [W | w]
    T El[SHE ? 1 : Dm::NFACE * Dm::N * Dm::NF];  // oriented face tables of the element
    T FV[D * Dm::N * R];                         // velocity right-hand side
    T cf[Dm::NFACE * Dm::NFACE];                 // s_f s_g (n_f . n_g) / (a rho |J|)
    T dv[Dm::N];                                 // inverse pivots
    double geo[GEOM_STRIDE];
    int pf[Dm::NFACE];                           // orientation of each face
};

// LDS plan of the condensation kernel.  Target occupancy: three wavefronts per SIMD in FP32,
// two in FP64 (the register budgets of the two instantiations).  In order of preference the
// workgroup shares in LDS, beside Sr: the face tables of all orientations (SHE) and the upper
// triangles of the reference tables of S (TBL).  With TBL no global load other than the
// one-element-ahead prefetch happens inside an element; this matters because vector loads and
// stores share one in-order counter, so a load issued after an element's stores cannot be used
// before those stores complete.  The first configuration that fits at the target wavefronts per
// CU (LDS allocated in 512-byte granules), with 4, 8 or 12 wavefronts per workgroup (whole
// wavefronts per SIMD), wins;
// failing all, every wavefront gathers the oriented tables of its element.
template <int D, int K, int R, typename T, bool SHE, bool TBL>
constexpr int ac_block_lds(int wpb) {
    using Dm = AcDims<D, K, R>;
    const int np = Dm::N * (Dm::N + 1) / 2;
    const int b = (int)((D * Dm::N * Dm::N + (SHE ? Dm::NFACE * Dm::NPERM * Dm::N * Dm::NF : 0) +
                         (TBL ? (Dm::NFACE + Dm::NPAIR) * np : 0)) * sizeof(T) +
                        wpb * sizeof(AcScratch<D, K, R, T, SHE>));
    return (b + 511) / 512 * 512;
}
template <int D, int K, int R, typename T, bool SHE, bool TBL>
constexpr int ac_fit_wpb(int waves) {   // wavefronts per workgroup, 0 if none fits
    const int cand[3] = {4, 8, 12};
    for (int i = 0; i < 3; ++i)
        if (waves % cand[i] == 0 && (waves / cand[i]) * ac_block_lds<D, K, R, T, SHE, TBL>(cand[i]) <= 160 * 1024)
            return cand[i];
    return 0;
}
template <int D, int K, int R, typename T>
struct AcPlan {
    static constexpr int WAVES = sizeof(T) == 4 ? 12 : 8;   // per CU
    static constexpr int W_ST = ac_fit_wpb<D, K, R, T, true, true>(WAVES);
    static constexpr int W_S = ac_fit_wpb<D, K, R, T, true, false>(WAVES);
    static constexpr bool SHE = W_ST > 0 || W_S > 0;
    static constexpr bool TBL = W_ST > 0;
    static constexpr int WPB_G = (4 * (int)sizeof(AcScratch<D, K, R, T, false>) + D * dimp(K, D) * dimp(K, D) * (int)sizeof(T) <= 80 * 1024) ? 4
                                 : (2 * (int)sizeof(AcScratch<D, K, R, T, false>) + D * dimp(K, D) * dimp(K, D) * (int)sizeof(T) <= 80 * 1024) ? 2 : 1;
    static constexpr int WPB = W_ST ? W_ST : (W_S ? W_S : WPB_G);
    static constexpr int MINB = SHE ? WAVES / WPB : (sizeof(T) == 4 ? 3 : 2);
};

// Row and column (i <= j) of entry q of the row-major upper triangle of an n x n matrix: the
// float root estimate of the row is corrected against the exact row offsets.
__device__ __forceinline__ void upper_pair(int q, int n, int& i, int& j) {
    const float b = 2.f * n + 1.f;
    int r = (int)((b - __builtin_amdgcn_sqrtf(b * b - 8.f * q)) * 0.5f);
    r = max(0, min(r, n - 1));
    if (r + 1 < n && (r + 1) * n - (r + 1) * r / 2 <= q) ++r;
    if (r * n - r * (r - 1) / 2 > q) --r;
    i = r;
    j = q - (r * n - r * (r - 1) / 2) + r;
}

// Broadcast of lane `src`'s value (src a compile-time constant after unrolling).
__device__ __forceinline__ double bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

template <int D, int K, int R, typename T, int WPB, bool SHE, bool TBL, int MINB, bool SU>
__global__ __launch_bounds__(64 * WPB, MINB) void condense_acoustic_kernel(
    int64_t ne, double a_in, const double* __restrict__ geom, const int32_t* __restrict__ eperm,
    const T* __restrict__ Sr, const T* __restrict__ Mf, const T* __restrict__ Tsym,
    const T* __restrict__ Ef, const double* __restrict__ f_loc, T* __restrict__ Ke,
    T* __restrict__ re, T* __restrict__ Zs, T* __restrict__ zs, T* __restrict__ Lout,
    int* __restrict__ status) {
    using Dm = AcDims<D, K, R>;
    using MF = Mfma<T>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, TT = Dm::TT, C = Dm::C;
    constexpr int NLOC = Dm::NLOC, NPERM = Dm::NPERM, NPAIR = Dm::NPAIR;
    constexpr int NC = N + C;                 // columns of the augmented matrix [S | B~ | f~]
    constexpr int P = (NC + 63) / 64;         // columns held per lane
    constexpr int SB0 = N / 64, SB1 = (NC - 1) / 64;   // slots holding [B~ | f~]
    static_assert(N <= 64, "pivot columns must sit in the first register slot");

    __shared__ T Srs[D * N * N];
    constexpr int NP = N * (N + 1) / 2;       // entries of an upper triangle
    __shared__ T Efs[SHE ? NFACE * NPERM * N * NF : 1];
    __shared__ T Tbs[TBL ? (NFACE + NPAIR) * NP : 1];   // upper triangles of Mf_f, then Tsym_c
    __shared__ AcScratch<D, K, R, T, SHE> scr_all[WPB];

    for (int idx = threadIdx.x; idx < D * N * N; idx += 64 * WPB) Srs[idx] = Sr[idx];
    if (SHE)
        for (int idx = threadIdx.x; idx < NFACE * NPERM * N * NF; idx += 64 * WPB) Efs[idx] = Ef[idx];
    if (TBL)
        for (int q = threadIdx.x; q < NP; q += 64 * WPB) {
            int i, j;
            upper_pair(q, N, i, j);
            for (int f = 0; f < NFACE; ++f) Tbs[f * NP + q] = Mf[f * N * N + i * N + j];
            for (int c = 0; c < NPAIR; ++c) Tbs[(NFACE + c) * NP + q] = Tsym[c * N * N + i * N + j];
        }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    AcScratch<D, K, R, T, SHE>& sc = scr_all[wave];
    T* Sb = sc.Sb;
    T* X = sc.X;
    T* El = sc.El;
    T* FV = sc.FV;
    const T a = (T)a_in;
    const int lc = lane & 15, lk = lane >> 4;

    // Inputs of the next element (geometry record, face orientations, right-hand side) are
    // loaded into registers while the current one is condensed.
    constexpr int PF = (NLOC * R + 63) / 64;
    const int64_t stride = (int64_t)gridDim.x * WPB;
    double rgeo = 0.0, rf[PF];
    int rperm = 0;
    auto issue = [&](int64_t en) {
        if (lane < GEOM_STRIDE) rgeo = geom[en * GEOM_STRIDE + lane];
        if (lane < NFACE) rperm = eperm[en * NFACE + lane];
        const double* fe = f_loc + (size_t)en * NLOC * R;
#pragma unroll
        for (int t = 0; t < PF; ++t) rf[t] = fe[min(lane + 64 * t, NLOC * R - 1)];
    };
    int64_t e = (int64_t)blockIdx.x * WPB + wave;
    if (e < ne) issue(e);
    for (; e < ne; e += stride) {
        // ------------------------------------------------------------ load
        if (lane < GEOM_STRIDE) sc.geo[lane] = rgeo;
        if (lane < NFACE) sc.pf[lane] = rperm;
#pragma unroll
        for (int t = 0; t < PF; ++t) {
            const int idx = lane + 64 * t;
            if (idx < D * N * R) FV[idx] = (T)rf[t];
            else if (idx < NLOC * R) {
                const int j = idx - D * N * R;
                X[(j / R) * C + TT + j % R] = (T)rf[t];
            }
        }
        wsync();
        if (!SHE) {
            for (int idx = lane; idx < NFACE * N * NF; idx += 64) {
                const int f = idx / (N * NF);
                El[idx] = Ef[(size_t)(f * NPERM + sc.pf[f]) * N * NF + (idx - f * N * NF)];
            }
            wsync();
        }
        if (e + stride < ne) issue(e + stride);
        // oriented face table of local face f (row-major N x NF)
        auto EF = [&](int f) -> const T* { return SHE ? &Efs[(f * NPERM + sc.pf[f]) * N * NF] : &El[f * N * NF]; };

        const T J = (T)sc.geo[0];
        T G[D][D], sf[NFACE], nf[NFACE][D];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int x = 0; x < D; ++x) G[r][x] = (T)sc.geo[1 + r * D + x];
#pragma unroll
        for (int f = 0; f < NFACE; ++f) {
            sf[f] = (T)sc.geo[1 + D * D + f];
#pragma unroll
            for (int x = 0; x < D; ++x) nf[f][x] = (T)sc.geo[1 + D * D + NFACE + f * D + x];
        }
        const T rho = (T)sc.geo[GEO_PAR], cc = (T)sc.geo[GEO_PAR + 1];
        const T tau = (T)sc.geo[GEO_STAB];
        const T inv_arho = T(1) / (a * rho);
        const T inv_av = inv_arho / J;          // 1 / (a rho |J|)
        const T alpha_p = a * J / (rho * cc * cc);

        // face-pair coefficients of the velocity part of K; G f_v for f~
        if (lane < NFACE * NFACE) {
            const int f = lane / NFACE, g = lane % NFACE;
            T nn = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) nn += (T)sc.geo[1 + D * D + NFACE + f * D + x] * (T)sc.geo[1 + D * D + NFACE + g * D + x];
            sc.cf[lane] = inv_av * (T)sc.geo[1 + D * D + f] * (T)sc.geo[1 + D * D + g] * nn;
        }
        for (int idx = lane; idx < D * N * R; idx += 64) {
            const int r = idx / (N * R), jq = idx - r * N * R;
            T g = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) g += G[r][x] * FV[x * N * R + jq];
            Sb[idx] = g * inv_arho;
        }

        // ------------------------------------------------------------ B~ = [-s_f W_f E_f]_f
        // W_f = tau I + (1/(a rho)) sum_r beta_fr Sr_r, formed in the MFMA operand itself;
        // all faces share the Sr reads of one (row tile, k) step.
        {
            constexpr int TM = (N + 15) / 16, TK = (N + 3) / 4;
            T beta[NFACE][D];
#pragma unroll
            for (int f = 0; f < NFACE; ++f)
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    T b = 0;
#pragma unroll
                    for (int x = 0; x < D; ++x) b += G[r][x] * nf[f][x];
                    beta[f][r] = b * inv_arho;
                }
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                typename MF::acc acc[NFACE];
#pragma unroll
                for (int f = 0; f < NFACE; ++f) acc[f] = MF::zero();
                const int am = tm * 16 + lc;
#pragma unroll
                for (int tk = 0; tk < TK; ++tk) {
                    const int k = tk * 4 + lk;
                    const bool aok = am < N && k < N, bok = lc < NF && k < N;
                    T sv[D];
#pragma unroll
                    for (int r = 0; r < D; ++r) sv[r] = aok ? Srs[(r * N + am) * N + k] : T(0);
                    const T dg = (aok && am == k) ? tau : T(0);
#pragma unroll
                    for (int f = 0; f < NFACE; ++f) {
                        T av = dg;
#pragma unroll
                        for (int r = 0; r < D; ++r) av += beta[f][r] * sv[r];
                        const T bv = bok ? EF(f)[k * NF + lc] : T(0);
                        acc[f] = MF::mac(av, bv, acc[f]);
                    }
                }
                if (lc < NF) {
#pragma unroll
                    for (int f = 0; f < NFACE; ++f)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = tm * 16 + MF::row(lane, v);
                            if (i < N) X[i * C + f * NF + lc] = -sf[f] * acc[f][v];
                        }
                }
            }
        }
        wsync();

        // ------------------------------------------------------------ f~ = f_p - sum_r Sr_r (G f_v)_r / (a rho)
        for (int idx = lane; idx < N * R; idx += 64) {
            const int i = idx / R, q = idx % R;
            T acc = 0;
#pragma unroll
            for (int r = 0; r < D; ++r) {
                const T* Srow = &Srs[(r * N + i) * N];
#pragma unroll
                for (int j = 0; j < N; ++j) acc += Srow[j] * Sb[(r * N + j) * R + q];
            }
            X[i * C + TT + q] -= acc;
        }
        wsync();

        // ------------------------------------------------------------ S
        {
            T gam[NPAIR];
            int c = 0;
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int s = r; s < D; ++s, ++c) {
                    T g = 0;
#pragma unroll
                    for (int x = 0; x < D; ++x) g += G[r][x] * G[s][x];
                    gam[c] = g * J * inv_arho;
                }
            // S and the tables are symmetric: the upper triangle is formed and mirrored
            for (int q = lane; q < NP; q += 64) {
                int i, j;
                upper_pair(q, N, i, j);
                const int idx = i * N + j;
                T s = (i == j) ? alpha_p : T(0);
                T fm = 0;
#pragma unroll
                for (int f = 0; f < NFACE; ++f) fm += sf[f] * (TBL ? Tbs[f * NP + q] : Mf[f * N * N + idx]);
                s += tau * fm;
#pragma unroll
                for (int c2 = 0; c2 < NPAIR; ++c2)
                    s += gam[c2] * (TBL ? Tbs[(NFACE + c2) * NP + q] : Tsym[c2 * N * N + idx]);
                Sb[idx] = s;
                Sb[j * N + i] = s;
            }
        }
        wsync();

        // ------------------------------------------------------------ elimination in registers
        // Lane l holds columns l, l+64, ... of [S | B~ | f~].  Gaussian elimination
        // without pivoting (S is SPD): S = L_u U with L_u unit lower, U = diag(d) L_u^T.  Pivot
        // column j sits in lane j; its entries reach the other lanes through readlane broadcasts.
        //   forward:  Y = L_u^{-1} [B~ | f~]; row j of diag(d)^{-1/2} Y is final at step j: W;
        //   backward: [Z_p | z_p] = U^{-1} Y.
        // With SU (mixed precision, or cached factors) U, with 1/d_j in place of its diagonal,
        // is kept for the refinement and for right-hand-side condensations (Lout, column-major
        // N x N: each column contiguous, zero below the diagonal).
        T x[P][N];
        {
            T dmax = lane < N ? fabs(Sb[min(lane, N - 1) * (N + 1)]) : T(0);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
            const T ptol = T(64 * N) * eps_of<T>() * dmax;
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int col = s * 64 + lane;
#pragma unroll
                for (int i = 0; i < N; ++i)
                    x[s][i] = col < N    ? Sb[i * N + min(col, N - 1)]
                              : col < NC ? X[i * C + min(max(col - N, 0), C - 1)]
                                         : (col - NC == i ? T(1) : T(0));   // padding lanes
            }
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const T p = bcast(x[0][j], j);
                const T ip = pivot_rcp(p);
                if (lane == 0) {
                    if (!(p > ptol && p - p == T(0))) atomicOr(status, 1);
                    sc.dv[j] = ip;
                }
                const T sq = pivot_sqrt(ip);
                T t[P];
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    const int col = s * 64 + lane;
                    if (col >= N && col < NC) X[j * C + col - N] = x[s][j] * sq;
                    t[s] = x[s][j] * ip;
                }
#pragma unroll
                for (int i = j + 1; i < N; ++i) {
                    const T aij = bcast(x[0][i], j);
#pragma unroll
                    for (int s = 0; s < P; ++s) x[s][i] -= aij * t[s];
                }
            }
        }
        wsync();
        if constexpr (SU) {
            if (Lout && lane < N) {
                T* Le = Lout + (size_t)e * N * N;
#pragma unroll
                for (int i = 0; i < N; ++i) Le[lane * N + i] = i < lane ? x[0][i] : (i == lane ? sc.dv[lane] : T(0));
            }
        }
        {
#pragma unroll
            for (int j = N - 1; j >= 0; --j) {
                const T ip = sc.dv[j];
                T t[P];
#pragma unroll
                for (int s = SB0; s <= SB1; ++s) {
                    const int col = s * 64 + lane;
                    const bool rhs = col >= N && col < NC;
                    const T z = x[s][j] * ip;
                    t[s] = rhs ? z : T(0);
                    if (rhs) x[s][j] = z;
                }
#pragma unroll
                for (int i = 0; i < j; ++i) {
                    const T uij = bcast(x[0][i], j);
#pragma unroll
                    for (int s = SB0; s <= SB1; ++s) x[s][i] -= uij * t[s];
                }
            }
            T* Zse = Zs + (size_t)e * N * TT;
            T* zse = zs + (size_t)e * NLOC * R;
#pragma unroll
            for (int s = SB0; s <= SB1; ++s) {
                const int c = s * 64 + lane - N;
                if (c >= 0 && c < TT) {
#pragma unroll
                    for (int i = 0; i < N; ++i) Zse[c * N + i] = x[s][i];
                } else if (c >= TT && c < C) {
#pragma unroll
                    for (int i = 0; i < N; ++i) zse[(D * N + i) * R + (c - TT)] = x[s][i];
                }
            }
            // velocity rows of z: D1^{-1} f_v (the coupling to p is applied at recovery)
            for (int idx = lane; idx < D * N * R; idx += 64) zse[idx] = FV[idx] * inv_av;
        }

        // ------------------------------------------------------------ K_e
        // K = D - (1/(a rho |J|)) [s_f s_g (n_f.n_g) E_f^T E_g] + W^T W: two MFMA chains per
        // 16x16 output tile (inner dimension N).  K_e is symmetric: only the tiles on and above
        // the diagonal are formed and stored.  In FP64 the tiles are unrolled (their MFMA chains
        // overlap) and the A operands of a row tile are read once for all its column tiles; the
        // FP32 instantiation, at three wavefronts per SIMD, has no registers for that and forms
        // one tile at a time.
        if constexpr (sizeof(T) == 8) {
            {
                constexpr int TA = (TT + 15) / 16, TK = (N + 3) / 4;
                T* Kee = Ke + (size_t)e * TT * TT;
#pragma unroll
                for (int ta = 0; ta < TA; ++ta) {
                    const int am = ta * 16 + lc;                       // this lane's A row
                    const bool aok = am < TT;
                    const int fam = aok ? am / NF : 0, lam_ = aok ? am % NF : 0;
                    const T* Ea = EF(fam) + lam_;
                    T xa[TK], ea[TK];
#pragma unroll
                    for (int tk = 0; tk < TK; ++tk) {
                        const int k = tk * 4 + lk;
                        const bool ok = aok && k < N;
                        xa[tk] = ok ? X[k * C + am] : T(0);
                        ea[tk] = ok ? Ea[k * NF] : T(0);
                    }
#pragma unroll
                    for (int tb = ta; tb < TA; ++tb) {
                        const int bn = tb * 16 + lc;                   // this lane's B column
                        const bool bok = bn < TT;
                        const int fbn = bok ? bn / NF : 0, lbn = bok ? bn % NF : 0;
                        const T* Eb = EF(fbn) + lbn;
                        typename MF::acc ww = MF::zero(), ee = MF::zero();
#pragma unroll
                        for (int tk = 0; tk < TK; ++tk) {
                            const int k = tk * 4 + lk;
                            const bool ok = bok && k < N;
                            const T xb = ok ? X[k * C + bn] : T(0);
                            const T eb = ok ? Eb[k * NF] : T(0);
                            ww = MF::mac(xa[tk], xb, ww);
                            ee = MF::mac(ea[tk], eb, ee);
                        }
                        if (bok && tb >= ta) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int ar = ta * 16 + MF::row(lane, v);
                                if (ar >= TT) continue;
                                const int fa = ar / NF;
                                T val = ww[v] - sc.cf[fa * NFACE + fbn] * ee[v];
                                if (ar == bn) val -= tau * (T)sc.geo[1 + D * D + fa];
                                Kee[ar * TT + bn] = val;
                            }
                        }
                    }
                }
            }
        } else {
            {
                constexpr int TA = (TT + 15) / 16, TK = (N + 3) / 4;
                T* Kee = Ke + (size_t)e * TT * TT;
#pragma unroll 1
                for (int ta = 0; ta < TA; ++ta) {
                    const int am = ta * 16 + lc;                       // this lane's A row
                    const bool aok = am < TT;
                    const int fam = aok ? am / NF : 0, lam_ = aok ? am % NF : 0;
                    const T* Ea = EF(fam) + lam_;
#pragma unroll 1
                    for (int tb = ta; tb < TA; ++tb) {
                        const int bn = tb * 16 + lc;                   // this lane's B column
                        const bool bok = bn < TT;
                        const int fbn = bok ? bn / NF : 0, lbn = bok ? bn % NF : 0;
                        const T* Eb = EF(fbn) + lbn;
                        typename MF::acc ww = MF::zero(), ee = MF::zero();
#pragma unroll
                        for (int tk = 0; tk < TK; ++tk) {
                            const int k = tk * 4 + lk;
                            const bool kok = k < N;
                            const T xa = (aok && kok) ? X[k * C + am] : T(0);
                            const T xb = (bok && kok) ? X[k * C + bn] : T(0);
                            const T ea = (aok && kok) ? Ea[k * NF] : T(0);
                            const T eb = (bok && kok) ? Eb[k * NF] : T(0);
                            ww = MF::mac(xa, xb, ww);
                            ee = MF::mac(ea, eb, ee);
                        }
                        if (bok) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int ar = ta * 16 + MF::row(lane, v);
                                if (ar >= TT) continue;
                                const int fa = ar / NF;
                                T val = ww[v] - sc.cf[fa * NFACE + fbn] * ee[v];
                                if (ar == bn) val -= tau * (T)sc.geo[1 + D * D + fa];
                                Kee[ar * TT + bn] = val;
                            }
                        }
                    }
                }
            }
        }

        // ------------------------------------------------------------ r_e
        // r_e = -(1/(a rho |J|)) B_v^T f_v + W^T w
        for (int idx = lane; idx < NFACE * N * R; idx += 64) {
            const int f = idx / (N * R), iq = idx - f * N * R;
            T s = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) s += (T)sc.geo[1 + D * D + NFACE + f * D + x] * FV[x * N * R + iq];
            Sb[idx] = s;
        }
        wsync();
        {
            T* ree = re + (size_t)e * TT * R;
            for (int idx = lane; idx < TT * R; idx += 64) {
                const int aa = idx / R, q = idx % R;
                const int f = aa / NF, l = aa % NF;
                T acc = 0, accv = 0;
                const T* Er = EF(f) + l;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    acc += X[i * C + aa] * X[i * C + TT + q];
                    accv += Er[i * NF] * Sb[(f * N + i) * R + q];
                }
                ree[idx] = acc - inv_av * (T)sc.geo[1 + D * D + f] * accv;
            }
        }
        wsync();
    }
}

// Right-hand-side condensation with the factors of the last condensation at the same stage
// coefficient (the stage matrices depend on a only, so Z_p, U and K_e stay valid).  For a new f:
//   f~  = f_p - (1/(a rho)) sum_r Sr_r (G f_v)_r,
//   z_p = S^{-1} f~  (forward substitution with L_u, backward with U, from the stored U),
//   z_v = f_v / (a rho |J|),
//   r_e = Z_p^T f~ - (1/(a rho |J|)) B_v^T f_v     (W^T w = B~^T S^{-1} f~ = Z_p^T f~, S symmetric),
// all in the factors' precision T.  One element per wavefront; Sr in LDS, U staged per
// wavefront, Z_p (column-major) read by its columns, the oriented face tables through L2.
template <int D, int K, int R, typename T>
struct RhScratch {
    using Dm = AcDims<D, K, R>;
    double geo[GEOM_STRIDE];
    T fv[D * Dm::N];              // f_v
    T gf[D * Dm::N];              // (G f_v)_r / (a rho)
    T nf[Dm::NFACE * Dm::N];      // n_f . f_v
    T ul[Dm::N * Dm::N];          // U, column-major
    int pf[Dm::NFACE];
};

template <int D, int K, int R, typename T, int WPB>
__global__ __launch_bounds__(64 * WPB, 2) void rhs_acoustic_kernel(
    int64_t ne, double a_in, const double* __restrict__ geom, const int32_t* __restrict__ eperm,
    const T* __restrict__ Sr, const T* __restrict__ Ef, const T* __restrict__ Zs, const T* __restrict__ Us,
    const double* __restrict__ f_loc, T* __restrict__ re, T* __restrict__ zs) {
    using Dm = AcDims<D, K, R>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, TT = Dm::TT, NLOC = Dm::NLOC;
    constexpr int NPERM = Dm::NPERM;
    static_assert(R == 1 && TT <= 64 && N <= 64, "one right-hand side; trace and Schur vectors fit a wavefront");
    __shared__ T Srs[D * N * N];
    __shared__ RhScratch<D, K, R, T> scr_all[WPB];
    for (int idx = threadIdx.x; idx < D * N * N; idx += 64 * WPB) Srs[idx] = Sr[idx];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    RhScratch<D, K, R, T>& sc = scr_all[wave];
    const int il = min(lane, N - 1), al = min(lane, TT - 1);
    const T a = (T)a_in;
    for (int64_t e = (int64_t)blockIdx.x * WPB + wave; e < ne; e += (int64_t)gridDim.x * WPB) {
        const double* fe = f_loc + (size_t)e * NLOC;
        if (lane < GEOM_STRIDE) sc.geo[lane] = geom[e * GEOM_STRIDE + lane];
        if (lane < NFACE) sc.pf[lane] = eperm[e * NFACE + lane];
        for (int idx = lane; idx < D * N; idx += 64) sc.fv[idx] = (T)fe[idx];
        for (int idx = lane; idx < N * N; idx += 64) sc.ul[idx] = Us[(size_t)e * N * N + idx];
        const T fpv = (T)fe[D * N + il];
        wsync();
        const double* g = sc.geo;
        const T J = (T)g[0], rho = (T)g[GEO_PAR];
        const T inv_arho = T(1) / (a * rho), inv_av = inv_arho / J;
        for (int idx = lane; idx < D * N; idx += 64) {
            const int r = idx / N, j = idx - r * N;
            T s = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) s += (T)g[1 + r * D + x] * sc.fv[x * N + j];
            sc.gf[idx] = s * inv_arho;
        }
        for (int idx = lane; idx < NFACE * N; idx += 64) {
            const int f = idx / N, i = idx - f * N;
            T s = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) s += (T)g[1 + D * D + NFACE + f * D + x] * sc.fv[x * N + i];
            sc.nf[idx] = s;
        }
        wsync();
        // f~ (lane i)
        T ft = fpv;
#pragma unroll 6
        for (int rj = 0; rj < D * N; ++rj) {
            const int r = rj / N, j = rj - r * N;
            ft -= Srs[(r * N + il) * N + j] * sc.gf[rj];
        }
        // z_p = S^{-1} f~ by forward substitution with L_u (L_u[i][j] = U[j][i] / d_j) and
        // backward substitution with U; lane i holds entry i, U is read from LDS (column-major:
        // U[j][i] = ul[i N + j]) and 1/d_i sits on its diagonal
        const T dl = sc.ul[il * N + il];
        T zv = ft;
#pragma unroll 4
        for (int j = 0; j < N; ++j) zv -= (j < lane ? sc.ul[il * N + j] : T(0)) * bcast(zv * dl, j);
#pragma unroll 4
        for (int j = N - 1; j >= 0; --j) {
            const T zj = bcast(zv * dl, j);
            zv = lane == j ? zj : zv - (j > lane ? sc.ul[j * N + il] : T(0)) * zj;
        }
        // r_e (lane a): Z_p column a dot f~, minus the velocity-block term
        {
            const int fc = al / NF, l = al - fc * NF;
            const T* Zc = Zs + ((size_t)e * TT + al) * N;
            const T* Ec = Ef + (size_t)(fc * NPERM + sc.pf[fc]) * N * NF + l;
            const T zf = dot4<N, T>([&](int i) { return Zc[i] * bcast(ft, i); });
            const T bf = dot4<N, T>([&](int i) { return Ec[i * NF] * sc.nf[fc * N + i]; });
            if (lane < TT) re[(size_t)e * TT + lane] = zf - inv_av * (T)g[1 + D * D + fc] * bf;
        }
        T* ze = zs + (size_t)e * NLOC;
        for (int idx = lane; idx < D * N; idx += 64) ze[idx] = sc.fv[idx] * inv_av;
        if (lane < N) ze[D * N + lane] = zv;
        wsync();
    }
}

// Mixed-precision refinement step on the full stage system (FP64 residual, low-precision
// correction factors).  The velocity block of A is a rho |J| I, so for given (p, lam) the
// velocity that satisfies the first block row exactly is
//   v_x = (f_vx + |J| sum_r G_rx Sr_r^T p - sum_f n_fx s_f E_f lam_f) / (a rho |J|),
// and the refinement iterates on (p, lam) only; the velocity residual is zero up to FP64
// rounding.  With the face trace of P_k inside the face space, Mf_f = E_f E_f^T, so the face
// terms of the pressure row share ep_f = E_f^T p with the trace row.  One call, per element:
//   p   <- p_prev + z'_p - Z_p dlam_e       (correction through the stored factors; mode 1, the
//                                            first call, starts from p_prev = 0, z'_p = z_p,
//                                            dlam = lam; mode 2 applies no correction)
//   v   <- closed form above (FP64), u = (v, p) written back
//   s_p  = f_p - |J| sum_r Sr_r (G v)_r - alpha p + tau sum_f s_f E_f (lam_f - ep_f)
//   t_e  = s_f (E_f^T (n_f . v) - tau (lam_f - ep_f))                (= C u + D lam, element part)
//   re64 = Z_p^T s_p - t_e                   (element part of the trace residual of the correction)
//   z'_p = S^{-1} s_p                        (two triangular solves with the stored factor U)
// and the per-element norms |du| and |u|.  RM selects the residual work: 0 stops after the
// recovery (p, v), the plain recovery of the condensed solve; 1 forms everything above, or, with
// the run-time flag chk (the convergence check of the refinement), s_p and t_e only: re64 = -t_e
// (the element part of the FP64 trace residual) and |s_p| per element in place of |du| (the
// velocity rows of the residual vanish by construction).  The check is a run-time branch of the
// RM = 1 kernel rather than an instantiation of its own: compiled separately it spilled registers.
//
// Every global read of an element is issued one element ahead into registers (software
// pipeline, one element per wavefront), so the compute phases read LDS only.  The oriented
// face tables of all orientations are shared by the workgroup when they are small.

// row stride of the refinement kernel's LDS copy of Sr: 2 x odd doubles (16-byte aligned rows
// whose 128-bit reads by a lane per row hit distinct LDS banks for eight consecutive lanes)
constexpr int rf_sr_stride(int n) { return ((n + 1) / 2 % 2 == 1) ? (n + 1) / 2 * 2 : (n + 1) / 2 * 2 + 2; }

template <int D, int K>
constexpr bool rf_shared_faces() {
    return (D + 1) * ((D == 3) ? 6 : 2) * dimp(K, D) * dimp(K, D - 1) * 8 <= 48 * 1024;
}

// per-wavefront LDS scratch of the refinement/recovery kernel
template <int D, int K, int R, typename T, int RM>
struct RfScratch {
    using Dm = AcDims<D, K, R>;
    static constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, TT = Dm::TT, NLOC = Dm::NLOC;
    static constexpr bool SHE = rf_shared_faces<D, K>();
    double geo[GEOM_STRIDE];
    double lm[TT * R];            // lam_e
    double uo[NLOC * R];          // u_e on entry
    double ff[NLOC * R];          // f_e
    double ef[NFACE * N * R];     // E_f lam_f
    double yp[D * N * R];         // Sr_r^T p
    double vv[D * N * R];         // v
    double nv[NFACE * N * R];     // n_f . v
    double El[SHE ? 1 : NFACE * N * NF];
    // Z_p, rows padded so that a lane per row reads distinct LDS banks: FP64 an odd stride;
    // FP32 a multiple of four floats with an odd quotient, so rows stay 16-byte aligned for
    // 128-bit reads and eight consecutive lanes cover the 32 banks once
    static constexpr int ZS = sizeof(T) == 8 ? ((Dm::TT % 2 == 0) ? Dm::TT + 1 : Dm::TT)
                                             : ((Dm::TT + 3) / 4 % 2 == 1 ? (Dm::TT + 3) / 4 * 4 : (Dm::TT + 3) / 4 * 4 + 4);
    alignas(16) T Zl[N * ZS];
    T zb[N * R];                  // z'_p on entry
    T Ll[RM == 1 ? N * N : 1];      // U = diag(d) L_u^T of S = L_u diag(d) L_u^T, 1/d_j on the
                                  // diagonal, column-major
    int fq[32][8];                // face ids [0..NFACE) and orientations [4..4+NFACE) of the
                                  // next 32 elements of this wavefront
    int fc[8];                    // the same for the element being computed
};

template <int M>
struct PerLane {
    static constexpr int n = (M + 63) / 64;
};

// sum_{j < L} term(j) with four independent accumulators of type A (FMA chains of a quarter of
// the length; the summation order is fixed)
template <int L, typename A = double, typename F>
__device__ __forceinline__ A dot4(F term) {
    A a0 = A(0), a1 = A(0), a2 = A(0), a3 = A(0);
#pragma unroll
    for (int j = 0; j + 3 < L; j += 4) {
        a0 += term(j);
        a1 += term(j + 1);
        a2 += term(j + 2);
        a3 += term(j + 3);
    }
#pragma unroll
    for (int j = L & ~3; j < L; ++j) a0 += term(j);
    return (a0 + a1) + (a2 + a3);
}

template <int D, int K, int R, typename T, int WPB, int RM>
__global__ __launch_bounds__(64 * WPB) void refine_acoustic_kernel(
    int64_t ne, double a, const double* __restrict__ geom, const int32_t* __restrict__ eperm,
    const int32_t* __restrict__ eface, const double* __restrict__ Sr, const double* __restrict__ Ef,
    const T* __restrict__ Zs, const T* __restrict__ Lst, const double* __restrict__ f,
    const double* __restrict__ lam, const double* __restrict__ dlam, int mode, int chk, T* __restrict__ zb,
    double* __restrict__ u, double* __restrict__ re64, double* __restrict__ nrm) {
    using Dm = AcDims<D, K, R>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, TT = Dm::TT;
    constexpr int NLOC = Dm::NLOC, NPERM = Dm::NPERM;
    constexpr int NEL = NFACE * N * NF, NZ = N * TT, NLL = RM == 1 ? N * N : 0;
    constexpr bool SHE = rf_shared_faces<D, K>();
    constexpr int PT = PerLane<TT * R>::n, PE = SHE ? 0 : PerLane<NEL>::n, PZ = PerLane<NZ>::n;
    constexpr int PB = PerLane<N * R>::n, PU = PerLane<NLOC * R>::n, PL = PerLane<NLL>::n;
    using Scr = RfScratch<D, K, R, T, RM>;
    constexpr int SDN = PerLane<D * N>::n;
    static_assert(R == 1 && TT <= 64 && N <= 64, "one right-hand side; trace and Schur vectors fit a wavefront");
    constexpr int SS = rf_sr_stride(N);
    __shared__ double Srs[D * N * SS];
    __shared__ double Efs[SHE ? NFACE * NPERM * N * NF : 1];
    __shared__ Scr scr_all[WPB];
    for (int idx = threadIdx.x; idx < D * N * N; idx += 64 * WPB) Srs[(idx / N) * SS + idx % N] = Sr[idx];
    if (SHE)
        for (int idx = threadIdx.x; idx < NFACE * NPERM * N * NF; idx += 64 * WPB) Efs[idx] = Ef[idx];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Scr& sc = scr_all[wave];
    const double* g = sc.geo;
    const int64_t stride = (int64_t)gridDim.x * WPB;

    // ---- registers of the element in flight
    double rgeo = 0.0, rlm[PT], rdl[PT], rel[PE > 0 ? PE : 1], ru[PU], rf[PU];
    T rz[PZ], rzb[PB], rl[PL > 0 ? PL : 1];
    // Face ids and orientations are staged through LDS 32 elements at a time (one vector load
    // per lane), so the gathers of an element never wait on a load of the same pass.
    auto load_faces = [&](int64_t e0) {
        const int k = lane >> 1, part = lane & 1;
        const int64_t ek = e0 + (int64_t)k * stride;
        int v[NFACE];
#pragma unroll
        for (int fc = 0; fc < NFACE; ++fc)
            v[fc] = ek < ne ? (part ? eperm : eface)[ek * NFACE + fc] : 0;
#pragma unroll
        for (int fc = 0; fc < NFACE; ++fc) sc.fq[k][part * 4 + fc] = v[fc];
    };
    auto issue = [&](int64_t en, int k) {
        if (lane < GEOM_STRIDE) rgeo = geom[en * GEOM_STRIDE + lane];
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int idx = min(lane + 64 * t, TT * R - 1);
            const int c = idx / R, q = idx % R;
            const int64_t off = ((int64_t)sc.fq[k][c / NF] * NF + c % NF) * R + q;
            rlm[t] = lam[off];
            rdl[t] = dlam[off];
        }
        if (!SHE)
#pragma unroll
            for (int t = 0; t < PE; ++t) {
                const int idx = min(lane + 64 * t, NEL - 1);
                const int fc = idx / (N * NF);
                rel[t] = Ef[(size_t)(fc * NPERM + sc.fq[k][4 + fc]) * N * NF + (idx - fc * N * NF)];
            }
        const T* Zse = Zs + (size_t)en * NZ;
#pragma unroll
        for (int t = 0; t < PZ; ++t) rz[t] = Zse[min(lane + 64 * t, NZ - 1)];
        const T* zbe = zb + (size_t)en * NLOC * R + D * N * R;
#pragma unroll
        for (int t = 0; t < PB; ++t) rzb[t] = zbe[min(lane + 64 * t, N * R - 1)];
        const double* ue = u + (size_t)en * NLOC * R;
        // without f (FP64 recovery) the velocity rows of z, D1^{-1} f_v, take its place
        const T* zve = zb + (size_t)en * NLOC * R;
#pragma unroll
        for (int t = 0; t < PU; ++t) {
            const int idx = min(lane + 64 * t, NLOC * R - 1);
            ru[t] = mode == 1 ? 0.0 : ue[idx];
            if (f) rf[t] = f[(size_t)en * NLOC * R + idx];
            else rf[t] = idx < D * N * R ? (double)zve[idx] : 0.0;
        }
        if (RM == 1 && !chk) {
            const T* Le = Lst + (size_t)en * NLL;
#pragma unroll
            for (int t = 0; t < PL; ++t) rl[t] = Le[min(lane + 64 * t, NLL - 1)];
        }
    };
    auto commit = [&]() {
        if (lane < GEOM_STRIDE) sc.geo[lane] = rgeo;
#pragma unroll
        for (int t = 0; t < PT; ++t)
            if (lane + 64 * t < TT * R) sc.lm[lane + 64 * t] = rlm[t];
        if (!SHE)
#pragma unroll
            for (int t = 0; t < PE; ++t)
                if (lane + 64 * t < NEL) sc.El[lane + 64 * t] = rel[t];
#pragma unroll
        for (int t = 0; t < PZ; ++t)
            if (lane + 64 * t < NZ) {
                const int idx = lane + 64 * t;
                sc.Zl[(idx % N) * Scr::ZS + idx / N] = rz[t];   // Z_p is stored column-major
            }
#pragma unroll
        for (int t = 0; t < PB; ++t)
            if (lane + 64 * t < N * R) sc.zb[lane + 64 * t] = rzb[t];
#pragma unroll
        for (int t = 0; t < PU; ++t)
            if (lane + 64 * t < NLOC * R) {
                sc.uo[lane + 64 * t] = ru[t];
                sc.ff[lane + 64 * t] = rf[t];
            }
        if (RM == 1 && !chk)
#pragma unroll
            for (int t = 0; t < PL; ++t)
                if (lane + 64 * t < NLL) sc.Ll[lane + 64 * t] = rl[t];
    };

    int64_t e = (int64_t)blockIdx.x * WPB + wave;
    if (e < ne) {
        load_faces(e);
        wsync();
        issue(e, 0);
    }
    for (int it = 0; e < ne; e += stride, ++it) {
        commit();
        const double lmv = rlm[0], dlv = rdl[0];   // lam_e, dlam_e: entry c in lane c
        if (lane < 8) sc.fc[lane] = sc.fq[it & 31][lane];
        const int kn = (it + 1) & 31;
        if (kn == 0) load_faces(e + stride);
        wsync();
        if (e + stride < ne) issue(e + stride, kn);
        // oriented face table of local face fc of this element
        auto Eface = [&](int fc) -> const double* {
            return SHE ? &Efs[(fc * NPERM + sc.fc[4 + fc]) * N * NF] : &sc.El[fc * N * NF];
        };
        double* ue = u + (size_t)e * NLOC;
        const double J = g[0];
        const double rho = g[GEO_PAR], cc = g[GEO_PAR + 1], tau = g[GEO_STAB];
        const double inv_av = 1.0 / (a * rho * J), alpha_p = a * J / (rho * cc * cc);
        double dn = 0.0, un = 0.0;
        // Vectors that a phase needs whole (p, G v, lam - E^T p, s_p, S^{-1} s_p) stay in
        // registers, entry m in lane m % 64 of slot m / 64, and reach the other lanes by readlane;
        // only the lane-varying operands (reference tables, Z_p, U) are read from LDS.
        // Phases that broadcast by readlane run in uniform control flow (every lane computes,
        // with clamped indices; only the stores are masked), so the source lanes are active.
        const int il = min(lane, N - 1), al = min(lane, TT - 1);
        // The products with the stored factors (Z_p dlam here, Z_p^T s_p below) are taken in
        // their precision T: in mixed precision they carry the FP32 factors' error anyway, which
        // the refinement removes, while the sums with p and the residuals stay FP64.
        // ---- p = p_prev + z'_p - Z_p dlam (lane i) ; E_f lam_f
        double pv;
        {
            double s = 0.0;
            const T dlt = (T)dlv;
            if (mode != 2)
                s = (double)(sc.zb[il] - dot4<TT, T>([&](int c) { return sc.Zl[il * Scr::ZS + c] * bcast(dlt, c); }));
            pv = sc.uo[D * N + il] + s;
            if (lane < N) {
                ue[D * N + lane] = pv;
                dn += s * s;
                un += pv * pv;
            }
        }
#pragma unroll
        for (int t = 0; t < PerLane<NFACE * N>::n; ++t) {
            const int idx = lane + 64 * t;
            if (idx < NFACE * N) {
                const int fc = idx / N, i = idx - fc * N;
                const double* Er = Eface(fc) + i * NF;
                sc.ef[idx] = dot4<NF>([&](int l) { return Er[l] * sc.lm[fc * NF + l]; });
            }
        }
        // ---- Sr_r^T p ; lam - E_f^T p
#pragma unroll
        for (int t = 0; t < SDN; ++t) {
            const int idx = min(lane + 64 * t, D * N - 1);
            const int r = idx / N, i = idx - r * N;
            const double y = dot4<N>([&](int j) { return Srs[(r * N + j) * SS + i] * bcast(pv, j); });
            if (lane + 64 * t < D * N) sc.yp[idx] = y;
        }
        double epv = 0.0;
        if (RM != 0) {
            const int fc = al / NF, l = al - fc * NF;
            const double* Ec = Eface(fc) + l;
            epv = lmv - dot4<N>([&](int i) { return Ec[i * NF] * bcast(pv, i); });
        }
        wsync();
        // ---- v in closed form
#pragma unroll
        for (int t = 0; t < SDN; ++t) {
            const int idx = lane + 64 * t;
            if (idx < D * N) {
                const int x = idx / N, i = idx - x * N;
                double s = f ? sc.ff[idx] : 0.0;
#pragma unroll
                for (int r = 0; r < D; ++r) s += J * g[1 + r * D + x] * sc.yp[r * N + i];
#pragma unroll
                for (int fc = 0; fc < NFACE; ++fc)
                    s -= g[1 + D * D + NFACE + fc * D + x] * g[1 + D * D + fc] * sc.ef[fc * N + i];
                const double v = f ? s * inv_av : sc.ff[idx] + s * inv_av;
                sc.vv[idx] = v;
                const double dd = v - sc.uo[idx];
                dn += dd * dd;
                un += v * v;
                ue[idx] = v;
            }
        }
        if (RM != 0) {
            wsync();
            // ---- G v (registers) ; n_f . v
            double gvv[SDN];
#pragma unroll
            for (int t = 0; t < SDN; ++t) {
                const int idx = min(lane + 64 * t, D * N - 1);
                const int r = idx / N, i = idx - r * N;
                double s = 0.0;
#pragma unroll
                for (int x = 0; x < D; ++x) s += g[1 + r * D + x] * sc.vv[x * N + i];
                gvv[t] = s;
            }
#pragma unroll
            for (int t = 0; t < PerLane<NFACE * N>::n; ++t) {
                const int idx = lane + 64 * t;
                if (idx < NFACE * N) {
                    const int fc = idx / N, i = idx - fc * N;
                    double s = 0.0;
#pragma unroll
                    for (int x = 0; x < D; ++x) s += g[1 + D * D + NFACE + fc * D + x] * sc.vv[x * N + i];
                    sc.nv[idx] = s;
                }
            }
            wsync();
            // ---- s_p (lane i) ; t_e (lane a)
            double spv;
            {
                const int i = il;
                const double qv = dot4<D * N>([&](int rj) {
                    const int r = rj / N, j = rj - r * N;
                    return Srs[(r * N + i) * SS + j] * bcast(gvv[rj / 64], rj % 64);
                });
                const double fe = dot4<NFACE * NF>([&](int fl) {
                    const int fc = fl / NF, l = fl - fc * NF;
                    return g[1 + D * D + fc] * Eface(fc)[i * NF + l] * bcast(epv, fl);
                });
                spv = sc.ff[D * N + i] - J * qv - alpha_p * pv + tau * fe;
            }
            double tev;
            {
                const int fc = al / NF, l = al - fc * NF;
                const double* Ec = Eface(fc) + l;
                const double s = dot4<N>([&](int i) { return Ec[i * NF] * sc.nv[fc * N + i]; });
                tev = g[1 + D * D + fc] * (s - tau * epv);
            }
            if (chk) {   // convergence check: the residual only; |s_p|^2 replaces |du|^2
                dn = lane < N ? spv * spv : 0.0;
                if (lane < TT) re64[(size_t)e * TT + lane] = -tev;
            } else {
            // ---- re64 = Z_p^T s_p - t_e ; z'_p = S^{-1} s_p
            {
                const T spt = (T)spv;
                const double s = (double)dot4<N, T>([&](int i) { return sc.Zl[i * Scr::ZS + al] * bcast(spt, i); });
                if (lane < TT) re64[(size_t)e * TT + lane] = s - tev;
            }
            // z'_p = S^{-1} s_p with S = L_u diag(d) L_u^T, U = diag(d) L_u^T stored with 1/d_j on
            // its diagonal: w = L_u^{-1} s_p column by column (L_u[i][j] = U[j][i] / d_j), then
            // U z = w from the last column back.
            // Lane i first takes column i of U above the diagonal, row i right of it and 1/d_i
            // into registers, so that a step of either solve is one multiply, one broadcast
            // and one FMA.  The solves run in the precision of the factor (and of the stored
            // correction), T.
            {
            T cu[N], ru_[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                cu[j] = j < lane ? sc.Ll[il * N + j] : T(0);   // U is stored column-major
                ru_[j] = j > lane ? sc.Ll[j * N + il] : T(0);
            }
            const T dl = sc.Ll[il * N + il];
            T zv = (T)spv;
#pragma unroll
            for (int j = 0; j < N; ++j) zv -= cu[j] * bcast(zv * dl, j);
#pragma unroll
            for (int j = N - 1; j >= 0; --j) {
                const T zj = bcast(zv * dl, j);
                zv = lane == j ? zj : zv - ru_[j] * zj;
            }
            T* zbe = zb + (size_t)e * NLOC + D * N;
            if (lane < N) zbe[lane] = (T)zv;
            }
            }
        }
        // ---- per-element norms of the correction and of u (check mode: and of s_p)
        if (nrm) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                dn += __shfl_xor(dn, off, 64);
                un += __shfl_xor(un, off, 64);
            }
            if (lane == 0) {
                nrm[chk ? 2 * ne + e : e] = sqrt(dn);
                nrm[ne + e] = sqrt(un);
            }
        }
        wsync();
    }
}

template <int D, int K, int R, typename T>
int launch_ac(hdg_ctx* c, double a, const double* f_loc, const T* Sr, const T* Mf, const T* Tsym,
              const T* Ef) {
    using Pl = AcPlan<D, K, R, T>;
    constexpr int WPB = Pl::WPB;
    // U is stored in mixed precision (refinement) and with cached factors; the FP64 kernel
    // without it is a separate instantiation
    auto launch = [&](auto kern) {
        const int64_t groups = (c->n_elem + WPB - 1) / WPB;
        const int grid = (int)std::min<int64_t>(groups, resident_groups((const void*)kern, 64 * WPB));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WPB), 0, c->stream, c->n_elem, a, c->d_geom,
                           c->d_eperm, Sr, Mf, Tsym, Ef, f_loc, (T*)c->d_Ke, (T*)c->d_re, (T*)c->d_Zt,
                           (T*)c->d_z, (T*)c->d_LU, c->d_status);
        return (int)hipGetLastError();
    };
    if constexpr (sizeof(T) == 4) {
        return launch(condense_acoustic_kernel<D, K, R, T, WPB, Pl::SHE, Pl::TBL, Pl::MINB, true>);
    } else {
        if (c->cache_factors && c->d_LU)
            return launch(condense_acoustic_kernel<D, K, R, T, WPB, Pl::SHE, Pl::TBL, Pl::MINB, true>);
        return launch(condense_acoustic_kernel<D, K, R, T, WPB, Pl::SHE, Pl::TBL, Pl::MINB, false>);
    }
}

// wavefronts per workgroup of the refinement kernel: as many as fit next to the shared tables
// in the 160 KB of LDS of a CU (one workgroup per CU), at most 8
template <int D, int K, typename T, int RM>
constexpr int rf_wpb() {
    constexpr int N = dimp(K, D), NF = dimp(K, D - 1);
    constexpr int sb = (int)sizeof(RfScratch<D, K, 1, T, RM>);
    constexpr int tb = (D * N * rf_sr_stride(N) + (rf_shared_faces<D, K>() ? (D + 1) * ((D == 3) ? 6 : 2) * N * NF : 0)) * 8;
    constexpr int w = (160 * 1024 - tb) / sb;
    return w >= 8 ? 8 : (w < 1 ? 1 : w);
}

template <int D, int K, int R, typename T, int RM>
int launch_ac_ref(hdg_ctx* c, const double* lam, const double* dlam, int mode, double* u, double* nrm,
                  int chk = 0) {
    constexpr int WPB = rf_wpb<D, K, T, RM>();
    // the residual needs the FP64 right-hand side, the inverse factor and the residual buffer,
    // which exist in mixed precision only; the plain recovery reads none of them
    if (RM != 0 && (!c->d_f_saved || !c->d_LU || !c->d_re64)) return -1;
    if (chk && (RM != 1 || !nrm)) return -1;
    if (mode != 1 && !c->d_f_saved) return -1;
    int64_t groups = (c->n_elem + WPB - 1) / WPB;
    static const int resident =
        resident_groups((const void*)refine_acoustic_kernel<D, K, R, T, WPB, RM>, 64 * WPB);
    int grid = (int)std::min<int64_t>(groups, resident);
    hipLaunchKernelGGL((refine_acoustic_kernel<D, K, R, T, WPB, RM>), dim3(grid), dim3(64 * WPB), 0,
                       c->stream, c->n_elem, c->last_a, c->d_geom, c->d_eperm, c->d_eface, c->tab.Sr, c->tab.Ef,
                       (const T*)c->d_Zt, (const T*)(RM == 1 ? c->d_LU : nullptr), c->d_f_saved, lam, dlam, mode,
                       chk, (T*)c->d_z, u, RM != 0 ? c->d_re64 : nullptr, nrm);
    return (int)hipGetLastError();
}

#define HDG_AC_CASES(X) X(2, 1, 1) X(2, 2, 1) X(2, 3, 1) X(2, 4, 1) X(3, 1, 1) X(3, 2, 1) X(3, 3, 1) X(3, 4, 1)

template <typename T>
int dispatch_ac(hdg_ctx* c, double a, const double* f_loc, const T* Sr, const T* Mf, const T* Tsym,
                const T* Ef) {
    const int D = c->dim, K = c->k, R = c->nrhs;
#define HDG_CASE(DD, KK, RR) \
    if (D == DD && K == KK && R == RR) return launch_ac<DD, KK, RR, T>(c, a, f_loc, Sr, Mf, Tsym, Ef);
    HDG_AC_CASES(HDG_CASE)
#undef HDG_CASE
    return -1;
}

int dispatch_ac_ref(hdg_ctx* c, const double* lam, const double* dlam, int mode, int resid, double* u,
                    double* nrm) {
    const int D = c->dim, K = c->k, R = c->nrhs;
#define HDG_CASE(DD, KK, RR)                                                                     \
    if (D == DD && K == KK && R == RR) {                                                         \
        if (c->precision == HDG_FP64) return launch_ac_ref<DD, KK, RR, double, 0>(c, lam, dlam, mode, u, nrm); \
        if (resid == 1) return launch_ac_ref<DD, KK, RR, float, 1>(c, lam, dlam, mode, u, nrm);  \
        if (resid == 2) return launch_ac_ref<DD, KK, RR, float, 1>(c, lam, dlam, mode, u, nrm, 1); \
        return launch_ac_ref<DD, KK, RR, float, 0>(c, lam, dlam, mode, u, nrm);                  \
    }
    HDG_AC_CASES(HDG_CASE)
#undef HDG_CASE
    return -1;
}

}  // namespace

int launch_refine_acoustic(hdg_ctx* c, const double* lam, const double* dlam, int mode, int resid,
                           double* u, double* nrm) {
    if (c->physics != HDG_ACOUSTIC || resid < 0 || resid > 2) return -1;
    if (c->precision == HDG_FP64 && resid) return -1;
    return dispatch_ac_ref(c, lam, dlam, mode, resid, u, nrm);
}

template <int D, int K, int R, typename T>
int launch_rh(hdg_ctx* c, double a, const double* f_loc, const T* Sr, const T* Ef) {
    constexpr int WPB = 8;
    auto kern = rhs_acoustic_kernel<D, K, R, T, WPB>;
    const int64_t groups = (c->n_elem + WPB - 1) / WPB;
    const int grid = (int)std::min<int64_t>(groups, resident_groups((const void*)kern, 64 * WPB));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WPB), 0, c->stream, c->n_elem, a, c->d_geom, c->d_eperm, Sr, Ef,
                       (const T*)c->d_Zt, (const T*)c->d_LU, f_loc, (T*)c->d_re, (T*)c->d_z);
    return (int)hipGetLastError();
}

template <typename T>
int dispatch_rh(hdg_ctx* c, double a, const double* f_loc, const T* Sr, const T* Ef) {
    const int D = c->dim, K = c->k, R = c->nrhs;
#define HDG_CASE(DD, KK, RR) \
    if (D == DD && K == KK && R == RR) return launch_rh<DD, KK, RR, T>(c, a, f_loc, Sr, Ef);
    HDG_AC_CASES(HDG_CASE)
#undef HDG_CASE
    return -1;
}

int launch_condense_acoustic(hdg_ctx* c, double a, const double* f_loc) {
    c->ke_tile = 16;
    if (c->precision == HDG_FP64)
        return dispatch_ac<double>(c, a, f_loc, c->tab.Sr, c->tab.Mf, c->tab.Tsym, c->tab.Ef);
    return dispatch_ac<float>(c, a, f_loc, c->tab.Sr32, c->tab.Mf32, c->tab.Tsym32, c->tab.Ef32);
}

int launch_condense_rhs_acoustic(hdg_ctx* c, double a, const double* f_loc) {
    if (!c->d_LU) return -1;
    if (c->precision == HDG_FP64) return dispatch_rh<double>(c, a, f_loc, c->tab.Sr, c->tab.Ef);
    return dispatch_rh<float>(c, a, f_loc, c->tab.Sr32, c->tab.Ef32);
}

}  // namespace hdg
