// Block-structured HDG condensation / recovery / refinement kernels for gfx950: elastodynamics,
// Maxwell, and acoustics on meshes of variable polynomial degree or with several right-hand
// sides.
//
// All three physics share one block structure of the element stage matrix (unknowns
// u = [u1 (M1 flux-like components), u2 (M2 components)], trace lam with MT components):
//   A = [[D1, X], [-X^T, A22]],   D1 = |J| dmat (x) I_N,   X = |J| sum_r c_r (x) Sr_r^T,
//   B = [B1; B2] with B1_a[(f,c)] = b1[a][f,c] s_f E_f,  B2_b[(f,c)] = b2[b][f,c] s_f E_f,
//   C = [j1 B1^T, j2 B2^T] (j2 = -j1),   D = dface s_f I per face block,
//   A22 = |J| amass (x) I + sum_f s_f af_f (x) Mf_f.
//   elastic (u1 = stress s11..s12 with the symmetric test tensors, u2 = velocity, trace v_hat):
//     dmat = a Acomp (compliance in the weighted symmetric basis), c_r[a][x] = sum_b E_a[x][b] G_rb,
//     b1[a][f,y] = -(E_a n_f)_y, b2[x][f,y] = -S delta_xy, amass = a rho I, af_f = S I,
//     dface = S, j1 = -1.
//   maxwell (u1 = H, u2 = E, trace E_hat^t in the face frame (t1, t2)):
//     dmat = a mu I, c_r[y][x] = sum_s eps_{x s y} G_rs, b1[y][f,c] = (n_f x t_fc)_y,
//     b2[x][f,c] = -tau t_fc,x, amass = (a eps + sigma) I, af_f = tau (I - n_f n_f^T),
//     dface = tau, j1 = -1.
//   acoustic (u1 = velocity, u2 = pressure, trace p_hat):
//     dmat = a rho I, c_r[x][0] = -G_rx, b1[x][f] = n_fx, b2[0][f] = -tau, amass = a/(rho c^2),
//     af_f = tau, dface = -tau, j1 = +1.
//   GLM-Maxwell (section 5.2 with the multiplier phi of section 5.1.2; u1 = H, u2 = [E, phi]):
//     as Maxwell for H and E; the phi equation (dmax3) enters with its sign reversed, so that
//     A22 stays symmetric: A22 gains the skew-free coupling Y of E and phi,
//       Y[phi][E_x] = Y[E_x][phi]^T = -|J| sum_r G_rx Sr_r   (-(phi, div v) and -(div E, psi)),
//     amass[phi][phi] = -(a/alpha_1^2 + 1/alpha_2^2), af_f[phi][phi] = -1/alpha_3^2, and the phi
//     rows of f2 change sign.  The Schur block S is then quasi-definite (SPD in E, negative
//     definite in phi after elimination), factored without pivoting as S = L Sigma L^T with
//     Sigma = diag(sign of the pivots); phi is eliminated locally with the rest of the Schur
//     block, so the trace system keeps its size (section 5.2).
// Variable degree (acoustic): the face tables are built at the largest element degree of the
// mesh and the modes of a face above its own degree (the larger degree of its two elements)
// are masked out; elements are launched by degree class through an element list, local
// vectors are addressed through compact offsets, and per-element outputs use the strides of
// the largest class.
// LU without pivoting of A with the D1 block first (closed form) leaves the SPD Schur block
//   S   = A22 + X^T D1^{-1} X = A22 + |J| sum_{r,r'} (c_r^T dmat^{-1} c_r') (x) Sr_r Sr_r'^T
//   B~2 = B2 + X^T D1^{-1} B1,  f~2 = f2 + X^T D1^{-1} f1,
// and with S = L L^T, W = L^{-1} B~2, w = L^{-1} f~2:
//   K_e = D - j1 B1^T D1^{-1} B1 - j2 W^T W,   r_e = -j1 B1^T D1^{-1} f1 - j2 W^T w,
//   Z2 = L^{-T} W, z2 = L^{-T} w, z1 = D1^{-1} f1 (the coupling -D1^{-1}(B1 lam + X u2) is applied
//   at recovery).  One element per workgroup of 256 threads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "internal.h"
#include "mfma.h"
#include "physics.h"

namespace hdg {

namespace {

constexpr int NWG_DEF = 4;   // wavefronts per element workgroup of the condensation (schedules 0-2)
constexpr int PH_ACOUSTIC = 0, PH_ELASTIC = 1, PH_MAXWELL = 2, PH_GLM = 3;
// GLM coefficients alpha_1, alpha_2, alpha_3 of (dmax3): section 5.4 runs all three at 1
constexpr double GLM_A1 = 1.0, GLM_A2 = 1.0, GLM_A3 = 1.0;

// Broadcast of lane `src`'s value within the wavefront (src uniform)
__device__ __forceinline__ double wbcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wbcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Reciprocal of a pivot: the hardware reciprocal, refined by two Newton steps in FP64 (to the
// rounding of a division); in FP32 the hardware value (within one ulp), as the FP32 factors are
// refined in FP64 anyway.
__device__ __forceinline__ double piv_rcp(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float piv_rcp(float p) { return __builtin_amdgcn_rcpf(p); }

template <int PHYS>
struct PhysDims;
template <>
struct PhysDims<PH_ACOUSTIC> {
    static constexpr int M1 = 3, M2 = 1, MT = 1;
};
template <>
struct PhysDims<PH_ELASTIC> {
    static constexpr int M1 = 6, M2 = 3, MT = 3;
};
template <>
struct PhysDims<PH_MAXWELL> {
    static constexpr int M1 = 3, M2 = 3, MT = 2;
};
template <>
struct PhysDims<PH_GLM> {
    static constexpr int M1 = 3, M2 = 4, MT = 2;
};

template <int PHYS, int K, int KF, int R>
struct GDims {
    static constexpr int D = 3, NFACE = 4, NPERM = 6;
    static constexpr int M1 = PhysDims<PHYS>::M1, M2 = PhysDims<PHYS>::M2, MT = PhysDims<PHYS>::MT;
    static constexpr int N = dimp(K, 3), NF = dimp(KF, 2);
    static constexpr int N1 = M1 * N, N2 = M2 * N, NLOC = N1 + N2;
    static constexpr int NFC = NFACE * MT;             // (face, component) pairs
    static constexpr int TT = NFC * NF;
    static constexpr int C = TT + R;
    static constexpr int HV = D * M2 * N * R;
    static constexpr int SBUF = (N2 * N2 > HV) ? N2 * N2 : HV;   // HV, then the Schur block
};

template <int PHYS>
struct Coef {
    static constexpr int M1 = PhysDims<PHYS>::M1, M2 = PhysDims<PHYS>::M2, MT = PhysDims<PHYS>::MT;
    static constexpr int NFC = 4 * MT;
    double d1inv[M1][M1];
    double dmat[M1][M1];       // D1 = |J| dmat (x) I
    double c[3][M1][M2];
    double cd[3][M1][M2];      // dmat^{-1} c_r
    double b1[M1][NFC];
    double bd[M1][NFC];        // dmat^{-1} b1
    double b2[M2][NFC];
    double amass[M2][M2];
    double af[4][M2][M2];
    double Gam[M2][M2][9];     // c_r^T dmat^{-1} c_r'
    double kap[M2][NFC][3];    // c_r^T dmat^{-1} b1
    double g1[NFC][NFC];       // b1^T dmat^{-1} b1
    double dface;
    double j1;
    double y[3][M2][M2];       // GLM: coefficient of |J| Sr_r[i][j] in block (b, gm) of A22
    double f2s[M2];            // sign of the rows of f2 (GLM: -1 on phi)
};

// primary coefficients from the geometry record, material and (Maxwell) face frames
template <int PHYS>
__device__ void coef_primary(const double* g, const double* frm, double a, Coef<PHYS>& cf) {
    constexpr int M1 = Coef<PHYS>::M1, M2 = Coef<PHYS>::M2, MT = Coef<PHYS>::MT, NFC = Coef<PHYS>::NFC;
    double G[3][3], n[4][3];
    for (int r = 0; r < 3; ++r)
        for (int x = 0; x < 3; ++x) G[r][x] = g[1 + r * 3 + x];
    for (int f = 0; f < 4; ++f)
        for (int x = 0; x < 3; ++x) n[f][x] = g[14 + f * 3 + x];
    for (int a1 = 0; a1 < M1; ++a1)
        for (int a2 = 0; a2 < M1; ++a2) cf.d1inv[a1][a2] = cf.dmat[a1][a2] = 0.0;
    for (int b = 0; b < M2; ++b)
        for (int b2 = 0; b2 < M2; ++b2) {
            cf.amass[b][b2] = 0.0;
            for (int f = 0; f < 4; ++f) cf.af[f][b][b2] = 0.0;
        }
    cf.j1 = -1.0;
    for (int r = 0; r < 3; ++r)
        for (int b = 0; b < M2; ++b)
            for (int b2 = 0; b2 < M2; ++b2) cf.y[r][b][b2] = 0.0;
    for (int b = 0; b < M2; ++b) cf.f2s[b] = 1.0;
    if constexpr (PHYS == PH_ACOUSTIC) {
        const double rho = g[GEO_PAR], cc = g[GEO_PAR + 1], tau = g[GEO_STAB];
        for (int x = 0; x < 3; ++x) {
            cf.dmat[x][x] = a * rho;
            cf.d1inv[x][x] = 1.0 / (a * rho);
        }
        for (int r = 0; r < 3; ++r)
            for (int x = 0; x < 3; ++x) cf.c[r][x][0] = -G[r][x];
        for (int x = 0; x < 3; ++x)
            for (int f = 0; f < 4; ++f) cf.b1[x][f] = n[f][x];
        for (int f = 0; f < 4; ++f) {
            cf.b2[0][f] = -tau;
            cf.af[f][0][0] = tau;
        }
        cf.amass[0][0] = a / (rho * cc * cc);
        cf.dface = -tau;
        cf.j1 = 1.0;
    } else if constexpr (PHYS == PH_ELASTIC) {
        const double rho = g[GEO_PAR], lam = g[GEO_PAR + 1], mu = g[GEO_PAR + 2], S = g[GEO_STAB];
        // stress pairs (0,0),(1,1),(2,2),(1,2),(0,2),(0,1); E_a = e_i e_j^T + e_j e_i^T (i != j)
        const int pi[6] = {0, 1, 2, 1, 0, 0}, pj[6] = {0, 1, 2, 2, 2, 1};
        auto Ea = [&](int al, int x, int b) {
            return ((x == pi[al] && b == pj[al]) || (x == pj[al] && b == pi[al])) ? 1.0 : 0.0;
        };
        // dmat^{-1} = (2 mu W^{-1} + lambda t t^T) / a,  W = diag(1,1,1,2,2,2), t = (1,1,1,0,0,0)
        for (int a1 = 0; a1 < 6; ++a1)
            for (int a2 = 0; a2 < 6; ++a2) {
                double v = 0.0;
                if (a1 < 3 && a2 < 3) v = lam + (a1 == a2 ? 2.0 * mu : 0.0);
                else if (a1 == a2) v = mu;
                cf.d1inv[a1][a2] = v / a;
                // dmat = a Acomp: (E_a : E_b - lambda/(3 lambda + 2 mu) tr E_a tr E_b) / (2 mu)
                const double ee = (a1 == a2) ? (a1 < 3 ? 1.0 : 2.0) : 0.0;
                const double tt = (a1 < 3 && a2 < 3) ? 1.0 : 0.0;
                cf.dmat[a1][a2] = a * (ee - lam / (3.0 * lam + 2.0 * mu) * tt) / (2.0 * mu);
            }
        for (int r = 0; r < 3; ++r)
            for (int al = 0; al < 6; ++al)
                for (int x = 0; x < 3; ++x) {
                    double s = 0.0;
                    for (int b = 0; b < 3; ++b) s += Ea(al, x, b) * G[r][b];
                    cf.c[r][al][x] = s;
                }
        for (int al = 0; al < 6; ++al)
            for (int f = 0; f < 4; ++f)
                for (int y = 0; y < 3; ++y) {
                    double s = 0.0;
                    for (int b = 0; b < 3; ++b) s += Ea(al, y, b) * n[f][b];
                    cf.b1[al][f * 3 + y] = -s;
                }
        for (int x = 0; x < 3; ++x)
            for (int fc = 0; fc < NFC; ++fc) cf.b2[x][fc] = (fc % 3 == x) ? -S : 0.0;
        for (int x = 0; x < 3; ++x) {
            cf.amass[x][x] = a * rho;
            for (int f = 0; f < 4; ++f) cf.af[f][x][x] = S;
        }
        cf.dface = S;
    } else {
        const double eps = g[GEO_PAR], mu = g[GEO_PAR + 1], sig = g[GEO_PAR + 2], tau = g[GEO_STAB];
        for (int y = 0; y < 3; ++y) {
            cf.d1inv[y][y] = 1.0 / (a * mu);
            cf.dmat[y][y] = a * mu;
        }
        auto lc = [](int i, int j, int k) { return (double)((i - j) * (j - k) * (k - i)) / 2.0; };
        for (int r = 0; r < 3; ++r)
            for (int y = 0; y < 3; ++y)
                for (int x = 0; x < M2; ++x) {
                    double s = 0.0;
                    if (x < 3)
                        for (int sx = 0; sx < 3; ++sx) s += lc(x, sx, y) * G[r][sx];
                    cf.c[r][y][x] = s;
                }
        for (int f = 0; f < 4; ++f)
            for (int cc = 0; cc < 2; ++cc) {
                const double* t = frm + f * 6 + cc * 3;
                const double w[3] = {n[f][1] * t[2] - n[f][2] * t[1], n[f][2] * t[0] - n[f][0] * t[2],
                                     n[f][0] * t[1] - n[f][1] * t[0]};
                for (int y = 0; y < 3; ++y) cf.b1[y][f * 2 + cc] = w[y];
                for (int y = 0; y < M2; ++y) cf.b2[y][f * 2 + cc] = y < 3 ? -tau * t[y] : 0.0;
            }
        for (int x = 0; x < 3; ++x) {
            cf.amass[x][x] = a * eps + sig;
            for (int f = 0; f < 4; ++f)
                for (int z = 0; z < 3; ++z) cf.af[f][x][z] = tau * ((x == z ? 1.0 : 0.0) - n[f][x] * n[f][z]);
        }
        cf.dface = tau;
        if constexpr (PHYS == PH_GLM) {
            constexpr int P = 3;   // phi
            cf.amass[P][P] = -(a / (GLM_A1 * GLM_A1) + 1.0 / (GLM_A2 * GLM_A2));
            for (int f = 0; f < 4; ++f) cf.af[f][P][P] = -1.0 / (GLM_A3 * GLM_A3);
            for (int r = 0; r < 3; ++r)
                for (int x = 0; x < 3; ++x) {
                    cf.y[r][P][x] = -G[r][x];   // -(div E, psi)  in the reversed phi row
                    cf.y[r][x][P] = 0.0;        // -(phi, div v) is its transpose (Sr_r^T), see form_s
                }
            cf.f2s[P] = -1.0;
        }
    }
    (void)MT;
}

// derived coefficient products, spread over the threads of a group (stride nthr)
template <int PHYS>
__device__ void coef_derived_a(Coef<PHYS>& cf, int t, int nthr) {
    constexpr int M1 = Coef<PHYS>::M1, M2 = Coef<PHYS>::M2, NFC = Coef<PHYS>::NFC;
    for (int idx = t; idx < 3 * M1 * M2; idx += nthr) {
        const int r = idx / (M1 * M2), al = (idx / M2) % M1, b = idx % M2;
        double s = 0.0;
        for (int a2 = 0; a2 < M1; ++a2) s += cf.d1inv[al][a2] * cf.c[r][a2][b];
        cf.cd[r][al][b] = s;
    }
    for (int idx = t; idx < M1 * NFC; idx += nthr) {
        const int al = idx / NFC, fc = idx % NFC;
        double s = 0.0;
        for (int a2 = 0; a2 < M1; ++a2) s += cf.d1inv[al][a2] * cf.b1[a2][fc];
        cf.bd[al][fc] = s;
    }
}

template <int PHYS>
__device__ void coef_derived_b(Coef<PHYS>& cf, int t, int nthr) {
    constexpr int M1 = Coef<PHYS>::M1, M2 = Coef<PHYS>::M2, NFC = Coef<PHYS>::NFC;
    for (int idx = t; idx < M2 * M2 * 9; idx += nthr) {
        const int b = idx / (M2 * 9), gm = (idx / 9) % M2, rr = idx % 9;
        const int r = rr / 3, r2 = rr % 3;
        double s = 0.0;
        for (int al = 0; al < M1; ++al) s += cf.c[r][al][b] * cf.cd[r2][al][gm];
        cf.Gam[b][gm][rr] = s;
    }
    for (int idx = t; idx < M2 * NFC * 3; idx += nthr) {
        const int b = idx / (NFC * 3), fc = (idx / 3) % NFC, r = idx % 3;
        double s = 0.0;
        for (int al = 0; al < M1; ++al) s += cf.c[r][al][b] * cf.bd[al][fc];
        cf.kap[b][fc][r] = s;
    }
    for (int idx = t; idx < NFC * NFC; idx += nthr) {
        const int fc = idx / NFC, gd = idx % NFC;
        double s = 0.0;
        for (int al = 0; al < M1; ++al) s += cf.b1[al][fc] * cf.bd[al][gd];
        cf.g1[fc][gd] = s;
    }
}

// Addressing of meshes of variable degree (all null / zero on a mesh of uniform degree).
struct VarArgs {
    const int32_t* elist;    // elements of the launched degree class (null: 0 .. count-1)
    const int64_t* loc_off;  // compact local dof offsets (null: e * NLOC)
    const int8_t* efnf;      // [e][4] size of the face space of each local face (null: NF)
    int64_t strZ, strz, strL;   // per-element strides of Z, z, L (0: the class's own sizes)
};

template <typename T>
__device__ __forceinline__ T geps() {
    return sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7);
}

// SG: 0 all scratch in LDS; 1 the [B~2 | f~2] block in global scratch; 2 also the Schur block
// buffer and f1 (per workgroup, when the LDS cannot hold them).
template <int PHYS, int K, int KF, int R>
constexpr int64_t gen_gstride(int SG) {
    using Dm = GDims<PHYS, K, KF, R>;
    return (SG >= 1 ? (int64_t)Dm::N2 * Dm::C : 0) + (SG >= 2 ? (int64_t)Dm::SBUF + Dm::N1 * R : 0);
}

// TBL: the Sr tables staged in LDS once per workgroup (true) or read through L1/L2 (false, which
// leaves more LDS for workgroups per CU).  BF (T = float): the matrix-core products (B~2 tiles,
// the strip updates of the triangular solves, the K_e tiles) run as split-BF16 products on the
// BF16 matrix cores with FP32 accumulation (bf16x3_mac16); the factorisation stays FP32.  NW:
// wavefronts per workgroup (one element per workgroup); the tile loops spread over all of them,
// the pivot steps stay on wavefront 0.
template <int PHYS, int K, int KF, int R, typename T, int SG, bool TBL, bool BF = false, int NW = NWG_DEF>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void condense_general_kernel(
    int64_t ne, double a, const double* __restrict__ geom, const double* __restrict__ eframe,
    const int32_t* __restrict__ eperm, const T* __restrict__ Sr, const T* __restrict__ Mf,
    const T* __restrict__ Tfull, const T* __restrict__ Ef, const double* __restrict__ f_loc,
    T* __restrict__ Ke, T* __restrict__ re, T* __restrict__ Zs, T* __restrict__ zs, T* __restrict__ Lout,
    T* __restrict__ Xglob, int* __restrict__ status, VarArgs va) {
    using Dm = GDims<PHYS, K, KF, R>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, NPERM = Dm::NPERM, D = Dm::D;
    constexpr int M1 = Dm::M1, M2 = Dm::M2, MT = Dm::MT, N1 = Dm::N1, N2 = Dm::N2, NLOC = Dm::NLOC;
    constexpr int NFC = Dm::NFC, TT = Dm::TT, C = Dm::C;
    constexpr int NTG = 64 * NW, NWG = NW;   // threads and wavefronts of the workgroup
    static_assert(NW >= 2 && 64 * NW >= GEOM_STRIDE, "the loads assume at least two wavefronts");

    __shared__ T Srl[TBL ? D * N * N : 1];
    const T* Srs = TBL ? Srl : Sr;
    __shared__ T Sbl[SG >= 2 ? 1 : Dm::SBUF];
    __shared__ T El[NFACE * N * NF];
    __shared__ T F1l[SG >= 2 ? 1 : N1 * R];
    __shared__ T Xl[SG >= 1 ? 1 : N2 * C];
    __shared__ Coef<PHYS> cf;
    __shared__ double geo[GEOM_STRIDE];
    __shared__ double frm[24];
    __shared__ T dinv[N2];
    __shared__ T sgn[N2];   // signs of the Schur block's pivots (all +1 unless GLM)
    // Schur blocks of at most 64 unknowns with one right-hand side: the one-wavefront register
    // Cholesky runs while the other wavefronts form B~2 and f~2 (HV then has its own buffer)
    constexpr bool OVL = (N2 <= 64 && R == 1);
    __shared__ T HVl[OVL ? Dm::HV : 1];
    T* gsc = Xglob + (size_t)blockIdx.x * gen_gstride<PHYS, K, KF, R>(SG);
    T* X = SG >= 1 ? gsc : Xl;
    T* Sb = SG >= 2 ? gsc + (int64_t)N2 * C : Sbl;
    T* F1 = SG >= 2 ? gsc + (int64_t)N2 * C + Dm::SBUF : F1l;
    const int64_t strZ = va.strZ ? va.strZ : (int64_t)N2 * TT, strz = va.strz ? va.strz : (int64_t)NLOC * R;
    const int64_t strL = va.strL ? va.strL : (int64_t)N2 * N2;
    const int tid = threadIdx.x;

    if (TBL)
        for (int idx = tid; idx < D * N * N; idx += NTG) Srl[idx] = Sr[idx];

    for (int64_t ie = blockIdx.x; ie < ne; ie += gridDim.x) {
        const int64_t e = va.elist ? (int64_t)va.elist[ie] : ie;
        __syncthreads();
        // ------------------------------------------------------------ load
        if (tid < GEOM_STRIDE) geo[tid] = geom[e * GEOM_STRIDE + tid];
        if (PHYS >= PH_MAXWELL && tid >= 64 && tid < 64 + 24) frm[tid - 64] = eframe[e * 24 + tid - 64];
        for (int idx = tid; idx < NFACE * N * NF; idx += NTG) {
            const int f = idx / (N * NF);
            const int p = eperm[e * NFACE + f];
            const int nfv = va.efnf ? (int)va.efnf[e * NFACE + f] : NF;
            El[idx] = (idx % NF) < nfv ? Ef[(size_t)(f * NPERM + p) * N * NF + (idx - f * N * NF)] : T(0);
        }
        const double* fe = f_loc + (va.loc_off ? va.loc_off[e] : e * NLOC) * R;
        for (int idx = tid; idx < N1 * R; idx += NTG) F1[idx] = (T)fe[idx];
        __syncthreads();
        if (tid == 0) coef_primary<PHYS>(geo, frm, a, cf);
        __syncthreads();
        for (int idx = tid; idx < N2 * R; idx += NTG)
            X[(idx / R) * C + TT + idx % R] = (T)(cf.f2s[idx / (N * R)] * fe[N1 * R + idx]);
        coef_derived_a<PHYS>(cf, tid, NTG);
        __syncthreads();
        coef_derived_b<PHYS>(cf, tid, NTG);
        __syncthreads();
        const T J = (T)geo[0];
        const T invJ = T(1) / J;

        // ------------------------------------------------------------ Sr_r E_f and the f1 coupling
        T* HV = OVL ? HVl : Sb;           // [r][b][j][q] = sum_a cd[r][a][b] f1_a[j][q]
        const int wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
        using MF = Mfma<T>;
        for (int idx = tid; idx < Dm::HV; idx += NTG) {
            const int r = idx / (M2 * N * R), b = (idx / (N * R)) % M2, jq = idx % (N * R);
            T acc = 0;
#pragma unroll
            for (int al = 0; al < M1; ++al) acc += (T)cf.cd[r][al][b] * F1[al * N * R + jq];
            HV[idx] = acc;
        }
        __syncthreads();
        // B~2 and f~2 by the wavefronts [w0, w0 + nw) of the workgroup
        auto form_b2 = [&](int w0, int nw) {
            // ------------------------------------------------------------ B~2 and f~2
            // B~2 block (component b, face component fc) = s_f W_{b,fc} E_f with
            // W_{b,fc} = b2[b][fc] I + sum_r kap[b][fc][r] Sr_r formed inside the A operand: one
            // MFMA chain over the N modes per 16 x 16 tile.  With many right-hand sides and one
            // Schur component the f~2 columns are the product [Sr_0 Sr_1 Sr_2] HV, formed as MFMA
            // tiles over the flattened (r, j) index; otherwise one entry per thread.
            constexpr bool FMF = (R >= 16 && M2 == 1);
            {
                constexpr int NIT = (N + 15) / 16, NLT = (NF + 15) / 16;
                for (int t = wv - w0; t >= 0 && t < M2 * NFC * NIT * NLT; t += nw) {
                    const int bfc = t / (NIT * NLT), it = (t / NLT) % NIT, lt = t % NLT;
                    const int b = bfc / NFC, fc = bfc % NFC, f = fc / MT;
                    const T b2 = (T)cf.b2[b][fc], c0 = (T)cf.kap[b][fc][0], c1 = (T)cf.kap[b][fc][1],
                            c2 = (T)cf.kap[b][fc][2];
                    const int ia = min(it * 16 + li, N - 1), lb = min(lt * 16 + li, NF - 1);
                    const T* A0 = &Srs[ia * N];
                    const T* A1 = &Srs[(N + ia) * N];
                    const T* A2 = &Srs[(2 * N + ia) * N];
                    const T* Bc = &El[f * N * NF + lb];
                    typename MF::acc acc = MF::zero();
                    if constexpr (BF) {
                        for (int j0 = 0; j0 < N; j0 += 16) {
                            float av[4], bv[4];
    #pragma unroll
                            for (int t4 = 0; t4 < 4; ++t4) {
                                const int j = j0 + 4 * lk + t4, jc = min(j, N - 1);
                                const T v = c0 * A0[jc] + c1 * A1[jc] + c2 * A2[jc] + (ia == j ? b2 : T(0));
                                av[t4] = j < N ? v : T(0);
                                bv[t4] = j < N ? Bc[jc * NF] : T(0);
                            }
                            acc = bf16x3_mac16(av, bv, acc);
                        }
                    } else {
    #pragma unroll 4
                        for (int j0 = 0; j0 < N; j0 += 4) {
                            const int j = j0 + lk, jc = min(j, N - 1);
                            T av = c0 * A0[jc] + c1 * A1[jc] + c2 * A2[jc] + (ia == j ? b2 : T(0));
                            av = j < N ? av : T(0);
                            acc = MF::mac(av, Bc[jc * NF], acc);
                        }
                    }
                    const T sf = (T)geo[1 + D * D + f];
                    const int l = lt * 16 + li;
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = it * 16 + MF::row(lane, v);
                        if (i < N && l < NF) X[(b * N + i) * C + fc * NF + l] = sf * acc[v];
                    }
                }
            }
            if constexpr (!FMF) {
                for (int idx = tid - 64 * w0; idx >= 0 && idx < N2 * R; idx += 64 * nw) {
                    const int row = idx / R, q = idx % R;
                    const int b = row / N, i = row % N;
                    T acc = 0;
    #pragma unroll
                    for (int r = 0; r < D; ++r) {
                        const T* Srow = &Srs[(r * N + i) * N];
                        for (int j = 0; j < N; ++j) acc += Srow[j] * HV[((r * M2 + b) * N + j) * R + q];
                    }
                    X[row * C + TT + q] += acc;
                }
            }
            if constexpr (FMF) {
                constexpr int NIT = (N + 15) / 16, NQT = R / 16, KK = D * N;
                for (int t = wv - w0; t >= 0 && t < NIT * NQT; t += nw) {
                    const int it = t / NQT, q0 = (t % NQT) * 16;
                    const int ia = min(it * 16 + li, N - 1);
                    typename MF::acc acc;
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = min(it * 16 + MF::row(lane, v), N - 1);
                        acc[v] = X[i * C + TT + q0 + li];
                    }
    #pragma unroll 4
                    for (int k0 = 0; k0 < KK; k0 += 4) {
                        const int kk = min(k0 + lk, KK - 1);
                        const int r = kk / N, j = kk - r * N;
                        const T av = k0 + lk < KK ? Srs[(r * N + ia) * N + j] : T(0);
                        acc = MF::mac(av, HV[kk * R + q0 + li], acc);
                    }
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = it * 16 + MF::row(lane, v);
                        if (i < N) X[i * C + TT + q0 + li] = acc[v];
                    }
                }
            }
        };
        auto form_s = [&]() {
            // ------------------------------------------------------------ S
            // the reference tables depend on the mode pair (i, j) only: each is read once per pair
            // and serves every component pair (b, gm)
            for (int idx = tid; idx < N * N; idx += NTG) {
                const int i = idx / N, j = idx % N;
                T mf[NFACE], tf[9];
    #pragma unroll
                for (int f = 0; f < NFACE; ++f) mf[f] = (T)geo[1 + D * D + f] * Mf[(f * N + i) * N + j];
    #pragma unroll
                for (int rr = 0; rr < 9; ++rr) tf[rr] = Tfull[(rr * N + i) * N + j];
                T sij[3], sji[3];
                if constexpr (PHYS == PH_GLM)
    #pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        sij[r] = Srs[(r * N + i) * N + j];
                        sji[r] = Srs[(r * N + j) * N + i];
                    }
                auto put = [&](int b, int gm) {
                    T s = (i == j) ? J * (T)cf.amass[b][gm] : T(0);
    #pragma unroll
                    for (int f = 0; f < NFACE; ++f) s += (T)cf.af[f][b][gm] * mf[f];
                    T q = 0;
    #pragma unroll
                    for (int rr = 0; rr < 9; ++rr) q += (T)cf.Gam[b][gm][rr] * tf[rr];
                    if constexpr (PHYS == PH_GLM)   // the E-phi coupling Y and its transpose
    #pragma unroll
                        for (int r = 0; r < 3; ++r) q += (T)cf.y[r][b][gm] * sij[r] + (T)cf.y[r][gm][b] * sji[r];
                    Sb[(b * N + i) * N2 + gm * N + j] = s + J * q;
                };
                // FP64 keeps the component-pair loop rolled (unrolled, its registers spill)
                if constexpr (sizeof(T) == 4) {
    #pragma unroll
                    for (int b = 0; b < M2; ++b)
    #pragma unroll
                        for (int gm = 0; gm < M2; ++gm) put(b, gm);
                } else {
    #pragma unroll 1
                    for (int b = 0; b < M2; ++b)
    #pragma unroll 1
                        for (int gm = 0; gm < M2; ++gm) put(b, gm);
                }
            }
        };
        // ------------------------------------------------------------ Cholesky S = L L^T
        // N2 <= 64: one wavefront, lane c holding column c of S in registers, Gaussian
        // elimination without pivoting (S = L_u diag(d) L_u^T) with readlane broadcasts; lane c
        // then writes row c of L = L_u diag(d)^{1/2} (L[c][j] = U[j][c] / sqrt(d_j), U =
        // diag(d) L_u^T the eliminated rows).  Larger blocks: right-looking with barriers.
        auto chol_small = [&]() {   // wavefront 0
            if constexpr (N2 <= 64) {
                const int cl = min(lane, N2 - 1);
                T x[N2];
#pragma unroll
                for (int i = 0; i < N2; ++i) x[i] = Sb[cl * N2 + i];   // row cl = column cl
                T dmax = lane < N2 ? fabs(Sb[cl * N2 + cl]) : T(0);
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
                const T ptol = T(64 * N2) * geps<T>() * dmax;
                T dl = T(1);
                bool bad = false;
#pragma unroll
                for (int j = 0; j < N2; ++j) {
                    const T p = wbcast(x[j], j);
                    bad |= !(fabs(p) > ptol && p - p == T(0)) || (PHYS != PH_GLM && !(p > T(0)));
                    dl = lane == j ? p : dl;
                    const T t = x[j] * piv_rcp(p);
#pragma unroll
                    for (int i = j + 1; i < N2; ++i) x[i] -= wbcast(x[i], j) * t;
                }
                if (bad && lane == 0) atomicOr(status, 1);
                // L[c][j] = U[j][c] sign(d_j) / sqrt|d_j|  (S = L Sigma L^T, Sigma = sign(d))
                const T sg = dl < T(0) ? T(-1) : T(1);
                const T isq = sg / sqrt(fabs(dl));
                if (lane < N2) sgn[lane] = sg;
#pragma unroll
                for (int j = 0; j < N2; ++j) {
                    const T sj = wbcast(isq, j);
                    if (lane < N2 && j <= lane) Sb[lane * N2 + j] = x[j] * sj;
                }
            }
        };
        if constexpr (OVL) {
            form_s();
            __syncthreads();
            if (wv == 0) chol_small();
            else form_b2(1, NWG - 1);
            __syncthreads();
        } else if constexpr (N2 <= 64) {
            form_b2(0, NWG);
            __syncthreads();
            form_s();
            __syncthreads();
            if (wv == 0) chol_small();
            __syncthreads();
        } else
        {
            form_b2(0, NWG);
            __syncthreads();
            form_s();
            __syncthreads();
            // Blocked right-looking factorisation S = L Sigma L^T (Sigma = sign of the pivots, the
            // identity unless GLM) in panels of 16 columns, three barriers per panel:
            //   (1) wavefront 0 eliminates the diagonal block in registers (lane c holds column c)
            //       and writes L11 = L_u |d|^{1/2} with the signs;
            //   (2) one thread per row below: L21 = S21 L11^{-T} Sigma1 (forward substitution);
            //   (3) the trailing lower triangle S22 -= L21 Sigma1 L21^T as 16 x 16 matrix-core
            //       tiles (k = the 16 panel columns), the tiles spread over the wavefronts.
            // The lower triangle of Sb then holds L (diagonal sqrt|d_j|); the upper triangle is
            // not read.  Same factors as the unblocked elimination up to rounding order.
            T dmax = 0;
            for (int i = 0; i < N2; ++i) dmax = fmax(dmax, fabs(Sb[i * N2 + i]));
            const T ptol = T(64 * N2) * geps<T>() * dmax;
            constexpr int PW = 16, NPAN = (N2 + PW - 1) / PW;
            for (int pn = 0; pn < NPAN; ++pn) {
                const int j0 = pn * PW, b = min(PW, N2 - j0), j1 = j0 + b;
                if (wv == 0) {   // (1)
                    const int c = min(lane, b - 1);
                    T x[PW];
#pragma unroll
                    for (int i = 0; i < PW; ++i) {
                        const int ii = min(i, b - 1);
                        x[i] = i >= b ? T(0) : (ii >= c ? Sb[(j0 + ii) * N2 + j0 + c] : Sb[(j0 + c) * N2 + j0 + ii]);
                    }
                    T dl = T(1);
                    bool bad = false;
#pragma unroll
                    for (int j = 0; j < PW; ++j) {
                        if (j < b) {
                            const T pv = wbcast(x[j], j);
                            bad |= !(fabs(pv) > ptol && pv - pv == T(0)) || (PHYS != PH_GLM && !(pv > T(0)));
                            dl = lane == j ? pv : dl;
                            const T t = x[j] * piv_rcp(pv);
#pragma unroll
                            for (int i = j + 1; i < PW; ++i) x[i] -= wbcast(x[i], j) * t;
                        }
                    }
                    if (bad && lane == 0) atomicOr(status, 1);
                    const T sg = dl < T(0) ? T(-1) : T(1);
                    const T isq = sg / sqrt(fabs(dl));
                    if (lane < b) {
                        sgn[j0 + lane] = sg;
                        dinv[j0 + lane] = fabs(isq);   // 1 / L[j][j]
                    }
#pragma unroll
                    for (int j = 0; j < PW; ++j) {
                        const T sj = wbcast(isq, j);
                        if (lane < b && j <= lane) Sb[(j0 + lane) * N2 + j0 + j] = x[j] * sj;
                    }
                }
                __syncthreads();
                for (int i = j1 + tid; i < N2; i += NTG) {   // (2)
                    T y[PW];
#pragma unroll
                    for (int c = 0; c < PW; ++c) {
                        if (c < b) {
                            T sv = Sb[i * N2 + j0 + c];
#pragma unroll
                            for (int j = 0; j < c; ++j) sv -= Sb[(j0 + c) * N2 + j0 + j] * y[j];
                            y[c] = sv * dinv[j0 + c];
                        } else {
                            y[c] = T(0);
                        }
                    }
#pragma unroll
                    for (int c = 0; c < PW; ++c)
                        if (c < b) Sb[i * N2 + j0 + c] = y[c] * sgn[j0 + c];
                }
                __syncthreads();
                {   // (3)
                    const int nt = (N2 - j1 + 15) / 16, ntile = nt * (nt + 1) / 2;
                    for (int t = wv; t < ntile; t += NWG) {
                        int ti = 0;
                        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
                        const int tm = t - ti * (ti + 1) / 2;
                        const int i0 = j1 + 16 * ti, m0 = j1 + 16 * tm;
                        const int ia = min(i0 + li, N2 - 1), mb = min(m0 + li, N2 - 1);
                        const bool aok = i0 + li < N2, bok = m0 + li < N2;
                        typename MF::acc acc;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = i0 + MF::row(lane, v);
                            acc[v] = (i < N2 && bok) ? Sb[i * N2 + mb] : T(0);
                        }
#pragma unroll
                        for (int kk = 0; kk < PW / 4; ++kk) {
                            const int c = 4 * kk + lk;
                            const T av = (aok && c < b) ? -Sb[ia * N2 + j0 + c] * sgn[j0 + c] : T(0);
                            const T bv = (bok && c < b) ? Sb[mb * N2 + j0 + c] : T(0);
                            acc = MF::mac(av, bv, acc);
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = i0 + MF::row(lane, v);
                            if (i < N2 && bok && m0 + li <= i) Sb[i * N2 + mb] = acc[v];
                        }
                    }
                }
                __syncthreads();
            }
        }
        // the stored factor carries sign(d_j) on its diagonal (negative only for GLM's phi pivots)
        if (Lout)
            for (int idx = tid; idx < N2 * N2; idx += NTG) {
                const int i = idx / N2;
                Lout[e * strL + idx] = (idx == i * N2 + i) ? sgn[i] * Sb[idx] : Sb[idx];
            }
        // ------------------------------------------------------------ [W | w] = L^{-1} [B~2 | f~2]
        // Blocks of 16 rows: the diagonal block is solved one column per thread in registers
        // (factor entries by LDS broadcast), then the rows below are updated as MFMA tiles,
        // X[below] -= L[below][block] X[block], one wavefront per strip of tiles.  The upper
        // triangle of Sb receives L^T for the backward solve.
        constexpr int BR = 16, NBR = (N2 + BR - 1) / BR, NCT = (C + 15) / 16;
        __syncthreads();
        for (int idx = tid; idx < N2 * N2; idx += NTG) {
            const int i = idx / N2, m = idx - i * N2;
            if (m > i) Sb[idx] = Sb[m * N2 + i];
        }
        for (int i = tid; i < N2; i += NTG) dinv[i] = T(1) / Sb[i * N2 + i];
        __syncthreads();
        // X[i0.., c0..] -= sum_k F[i][r0 + k] X[r0 + k][c0..] for a strip of up to SW 16 x 16
        // tiles at column tiles ct0.. (F = L or L^T as stored in Sb; rows at or past N2 are read
        // clamped and not written; k < BR).  Every load of the strip (its A operands, the tiles
        // and their B operands) is issued before the first MFMA and every store after the last,
        // so the strip waits on one round of (L2) latency instead of one per tile.
        constexpr int SW = 4, NCS = (NCT + SW - 1) / SW;
        auto strip_update = [&](int i0, int ct0, int r0) {
            const int ia = min(i0 + li, N2 - 1);
            if constexpr (BF) {   // the k-range of 16 rows as one split-BF16 product per tile
                float av[4];
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const int kr = r0 + 4 * lk + t4;
                    av[t4] = kr < N2 ? -Sb[ia * N2 + kr] : T(0);
                }
                typename MF::acc acc[SW];
                float bv[SW][4];
#pragma unroll
                for (int u = 0; u < SW; ++u) {
                    const int cb = min((ct0 + u) * 16 + li, C - 1);
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = X[min(i0 + MF::row(lane, v), N2 - 1) * C + cb];
#pragma unroll
                    for (int t4 = 0; t4 < 4; ++t4) bv[u][t4] = X[min(r0 + 4 * lk + t4, N2 - 1) * C + cb];
                }
#pragma unroll
                for (int u = 0; u < SW; ++u) acc[u] = bf16x3_mac16(av, bv[u], acc[u]);
#pragma unroll
                for (int u = 0; u < SW; ++u) {
                    const int c = (ct0 + u) * 16 + li;
                    if (ct0 + u < NCT && c < C)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = i0 + MF::row(lane, v);
                            if (i < N2) X[i * C + c] = acc[u][v];
                        }
                }
                return;
            }
            T av[BR / 4];
#pragma unroll
            for (int k = 0; k < BR / 4; ++k) {
                const int kr = min(r0 + 4 * k + lk, N2 - 1);
                av[k] = r0 + 4 * k + lk < N2 ? -Sb[ia * N2 + kr] : T(0);
            }
            typename MF::acc acc[SW];
            T bv[SW][BR / 4];
#pragma unroll
            for (int u = 0; u < SW; ++u) {
                const int cb = min((ct0 + u) * 16 + li, C - 1);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = X[min(i0 + MF::row(lane, v), N2 - 1) * C + cb];
#pragma unroll
                for (int k = 0; k < BR / 4; ++k) bv[u][k] = X[min(r0 + 4 * k + lk, N2 - 1) * C + cb];
            }
#pragma unroll
            for (int u = 0; u < SW; ++u)
#pragma unroll
                for (int k = 0; k < BR / 4; ++k) acc[u] = MF::mac(av[k], bv[u][k], acc[u]);
#pragma unroll
            for (int u = 0; u < SW; ++u) {
                const int c = (ct0 + u) * 16 + li;
                if (ct0 + u < NCT && c < C)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = i0 + MF::row(lane, v);
                        if (i < N2) X[i * C + c] = acc[u][v];
                    }
            }
        };
#pragma unroll 1
        for (int kb = 0; kb < NBR; ++kb) {
            const int r0 = kb * BR;
            for (int c = tid; c < C; c += NTG) {
                T xb[BR];
#pragma unroll
                for (int u = 0; u < BR; ++u) xb[u] = r0 + u < N2 ? X[(r0 + u) * C + c] : T(0);
#pragma unroll
                for (int u = 0; u < BR; ++u) {
                    if (r0 + u >= N2) break;
                    const T* Lr = &Sb[(r0 + u) * N2 + r0];
                    T s = xb[u];
#pragma unroll
                    for (int m = 0; m < u; ++m) s -= Lr[m] * xb[m];
                    xb[u] = s * dinv[r0 + u];
                    X[(r0 + u) * C + c] = xb[u];
                }
            }
            __syncthreads();
            const int nrt = (N2 - r0 - BR + 15) / 16;   // row tiles below the block (<= 0: none)
            for (int t = wv; t < nrt * NCS; t += NWG) strip_update(r0 + BR + (t / NCS) * 16, (t % NCS) * SW, r0);
            __syncthreads();
        }
        // ------------------------------------------------------------ K_e, r_e
        // K_e = D - j1 B1^T D1^{-1} B1 - j2 W^T W on the upper 16 x 16 tiles (mirrored on
        // store): one wavefront per tile, two MFMA chains (W^T W over the N2 rows of W, and
        // E_fa^T E_fb over the N volume modes, scaled per face pair in the epilogue).
        {
            const T j1 = (T)cf.j1;
            const T j2 = -j1;
            constexpr int NTT = (TT + 15) / 16, NPAIR = NTT * (NTT + 1) / 2;
            T* Kee = Ke + (size_t)e * TT * TT;
            for (int pr = wv; pr < NPAIR; pr += NWG) {
                int ta = 0, rem = pr;
                while (rem >= NTT - ta) {
                    rem -= NTT - ta;
                    ++ta;
                }
                const int tb = ta + rem;
                const int a0 = ta * 16, b0 = tb * 16;
                const int ca = min(a0 + li, TT - 1), cb = min(b0 + li, TT - 1);
                typename MF::acc w0 = MF::zero(), w1 = MF::zero(), ee = MF::zero();
                if constexpr (BF) {
                    for (int k0 = 0; k0 < N2; k0 += 16) {
                        float av[4], bv[4];
#pragma unroll
                        for (int t4 = 0; t4 < 4; ++t4) {
                            const int r = k0 + 4 * lk + t4, rc = min(r, N2 - 1);
                            T x = r < N2 ? X[rc * C + ca] : T(0);
                            if constexpr (PHYS == PH_GLM) x *= sgn[rc];
                            av[t4] = x;
                            bv[t4] = X[rc * C + cb];
                        }
                        w0 = bf16x3_mac16(av, bv, w0);
                    }
                    const int fa = ca / NF / MT, la = ca % NF, fb = cb / NF / MT, lb = cb % NF;
                    for (int k0 = 0; k0 < N; k0 += 16) {
                        float av[4], bv[4];
#pragma unroll
                        for (int t4 = 0; t4 < 4; ++t4) {
                            const int i = k0 + 4 * lk + t4, ic = min(i, N - 1);
                            av[t4] = i < N ? El[(fa * N + ic) * NF + la] : T(0);
                            bv[t4] = El[(fb * N + ic) * NF + lb];
                        }
                        ee = bf16x3_mac16(av, bv, ee);
                    }
                } else {
#pragma unroll 2
                for (int k0 = 0; k0 < N2; k0 += 8) {
                    const int r = k0 + lk, r2 = k0 + 4 + lk;
                    const int rc = min(r, N2 - 1), rc2 = min(r2, N2 - 1);
                    T av = r < N2 ? X[rc * C + ca] : T(0);
                    T av2 = r2 < N2 ? X[rc2 * C + ca] : T(0);
                    if constexpr (PHYS == PH_GLM) {   // W^T Sigma W
                        av *= sgn[rc];
                        av2 *= sgn[rc2];
                    }
                    w0 = MF::mac(av, X[rc * C + cb], w0);
                    w1 = MF::mac(av2, X[rc2 * C + cb], w1);
                }
                const int fa = ca / NF / MT, la = ca % NF, fb = cb / NF / MT, lb = cb % NF;
#pragma unroll 2
                for (int k0 = 0; k0 < N; k0 += 4) {
                    const int i = k0 + lk, ic = min(i, N - 1);
                    const T av = i < N ? El[(fa * N + ic) * NF + la] : T(0);
                    ee = MF::mac(av, El[(fb * N + ic) * NF + lb], ee);
                }
                }
                const int bb = b0 + li;
                if (bb < TT) {
                    const int fcb = bb / NF;
                    const T sb = (T)geo[1 + D * D + fcb / MT];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int aa = a0 + MF::row(lane, v);
                        // a diagonal tile keeps its upper triangle and mirrors it, so K_e is
                        // symmetric to the last bit also where the two triangles' products round
                        // differently (the split-BF16 products)
                        if (aa >= TT || (ta == tb && aa > bb)) continue;
                        const int fca = aa / NF;
                        const T sa = (T)geo[1 + D * D + fca / MT];
                        T val = -j1 * invJ * sa * sb * (T)cf.g1[fca][fcb] * ee[v] - j2 * (w0[v] + w1[v]);
                        if (aa == bb) val += (T)cf.dface * sa;
                        Kee[aa * TT + bb] = val;
                        if (aa != bb) Kee[bb * TT + aa] = val;
                    }
                }
            }
            T* ree = re + (size_t)e * TT * R;
            if constexpr (R >= 16) {
                // r_e = -j1 (1/|J|) s_f E_f^T (sum_a bd[a][fc] f1_a) - j2 W^T w as 16 x 16 MFMA
                // tiles (rows: trace unknowns, columns: right-hand sides); the bd factor of a row
                // is folded into that row's A operand.
                constexpr int NQT = R / 16;
                for (int t = wv; t < NTT * NQT; t += NWG) {
                    const int a0 = (t / NQT) * 16, q0 = (t % NQT) * 16;
                    const int ca = min(a0 + li, TT - 1);
                    typename MF::acc acc = MF::zero(), accb = MF::zero();
#pragma unroll 2
                    for (int k0 = 0; k0 < N2; k0 += 4) {
                        const int r = k0 + lk, rc = min(r, N2 - 1);
                        const T av = r < N2 ? X[rc * C + ca] : T(0);
                        acc = MF::mac(av, X[rc * C + TT + q0 + li], acc);
                    }
                    const int fc = ca / NF, f = fc / MT, l = ca % NF;
#pragma unroll
                    for (int al = 0; al < M1; ++al) {
                        const T bdv = (T)cf.bd[al][fc];
#pragma unroll 2
                        for (int k0 = 0; k0 < N; k0 += 4) {
                            const int i = k0 + lk, ic = min(i, N - 1);
                            const T av = i < N ? bdv * El[(f * N + ic) * NF + l] : T(0);
                            accb = MF::mac(av, F1[(al * N + ic) * R + q0 + li], accb);
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int aa = a0 + MF::row(lane, v);
                        if (aa >= TT) continue;
                        const int fr = (aa / NF) / MT;
                        ree[aa * R + q0 + li] = -j1 * invJ * (T)geo[1 + D * D + fr] * accb[v] - j2 * acc[v];
                    }
                }
            } else {
                for (int idx = tid; idx < TT * R; idx += NTG) {
                    const int aa = idx / R, q = idx % R;
                    const int fc = aa / NF, l = aa % NF, f = fc / MT;
                    T acc = 0, accb = 0;
                    for (int row = 0; row < N2; ++row) {
                        T w = X[row * C + aa] * X[row * C + TT + q];
                        if constexpr (PHYS == PH_GLM) w *= sgn[row];
                        acc += w;
                    }
                    for (int i = 0; i < N; ++i) {
                        T fb = 0;
#pragma unroll
                        for (int al = 0; al < M1; ++al) fb += (T)cf.bd[al][fc] * F1[(al * N + i) * R + q];
                        accb += El[(f * N + i) * NF + l] * fb;
                    }
                    ree[idx] = -j1 * invJ * (T)geo[1 + D * D + f] * accb - j2 * acc;
                }
            }
        }
        __syncthreads();
        if constexpr (PHYS == PH_GLM) {   // Z2 = L^{-T} Sigma W
            for (int idx = tid; idx < N2 * C; idx += NTG) X[idx] *= sgn[idx / C];
            __syncthreads();
        }
        // ------------------------------------------------------------ Z2 = L^{-T} W, z2 = L^{-T} w
        // The same by blocks of rows from the bottom, with L^T from the upper triangle of Sb:
        // the diagonal block in registers, then the rows above as MFMA tiles.
#pragma unroll 1
        for (int kb = NBR - 1; kb >= 0; --kb) {
            const int r0 = kb * BR;
            for (int c = tid; c < C; c += NTG) {
                T xb[BR];
#pragma unroll
                for (int u = 0; u < BR; ++u) xb[u] = r0 + u < N2 ? X[(r0 + u) * C + c] : T(0);
#pragma unroll
                for (int u = BR - 1; u >= 0; --u) {
                    if (r0 + u >= N2) continue;
                    const T* Lr = &Sb[(r0 + u) * N2 + r0];   // row r0+u of L^T
                    T s = xb[u];
#pragma unroll
                    for (int m = u + 1; m < BR; ++m) s -= (r0 + m < N2 ? Lr[m] : T(0)) * xb[m];
                    xb[u] = s * dinv[r0 + u];
                    X[(r0 + u) * C + c] = xb[u];
                }
            }
            __syncthreads();
            for (int t = wv; t < (r0 / 16) * NCS; t += NWG) strip_update((t / NCS) * 16, (t % NCS) * SW, r0);
            __syncthreads();
        }
        T* Zse = Zs + e * strZ;
        for (int idx = tid; idx < N2 * TT; idx += NTG) Zse[idx] = X[(idx / TT) * C + idx % TT];
        T* zse = zs + e * strz;
        for (int idx = tid; idx < N2 * R; idx += NTG) zse[N1 * R + idx] = X[(idx / R) * C + TT + idx % R];
        for (int idx = tid; idx < N1 * R; idx += NTG) {
            const int al = idx / (N * R), iq = idx % (N * R);
            T s = 0;
#pragma unroll
            for (int a2 = 0; a2 < M1; ++a2) s += (T)cf.d1inv[al][a2] * F1[a2 * N * R + iq];
            zse[idx] = s * invJ;
        }
    }
}

// Recovery, one right-hand-side column at a time: u2 = z2 - Z2 lam_e ;
// u1_a = z1_a - (1/|J|) sum_fc bd[a][fc] s_f E_f lam_fc - sum_{r,b} cd[r][a][b] Sr_r^T u2_b
template <int PHYS, int K, int KF, int R, typename T, int WPB>
__global__ __launch_bounds__(64 * WPB) void recover_general_kernel(
    int64_t ne, double a, const double* __restrict__ geom, const double* __restrict__ eframe,
    const int32_t* __restrict__ eperm, const int32_t* __restrict__ eface, const T* __restrict__ Sr,
    const T* __restrict__ Ef, const T* __restrict__ Zs, const T* __restrict__ zs,
    const double* __restrict__ lam, double* __restrict__ u, VarArgs va) {
    using Dm = GDims<PHYS, K, KF, R>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, NPERM = Dm::NPERM, D = Dm::D;
    constexpr int M1 = Dm::M1, M2 = Dm::M2, MT = Dm::MT, N1 = Dm::N1, N2 = Dm::N2, NLOC = Dm::NLOC;
    constexpr int NFC = Dm::NFC, TT = Dm::TT;
    struct Scr {
        double geo[GEOM_STRIDE];
        double frm[24];
        double lm[TT];
        double u2[N2];
        double ef[NFC * N];
        double yu[D * M2 * N];
        int nfv[NFACE];
        Coef<PHYS> cf;
    };
    __shared__ double Srs[D * N * N];
    __shared__ Scr scr_all[WPB];
    for (int idx = threadIdx.x; idx < D * N * N; idx += 64 * WPB) Srs[idx] = (double)Sr[idx];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Scr& sc = scr_all[wave];
    const int64_t strZ = va.strZ ? va.strZ : (int64_t)N2 * TT, strz = va.strz ? va.strz : (int64_t)NLOC * R;
    auto ws = []() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (int64_t ie = (int64_t)blockIdx.x * WPB + wave; ie < ne; ie += (int64_t)gridDim.x * WPB) {
        const int64_t e = va.elist ? (int64_t)va.elist[ie] : ie;
        if (lane < GEOM_STRIDE) sc.geo[lane] = geom[e * GEOM_STRIDE + lane];
        if (PHYS >= PH_MAXWELL && lane < 24) sc.frm[lane] = eframe[e * 24 + lane];
        if (lane < NFACE) sc.nfv[lane] = va.efnf ? (int)va.efnf[e * NFACE + lane] : NF;
        ws();
        if (lane == 0) coef_primary<PHYS>(sc.geo, sc.frm, a, sc.cf);
        ws();
        coef_derived_a<PHYS>(sc.cf, lane, 64);
        const T* Zse = Zs + e * strZ;
        const T* zse = zs + e * strz;
        double* ue = u + (va.loc_off ? va.loc_off[e] : e * NLOC) * R;
        const double invJ = 1.0 / sc.geo[0];
#pragma unroll 1
        for (int q = 0; q < R; ++q) {
            for (int c = lane; c < TT; c += 64) {
                const int f = c / (MT * NF), l = c % NF;
                const int32_t F = eface[e * NFACE + f];
                sc.lm[c] = l < sc.nfv[f] ? lam[((int64_t)F * MT * NF + c % (MT * NF)) * R + q] : 0.0;
            }
            ws();
            for (int row = lane; row < N2; row += 64) {
                double acc = (double)zse[(N1 + row) * R + q];
                const T* Zr = Zse + row * TT;
                for (int c = 0; c < TT; ++c) acc -= (double)Zr[c] * sc.lm[c];
                sc.u2[row] = acc;
                ue[(N1 + row) * R + q] = acc;
            }
            for (int idx = lane; idx < NFC * N; idx += 64) {
                const int fc = idx / N, i = idx % N;
                const int f = fc / MT, p = eperm[e * NFACE + f];
                const T* Er = Ef + (size_t)(f * NPERM + p) * N * NF + i * NF;
                double s = 0.0;
                for (int l = 0; l < NF; ++l) s += (double)Er[l] * sc.lm[fc * NF + l];
                sc.ef[idx] = s * sc.geo[1 + D * D + f];
            }
            ws();
            for (int idx = lane; idx < D * M2 * N; idx += 64) {
                const int r = idx / (M2 * N), b = (idx / N) % M2, i = idx % N;
                double s = 0.0;
                for (int j = 0; j < N; ++j) s += Srs[(r * N + j) * N + i] * sc.u2[b * N + j];
                sc.yu[idx] = s;
            }
            ws();
            for (int idx = lane; idx < N1; idx += 64) {
                const int al = idx / N, i = idx % N;
                double s1 = 0.0, s2 = 0.0;
                for (int fc = 0; fc < NFC; ++fc) s1 += sc.cf.bd[al][fc] * sc.ef[fc * N + i];
                for (int r = 0; r < D; ++r)
                    for (int b = 0; b < M2; ++b) s2 += sc.cf.cd[r][al][b] * sc.yu[(r * M2 + b) * N + i];
                ue[idx * R + q] = (double)zse[idx * R + q] - invJ * s1 - s2;
            }
            ws();
        }
    }
}

// Mixed-precision refinement step (FP64 residual of the full stage system, correction through
// the stored FP32 factors), one right-hand-side column at a time:
//   s1 = f1 - |J| (dmat (x) I) u1 - X u2 - B1 lam,   s2 = f2 + X^T u1 - A22 u2 - B2 lam
//   t_e = j1 B1^T u1 + j2 B2^T u2 + D lam
//   s~2 = s2 + X^T D1^{-1} s1,  z' = [D1^{-1} s1 ; L^{-T} L^{-1} s~2]
//   re64 = -j1 B1^T D1^{-1} s1 - j2 Z2^T s~2 - t_e
// One element per wavefront; operator applications staged as short products with lanes over
// their outputs; the triangular solves are column-oriented with lanes over rows.  TL: the
// reference tables Sr, Mf are staged in LDS (otherwise read through the caches).  CHK (the
// convergence check of the refinement): stop after s and t_e, write re64 = -t_e (the element
// part of the FP64 trace residual) and nrm[e][q] = |s| of the element's rows.
template <int PHYS, int K, int KF, int R, typename T, int WPB, bool TL, bool CHK>
__global__ __launch_bounds__(64 * WPB) void refine_general_kernel(
    int64_t ne, double a, const double* __restrict__ geom, const double* __restrict__ eframe,
    const int32_t* __restrict__ eperm, const int32_t* __restrict__ eface, const double* __restrict__ Sr,
    const double* __restrict__ Mf, const double* __restrict__ Ef, const T* __restrict__ Zs,
    const T* __restrict__ Lst, const double* __restrict__ u, const double* __restrict__ lam,
    const double* __restrict__ f, T* __restrict__ zout, double* __restrict__ re64, double* __restrict__ nrm,
    int zero_state, VarArgs va) {
    using Dm = GDims<PHYS, K, KF, R>;
    constexpr int N = Dm::N, NF = Dm::NF, NFACE = Dm::NFACE, NPERM = Dm::NPERM, D = Dm::D;
    constexpr int M1 = Dm::M1, M2 = Dm::M2, MT = Dm::MT, N1 = Dm::N1, N2 = Dm::N2, NLOC = Dm::NLOC;
    constexpr int NFC = Dm::NFC, TT = Dm::TT;
    struct Scr {
        double geo[GEOM_STRIDE];
        double frm[24];
        double uu[NLOC];
        double su[NLOC];
        double lm[TT];
        double ef[NFC * N];        // s_f E_f lam_fc
        double yu[D * M2 * N];     // Sr_r^T u2_b
        double gu[D * M2 * N];     // sum_a c[r][a][b] u1_a, later sum_a cd[r][a][b] s1_a
        double mu[NFACE * M2 * N]; // Mf_f u2_b
        double st[N2];             // s~2, then S^{-1} s~2
        double te[TT];
        int pf[NFACE];             // orientation of each local face (oriented face tables are
                                   // read through L1/L2; modes past a face's space meet zero
                                   // traces or are masked on store)
        int nfv[NFACE];
        Coef<PHYS> cf;
    };
    __shared__ double Srl[TL ? D * N * N : 1];
    __shared__ double Mfl[TL ? NFACE * N * N : 1];
    __shared__ Scr scr_all[WPB];
    if (TL) {
        for (int idx = threadIdx.x; idx < D * N * N; idx += 64 * WPB) Srl[idx] = Sr[idx];
        for (int idx = threadIdx.x; idx < NFACE * N * N; idx += 64 * WPB) Mfl[idx] = Mf[idx];
    }
    __syncthreads();
    const double* Srs = TL ? Srl : Sr;
    const double* Mfs = TL ? Mfl : Mf;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Scr& sc = scr_all[wave];
    const int64_t strZ = va.strZ ? va.strZ : (int64_t)N2 * TT, strz = va.strz ? va.strz : (int64_t)NLOC * R;
    const int64_t strL = va.strL ? va.strL : (int64_t)N2 * N2;
    auto ws = []() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (int64_t ie = (int64_t)blockIdx.x * WPB + wave; ie < ne; ie += (int64_t)gridDim.x * WPB) {
        const int64_t e = va.elist ? (int64_t)va.elist[ie] : ie;
        const int64_t loc = (va.loc_off ? va.loc_off[e] : e * NLOC) * R;
        if (lane < GEOM_STRIDE) sc.geo[lane] = geom[e * GEOM_STRIDE + lane];
        if (PHYS >= PH_MAXWELL && lane < 24) sc.frm[lane] = eframe[e * 24 + lane];
        if (lane < NFACE) sc.nfv[lane] = va.efnf ? (int)va.efnf[e * NFACE + lane] : NF;
        if (lane < NFACE) sc.pf[lane] = eperm[e * NFACE + lane];
        ws();
        if (lane == 0) coef_primary<PHYS>(sc.geo, sc.frm, a, sc.cf);
        ws();
        coef_derived_a<PHYS>(sc.cf, lane, 64);
        const double J = sc.geo[0];
        const double j1 = sc.cf.j1, j2 = -j1;
        const T* Zse = Zs + e * strZ;
        const T* L = Lst + e * strL;
        T* ze = zout + e * strz;
        const double* u1 = sc.uu;
        const double* u2 = sc.uu + N1;
        const double* s1 = sc.su;
        const double* s2 = sc.su + N1;
#pragma unroll 1
        for (int q = 0; q < R; ++q) {
            for (int idx = lane; idx < NLOC; idx += 64) {
                sc.uu[idx] = zero_state ? 0.0 : u[loc + (int64_t)idx * R + q];
                sc.su[idx] = (idx >= N1 ? sc.cf.f2s[(idx - N1) / N] : 1.0) * f[loc + (int64_t)idx * R + q];
            }
            for (int c = lane; c < TT; c += 64) {
                const int fo = c / (MT * NF), l = c % NF;
                const int32_t F = eface[e * NFACE + fo];
                sc.lm[c] = (l < sc.nfv[fo] && !zero_state) ? lam[((int64_t)F * MT * NF + c % (MT * NF)) * R + q] : 0.0;
            }
            ws();
            // ---- stage 1: E_f lam, Sr^T u2, c-weighted u1, Mf u2
            for (int idx = lane; idx < NFC * N; idx += 64) {
                const int fc = idx / N, i = idx % N;
                const int fo = fc / MT;
                double s = 0.0;
                for (int l = 0; l < NF; ++l) s += Ef[((size_t)(fo * NPERM + sc.pf[fo]) * N + i) * NF + l] * sc.lm[fc * NF + l];
                sc.ef[idx] = sc.geo[1 + D * D + fo] * s;
            }
            for (int idx = lane; idx < D * M2 * N; idx += 64) {
                const int r = idx / (M2 * N), b = (idx / N) % M2, i = idx % N;
                double y = 0.0, gg = 0.0;
                for (int j = 0; j < N; ++j) y += Srs[(r * N + j) * N + i] * u2[b * N + j];
                for (int al = 0; al < M1; ++al) gg += sc.cf.c[r][al][b] * u1[al * N + i];
                sc.yu[idx] = y;
                sc.gu[idx] = gg;
            }
            for (int idx = lane; idx < NFACE * M2 * N; idx += 64) {
                const int fa = idx / (M2 * N), b = (idx / N) % M2, i = idx % N;
                double s = 0.0;
                for (int j = 0; j < N; ++j) s += Mfs[(fa * N + i) * N + j] * u2[b * N + j];
                sc.mu[idx] = s;
            }
            ws();
            // ---- stage 2: s = f - A u - B lam ; t_e = j1 B1^T u1 + j2 B2^T u2 + D lam
            for (int row = lane; row < NLOC; row += 64) {
                double Au;
                if (row < N1) {
                    const int al = row / N, i = row % N;
                    double s = 0.0;
                    for (int a2 = 0; a2 < M1; ++a2) s += sc.cf.dmat[al][a2] * u1[a2 * N + i];
                    Au = J * s;
                    double x = 0.0;
                    for (int r = 0; r < D; ++r)
                        for (int b = 0; b < M2; ++b) x += sc.cf.c[r][al][b] * sc.yu[(r * M2 + b) * N + i];
                    Au += J * x;
                    for (int fc = 0; fc < NFC; ++fc) Au += sc.cf.b1[al][fc] * sc.ef[fc * N + i];
                } else {
                    const int b = (row - N1) / N, i = (row - N1) % N;
                    double xt = 0.0;
                    for (int r = 0; r < D; ++r) {
                        const double* Srow = &Srs[(r * N + i) * N];
                        for (int j = 0; j < N; ++j) xt += Srow[j] * sc.gu[(r * M2 + b) * N + j];
                    }
                    double s = 0.0;
                    for (int gm = 0; gm < M2; ++gm) {
                        s += J * sc.cf.amass[b][gm] * u2[gm * N + i];
                        for (int fa = 0; fa < NFACE; ++fa)
                            s += sc.geo[1 + D * D + fa] * sc.cf.af[fa][b][gm] * sc.mu[(fa * M2 + gm) * N + i];
                    }
                    for (int fc = 0; fc < NFC; ++fc) s += sc.cf.b2[b][fc] * sc.ef[fc * N + i];
                    if constexpr (PHYS == PH_GLM) {   // E-phi coupling: J sum_r (y Sr_r + y^T Sr_r^T) u2
                        double yv = 0.0;
                        for (int r = 0; r < D; ++r)
                            for (int gm = 0; gm < M2; ++gm) {
                                const double c1 = sc.cf.y[r][b][gm], c2 = sc.cf.y[r][gm][b];
                                if (c1 != 0.0) {
                                    const double* Srow = &Srs[(r * N + i) * N];
                                    double t = 0.0;
                                    for (int j = 0; j < N; ++j) t += Srow[j] * u2[gm * N + j];
                                    yv += c1 * t;
                                }
                                yv += c2 * sc.yu[(r * M2 + gm) * N + i];
                            }
                        s += J * yv;
                    }
                    Au = -J * xt + s;
                }
                sc.su[row] -= Au;
            }
            for (int aa = lane; aa < TT; aa += 64) {
                const int fc = aa / NF, l = aa % NF, fo = fc / MT;
                double s = 0.0;
                for (int i = 0; i < N; ++i) {
                    double w = 0.0;
                    for (int al = 0; al < M1; ++al) w += j1 * sc.cf.b1[al][fc] * u1[al * N + i];
                    for (int b = 0; b < M2; ++b) w += j2 * sc.cf.b2[b][fc] * u2[b * N + i];
                    s += Ef[((size_t)(fo * NPERM + sc.pf[fo]) * N + i) * NF + l] * w;
                }
                const double sf = sc.geo[1 + D * D + fo];
                sc.te[aa] = sf * s + sc.cf.dface * sf * sc.lm[aa];
            }
            ws();
            if constexpr (CHK) {
                double sq = 0.0;
                for (int idx = lane; idx < NLOC; idx += 64) sq += sc.su[idx] * sc.su[idx];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
                if (lane == 0) nrm[e * R + q] = sqrt(sq);
                for (int aa = lane; aa < TT; aa += 64) {
                    const int l = aa % NF, fo = (aa / NF) / MT;
                    re64[(e * TT + aa) * R + q] = l < sc.nfv[fo] ? -sc.te[aa] : 0.0;
                }
                ws();
                continue;
            }
            // ---- stage 3: cd-weighted s1, then s~2
            for (int idx = lane; idx < D * M2 * N; idx += 64) {
                const int r = idx / (M2 * N), b = (idx / N) % M2, i = idx % N;
                double gg = 0.0;
                for (int al = 0; al < M1; ++al) gg += sc.cf.cd[r][al][b] * s1[al * N + i];
                sc.gu[idx] = gg;
            }
            ws();
            for (int idx = lane; idx < N2; idx += 64) {
                const int b = idx / N, i = idx % N;
                double acc = 0.0;
                for (int r = 0; r < D; ++r) {
                    const double* Srow = &Srs[(r * N + i) * N];
                    for (int j = 0; j < N; ++j) acc += Srow[j] * sc.gu[(r * M2 + b) * N + j];
                }
                sc.st[idx] = s2[idx] + acc;
            }
            ws();
            // ---- re64 = -j1 B1^T D1^{-1} s1 - j2 Z2^T s~2 - t_e (zero on masked face modes)
            for (int aa = lane; aa < TT; aa += 64) {
                const int fc = aa / NF, l = aa % NF, fo = fc / MT;
                double rb = 0.0, zt = 0.0;
                for (int i = 0; i < N; ++i) {
                    double w = 0.0;
                    for (int al = 0; al < M1; ++al) w += sc.cf.bd[al][fc] * s1[al * N + i];
                    rb += Ef[((size_t)(fo * NPERM + sc.pf[fo]) * N + i) * NF + l] * w;
                }
                for (int row = 0; row < N2; ++row) zt += (double)Zse[row * TT + aa] * sc.st[row];
                const double v = -j1 * sc.geo[1 + D * D + fo] / J * rb - j2 * zt - sc.te[aa];
                re64[(e * TT + aa) * R + q] = l < sc.nfv[fo] ? v : 0.0;
            }
            // ---- z' = [D1^{-1} s1 ; S^{-1} s~2]
            for (int idx = lane; idx < N1; idx += 64) {
                const int al = idx / N, i = idx % N;
                double s = 0.0;
                for (int a2 = 0; a2 < M1; ++a2) s += sc.cf.d1inv[al][a2] * s1[a2 * N + i];
                ze[idx * R + q] = (T)(s / J);
            }
            ws();
            // ---- z2' = S^{-1} s~2 = L^{-T} L^{-1} s~2, one row per lane (rows lane + 64 s): the
            // entry each step solves for is broadcast by readlane, and the factor entries come
            // from the factor's global copy (L2-resident), independent of the substitution
            // chain, so their loads run ahead of it
            {
                constexpr int PS = (N2 + 63) / 64;
                double sv[PS], rd[PS];
                double sg[PS];   // signs of the pivots, stored on the factor's diagonal
#pragma unroll
                for (int t = 0; t < PS; ++t) {
                    const int i = min(lane + 64 * t, N2 - 1);
                    sv[t] = sc.st[i];
                    const double dg = (double)L[i * N2 + i];
                    sg[t] = dg < 0.0 ? -1.0 : 1.0;
                    rd[t] = 1.0 / fabs(dg);
                }
#pragma unroll 4
                for (int j = 0; j < N2; ++j) {       // forward: L y = s~2
                    double yj = 0.0;
#pragma unroll
                    for (int t = 0; t < PS; ++t)
                        if (t == (j >> 6)) yj = wbcast(sv[t] * rd[t], j & 63);
#pragma unroll
                    for (int t = 0; t < PS; ++t) {
                        const int i = lane + 64 * t;
                        const double lij = (double)L[min(i, N2 - 1) * N2 + j];
                        sv[t] = i == j ? yj : (i > j ? sv[t] - lij * yj : sv[t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < PS; ++t) sv[t] *= sg[t];   // y <- Sigma y (S^{-1} = L^{-T} Sigma L^{-1})
#pragma unroll 4
                for (int j = N2 - 1; j >= 0; --j) {  // backward: L^T x = y
                    double xj = 0.0;
#pragma unroll
                    for (int t = 0; t < PS; ++t)
                        if (t == (j >> 6)) xj = wbcast(sv[t] * rd[t], j & 63);
#pragma unroll
                    for (int t = 0; t < PS; ++t) {
                        const int i = lane + 64 * t;
                        const double lji = (double)L[j * N2 + min(i, N2 - 1)];
                        sv[t] = i == j ? xj : (i < j ? sv[t] - lji * xj : sv[t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < PS; ++t)
                    if (lane + 64 * t < N2) ze[(N1 + lane + 64 * t) * R + q] = (T)sv[t];
            }
            ws();
        }
    }
}

// ---------------------------------------------------------------------------------- launches
template <typename T>
struct TabOf;
template <>
struct TabOf<double> {
    static const double* Sr(const DeviceTables& t) { return t.Sr; }
    static const double* Mf(const DeviceTables& t) { return t.Mf; }
    static const double* Tf(const DeviceTables& t) { return t.Tfull; }
    static const double* Ef(const DeviceTables& t) { return t.Ef; }
};
template <>
struct TabOf<float> {
    static const float* Sr(const DeviceTables& t) { return t.Sr32; }
    static const float* Mf(const DeviceTables& t) { return t.Mf32; }
    static const float* Tf(const DeviceTables& t) { return t.Tfull32; }
    static const float* Ef(const DeviceTables& t) { return t.Ef32; }
};

VarArgs var_args(const hdg_ctx* c, const int32_t* elist) {
    VarArgs va{};
    va.elist = elist;
    if (c->vardeg) {
        va.loc_off = c->d_loc_off;
        va.efnf = c->d_efnf;
        va.strZ = (int64_t)c->Ns * c->n_tr;
        va.strz = (int64_t)c->n_loc * c->nrhs;
        va.strL = (int64_t)c->Ns * c->Ns;
    }
    return va;
}

// Launch schedules of the condensation kernel: SG places the element buffers (see
// gen_gstride) and TBL the Sr tables.  LDS bytes of a workgroup for each placement:
template <int PHYS, int K, int KF, int R, typename T>
constexpr size_t gen_lds(int SG, bool TBL) {
    using Dm = GDims<PHYS, K, KF, R>;
    const size_t base = sizeof(T) * ((TBL ? Dm::D * Dm::N * Dm::N : 0) + Dm::NFACE * Dm::N * Dm::NF + Dm::N2) +
                        sizeof(Coef<PHYS>) + 8 * 64;
    const size_t mid = base + sizeof(T) * (Dm::SBUF + Dm::N1 * R);
    const size_t all = mid + sizeof(T) * Dm::N2 * Dm::C;
    return SG == 0 ? all : (SG == 1 ? mid : base);
}
constexpr size_t LDS_SHARE = 75 * 1024;    // two workgroups per CU
constexpr size_t LDS_CU = 159 * 1024;      // one workgroup per CU (160 KB less slack)
template <int PHYS, int K, int KF, int R, typename T>
constexpr int gen_fit(size_t cap, bool tbl) {
    return gen_lds<PHYS, K, KF, R, T>(0, tbl) <= cap ? 0 : (gen_lds<PHYS, K, KF, R, T>(1, tbl) <= cap ? 1 : 2);
}
// schedule 0 (default): tables in LDS and at most 75 KB of LDS per workgroup, so that two
// workgroups share a CU, the element buffers that do not fit in global scratch (L2-resident);
// schedule 1: tables in LDS and the fewest buffers in global scratch that fit a whole CU's LDS
// (one workgroup per CU); schedule 2: tables through L1/L2 and the 75 KB rule; schedules 3 and 4:
// eight wavefronts per workgroup instead of four (one element per CU, its tile work spread over
// two wavefronts per SIMD) with the tables in LDS (schedule 1's placement) or through L1/L2 and
// the element buffers in a whole CU's LDS.  Schedules 0-2 run four wavefronts per workgroup.
// Schedule 1 is not built where it repeats schedule 0's placement.
constexpr int GEN_NSCHED = 5;
template <int PHYS, int K, int KF, int R, typename T>
constexpr int gen_sg(int sched) {
    return sched == 0 ? gen_fit<PHYS, K, KF, R, T>(LDS_SHARE, true)
                      : (sched == 1 || sched == 3 ? gen_fit<PHYS, K, KF, R, T>(LDS_CU, true)
                                                  : (sched == 4 ? gen_fit<PHYS, K, KF, R, T>(LDS_CU, false)
                                                                : gen_fit<PHYS, K, KF, R, T>(LDS_SHARE, false)));
}
constexpr int gen_waves(int sched) { return sched >= 3 ? 8 : NWG_DEF; }
template <int PHYS, int K, int KF, int R, typename T>
constexpr bool gen_built(int sched) {
    return sched == 0 || (sched == 1 && gen_sg<PHYS, K, KF, R, T>(1) != gen_sg<PHYS, K, KF, R, T>(0)) ||
           (sched >= 2 && sched < GEN_NSCHED);
}
template <int PHYS, int K, int KF, int R>
int gen_grid(int64_t n) {
    return (int)std::min<int64_t>(n, 256 * 8);
}
// global scratch bytes a launch of `n` elements needs under schedule `sched`
template <int PHYS, int K, int KF, int R, typename T>
size_t gen_scratch(int64_t n, int sched) {
    return (size_t)gen_grid<PHYS, K, KF, R>(n) * gen_gstride<PHYS, K, KF, R>(gen_sg<PHYS, K, KF, R, T>(sched)) * sizeof(T);
}

template <int PHYS, int K, int KF, int R, typename T, int SG, bool TBL, bool BF, int NW = NWG_DEF>
int launch_gen_sg(hdg_ctx* c, double a, const double* f_loc, const DeviceTables& tb, const int32_t* elist,
                  int64_t n, T* scratch, hipStream_t st) {
    using TB = TabOf<T>;
    hipLaunchKernelGGL((condense_general_kernel<PHYS, K, KF, R, T, SG, TBL, BF, NW>),
                       dim3(gen_grid<PHYS, K, KF, R>(n)), dim3(64 * NW), 0, st, n, a, c->d_geom, c->d_eframe, c->d_eperm, TB::Sr(tb), TB::Mf(tb), TB::Tf(tb),
                       TB::Ef(tb), f_loc, (T*)c->d_Ke, (T*)c->d_re, (T*)c->d_Zt, (T*)c->d_z,
                       (T*)c->d_LU, scratch, c->d_status,
                       var_args(c, elist));
    return (int)hipGetLastError();
}

// schedule `sched` (0..4) of a class; a schedule that is not built falls back to 0
template <int PHYS, int K, int KF, int R, typename T, bool BF>
int launch_gen(hdg_ctx* c, double a, const double* f_loc, const DeviceTables& tb, const int32_t* elist, int64_t n,
               int sched, T* scratch, hipStream_t st) {
    constexpr int S0 = gen_sg<PHYS, K, KF, R, T>(0), S1 = gen_sg<PHYS, K, KF, R, T>(1), S2 = gen_sg<PHYS, K, KF, R, T>(2),
                  S4 = gen_sg<PHYS, K, KF, R, T>(4);
    if constexpr (gen_built<PHYS, K, KF, R, T>(1))
        if (sched == 1) return launch_gen_sg<PHYS, K, KF, R, T, S1, true, BF>(c, a, f_loc, tb, elist, n, scratch, st);
    if (sched == 2) return launch_gen_sg<PHYS, K, KF, R, T, S2, false, BF>(c, a, f_loc, tb, elist, n, scratch, st);
    if (sched == 3)
        return launch_gen_sg<PHYS, K, KF, R, T, S1, true, BF, gen_waves(3)>(c, a, f_loc, tb, elist, n, scratch, st);
    if (sched == 4)
        return launch_gen_sg<PHYS, K, KF, R, T, S4, false, BF, gen_waves(4)>(c, a, f_loc, tb, elist, n, scratch, st);
    return launch_gen_sg<PHYS, K, KF, R, T, S0, true, BF>(c, a, f_loc, tb, elist, n, scratch, st);
}

template <int PHYS, int K, int KF, int R, typename T>
int launch_gen_rec(hdg_ctx* c, const DeviceTables& tb, const int32_t* elist, int64_t n, const double* lam,
                   double* u) {
    constexpr int WPB = 2;
    int64_t groups = (n + WPB - 1) / WPB;
    int grid = (int)std::min<int64_t>(groups, 256 * 16);
    using TB = TabOf<T>;
    hipLaunchKernelGGL((recover_general_kernel<PHYS, K, KF, R, T, WPB>), dim3(grid), dim3(64 * WPB), 0, c->stream, n,
                       c->last_a, c->d_geom, c->d_eframe, c->d_eperm, c->d_eface, TB::Sr(tb), TB::Ef(tb),
                       (const T*)c->d_Zt, (const T*)c->d_z, lam, u, var_args(c, elist));
    return (int)hipGetLastError();
}

// f == nullptr: the saved right-hand side of the stage (refinement); zero_state: u = 0, lam = 0
// (the residual is then f itself, and the pass condenses the right-hand side f with the kept
// factors: z into the z buffer, r_e into re_out)
template <int PHYS, int K, int KF, int R, typename T>
int launch_gen_ref(hdg_ctx* c, const DeviceTables& tb, const int32_t* elist, int64_t n, const double* u,
                   const double* lam, bool chk, double* nrm, const double* f = nullptr, int zero_state = 0,
                   double* re_out = nullptr) {
    constexpr int WPB = 1;
    constexpr bool TL = false;   // tables read through L1/L2: more wavefronts per CU than with LDS copies
    const int grid = (int)std::min<int64_t>(n, 256 * 16);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WPB), 0, c->stream, n, c->last_a, c->d_geom, c->d_eframe,
                           c->d_eperm, c->d_eface, tb.Sr, tb.Mf, tb.Ef, (const T*)c->d_Zt, (const T*)c->d_LU, u,
                           lam, f ? f : c->d_f_saved, (T*)c->d_z, re_out ? re_out : c->d_re64, nrm, zero_state,
                           var_args(c, elist));
        return (int)hipGetLastError();
    };
    if (chk) return go(refine_general_kernel<PHYS, K, KF, R, T, WPB, TL, true>);
    return go(refine_general_kernel<PHYS, K, KF, R, T, WPB, TL, false>);
}

// built configurations: (physics, volume degree, face-table degree, right-hand sides).
// Uniform meshes use face degree = volume degree; meshes of variable degree (acoustic) use
// face tables of degree 5 for every class.
// The acoustic cases with 32 right-hand sides recover and refine in recover_mrhs.hip.
#define HDG_GEN_CASES_R1(X)                                                                         \
    X(1, 1, 1, 1) X(1, 2, 2, 1) X(1, 3, 3, 1) X(1, 4, 4, 1) X(2, 1, 1, 1) X(2, 2, 2, 1) X(2, 3, 3, 1) \
    X(3, 1, 1, 1) X(3, 2, 2, 1) X(3, 3, 3, 1)                                                         \
    X(0, 1, 5, 1) X(0, 2, 5, 1) X(0, 3, 5, 1) X(0, 4, 5, 1) X(0, 5, 5, 1)
#define HDG_GEN_CASES(X)                                                                            \
    HDG_GEN_CASES_R1(X)                                                                             \
    X(0, 1, 1, 32) X(0, 2, 2, 32) X(0, 3, 3, 32) X(0, 4, 4, 32)                                       \
    X(0, 1, 5, 32) X(0, 2, 5, 32) X(0, 3, 5, 32) X(0, 4, 5, 32) X(0, 5, 5, 32)

constexpr int VAR_KF = 5;
constexpr int NSCHED = GEN_NSCHED;   // launch schedules of the condensation (see gen_sg)

// Calls `fn(K, KF, tables, list, count)` for every launch of the current mesh: one per degree
// class on a mesh of variable degree, one for all elements otherwise.
template <typename Fn>
int for_each_class(hdg_ctx* c, Fn fn) {
    if (!c->vardeg) return fn(c->k, c->k, c->tab, (const int32_t*)nullptr, c->n_elem);
    for (int k = 1; k <= 5; ++k) {
        if (c->cls_n[k] == 0) continue;
        const int e = fn(k, VAR_KF, c->tabk[k], c->d_cls[k], c->cls_n[k]);
        if (e) return e;
    }
    return 0;
}

// One class launch (op 0), whether schedule g.sched is built for it (op 1) or its scratch need in
// bytes (op 2).
struct GenOp {
    int op = 0, sched = 0;
    double a = 0;
    const double* f_loc = nullptr;
    void* scratch = nullptr;
    hipStream_t st = nullptr;
    size_t out = 0;
};

// BF: the split-BF16 matrix-core products (float only; elastic, Maxwell, GLM-Maxwell)
template <typename T, bool BF = false>
int gen_class(hdg_ctx* c, int K, int KF, const DeviceTables& tb, const int32_t* el, int64_t n, GenOp& g) {
    const int P = c->physics, R = c->nrhs;
#define HDG_CASE(PP, KK, FF, RR)                                                                        \
    if (P == PP && K == KK && KF == FF && R == RR) {                                                     \
        if (g.op == 1) {                                                                                 \
            g.out = (size_t)(gen_built<PP, KK, FF, RR, T>(g.sched) ? 1 : 0);                             \
            return 0;                                                                                    \
        }                                                                                                \
        if (g.op == 2) {                                                                                 \
            g.out = std::max({gen_scratch<PP, KK, FF, RR, T>(n, 0), gen_scratch<PP, KK, FF, RR, T>(n, 1),  \
                              gen_scratch<PP, KK, FF, RR, T>(n, 2), gen_scratch<PP, KK, FF, RR, T>(n, 3),     \
                              gen_scratch<PP, KK, FF, RR, T>(n, 4)});                                    \
            return 0;                                                                                    \
        }                                                                                                \
        if constexpr (BF && (PP == 0 || sizeof(T) != 4)) return -1;                                     \
        else return launch_gen<PP, KK, FF, RR, T, BF>(c, g.a, g.f_loc, tb, el, n, g.sched, (T*)g.scratch, g.st); \
    }
    HDG_GEN_CASES(HDG_CASE)
#undef HDG_CASE
    return -1;
}

// Degree classes of the mesh: (K, KF, tables, element list, count) for class slot k.
struct ClassRef {
    int K, KF;
    const DeviceTables* tb;
    const int32_t* el;
    int64_t n;
};
std::vector<std::pair<int, ClassRef>> gen_classes(hdg_ctx* c) {
    std::vector<std::pair<int, ClassRef>> v;
    if (!c->vardeg) {
        v.push_back({c->k, ClassRef{c->k, c->k, &c->tab, nullptr, c->n_elem}});
        return v;
    }
    for (int k = 1; k <= 5; ++k)
        if (c->cls_n[k] > 0) v.push_back({k, ClassRef{k, VAR_KF, &c->tabk[k], c->d_cls[k], c->cls_n[k]}});
    return v;
}

template <typename T, bool BF>
int gen_run(hdg_ctx* c, const ClassRef& cr, int k, GenOp g) {
    g.op = 0;
    g.scratch = (char*)c->d_xscratch + c->xs_off[k];
    return gen_class<T, BF>(c, cr.K, cr.KF, *cr.tb, cr.el, cr.n, g);
}

template <typename T, bool BF = false>
int dispatch_gen(hdg_ctx* c, double a, const double* f_loc) {
    const int pi = c->precision == HDG_FP64 ? 1 : 0;
    auto classes = gen_classes(c);
    // per-class scratch regions (classes may run concurrently inside the graph)
    size_t total = 0;
    for (auto& [k, cr] : classes) {
        GenOp q;
        q.op = 2;
        if (gen_class<T>(c, cr.K, cr.KF, *cr.tb, cr.el, cr.n, q)) return -1;
        c->xs_off[k] = total;
        total += (q.out + 255) / 256 * 256;
    }
    if (total > c->xscratch_bytes) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        if (c->sgexec) {   // a captured step reads the old scratch
            (void)hipGraphExecDestroy(c->sgexec);
            c->sgexec = nullptr;
        }
        if (c->d_xscratch) {
            (void)hipStreamSynchronize(c->stream);
            dev_release(c, c->d_xscratch);
        }
        c->d_xscratch = nullptr;
        c->xscratch_bytes = 0;
        const int er = dev_malloc(c, &c->d_xscratch, total);
        if (er) return er;
        c->xscratch_bytes = total;
    }
    GenOp g;
    g.a = a;
    g.f_loc = f_loc;
    g.st = c->stream;
    // schedules: tuned on the first condensation of a class (or read from the table), else 0
    bool tuned = false;
    for (auto& [k, cr] : classes) {
        if (c->sched[pi][k] > 0) {   // read from a tune table: keep it only if it is built here
            GenOp q;
            q.op = 1;
            q.sched = c->sched[pi][k];
            (void)gen_class<T>(c, cr.K, cr.KF, *cr.tb, cr.el, cr.n, q);
            if (q.out == 0) c->sched[pi][k] = -1;
        }
        if (c->sched[pi][k] >= 0) continue;
        bool built[NSCHED];
        int ns = 0;
        for (int sc = 0; sc < NSCHED; ++sc) {
            GenOp q;
            q.op = 1;
            q.sched = sc;
            (void)gen_class<T>(c, cr.K, cr.KF, *cr.tb, cr.el, cr.n, q);
            built[sc] = q.out != 0;
            ns += built[sc];
        }
        if (!c->autotune || ns < 2) {
            c->sched[pi][k] = 0;
            continue;
        }
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
            if (t0) (void)hipEventDestroy(t0);
            return -1;
        }
        float best = 0;
        int bs = 0, err = 0;
        for (int s = 0; s < NSCHED && !err; ++s) {
            if (!built[s]) continue;
            float ms = 0, t = 0;
            for (int rep = 0; rep < 2 && !err; ++rep) {   // the first run warms caches and code
                g.sched = s;
                err = hipEventRecord(t0, c->stream);
                if (!err) err = gen_run<T, BF>(c, cr, k, g);
                if (!err) err = hipEventRecord(t1, c->stream);
                if (!err) err = hipEventSynchronize(t1);
                if (!err) err = hipEventElapsedTime(&t, t0, t1);
                ms = rep ? std::min(ms, t) : t;
            }
            c->sched_ms[pi][k][s] = ms;
            if (s == 0 || ms < best) {
                best = ms;
                bs = s;
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        if (err) return err;
        c->sched[pi][k] = (int8_t)bs;
        tuned = true;
    }
    if (tuned && !c->tune_path.empty()) write_tune_table(c);
    int key = 0;
    for (auto& [k, cr] : classes) key = key * NSCHED + c->sched[pi][k];

    if (!c->use_graph || !c->vardeg || !c->side[0]) {
        for (auto& [k, cr] : classes) {
            g.sched = c->sched[pi][k];
            const int e = gen_run<T, BF>(c, cr, k, g);
            if (e) return e;
        }
        return 0;
    }
    // one graph: fork from side[0] to a side stream per class, join back into side[0]
    if (!c->gexec || c->g_a != a || c->g_f != f_loc || c->g_sched != key) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        hipStream_t s0 = c->side[0];
        if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) return -1;
        int err = hipEventRecord(c->ev_fork, s0);
        int i = 0;
        for (auto& [k, cr] : classes) {
            hipStream_t si = c->side[1 + i % 5];
            if (!err) err = hipStreamWaitEvent(si, c->ev_fork, 0);
            g.st = si;
            g.sched = c->sched[pi][k];
            if (!err) err = gen_run<T, BF>(c, cr, k, g);
            if (!err) err = hipEventRecord(c->ev_join[i], si);
            if (!err) err = hipStreamWaitEvent(s0, c->ev_join[i], 0);
            ++i;
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(s0, &graph);
        if (err || ee != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return err ? err : (int)ee;
        }
        const hipError_t ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            c->gexec = nullptr;
            return (int)ie;
        }
        c->g_a = a;
        c->g_f = f_loc;
        c->g_sched = key;
    }
    if (hipEventRecord(c->ev_in, c->stream) != hipSuccess || hipStreamWaitEvent(c->side[0], c->ev_in, 0) != hipSuccess ||
        hipGraphLaunch(c->gexec, c->side[0]) != hipSuccess || hipEventRecord(c->ev_out, c->side[0]) != hipSuccess ||
        hipStreamWaitEvent(c->stream, c->ev_out, 0) != hipSuccess)
        return -1;
    return 0;
}

template <typename T>
int dispatch_gen_rec(hdg_ctx* c, const double* lam, double* u) {
    const int P = c->physics, R = c->nrhs;
    return for_each_class(c, [&](int K, int KF, const DeviceTables& tb, const int32_t* el, int64_t n) {
#define HDG_CASE(PP, KK, FF, RR) \
    if (P == PP && K == KK && KF == FF && R == RR) return launch_gen_rec<PP, KK, FF, RR, T>(c, tb, el, n, lam, u);
        HDG_GEN_CASES_R1(HDG_CASE)
#undef HDG_CASE
        return -1;
    });
}

int dispatch_gen_ref(hdg_ctx* c, const double* u, const double* lam, bool chk, double* nrm) {
    const int P = c->physics, R = c->nrhs;
    return for_each_class(c, [&](int K, int KF, const DeviceTables& tb, const int32_t* el, int64_t n) {
#define HDG_CASE(PP, KK, FF, RR) \
    if (P == PP && K == KK && KF == FF && R == RR)            \
        return launch_gen_ref<PP, KK, FF, RR, float>(c, tb, el, n, u, lam, chk, nrm);
        HDG_GEN_CASES_R1(HDG_CASE)
#undef HDG_CASE
        return -1;
    });
}

__global__ void narrow_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Right-hand-side condensation with the kept factors (one right-hand side): the refinement pass
// at u = 0, lam = 0 (z = A^{-1} f in the z buffer, r_e = -C A^{-1} f into d_re)
template <typename T>
int dispatch_gen_rhs(hdg_ctx* c, const double* f_loc) {
    const int P = c->physics, R = c->nrhs;
    double* re_out = sizeof(T) == 8 ? (double*)c->d_re : c->d_re64;
    int e = for_each_class(c, [&](int K, int KF, const DeviceTables& tb, const int32_t* el, int64_t n) {
#define HDG_CASE(PP, KK, FF, RR)                                                                              \
    if (P == PP && K == KK && KF == FF && R == RR)                                                            \
        return launch_gen_ref<PP, KK, FF, RR, T>(c, tb, el, n, nullptr, nullptr, false, nullptr, f_loc, 1, re_out);
        HDG_GEN_CASES_R1(HDG_CASE)
#undef HDG_CASE
        return -1;
    });
    if (e || sizeof(T) == 8) return e;
    const int64_t nr = c->n_elem * c->n_tr * R;
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, c->stream, nr, c->d_re64,
                       (float*)c->d_re);
    return (int)hipGetLastError();
}

}  // namespace

int launch_condense_rhs_general(hdg_ctx* c, const double* f_loc) {
    if (!c->d_LU || c->nrhs != 1 || mr_supported(c)) return -1;
    if (c->precision == HDG_FP64) return dispatch_gen_rhs<double>(c, f_loc);
    if (!c->d_re64) return -1;
    return dispatch_gen_rhs<float>(c, f_loc);
}

int launch_refine_general(hdg_ctx* c, const double* u, const double* lam, bool check, double* nrm) {
    if (c->precision == HDG_FP64 || (check && !nrm)) return -1;
    if (mr_supported(c)) return launch_refine_mr(c, u, lam, check, nrm);
    return dispatch_gen_ref(c, u, lam, check, nrm);
}

bool general_supported(int physics, int k, int kf, int nrhs) {
#define HDG_CASE(PP, KK, FF, RR) \
    if (physics == PP && k == KK && kf == FF && nrhs == RR) return true;
    HDG_GEN_CASES(HDG_CASE)
#undef HDG_CASE
    return false;
}

int var_face_degree() { return VAR_KF; }


int launch_condense_general(hdg_ctx* c, double a, const double* f_loc) {
    if (c->precision == HDG_FP64) return dispatch_gen<double>(c, a, f_loc);
    if (c->precision == HDG_MIXED_BF16) return dispatch_gen<float, true>(c, a, f_loc);
    return dispatch_gen<float>(c, a, f_loc);
}

int launch_recover_general(hdg_ctx* c, const double* lam, double* u) {
    if (mr_supported(c)) return launch_recover_mr(c, lam, u);
    if (c->precision == HDG_FP64) return dispatch_gen_rec<double>(c, lam, u);
    return dispatch_gen_rec<float>(c, lam, u);
}

}  // namespace hdg
