// Acoustic HDG recovery and mixed-precision refinement with 32 right-hand sides (meshes of
// uniform or variable polynomial degree), on the FP64 matrix cores of gfx950.
//
// With r right-hand sides every operator of the element stage system (App. A, acoustic blocks
// of the first-order system of Sec. 2) acts on an n x r block of vectors, so each application
// is a dense contraction.  The 32 columns of an element form two blocks of 16; one wavefront
// owns one (element, block) pair and every product is a chain of 16x16x4 FP64 MFMA tiles whose
// 16 columns are the right-hand sides of that block.
//
// Register layout of a block of vectors with n rows (the accumulator layout of the
// instruction): element v of tile t of lane l holds row 16 t + (l >> 4) + 4 v of column l & 15.
// Element s & 3 of tile s >> 2 is then exactly the B operand of k-step s (rows 4 s .. 4 s + 3),
// so the output of one product feeds the next without data movement.  Rows past n are kept at
// zero; A operands are read at clamped indices (finite values), so padded k columns meet zero
// B rows and padded output rows are dropped.  A operands come from the reference tables and the
// element factors through the caches, each 16-lane group reading consecutive addresses: Sr and
// the oriented face tables E_f are also kept transposed for the products that need the other
// orientation, and the face mass tables Mf are symmetric.
//
// Acoustic blocks (notation of condense_general.hip): u1 = velocity (3 N rows), u2 = pressure
// (N rows), G = J^{-1}, s_f face measure ratios, n_f unit outward normals, tau stabilisation,
// a stage coefficient, rho and c the material, amass = a / (rho c^2).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "physics.h"

namespace hdg {

namespace {

constexpr int MR_R = 32;      // right-hand sides
constexpr int MR_NPERM = 6;   // orientations of a triangular face

typedef double mfd4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mfd4 mma(double a, double b, mfd4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfd4 mzero() { return mfd4{0.0, 0.0, 0.0, 0.0}; }
// Product chain of S k-steps: load(s, a) fetches the NA A operands of step s into a[], mac(s, a)
// issues its MFMAs.  The operands of step s + 2 are fetched while step s computes (two register
// buffers); a scheduling fence after each step keeps the compiler from hoisting the loads of
// the whole unrolled chain to its top, which would exhaust the registers.
// The loads also take an opaque zero z, produced after the fence, into their addresses: the
// table loads are invariant, and without that dependence later passes still gather them at the
// top of the chain.
__device__ __forceinline__ unsigned mr_token() {
    unsigned z = 0;
    asm volatile("" : "+v"(z));
    return z;
}
template <int S, int NA, typename LoadF, typename MacF>
__device__ __forceinline__ void mr_chain(LoadF&& load, MacF&& mac) {
    double buf[2][NA];
    const unsigned z0 = mr_token();
    load(0, buf[0], z0);
    if constexpr (S > 1) load(1, buf[1], z0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        mac(s, buf[s & 1]);
        __builtin_amdgcn_sched_barrier(0);
        if (s + 2 < S) load(s + 2, buf[s & 1], mr_token());
    }
}

// Opaque copy of a uniform pointer: the table loads of an element then depend on the element
// loop, so they are not hoisted out of it (keeping whole tables live in registers).
template <typename P>
__device__ __forceinline__ P* opaque(P* p) {
    asm volatile("" : "+s"(p));
    return p;
}
// Opaque copy of the lane index, taken per element: the per-lane address offsets of the A
// operands are then computed next to their loads instead of all at once before the loop.
__device__ __forceinline__ int opaque_lane() {
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}

// Wave-uniform values loaded through vector memory (element indices, offsets, face data) moved
// to scalar registers, so that the addresses derived from them stay scalar.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)v), hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Clamped row index.  Per-lane offsets are unsigned 32-bit throughout, so that every load
// addresses a scalar base plus one 32-bit vector offset.
__device__ __forceinline__ unsigned cl(unsigned v, unsigned hi) { return v < hi ? v : hi; }

template <int K, int KF>
struct MrDims {
    static constexpr int N = dimp(K, 3), NF = dimp(KF, 2), TT = 4 * NF, N1 = 3 * N, NLOC = 4 * N;
    static constexpr int NT = (N + 15) / 16;     // row tiles of a volume vector
    static constexpr int KS = (N + 3) / 4;       // k-steps over a volume vector
    static constexpr int NTF = (NF + 15) / 16;   // row tiles of a face vector
    static constexpr int KSF = (NF + 3) / 4;     // k-steps over a face vector
    static constexpr int NP = 16 * NT;           // padded rows of a volume vector
    static constexpr int LS = NP + 1;            // LDS row stride of the Cholesky factor
};

struct MrArgs {
    const int32_t* elist;    // elements of the launched degree class (null: 0 .. n-1)
    const int64_t* loc_off;  // compact local dof offsets (null: e * NLOC)
    const int8_t* efnf;      // [e][4] size of the face space of each local face (null: NF)
    int64_t strZ, strz, strL;   // per-element strides of Z2, z and L
};

struct MrElem {
    double J, aro, tau, amass;
    double G[3][3], nf[4][3], sf[4];
};

__device__ __forceinline__ void mr_elem(const double* __restrict__ g, double a, MrElem& m) {
    m.J = g[0];
    for (int r = 0; r < 3; ++r)
        for (int x = 0; x < 3; ++x) m.G[r][x] = g[1 + 3 * r + x];
    for (int f = 0; f < 4; ++f) {
        m.sf[f] = g[10 + f];
        for (int x = 0; x < 3; ++x) m.nf[f][x] = g[14 + 3 * f + x];
    }
    const double rho = g[GEO_PAR], cc = g[GEO_PAR + 1];
    m.aro = a * rho;
    m.tau = g[GEO_STAB];
    m.amass = a / (rho * cc * cc);
}

// Recovery from the stored factors (T: their precision):
//   u2   = z2 - Z2 lam_e
//   u1_x = z1_x - (1/(a rho)) [ (1/|J|) sum_f s_f n_f,x E_f lam_f - sum_r G_rx Sr_r^T u2 ]
template <int K, int KF, typename T>
__global__ __launch_bounds__(256, 2) void recover_mr_kernel(
    int64_t ne, double a, const double* __restrict__ geom, const int32_t* __restrict__ eperm,
    const int32_t* __restrict__ eface, const double* __restrict__ Sr, const double* __restrict__ EfT,
    const T* __restrict__ Zs, const T* __restrict__ zs, const double* __restrict__ lam, double* __restrict__ u,
    MrArgs va) {
    using Dm = MrDims<K, KF>;
    constexpr int N = Dm::N, NF = Dm::NF, TT = Dm::TT, N1 = Dm::N1, NLOC = Dm::NLOC;
    constexpr int NT = Dm::NT, KS = Dm::KS, KSF = Dm::KSF, R = MR_R;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t w = (int64_t)blockIdx.x * wpb + wave; w < 2 * ne; w += (int64_t)gridDim.x * wpb) {
        const unsigned lane = opaque_lane(), lr = lane & 15, lg = lane >> 4;
        const int64_t ie = w >> 1;
        const unsigned q = (unsigned)(w & 1) * 16 + lr;
        const int64_t e = va.elist ? (int64_t)uni((int)va.elist[ie]) : ie;
        MrElem m;
        mr_elem(geom + e * GEOM_STRIDE, a, m);
        const T* Ze = Zs + e * va.strZ;
        const T* ze = zs + e * va.strz;
        double* ue = u + (va.loc_off ? uni(va.loc_off[e]) : e * NLOC) * R;
        const double* SrE = opaque(Sr);
        int64_t F[4];
        int nfv[4];
        const double* Et[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            F[f] = uni((int)eface[e * 4 + f]);
            nfv[f] = va.efnf ? uni((int)va.efnf[e * 4 + f]) : NF;
            Et[f] = EfT + (size_t)(f * MR_NPERM + uni((int)eperm[e * 4 + f])) * NF * N;
        }
        // trace value of face mode l as a B operand (0 past the face's space)
        auto lam_at = [&](int f, unsigned l, unsigned z) {
            const double v = (lam + F[f] * NF * R)[cl(l, NF - 1) * R + q + z];
            return l < (unsigned)nfv[f] ? v : 0.0;
        };
        // pressure
        double u2[NT][4];
        {
            mfd4 acc[NT];
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) acc[mt] = mzero();
            mr_chain<4 * KSF, NT + 1>(
                [&](int st, double* A, unsigned z) {
                    const int f = st / KSF;
                    const unsigned l = 4 * (st % KSF) + (lg + z);
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt)
                        A[mt] = (double)Ze[cl(16 * mt + (lr + z), N - 1) * TT + f * NF + cl(l, NF - 1)];
                    A[NT] = lam_at(f, l, z);
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt) acc[mt] = mma(A[mt], A[NT], acc[mt]);
                });
#pragma unroll
            for (int mt = 0; mt < NT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const unsigned orow = 16 * mt + lg + 4 * v;
                    double x = 0.0;
                    if (orow < (unsigned)N) {
                        x = (double)ze[(N1 + orow) * R + q] - acc[mt][v];
                        ue[(N1 + orow) * R + q] = x;
                    }
                    u2[mt][v] = x;
                }
        }
        // velocity
        const double invJ = 1.0 / m.J, iaro = 1.0 / m.aro;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            const unsigned i = cl(16 * mt + lr, N - 1);
            mfd4 aE[4], aS[3];
#pragma unroll
            for (int f = 0; f < 4; ++f) aE[f] = mzero();
#pragma unroll
            for (int r = 0; r < 3; ++r) aS[r] = mzero();
            mr_chain<KSF, 8>(
                [&](int s, double* A, unsigned z) {
                    const unsigned l = 4 * s + (lg + z);
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        A[f] = Et[f][cl(l, NF - 1) * N + (i + z)];
                        A[4 + f] = lam_at(f, l, z);
                    }
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int f = 0; f < 4; ++f) aE[f] = mma(A[f], A[4 + f], aE[f]);
                });
            mr_chain<KS, 3>(
                [&](int s, double* A, unsigned z) {
                    const unsigned j = cl(4 * s + (lg + z), N - 1);
#pragma unroll
                    for (int r = 0; r < 3; ++r) A[r] = SrE[(r * N + j) * N + (i + z)];
                },
                [&](int s, const double* A) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) aS[r] = mma(A[r], u2[s >> 2][s & 3], aS[r]);
                });
            const unsigned z = mr_token();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const unsigned orow = 16 * mt + lg + 4 * v;
                if (orow < (unsigned)N) {
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        double t1 = 0.0, t2 = 0.0;
#pragma unroll
                        for (int f = 0; f < 4; ++f) t1 += m.nf[f][x] * m.sf[f] * aE[f][v];
#pragma unroll
                        for (int r = 0; r < 3; ++r) t2 += m.G[r][x] * aS[r][v];
                        const unsigned o = (x * N + orow) * R + q;
                        ue[o] = (double)ze[o + z] - (t1 * invJ - t2) * iaro;
                    }
                }
            }
        }
    }
}

// Mixed-precision refinement step: FP64 residual of the full stage system, correction right-hand
// side through the stored FP32 factors (Z2, the Cholesky factor L of the Schur block):
//   s1_x = f1_x - |J| a rho u1_x + |J| sum_r G_rx Sr_r^T u2 - sum_f s_f n_f,x E_f lam_f
//   s2   = f2 - |J| sum_r Sr_r (sum_x G_rx u1_x) - |J| amass u2 - tau sum_f s_f Mf_f u2
//          + tau sum_f s_f E_f lam_f
//   te_f = s_f E_f^T (sum_x n_f,x u1_x + tau u2) - tau s_f lam_f            (trace residual)
//   z1'  = s1 / (|J| a rho), stored in FP32
//   st   = s2 - (1/(a rho)) sum_r Sr_r (sum_x G_rx s1_x)
//   re64_f = Z2_f^T st - (s_f / (|J| a rho)) E_f^T (sum_x n_f,x s1_x) - te_f  (0 on masked modes)
//   z2'  = L^{-T} L^{-1} st
// The residual is FP64 throughout; the velocity residual enters the correction (st, re64, z1')
// rounded to FP32 like the factors that correct it, read back from z1'.  The velocity u1 is
// streamed from memory as B operands; the pressure vectors u2 and s2 live in LDS in the register
// layout (element v of tile t of lane l at (4 t + v) 64 + l), read as B operands per k-step.
// The two wavefronts of a workgroup are the two column blocks of one element; they share the
// element's factor L, staged in LDS with its upper triangle and diagonal zeroed, for the
// substitutions (one row per step, the pivot row's values broadcast across the four row groups).
// CHK (the convergence check of the refinement): stop after the residuals, leave re64 = -te_f
// and write nrm[e][q] = |(s1, s2)| of element e, column q.
template <int K, int KF, bool CHK>
__global__ __launch_bounds__(128, 2) void refine_mr_kernel(
    int64_t ne, double a, const double* __restrict__ geom, const int32_t* __restrict__ eperm,
    const int32_t* __restrict__ eface, const double* __restrict__ Sr, const double* __restrict__ SrT,
    const double* __restrict__ Mf, const double* __restrict__ Ef, const double* __restrict__ EfT,
    const float* __restrict__ Zs, const float* __restrict__ Lst, const double* __restrict__ u,
    const double* __restrict__ lam, const double* __restrict__ f, float* __restrict__ zout,
    double* __restrict__ re64, double* __restrict__ nrm, MrArgs va) {
    using Dm = MrDims<K, KF>;
    constexpr int N = Dm::N, NF = Dm::NF, TT = Dm::TT, N1 = Dm::N1, NLOC = Dm::NLOC;
    constexpr int NT = Dm::NT, KS = Dm::KS, KSF = Dm::KSF, NTF = Dm::NTF, NP = Dm::NP, LS = Dm::LS;
    constexpr int R = MR_R, NV = NT * 4 * 64;
    __shared__ float Ls[NP * LS];
    __shared__ double dinv[NP];
    __shared__ double Vs[2][2][NV];   // [wavefront][u2, s2]
    const int cb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double* U2 = Vs[cb][0];
    double* S2 = Vs[cb][1];
    for (int64_t ie = blockIdx.x; ie < ne; ie += gridDim.x) {
        const unsigned lane = opaque_lane(), lr = lane & 15, lg = lane >> 4;
        const unsigned q = cb * 16 + lr;
        const int64_t e = va.elist ? (int64_t)uni((int)va.elist[ie]) : ie;
        const float* Le = Lst + e * va.strL;
        __syncthreads();   // both wavefronts are done with the previous element's factor
        for (int idx = threadIdx.x; idx < NP * NP; idx += 128) {
            const int i = idx / NP, j = idx % NP;
            Ls[i * LS + j] = (i < N && j < i) ? Le[i * N + j] : 0.f;
        }
        for (int i = threadIdx.x; i < NP; i += 128) dinv[i] = i < N ? 1.0 / (double)Le[i * N + i] : 0.0;

        MrElem m;
        mr_elem(geom + e * GEOM_STRIDE, a, m);
        const int64_t loc = (va.loc_off ? uni(va.loc_off[e]) : e * NLOC) * R;
        const double* ue = u + loc;
        const double* fe = f + loc;
        const float* Ze = Zs + e * va.strZ;
        float* zo = zout + e * va.strz;
        double* rq = re64 + e * TT * R;
        const double* SrE = opaque(Sr);
        const double* SrTE = opaque(SrT);
        const double* MfE = opaque(Mf);
        int64_t F[4];
        int nfv[4];
        const double *Eo[4], *Et[4];
#pragma unroll
        for (int fc = 0; fc < 4; ++fc) {
            F[fc] = uni((int)eface[e * 4 + fc]);
            nfv[fc] = va.efnf ? uni((int)va.efnf[e * 4 + fc]) : NF;
            const size_t off = (size_t)(fc * MR_NPERM + uni((int)eperm[e * 4 + fc])) * N * NF;
            Eo[fc] = Ef + off;
            Et[fc] = EfT + off;
        }
        // trace value of face mode l (0 past the face's space)
        auto lam_at = [&](int fc, unsigned l, unsigned z) {
            const double v = (lam + F[fc] * NF * R)[cl(l, NF - 1) * R + q + z];
            return l < (unsigned)nfv[fc] ? v : 0.0;
        };
        // k-step s of velocity component x (rows 4 s + lg) from u, zero past N
        auto u1_at = [&](int x, int s, unsigned z) {
            const double v = ue[(x * N + cl(4 * s + lg, N - 1)) * R + q + z];
            return 4 * s + lg < (unsigned)N ? v : 0.0;
        };
        // the same from the FP32 velocity residual, stored as z1' = s1 / (|J| a rho)
        const double jaro = m.J * m.aro, ijaro = 1.0 / jaro;
        auto s1_at = [&](int x, int s, unsigned z) {
            const double v = (double)zo[(x * N + cl(4 * s + lg, N - 1)) * R + q + z];
            return 4 * s + lg < (unsigned)N ? v * jaro : 0.0;
        };
        // element s of a vector held in LDS (k-step s as a B operand, or tile s >> 2, element s & 3)
        auto at = [&](const double* V, int s, unsigned z) { return V[s * 64 + lane + z]; };
#pragma unroll
        for (int t = 0; t < NT * 4; ++t) {
            const unsigned orow = 16 * (t >> 2) + lg + 4 * (t & 3);
            const double v = ue[(N1 + cl(orow, N - 1)) * R + q];
            U2[t * 64 + lane] = orow < (unsigned)N ? v : 0.0;
        }

        // trace residual, kept as -te_f in re64 until the end (two faces per pass)
#pragma unroll
        for (int fp = 0; fp < 2; ++fp) {
            mfd4 acc[2][NTF];
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int mt = 0; mt < NTF; ++mt) acc[k][mt] = mzero();
            mr_chain<KS, 2 * NTF + 4>(
                [&](int s, double* A, unsigned z) {
                    const unsigned i = cl(4 * s + lg + z, N - 1);
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int mt = 0; mt < NTF; ++mt)
                            A[k * NTF + mt] = Eo[2 * fp + k][i * NF + cl(16 * mt + lr + z, NF - 1)];
#pragma unroll
                    for (int x = 0; x < 3; ++x) A[2 * NTF + x] = u1_at(x, s, z);
                    A[2 * NTF + 3] = at(U2, s, z);
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int fc = 2 * fp + k;
                        const double b = m.nf[fc][0] * A[2 * NTF] + m.nf[fc][1] * A[2 * NTF + 1] +
                                         m.nf[fc][2] * A[2 * NTF + 2] + m.tau * A[2 * NTF + 3];
#pragma unroll
                        for (int mt = 0; mt < NTF; ++mt) acc[k][mt] = mma(A[k * NTF + mt], b, acc[k][mt]);
                    }
                });
            const unsigned z = mr_token();
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int mt = 0; mt < NTF; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int fc = 2 * fp + k;
                        const unsigned l = 16 * mt + lg + 4 * v;
                        if (l < (unsigned)NF) {
                            const double te = m.sf[fc] * (acc[k][mt][v] - m.tau * lam_at(fc, l, z));
                            rq[(fc * NF + l) * R + q] = l < (unsigned)nfv[fc] ? -te : 0.0;
                        }
                    }
        }
        // s2 <- f2 - |J| sum_r Sr_r (sum_x G_rx u1_x) - |J| amass u2
        {
            mfd4 acc[NT];
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) acc[mt] = mzero();
            mr_chain<KS, 3 * NT + 3>(
                [&](int s, double* A, unsigned z) {
                    const unsigned j = cl(4 * s + lg + z, N - 1);
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt)
                            A[r * NT + mt] = SrTE[(r * N + j) * N + cl(16 * mt + lr + z, N - 1)];
#pragma unroll
                    for (int x = 0; x < 3; ++x) A[3 * NT + x] = u1_at(x, s, z);
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const double b = m.G[r][0] * A[3 * NT] + m.G[r][1] * A[3 * NT + 1] + m.G[r][2] * A[3 * NT + 2];
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt) acc[mt] = mma(A[r * NT + mt], b, acc[mt]);
                    }
                });
            const unsigned z = mr_token();
#pragma unroll
            for (int mt = 0; mt < NT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const unsigned orow = 16 * mt + lg + 4 * v;
                    const double t = fe[(N1 + cl(orow, N - 1)) * R + q + z] - m.J * acc[mt][v] -
                                     m.J * m.amass * at(U2, 4 * mt + v, z);
                    S2[(4 * mt + v) * 64 + lane] = orow < (unsigned)N ? t : 0.0;
                }
        }
        // residuals, one row tile at a time: s1 (stored as z1') and s2
        double sq = 0.0;   // CHK: this lane's share of |(s1, s2)|^2 of column q
        double wsm[4];
#pragma unroll
        for (int fc = 0; fc < 4; ++fc) wsm[fc] = m.sf[fc] * m.tau;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            const unsigned i = cl(16 * mt + lr, N - 1);
            mfd4 aS[3], aM[4];
#pragma unroll
            for (int r = 0; r < 3; ++r) aS[r] = mzero();
#pragma unroll
            for (int fc = 0; fc < 4; ++fc) aM[fc] = mzero();
            mr_chain<KS, 8>(
                [&](int s, double* A, unsigned z) {
                    const unsigned j = cl(4 * s + lg + z, N - 1);
#pragma unroll
                    for (int r = 0; r < 3; ++r) A[r] = SrE[(r * N + j) * N + i + z];
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) A[3 + fc] = MfE[(fc * N + j) * N + i + z];
                    A[7] = at(U2, s, z);
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) aS[r] = mma(A[r], A[7], aS[r]);
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) aM[fc] = mma(A[3 + fc], A[7], aM[fc]);
                });
            double t1[3][4];   // volume part of s1 on this row tile
            {
                const unsigned z = mr_token();
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const unsigned oc = cl(16 * mt + lg + 4 * v, N - 1);
#pragma unroll
                    for (int x = 0; x < 3; ++x)
                        t1[x][v] = fe[(x * N + oc) * R + q + z] - jaro * ue[(x * N + oc) * R + q + z] +
                                   m.J * (m.G[0][x] * aS[0][v] + m.G[1][x] * aS[1][v] + m.G[2][x] * aS[2][v]);
                    double mm = 0.0;
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) mm += wsm[fc] * aM[fc][v];
                    S2[(4 * mt + v) * 64 + lane + z] -= mm;
                }
            }
            mfd4 aE[4];
#pragma unroll
            for (int fc = 0; fc < 4; ++fc) aE[fc] = mzero();
            mr_chain<KSF, 8>(
                [&](int s, double* A, unsigned z) {
                    const unsigned l = 4 * s + lg + z;
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) {
                        A[fc] = Et[fc][cl(l, NF - 1) * N + i + z];
                        A[4 + fc] = lam_at(fc, l, z);
                    }
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) aE[fc] = mma(A[fc], A[4 + fc], aE[fc]);
                });
            {
                const unsigned z = mr_token();
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const unsigned orow = 16 * mt + lg + 4 * v;
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        double t = t1[x][v];
#pragma unroll
                        for (int fc = 0; fc < 4; ++fc) t -= m.nf[fc][x] * m.sf[fc] * aE[fc][v];
                        if (orow < (unsigned)N) {
                            if (CHK) sq += t * t;
                            else zo[(x * N + orow) * R + q] = (float)(t * ijaro);
                        }
                    }
                    double t = 0.0;
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) t += wsm[fc] * aE[fc][v];
                    const double sv = S2[(4 * mt + v) * 64 + lane + z] + t;
                    S2[(4 * mt + v) * 64 + lane + z] = orow < (unsigned)N ? sv : 0.0;
                    if (CHK && orow < (unsigned)N) sq += sv * sv;
                }
            }
        }
        if constexpr (CHK) {
            // the four row groups of column q hold lanes lr, lr + 16, lr + 32, lr + 48
            sq += __shfl_xor(sq, 16, 64);
            sq += __shfl_xor(sq, 32, 64);
            if (lg == 0) nrm[e * R + q] = sqrt(sq);
            continue;
        }
        // st = s2 - (1/(a rho)) sum_r Sr_r (sum_x G_rx s1_x)
        {
            const double iaro = 1.0 / m.aro;
            mfd4 acc[NT];
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) acc[mt] = mzero();
            mr_chain<KS, 3 * NT + 3>(
                [&](int s, double* A, unsigned z) {
                    const unsigned j = cl(4 * s + lg + z, N - 1);
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt)
                            A[r * NT + mt] = SrTE[(r * N + j) * N + cl(16 * mt + lr + z, N - 1)];
#pragma unroll
                    for (int x = 0; x < 3; ++x) A[3 * NT + x] = s1_at(x, s, z);
                },
                [&](int, const double* A) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const double b = m.G[r][0] * A[3 * NT] + m.G[r][1] * A[3 * NT + 1] + m.G[r][2] * A[3 * NT + 2];
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt) acc[mt] = mma(A[r * NT + mt], b, acc[mt]);
                    }
                });
            const unsigned z = mr_token();
#pragma unroll
            for (int mt = 0; mt < NT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const bool ok = 16 * mt + lg + 4 * v < (unsigned)N;
                    const double t = S2[(4 * mt + v) * 64 + lane + z] - iaro * acc[mt][v];
                    S2[(4 * mt + v) * 64 + lane + z] = ok ? t : 0.0;
                }
        }
        // correction right-hand side of the trace system (two faces per pass)
#pragma unroll
        for (int fp = 0; fp < 2; ++fp) {
            mfd4 acc[2][NTF];
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int mt = 0; mt < NTF; ++mt) acc[k][mt] = mzero();
            mr_chain<KS, 4 * NTF + 4>(
                [&](int s, double* A, unsigned z) {
                    const unsigned i = cl(4 * s + lg + z, N - 1);
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int mt = 0; mt < NTF; ++mt) {
                            const int fc = 2 * fp + k;
                            const unsigned l = cl(16 * mt + lr + z, NF - 1);
                            A[k * NTF + mt] = (double)Ze[i * TT + fc * NF + l];
                            A[(2 + k) * NTF + mt] = Eo[fc][i * NF + l];
                        }
#pragma unroll
                    for (int x = 0; x < 3; ++x) A[4 * NTF + x] = s1_at(x, s, z);
                    A[4 * NTF + 3] = at(S2, s, z);
                },
                [&](int, const double* A) {
                    const double bst = A[4 * NTF + 3];
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int mt = 0; mt < NTF; ++mt) acc[k][mt] = mma(A[k * NTF + mt], bst, acc[k][mt]);
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int fc = 2 * fp + k;
                        const double b = -m.sf[fc] * ijaro *
                                         (m.nf[fc][0] * A[4 * NTF] + m.nf[fc][1] * A[4 * NTF + 1] +
                                          m.nf[fc][2] * A[4 * NTF + 2]);
#pragma unroll
                        for (int mt = 0; mt < NTF; ++mt) acc[k][mt] = mma(A[(2 + k) * NTF + mt], b, acc[k][mt]);
                    }
                });
            const unsigned z = mr_token();
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int mt = 0; mt < NTF; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int fc = 2 * fp + k;
                        const unsigned l = 16 * mt + lg + 4 * v;
                        if (l < (unsigned)NF) {
                            const unsigned o = (fc * NF + l) * R + q;
                            rq[o] = l < (unsigned)nfv[fc] ? acc[k][mt][v] + rq[o + z] : 0.0;
                        }
                    }
        }
        // z2' = L^{-T} L^{-1} st
        double st[NT][4];
#pragma unroll
        for (int t = 0; t < NT * 4; ++t) st[t >> 2][t & 3] = S2[t * 64 + lane];
        __syncthreads();   // factor staged
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const int t = r >> 4, vv = (r >> 2) & 3, g = r & 3;
            const unsigned z = mr_token();
            const double yv = st[t][vv] * dinv[r];
            const double y = __shfl(yv, lr + 16 * g);
            st[t][vv] = lg == (unsigned)g ? y : st[t][vv];
#pragma unroll
            for (int t2 = t; t2 < NT; ++t2)
#pragma unroll
                for (int v2 = (t2 == t ? vv : 0); v2 < 4; ++v2)
                    st[t2][v2] -= (double)Ls[(16 * t2 + lg + 4 * v2) * LS + r + z] * y;
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int r = N - 1; r >= 0; --r) {
            const int t = r >> 4, vv = (r >> 2) & 3, g = r & 3;
            const unsigned z = mr_token();
            const double xv = st[t][vv] * dinv[r];
            const double x = __shfl(xv, lr + 16 * g);
            st[t][vv] = lg == (unsigned)g ? x : st[t][vv];
#pragma unroll
            for (int t2 = 0; t2 <= t; ++t2)
#pragma unroll
                for (int v2 = 0; v2 < (t2 == t ? vv + 1 : 4); ++v2)
                    st[t2][v2] -= (double)Ls[r * LS + 16 * t2 + lg + 4 * v2 + z] * x;
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const unsigned orow = 16 * mt + lg + 4 * v;
                if (orow < (unsigned)N) zo[(N1 + orow) * R + q] = (float)st[mt][v];
            }
    }
}

MrArgs mr_args(const hdg_ctx* c, const int32_t* elist, int N, int NLOC, int TT) {
    MrArgs va{};
    va.elist = elist;
    if (c->vardeg) {
        va.loc_off = c->d_loc_off;
        va.efnf = c->d_efnf;
        va.strZ = (int64_t)c->Ns * c->n_tr;
        va.strz = (int64_t)c->n_loc * c->nrhs;
        va.strL = (int64_t)c->Ns * c->Ns;
    } else {
        va.strZ = (int64_t)N * TT;
        va.strz = (int64_t)NLOC * MR_R;
        va.strL = (int64_t)N * N;
    }
    return va;
}

template <int K, int KF, typename T>
int launch_rec_mr(hdg_ctx* c, const DeviceTables& tb, const int32_t* el, int64_t n, const double* lam, double* u) {
    using Dm = MrDims<K, KF>;
    constexpr int WPB = 4;
    const void* kern = (const void*)recover_mr_kernel<K, KF, T>;
    const int64_t groups = (2 * n + WPB - 1) / WPB;
    const int grid = (int)std::min<int64_t>(groups, resident_groups(kern, 64 * WPB));
    hipLaunchKernelGGL((recover_mr_kernel<K, KF, T>), dim3(grid), dim3(64 * WPB), 0, c->stream, n, c->last_a,
                       c->d_geom, c->d_eperm, c->d_eface, tb.Sr, tb.EfT, (const T*)c->d_Zt, (const T*)c->d_z, lam, u,
                       mr_args(c, el, Dm::N, Dm::NLOC, Dm::TT));
    return (int)hipGetLastError();
}

template <int K, int KF, bool CHK>
int launch_ref_mr(hdg_ctx* c, const DeviceTables& tb, const int32_t* el, int64_t n, const double* u,
                  const double* lam, double* nrm) {
    using Dm = MrDims<K, KF>;
    const void* kern = (const void*)refine_mr_kernel<K, KF, CHK>;
    const int grid = (int)std::min<int64_t>(n, resident_groups(kern, 128));
    hipLaunchKernelGGL((refine_mr_kernel<K, KF, CHK>), dim3(grid), dim3(128), 0, c->stream, n, c->last_a, c->d_geom,
                       c->d_eperm, c->d_eface, tb.Sr, tb.SrT, tb.Mf, tb.Ef, tb.EfT, (const float*)c->d_Zt,
                       (const float*)c->d_LU, u, lam, c->d_f_saved, (float*)c->d_z, c->d_re64, nrm,
                       mr_args(c, el, Dm::N, Dm::NLOC, Dm::TT));
    return (int)hipGetLastError();
}

// (volume degree, face-table degree) of the built configurations: uniform meshes use face
// degree = volume degree, meshes of variable degree face tables of degree 5 for every class
#define HDG_MR_CASES(X) X(1, 1) X(2, 2) X(3, 3) X(4, 4) X(1, 5) X(2, 5) X(3, 5) X(4, 5) X(5, 5)

template <typename Fn>
int mr_for_each_class(hdg_ctx* c, Fn fn) {
    if (!c->vardeg) return fn(c->k, c->k, c->tab, (const int32_t*)nullptr, c->n_elem);
    for (int k = 1; k <= 5; ++k) {
        if (c->cls_n[k] == 0) continue;
        const int e = fn(k, var_face_degree(), c->tabk[k], c->d_cls[k], c->cls_n[k]);
        if (e) return e;
    }
    return 0;
}

}  // namespace

bool mr_supported(const hdg_ctx* c) {
    return c->physics == HDG_ACOUSTIC && c->dim == 3 && c->nrhs == MR_R;
}

int launch_recover_mr(hdg_ctx* c, const double* lam, double* u) {
    const bool f64 = c->precision == HDG_FP64;
    return mr_for_each_class(c, [&](int K, int KF, const DeviceTables& tb, const int32_t* el, int64_t n) {
#define HDG_CASE(KK, FF)                                                              \
    if (K == KK && KF == FF)                                                          \
        return f64 ? launch_rec_mr<KK, FF, double>(c, tb, el, n, lam, u)             \
                   : launch_rec_mr<KK, FF, float>(c, tb, el, n, lam, u);
        HDG_MR_CASES(HDG_CASE)
#undef HDG_CASE
        return -1;
    });
}

int launch_refine_mr(hdg_ctx* c, const double* u, const double* lam, bool check, double* nrm) {
    if (c->precision == HDG_FP64 || (check && !nrm)) return -1;
    return mr_for_each_class(c, [&](int K, int KF, const DeviceTables& tb, const int32_t* el, int64_t n) {
#define HDG_CASE(KK, FF)                                                        \
    if (K == KK && KF == FF)                                                    \
        return check ? launch_ref_mr<KK, FF, true>(c, tb, el, n, u, lam, nrm)   \
                     : launch_ref_mr<KK, FF, false>(c, tb, el, n, u, lam, nrm);
        HDG_MR_CASES(HDG_CASE)
#undef HDG_CASE
        return -1;
    });
}

}  // namespace hdg
