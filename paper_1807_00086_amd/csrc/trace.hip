// Global trace system in FP64 (section 2.4.2): owner-computes assembly of the element Schur
// complements into face-block rows, block-Jacobi preconditioned conjugate gradients.
//
// BSR layout: row F has nslot = 1 + 2d blocks; slot 0 is the diagonal, slots 1 + s d + m are
// the other faces of the s-th neighbour element of F.  Blocks are stored column-major
// (bsr[F][slot][b][a] is entry (a, b)) so that the threads of one row block read adjacent
// words.  Dirichlet faces have identity rows; couplings to Dirichlet faces are moved to the
// right-hand side.  The system is assembled as K_sign * K so that it is positive definite.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

namespace hdg {

namespace {
constexpr int NT = 256;

// K_e[r][c] of an element matrix stored in full (ktile = 0) or as its tiles on and above the
// diagonal (symmetric K_e, tiles of ktile x ktile)
template <typename T>
__device__ __forceinline__ double kget(const T* K, int tt, int r, int c, int ktile) {
    return (ktile > 0 && r / ktile > c / ktile) ? (double)K[c * tt + r] : (double)K[r * tt + c];
}

// MAT = false: the right-hand side only (the matrix of an earlier assembly is kept)
// One workgroup per face (grid-stride).  The face's neighbour slots are resolved once per face
// into an LDS table (element, row and column offsets in K_e, valid columns, whether the
// neighbour is a Dirichlet face), so every matrix entry is one load of K_e after the table:
// the chain of dependent loads (neighbour face, its flag, then K_e) is not repeated per entry.
template <typename T, bool MAT>
__global__ __launch_bounds__(NT) void assemble_kernel(
    int64_t nf, int d, int bs, int tt, int R, double sign, int ktile, const int32_t* __restrict__ face_elem,
    const int32_t* __restrict__ face_lf, const uint8_t* __restrict__ face_bnd,
    const int32_t* __restrict__ eface, const T* __restrict__ Ke, const T* __restrict__ re,
    const double* __restrict__ lam_bnd, const int8_t* __restrict__ face_nf, double* __restrict__ bsr,
    double* __restrict__ rhs) {
    // face_nf (variable degree): modes of a face at or above its own size are padding and get
    // identity rows with a zero right-hand side.  face_bnd: 1 Dirichlet (identity rows, the
    // values moved to the neighbours' right-hand sides), 2 Neumann (the one element's flux rows
    // with lam_bnd, the tested flux datum, added to the right-hand side)
    constexpr int MS = 7;                       // slots of a block row (3D; 2D uses 5)
    __shared__ int32_t s_e[MS], s_r0[MS], s_c0[MS], s_nc[MS], s_F2[MS], s_dir[MS];
    const int nslot = 1 + 2 * d, nv = d + 1;
    for (int64_t F = blockIdx.x; F < nf; F += gridDim.x) {
        const bool bnd = face_bnd[F] == 1;
        const int nfF = face_nf ? (int)face_nf[F] : bs;
        const int32_t es[2] = {face_elem[2 * F], face_elem[2 * F + 1]};
        const int32_t ls[2] = {face_lf[2 * F], face_lf[2 * F + 1]};
        if (threadIdx.x >= 1 && threadIdx.x < nslot) {
            // slot 1 + s d + m: the m-th other face of the element on side s
            const int sl = threadIdx.x, sd = (sl - 1) / d, m = (sl - 1) % d;
            const int32_t e = es[sd];
            int32_t ee = -1, r0 = 0, c0 = 0, nc = 0, F2 = -1, dir = 0;
            if (e >= 0) {
                const int lf = ls[sd];
                const int q = (m < lf) ? m : m + 1;
                F2 = eface[(size_t)e * nv + q];
                dir = face_bnd[F2] == 1;
                ee = e;
                r0 = lf * bs;
                c0 = q * bs;
                nc = face_nf ? (int)face_nf[F2] : bs;
            }
            s_e[sl] = ee;
            s_r0[sl] = r0;
            s_c0[sl] = c0;
            s_nc[sl] = nc;
            s_F2[sl] = F2;
            s_dir[sl] = dir;
        }
        __syncthreads();
        double* B = bsr + (size_t)F * nslot * bs * bs;
        for (int idx = threadIdx.x; MAT && idx < nslot * bs * bs; idx += NT) {
            const int slot = idx / (bs * bs), rem = idx - slot * (bs * bs);
            const int b = rem / bs, a = rem - b * bs;   // column-major block
            double v = 0.0;
            if (slot == 0) {
                if (bnd || a >= nfF || b >= nfF) {
                    v = (a == b) ? 1.0 : 0.0;
                } else {
#pragma unroll
                    for (int sd = 0; sd < 2; ++sd) {
                        if (es[sd] < 0) continue;
                        const T* K = Ke + (size_t)es[sd] * tt * tt;
                        v += kget(K, tt, ls[sd] * bs + a, ls[sd] * bs + b, ktile);
                    }
                    v *= sign;
                }
            } else if (!bnd) {
                const int32_t e = s_e[slot];
                if (e >= 0 && !s_dir[slot] && a < nfF && b < s_nc[slot])
                    v = sign * kget(Ke + (size_t)e * tt * tt, tt, s_r0[slot] + a, s_c0[slot] + b, ktile);
            }
            B[idx] = v;
        }
        for (int idx = threadIdx.x; idx < bs * R; idx += NT) {
            const int a = idx / R, r = idx - a * R;
            double v;
            if (bnd) {
                v = a < nfF ? lam_bnd[((size_t)F * bs + a) * R + r] : 0.0;
            } else if (a >= nfF) {
                v = 0.0;
            } else {
                v = face_bnd[F] == 2 ? lam_bnd[((size_t)F * bs + a) * R + r] : 0.0;
                for (int sd = 0; sd < 2; ++sd) {
                    const int32_t e = es[sd];
                    if (e < 0) continue;
                    const int lf = ls[sd];
                    const T* K = Ke + (size_t)e * tt * tt;
                    double acc = (double)re[((size_t)e * tt + lf * bs + a) * R + r];
                    // Dirichlet neighbours of this element: their values move to this row
                    for (int m = 0; m < d; ++m) {
                        const int sl = 1 + sd * d + m;
                        if (!s_dir[sl]) continue;
                        const int32_t F2 = s_F2[sl];
                        const int c0 = s_c0[sl], nf2 = s_nc[sl];
                        for (int b = 0; b < nf2; ++b)
                            acc -= kget(K, tt, lf * bs + a, c0 + b, ktile) * lam_bnd[((size_t)F2 * bs + b) * R + r];
                    }
                    v += acc;
                }
                v *= sign;
            }
            rhs[((size_t)F * bs + a) * R + r] = v;
        }
        __syncthreads();   // the slot table is rewritten for the next face
    }
}

// Element-centric assembly of the matrix and the right-hand side (3D, uniform degree, one
// right-hand side, trace blocks of BS <= 10): the face-centric kernel reads each K_e once per
// face of the element, strips of rows whose lower tiles come from the mirrored upper tiles, so
// its loads fetch K_e more than twice over.  Here a wavefront reads its element's stored tiles
// once into LDS and scatters them: the off-diagonal blocks K_{F,G} (F, G faces of one element)
// belong to that element alone and are stored; a face's diagonal block and right-hand side
// receive one contribution per element of the face, added atomically onto what
// assemble_init_kernel wrote.  At most two contributions meet in one place (onto zero, or onto
// the Neumann datum of a face with one element) and IEEE addition is commutative, so the sums do
// not depend on the order of the atomics: every run gives the same bits.
template <int BS, bool MAT>
__global__ __launch_bounds__(NT) void assemble_init_kernel(int64_t nf, double sign, const int32_t* __restrict__ face_elem,
                                                           const uint8_t* __restrict__ face_bnd,
                                                           const double* __restrict__ lam_bnd,
                                                           double* __restrict__ bsr, double* __restrict__ rhs) {
    constexpr int BB = BS * BS, NS = 7, W = MAT ? BB : BS;   // threads per face
    const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (gid >= nf * W) return;
    const int64_t F = gid / W;
    const int rem = (int)(gid - F * W);
    const int fb = face_bnd[F];
    const bool dir = fb == 1;
    if (MAT) {
        const int b = rem / BS, a = rem - b * BS;
        double* B = bsr + (size_t)F * NS * BB + rem;
        B[0] = dir && a == b ? 1.0 : 0.0;
        // blocks no element writes: all of a Dirichlet row, the slots of a missing side
        const bool z0 = dir || face_elem[2 * F] < 0, z1 = dir || face_elem[2 * F + 1] < 0;
#pragma unroll
        for (int sl = 1; sl < NS; ++sl)
            if (sl <= 3 ? z0 : z1) B[(size_t)sl * BB] = 0.0;
    }
    if (rem < BS) {
        const double lb = fb ? lam_bnd[(size_t)F * BS + rem] : 0.0;
        rhs[(size_t)F * BS + rem] = dir ? lb : sign * lb;
    }
}

template <typename T, int BS, bool MAT>
__global__ __launch_bounds__(64) void assemble_elem_kernel(int64_t ne, int ktile, double sign,
                                                           const int32_t* __restrict__ face_elem,
                                                           const uint8_t* __restrict__ face_bnd,
                                                           const int32_t* __restrict__ eface,
                                                           const T* __restrict__ Ke, const T* __restrict__ re,
                                                           const double* __restrict__ lam_bnd,
                                                           double* __restrict__ bsr, double* __restrict__ rhs) {
    constexpr int NV = 4, TT = NV * BS, BB = BS * BS, NS = 7, LD = TT + 1, NL = (TT * TT + 63) / 64;
    __shared__ double Ks[TT * LD];   // odd row stride: a column read by consecutive rows spreads over the banks
    __shared__ int32_t sF[NV], sSide[NV], sDir[NV];
    const int lane = threadIdx.x;
    // K_e(r, c) as stored: row-major, only the tiles on and above the diagonal when ktile > 0
    auto kl = [&](int r, int c) -> double {
        return (ktile > 0 && r / ktile > c / ktile) ? Ks[c * LD + r] : Ks[r * LD + c];
    };
    for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
        if (lane < NV) {
            const int32_t F = eface[(size_t)e * NV + lane];
            sF[lane] = F;
            sSide[lane] = face_elem[2 * (size_t)F] == (int32_t)e ? 0 : 1;
            sDir[lane] = face_bnd[F] == 1;
        }
        __syncthreads();
        // the right-hand side alone reads K_e only next to Dirichlet faces
        const bool needK = MAT || sDir[0] || sDir[1] || sDir[2] || sDir[3];
        // the whole TT x TT region in one batch of loads (the entries below the stored tiles are
        // read and never used), so that every load of the element is in flight at once
        const T* K = Ke + (size_t)e * TT * TT;
        T kv[NL];
        if (needK) {
#pragma unroll
            for (int u = 0; u < NL; ++u) {
                const int idx = lane + 64 * u;
                kv[u] = idx < TT * TT ? K[idx] : T(0);
            }
#pragma unroll
            for (int u = 0; u < NL; ++u) {
                const int idx = lane + 64 * u;
                if (idx < TT * TT) {
                    const int r = idx / TT, c = idx - r * TT;
                    Ks[r * LD + c] = (double)kv[u];
                }
            }
        }
        __syncthreads();
        // matrix: block (i, q) of K_e goes to row F_i, the slot of face q (q == i: the diagonal)
        for (int idx = lane; MAT && idx < NV * NV * BB; idx += 64) {
            const int iq = idx / BB, rem = idx - iq * BB;
            const int i = iq / NV, q = iq - i * NV;
            if (sDir[i]) continue;
            const int b = rem / BS, a = rem - b * BS;
            const double v = sign * kl(i * BS + a, q * BS + b);
            double* Brow = bsr + (size_t)sF[i] * NS * BB + rem;
            if (q == i) {
                unsafeAtomicAdd(Brow, v);
            } else {
                const int sl = 1 + sSide[i] * 3 + (q < i ? q : q - 1);
                Brow[(size_t)sl * BB] = sDir[q] ? 0.0 : v;
            }
        }
        // right-hand side: r_e rows of face i, minus the couplings to Dirichlet faces times their
        // values
        for (int idx = lane; idx < NV * BS; idx += 64) {
            const int i = idx / BS, a = idx - i * BS;
            if (sDir[i]) continue;
            double acc = (double)re[(size_t)e * TT + i * BS + a];
            for (int q = 0; q < NV; ++q) {
                if (q == i || !sDir[q]) continue;
                const double* lb = lam_bnd + (size_t)sF[q] * BS;
                for (int b = 0; b < BS; ++b) acc -= kl(i * BS + a, q * BS + b) * lb[b];
            }
            unsafeAtomicAdd(rhs + (size_t)sF[i] * BS + a, sign * acc);
        }
        __syncthreads();   // Ks and the face table are rewritten for the next element
    }
}

// right-hand side of a correction equation (the trace rows of the FP64 residual): sum over the
// face's elements of the FP64 per-element contributions, plus the tested flux datum on Neumann
// faces; Dirichlet faces carry a zero correction
__global__ __launch_bounds__(NT) void assemble_rhs64_kernel(int64_t nf, int bs, int tt, int R, double sign,
                                                            const int32_t* __restrict__ face_elem,
                                                            const int32_t* __restrict__ face_lf,
                                                            const uint8_t* __restrict__ face_bnd,
                                                            const double* __restrict__ re64,
                                                            const double* __restrict__ lam_bnd,
                                                            double* __restrict__ rhs) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nf * bs * R) return;
    const int64_t F = gid / ((int64_t)bs * R);
    const int rem = (int)(gid % ((int64_t)bs * R));
    double v = 0.0;
    if (face_bnd[F] != 1) {
        if (face_bnd[F] == 2) v = lam_bnd[gid];
        for (int s = 0; s < 2; ++s) {
            const int32_t e = face_elem[2 * F + s];
            if (e < 0) continue;
            const int lf = face_lf[2 * F + s];
            v += re64[((size_t)e * tt + lf * bs) * R + rem];
        }
        v *= sign;
    }
    rhs[gid] = v;
}

// block sizes of the built 3D configurations (m_trace * N_F: acoustic k = 1..5, Maxwell
// k = 3, elastic k = 4) get the fixed-size kernels
#define HDG_BS_CASES(X) X(3) X(6) X(10) X(15) X(20) X(21) X(45)

// inverse of each diagonal block by Gauss-Jordan without pivoting (the blocks are SPD):
// one wavefront per face, the block and its inverse in LDS (bs <= 48)
constexpr int BI_MAX = 48;
__global__ __launch_bounds__(64) void block_inverse_kernel(int64_t nf, int nslot, int bs,
                                                           const double* __restrict__ bsr,
                                                           double* __restrict__ pinv) {
    __shared__ double M[BI_MAX * BI_MAX];
    __shared__ double V[BI_MAX * BI_MAX];
    __shared__ double fcol[BI_MAX];
    const int lane = threadIdx.x;
    for (int64_t F = blockIdx.x; F < nf; F += gridDim.x) {
        const double* A = bsr + (size_t)F * nslot * bs * bs;   // slot 0, column-major
        for (int i = lane; i < bs * bs; i += 64) {
            M[i] = A[i];
            V[i] = ((i % bs) == (i / bs)) ? 1.0 : 0.0;
        }
        __syncthreads();
        // column-major: entry (r, c) at c*bs + r
        for (int j = 0; j < bs; ++j) {
            const double ip = 1.0 / M[j * bs + j];
            __syncthreads();
            for (int c = lane; c < bs; c += 64) {
                M[c * bs + j] *= ip;
                V[c * bs + j] *= ip;
            }
            for (int r = lane; r < bs; r += 64) fcol[r] = M[j * bs + r];   // column j before elimination
            __syncthreads();
            for (int idx = lane; idx < bs * bs; idx += 64) {
                const int c = idx / bs, r = idx % bs;
                if (r == j) continue;
                const double fct = fcol[r];
                M[c * bs + r] -= fct * M[c * bs + j];
                V[c * bs + r] -= fct * V[c * bs + j];
            }
            __syncthreads();
        }
        double* Inv = pinv + (size_t)F * bs * bs;
        for (int i = lane; i < bs * bs; i += 64) Inv[i] = V[i];
        __syncthreads();
    }
}

// The same inverse for the built block sizes with the rows of a block in registers: a group of
// BS lanes per face (lane a holds row a of the block and of its inverse; 64 / BS faces per
// wavefront, the remaining lanes idle), the pivot row of each step broadcast by shuffles.  No LDS
// and no barriers.
template <int BS>
__global__ __launch_bounds__(NT) void block_inverse_rows_kernel(int64_t nf, int nslot, const double* __restrict__ bsr,
                                                                double* __restrict__ pinv) {
    constexpr int FPW = 64 / BS;
    const int lane = threadIdx.x & 63, fw = min(lane / BS, FPW), a = lane - fw * BS;
    const int64_t F = ((int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * FPW + fw;
    const bool ok = fw < FPW && F < nf;
    const int base = min(lane - a, 64 - BS);   // first lane of the group (idle lanes: any full group)
    const double* A = bsr + (size_t)(ok ? F : 0) * nslot * BS * BS + min(a, BS - 1);
    double m[BS], v[BS];
#pragma unroll
    for (int b = 0; b < BS; ++b) {
        m[b] = A[b * BS];
        v[b] = b == a ? 1.0 : 0.0;
    }
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const int src = base + j;
        const double ip = 1.0 / __shfl(m[j], src, 64);
        const double f = m[j] * ip;
        const bool piv = a == j;
#pragma unroll
        for (int b = j + 1; b < BS; ++b) {
            const double pb = __shfl(m[b], src, 64);
            m[b] = piv ? pb * ip : m[b] - f * pb;
        }
#pragma unroll
        for (int b = 0; b < BS; ++b) {
            const double pb = __shfl(v[b], src, 64);
            v[b] = piv ? pb * ip : v[b] - f * pb;
        }
    }
    if (ok) {
        double* out = pinv + (size_t)F * BS * BS + a;
#pragma unroll
        for (int b = 0; b < BS; ++b) out[b * BS] = v[b];
    }
}

// y = A x (one thread per row entry (F, a, r))
__global__ __launch_bounds__(NT) void bsr_spmv_kernel(int64_t nf, int nslot, int bs, int R,
                                                      const int32_t* __restrict__ cols,
                                                      const double* __restrict__ bsr,
                                                      const double* __restrict__ x, double* __restrict__ y,
                                                      const int* __restrict__ done) {
    if (done && *done) return;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = nf * bs * R;
    if (gid >= total) return;
    int r = (int)(gid % R);
    int64_t Fa = gid / R;
    int64_t F = Fa / bs;
    int a = (int)(Fa % bs);
    double acc = 0.0;
    for (int s = 0; s < nslot; ++s) {
        int32_t cF = cols[F * nslot + s];
        if (cF < 0) continue;
        const double* B = bsr + ((size_t)F * nslot + s) * bs * bs;
        const double* xv = x + (size_t)cF * bs * R + r;
        for (int b = 0; b < bs; ++b) acc += B[b * bs + a] * xv[b * R];
    }
    y[gid] = acc;
}

// The same with the block size and the blocks per row fixed at compile time: the row's
// NS * BS matrix loads are independent and unrolled (slots without a neighbour read a valid
// x entry whose product is discarded).
// M: precision of the stored blocks (FP64, or the FP32 copy used by the refinement's correction
// solves); products and sums in FP64.
template <int BS, int NS, typename M>
__global__ __launch_bounds__(NT) void bsr_spmv_fixed_kernel(int64_t nf, int R, const int32_t* __restrict__ cols,
                                                            const M* __restrict__ bsr,
                                                            const double* __restrict__ x, double* __restrict__ y,
                                                            const int* __restrict__ done) {
    if (done && *done) return;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nf * BS * R) return;
    const int r = (int)(gid % R);
    const int64_t Fa = gid / R;
    const int64_t F = Fa / BS;
    const int a = (int)(Fa % BS);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int32_t cF = cols[F * NS + s];
        const M* B = bsr + ((size_t)F * NS + s) * BS * BS + a;
        const double* xv = x + (size_t)max(cF, 0) * BS * R + r;
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < BS; ++b) t += (double)B[b * BS] * xv[b * R];
        acc += cF >= 0 ? t : 0.0;
    }
    y[gid] = acc;
}

// The same products for 32 right-hand sides: one wavefront per block row (face) F, its
// BS x 32 output as 16x16x4 FP64 MFMA tiles over (block rows, right-hand sides); the stored
// blocks are column-major (entry (a, b) at b BS + a), so the 16 lanes of an A-operand column
// read consecutive entries, and the B operands are 16 consecutive right-hand sides of a row of
// x.  NS = 1 with cols null applies the block diagonal (the preconditioner).  Rows and
// columns past BS are clamped on load (padded k rows of x are zero, padded output rows dropped).
// M = float reads the FP32 copy of the blocks and widens each entry to FP64 before the MFMA.
// DOT: the launch is grid-stride over faces and each workgroup also writes the partial sums per
// column of dv * y over its faces' rows to part[blk][32] (dv at the output rows: r for r.z
// after the preconditioner), reduced by dot_final_kernel.
typedef double mf64x4 __attribute__((ext_vector_type(4)));

template <int BS, int NS, typename M = double, bool DOT = false>
__global__ __launch_bounds__(256) void bsr_spmm32_kernel(int64_t nf, const int32_t* __restrict__ cols,
                                                         const M* __restrict__ bsr,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         const double* __restrict__ dv, double* __restrict__ part,
                                                         const int* __restrict__ done) {
    if (done && *done) return;
    constexpr int MT = (BS + 15) / 16, KS = (BS + 3) / 4, R = 32, SU = sizeof(M) == 4 ? 2 : 1;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double dacc[2] = {0.0, 0.0};
    auto face = [&](int64_t F) {
        mf64x4 acc[MT][2];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt][0] = acc[mt][1] = mf64x4{0.0, 0.0, 0.0, 0.0};
        // two slots in flight with FP32 blocks (2.61 -> 2.52 ms at 410k faces); FP64 blocks
        // measured no better unrolled
#pragma unroll SU
        for (int s = 0; s < NS; ++s) {
            const int cF = cols ? __builtin_amdgcn_readfirstlane(cols[F * NS + s]) : (int)F;
            if (cF < 0) continue;
            const M* B = bsr + ((size_t)F * NS + s) * BS * BS;
            const double* xv = x + (size_t)cF * BS * R;
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const int b = min(4 * kk + lg, BS - 1);
                const bool bok = 4 * kk + lg < BS;
                double xb[2];
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const double t = xv[b * R + 16 * nt + lr];
                    xb[nt] = bok ? t : 0.0;
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const double av = (double)B[b * BS + min(16 * mt + lr, BS - 1)];
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb[nt], acc[mt][nt], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int a = 16 * mt + lg + 4 * v;
                    if (a < BS) {
                        const size_t o = ((size_t)F * BS + a) * R + 16 * nt + lr;
                        y[o] = acc[mt][nt][v];
                        if (DOT) dacc[nt] += dv[o] * acc[mt][nt][v];
                    }
                }
    };
    if constexpr (!DOT) {   // one face per wavefront
        const int64_t F = (int64_t)blockIdx.x * 4 + wv;
        if (F >= nf) return;   // whole wavefronts
        face(F);
        return;
    } else {
        for (int64_t F = (int64_t)blockIdx.x * 4 + wv; F < nf; F += (int64_t)gridDim.x * 4) face(F);
        __shared__ double sh[4][R];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            double d = dacc[nt];
            d += __shfl_xor(d, 16);
            d += __shfl_xor(d, 32);
            if (lg == 0) sh[wv][16 * nt + lr] = d;
        }
        __syncthreads();
        if (threadIdx.x < R)
            part[(size_t)blockIdx.x * R + threadIdx.x] =
                sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
    }
}

template <int BS>
__global__ __launch_bounds__(NT) void block_apply_fixed_kernel(int64_t nf, int R, const double* __restrict__ pinv,
                                                               const double* __restrict__ x,
                                                               double* __restrict__ y, const int* __restrict__ done) {
    if (done && *done) return;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nf * BS * R) return;
    const int r = (int)(gid % R);
    const int64_t Fa = gid / R;
    const int64_t F = Fa / BS;
    const int a = (int)(Fa % BS);
    const double* B = pinv + (size_t)F * BS * BS + a;
    const double* xv = x + (size_t)F * BS * R + r;
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < BS; ++b) acc += B[b * BS] * xv[b * R];
    y[gid] = acc;
}

__global__ __launch_bounds__(NT) void block_apply_kernel(int64_t nf, int bs, int R,
                                                         const double* __restrict__ pinv,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ y, const int* __restrict__ done) {
    if (done && *done) return;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = nf * bs * R;
    if (gid >= total) return;
    int r = (int)(gid % R);
    int64_t Fa = gid / R;
    int64_t F = Fa / bs;
    int a = (int)(Fa % bs);
    const double* B = pinv + (size_t)F * bs * bs;
    const double* xv = x + (size_t)F * bs * R + r;
    double acc = 0.0;
    for (int b = 0; b < bs; ++b) acc += B[b * bs + a] * xv[b * R];
    y[gid] = acc;
}

// partial dot products per rhs column: out[blk][r]
__global__ __launch_bounds__(NT) void dot_partial_kernel(int64_t n, int R, const double* __restrict__ x,
                                                         const double* __restrict__ y,
                                                         double* __restrict__ part, const int* __restrict__ done) {
    if (done && *done) return;
    // thread t of a block owns column t % R of rows t / R, t / R + T, ... (T = NT / R rows per
    // pass): consecutive threads read consecutive entries of the row-major [n][R] vectors
    __shared__ double sh[NT];
    const int T = NT / R, t = threadIdx.x;
    double acc = 0.0;
    if (t < T * R) {
        const int r = t % R;
        for (int64_t i = (int64_t)blockIdx.x * T + t / R; i < n; i += (int64_t)gridDim.x * T)
            acc += x[i * R + r] * y[i * R + r];
    }
    sh[t] = acc;
    __syncthreads();
    if (R == 1) {
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (t < s) sh[t] += sh[t + s];
            __syncthreads();
        }
        if (t == 0) part[blockIdx.x] = sh[0];
    } else if (t < R) {
        double s = 0.0;
        for (int k = 0; k < T; ++k) s += sh[k * R + t];
        part[(size_t)blockIdx.x * R + t] = s;
    }
}

// partial column sums of the per-face partials part[F][32] of the 32-column sweeps: out[blk][r], in
// the thread layout of dot_partial_kernel
__global__ __launch_bounds__(NT) void colsum32_kernel(int64_t nf, const double* __restrict__ part,
                                                      double* __restrict__ out, const int* __restrict__ done) {
    if (done && *done) return;
    constexpr int R = 32, T = NT / R;
    __shared__ double sh[NT];
    const int t = threadIdx.x, r = t % R;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * T + t / R; i < nf; i += (int64_t)gridDim.x * T) acc += part[i * R + r];
    sh[t] = acc;
    __syncthreads();
    if (t < R) {
        double s = 0.0;
        for (int k = 0; k < T; ++k) s += sh[k * R + t];
        out[(size_t)blockIdx.x * R + t] = s;
    }
}

__global__ __launch_bounds__(NT) void dot_final_kernel(int nb, int R, const double* __restrict__ part,
                                                       double* __restrict__ out, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double sh[NT];
    if (R > 1) {   // thread t sums column t % R of rows t / R, t / R + NT / R, ...: coalesced reads
        const int T = NT / R, t = threadIdx.x;
        double acc = 0.0;
        if (t < T * R)
            for (int b = t / R; b < nb; b += T) acc += part[(size_t)b * R + t % R];
        sh[t] = acc;
        __syncthreads();
        if (t < R) {
            double s = 0.0;
            for (int k = 0; k < T; ++k) s += sh[k * R + t];
            out[t] = s;
        }
        return;
    }
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nb; b += NT) acc += part[(size_t)b * R + r];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[r] = sh[0];
        __syncthreads();
    }
}

// out = sum of nb partial sums (one column): 1024 threads, so that a few thousand partials take
// a few loads per thread
__global__ __launch_bounds__(1024) void sum_partials_kernel(int nb, const double* __restrict__ part,
                                                            double* __restrict__ out,
                                                            const int* __restrict__ done = nullptr) {
    if (done && *done) return;
    __shared__ double sh[16];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += 1024) acc += part[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += sh[w];
        *out = t;
    }
}

// CG update of one iteration in a single pass: x += alpha p (X), r -= alpha q (alpha = num/den per
// column), and the partial sums of the new r squared per column, in the thread layout of
// dot_partial_kernel (part[blk][r], reduced by dot_final_kernel)
template <bool X>
__device__ __forceinline__ void cg_update_body(int64_t n, int R, const double* __restrict__ num,
                                               const double* __restrict__ den, const double* __restrict__ p,
                                               const double* __restrict__ q, double* __restrict__ x,
                                               double* __restrict__ rv, double* __restrict__ part,
                                               const int* __restrict__ done, int* __restrict__ iters) {
    if (done && *done) return;
    if (iters && blockIdx.x == 0 && threadIdx.x == 0) ++*iters;
    __shared__ double sh[NT];
    const int T = NT / R, t = threadIdx.x;
    double acc = 0.0;
    if (t < T * R) {
        const int r = t % R;
        const double dd = den[r];
        const double al = (dd != 0.0) ? num[r] / dd : 0.0;
#pragma unroll 4
        for (int64_t i = (int64_t)blockIdx.x * T + t / R; i < n; i += (int64_t)gridDim.x * T) {
            const int64_t k = i * R + r;
            if constexpr (X) x[k] += al * p[k];
            const double rn = rv[k] - al * q[k];
            rv[k] = rn;
            acc += rn * rn;
        }
    }
    sh[t] = acc;
    __syncthreads();
    if (R == 1) {
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (t < s) sh[t] += sh[t + s];
            __syncthreads();
        }
        if (t == 0) part[blockIdx.x] = sh[0];
    } else if (t < R) {
        double s = 0.0;
        for (int k = 0; k < T; ++k) s += sh[k * R + t];
        part[(size_t)blockIdx.x * R + t] = s;
    }
}

__global__ __launch_bounds__(NT) void cg_update_kernel(int64_t n, int R, const double* __restrict__ num,
                                                       const double* __restrict__ den,
                                                       const double* __restrict__ p, const double* __restrict__ q,
                                                       double* __restrict__ x, double* __restrict__ rv,
                                                       double* __restrict__ part, const int* __restrict__ done,
                                                       int* __restrict__ iters) {
    cg_update_body<true>(n, R, num, den, p, q, x, rv, part, done, iters);
}

// the same without x (the 32-column SSOR CG applies x += alpha p in the next direction update)
__global__ __launch_bounds__(NT) void cg_resid_update_kernel(int64_t n, int R, const double* __restrict__ num,
                                                             const double* __restrict__ den,
                                                             const double* __restrict__ q, double* __restrict__ rv,
                                                             double* __restrict__ part) {
    cg_update_body<false>(n, R, num, den, nullptr, q, nullptr, rv, part, nullptr, nullptr);
}

// y += (num/den) x per column
__global__ __launch_bounds__(NT) void axpy_ratio_cols_kernel(int64_t n, int R, const double* __restrict__ num,
                                                             const double* __restrict__ den,
                                                             const double* __restrict__ x, double* __restrict__ y) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * R) return;
    const int r = (int)(gid % R);
    const double dd = den[r];
    y[gid] += (dd != 0.0 ? num[r] / dd : 0.0) * x[gid];
}

// p = z + beta p, beta = num/den per column
__global__ __launch_bounds__(NT) void xpby_cols_kernel(int64_t n, int R, const double* __restrict__ num,
                                                       const double* __restrict__ den,
                                                       const double* __restrict__ z, double* __restrict__ p,
                                                       const int* __restrict__ done) {
    if (done && *done) return;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * R) return;
    int r = (int)(gid % R);
    double dd = den[r];
    double be = (dd != 0.0) ? num[r] / dd : 0.0;
    p[gid] = z[gid] + be * p[gid];
}

__global__ __launch_bounds__(NT) void lincomb_kernel(int64_t n, double a, const double* __restrict__ x,
                                                     double b, const double* __restrict__ y,
                                                     double* __restrict__ out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n) return;
    out[gid] = a * x[gid] + (y ? b * y[gid] : 0.0);
}

__global__ __launch_bounds__(NT) void copy_bnd_kernel(int64_t nf, int bs, int R, const uint8_t* __restrict__ bnd,
                                                      const double* __restrict__ src, double* __restrict__ dst) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nf * bs * R) return;
    int64_t F = gid / ((int64_t)bs * R);
    if (bnd[F] == 1) dst[gid] = src[gid];   // Dirichlet values
}

// partial sums of squares per rhs column over the rows of the boundary faces only (the
// Dirichlet values and the tested Neumann data: the boundary part of the right-hand side),
// in the thread layout of dot_partial_kernel (rows are face-major: row / bs is the face)
__global__ __launch_bounds__(NT) void bnd_sq_partial_kernel(int64_t n, int R, int bs, const uint8_t* __restrict__ bnd,
                                                            const double* __restrict__ x, double* __restrict__ part) {
    __shared__ double sh[NT];
    const int T = NT / R, t = threadIdx.x;
    double acc = 0.0;
    if (t < T * R) {
        const int r = t % R;
        for (int64_t i = (int64_t)blockIdx.x * T + t / R; i < n; i += (int64_t)gridDim.x * T)
            if (bnd[i / bs]) acc += x[i * R + r] * x[i * R + r];
    }
    sh[t] = acc;
    __syncthreads();
    if (R == 1) {
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (t < s) sh[t] += sh[t + s];
            __syncthreads();
        }
        if (t == 0) part[blockIdx.x] = sh[0];
    } else if (t < R) {
        double s = 0.0;
        for (int k = 0; k < T; ++k) s += sh[k * R + t];
        part[(size_t)blockIdx.x * R + t] = s;
    }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

int resident_groups(const void* kernel, int block) {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return ncu * per_cu;
}

template <bool MAT>
static int launch_asm(hdg_ctx* c, const double* lam_bnd) {
    if (MAT) ++c->mat_version;
    if (c->dim == 3 && !c->d_face_nf && c->nrhs == 1 && c->n_tr == 4 * c->bs) {
        const int eg = (int)std::min<int64_t>(c->n_elem, 262144);
#define HDG_ASM_ELEM(B)                                                                                         \
        if (c->bs == B) {                                                                                      \
            hipLaunchKernelGGL((assemble_init_kernel<B, MAT>), dim3(nblk(c->n_faces * (MAT ? B * B : B))), dim3(NT), \
                               0, c->stream, c->n_faces, c->K_sign, c->d_face_elem, c->d_face_bnd, lam_bnd,     \
                               c->d_bsr, c->d_rhs);                                                            \
            if (c->precision == HDG_FP64)                                                                      \
                hipLaunchKernelGGL((assemble_elem_kernel<double, B, MAT>), dim3(eg), dim3(64), 0, c->stream,   \
                                   c->n_elem, c->ke_tile, c->K_sign, c->d_face_elem, c->d_face_bnd, c->d_eface, \
                                   (const double*)c->d_Ke, (const double*)c->d_re, lam_bnd, c->d_bsr, c->d_rhs); \
            else                                                                                               \
                hipLaunchKernelGGL((assemble_elem_kernel<float, B, MAT>), dim3(eg), dim3(64), 0, c->stream,    \
                                   c->n_elem, c->ke_tile, c->K_sign, c->d_face_elem, c->d_face_bnd, c->d_eface, \
                                   (const float*)c->d_Ke, (const float*)c->d_re, lam_bnd, c->d_bsr, c->d_rhs);  \
            return (int)hipGetLastError();                                                                     \
        }
        HDG_ASM_ELEM(3)
        HDG_ASM_ELEM(6)
        HDG_ASM_ELEM(10)
#undef HDG_ASM_ELEM
    }
    int grid = (int)std::min<int64_t>(c->n_faces, 65536);
    if (c->precision == HDG_FP64)
        hipLaunchKernelGGL((assemble_kernel<double, MAT>), dim3(grid), dim3(NT), 0, c->stream, c->n_faces, c->dim,
                           c->bs, c->n_tr, c->nrhs, c->K_sign, c->ke_tile, c->d_face_elem, c->d_face_lf, c->d_face_bnd,
                           c->d_eface, (const double*)c->d_Ke, (const double*)c->d_re, lam_bnd, c->d_face_nf,
                           c->d_bsr, c->d_rhs);
    else
        hipLaunchKernelGGL((assemble_kernel<float, MAT>), dim3(grid), dim3(NT), 0, c->stream, c->n_faces, c->dim,
                           c->bs, c->n_tr, c->nrhs, c->K_sign, c->ke_tile, c->d_face_elem, c->d_face_lf, c->d_face_bnd,
                           c->d_eface, (const float*)c->d_Ke, (const float*)c->d_re, lam_bnd, c->d_face_nf,
                           c->d_bsr, c->d_rhs);
    return (int)hipGetLastError();
}

int launch_assemble(hdg_ctx* c, const double* lam_bnd) { return launch_asm<true>(c, lam_bnd); }
int launch_assemble_rhs(hdg_ctx* c, const double* lam_bnd) { return launch_asm<false>(c, lam_bnd); }

int launch_assemble_rhs64(hdg_ctx* c, const double* re64, const double* lam_bnd) {
    const int64_t n = c->n_faces * c->bs * c->nrhs;
    hipLaunchKernelGGL(assemble_rhs64_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, c->bs, c->n_tr,
                       c->nrhs, c->K_sign, c->d_face_elem, c->d_face_lf, c->d_face_bnd, re64, lam_bnd, c->d_rhs);
    return (int)hipGetLastError();
}

int launch_block_inverse(hdg_ctx* c) {
    if (c->bs > BI_MAX) return -1;
    c->pinv_version = c->mat_version;
#define HDG_BS(B)                                                                                             \
    if (c->bs == B) {                                                                                         \
        constexpr int64_t FPB = (64 / B) * (NT / 64);                                                         \
        hipLaunchKernelGGL((block_inverse_rows_kernel<B>), dim3((unsigned)((c->n_faces + FPB - 1) / FPB)),     \
                           dim3(NT), 0, c->stream, c->n_faces, c->nslot, c->d_bsr, c->d_pinv);                 \
        return (int)hipGetLastError();                                                                        \
    }
    HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    int grid = (int)std::min<int64_t>(c->n_faces, 65536);
    hipLaunchKernelGGL(block_inverse_kernel, dim3(grid), dim3(64), 0, c->stream, c->n_faces, c->nslot, c->bs,
                       c->d_bsr, c->d_pinv);
    return (int)hipGetLastError();
}


static int64_t nblk_faces(const hdg_ctx* c) { return (c->n_faces + 3) / 4; }

// FP32 copy of the assembled trace matrix (mixed precision, 3D)
__global__ __launch_bounds__(NT) void to_f32_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

static void dot(hdg_ctx* c, const double* x, const double* y, double* out_dev);

// 32 right-hand sides: grid of the fused-dot launches (partials per workgroup in d_red)
static int dot_grid(const hdg_ctx* c) { return (int)std::max<int64_t>(1, std::min<int64_t>(nblk_faces(c), RED_MAX)); }

template <int BS, int NS, typename M>
static void launch_spmm32(hdg_ctx* c, const int32_t* cols, const M* blocks, const double* x, double* y,
                          double* dot_out) {
    if constexpr (NS == 1) {   // the fused dot is used for the preconditioner only
        if (dot_out) {
            const int g = dot_grid(c);
            hipLaunchKernelGGL((bsr_spmm32_kernel<BS, NS, M, true>), dim3(g), dim3(256), 0, c->stream,
                               c->n_faces, cols, blocks, x, y, x, c->d_red, c->cg_done);
            hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, g, 32, c->d_red, dot_out,
                               c->cg_done);
            return;
        }
    }
    hipLaunchKernelGGL((bsr_spmm32_kernel<BS, NS, M>), dim3(nblk_faces(c)), dim3(256), 0, c->stream, c->n_faces,
                       cols, blocks, x, y, (const double*)nullptr, (double*)nullptr, c->cg_done);
    if (dot_out) dot(c, x, y, dot_out);
}

static void spmv_other(hdg_ctx* c, const double* x, double* y, bool lowp);

// y = A x; with dot_out (device, R values) also dot_out = x . y per column.  The product keeps
// its one-face-per-wavefront grid and a separate dot: the grid-stride form with the dot in the
// epilogue measured slower (5.75 ms against 3.45 + 0.65 ms for FP64 blocks at 410k faces)
static void spmv(hdg_ctx* c, const double* x, double* y, bool lowp = false, double* dot_out = nullptr) {
    int64_t n = c->n_faces * c->bs * c->nrhs;
    if (c->nslot == 7 && c->nrhs == 32) {
#define HDG_BS(B)                                                                                          \
    if (c->bs == B) {                                                                                      \
        if (lowp && c->d_bsr32)                                                                            \
            launch_spmm32<B, 7, float>(c, c->d_bsr_cols, c->d_bsr32, x, y, dot_out);                        \
        else                                                                                               \
            launch_spmm32<B, 7, double>(c, c->d_bsr_cols, c->d_bsr, x, y, dot_out);                         \
        return;                                                                                            \
    }
        HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    }
    spmv_other(c, x, y, lowp);
    if (dot_out) dot(c, x, y, dot_out);
}

// one right-hand side, or neither 3D nor 32 right-hand sides
static void spmv_other(hdg_ctx* c, const double* x, double* y, bool lowp) {
    int64_t n = c->n_faces * c->bs * c->nrhs;
    if (c->nslot == 7) {
#define HDG_BS(B)                                                                                          \
    if (c->bs == B) {                                                                                      \
        if (lowp && c->d_bsr32)                                                                            \
            hipLaunchKernelGGL((bsr_spmv_fixed_kernel<B, 7, float>), dim3(nblk(n)), dim3(NT), 0, c->stream,  \
                               c->n_faces, c->nrhs, c->d_bsr_cols, c->d_bsr32, x, y, c->cg_done);          \
        else                                                                                               \
            hipLaunchKernelGGL((bsr_spmv_fixed_kernel<B, 7, double>), dim3(nblk(n)), dim3(NT), 0, c->stream, \
                               c->n_faces, c->nrhs, c->d_bsr_cols, c->d_bsr, x, y, c->cg_done);            \
        return;                                                                                            \
    }
        HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    }
    hipLaunchKernelGGL(bsr_spmv_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, c->nslot, c->bs,
                       c->nrhs, c->d_bsr_cols, c->d_bsr, x, y, c->cg_done);
}

static void precond_other(hdg_ctx* c, const double* x, double* y);

// y = P^-1 x (block Jacobi); with dot_out (device, R values) also dot_out = x . y per column
static void precond(hdg_ctx* c, const double* x, double* y, double* dot_out = nullptr) {
    if (c->nrhs == 32) {
#define HDG_BS(B)                                                                                          \
    if (c->bs == B) {                                                                                      \
        launch_spmm32<B, 1, double>(c, (const int32_t*)nullptr, c->d_pinv, x, y, dot_out);                 \
        return;                                                                                            \
    }
        HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    }
    precond_other(c, x, y);
    if (dot_out) dot(c, x, y, dot_out);
}

static void precond_other(hdg_ctx* c, const double* x, double* y) {
    int64_t n = c->n_faces * c->bs * c->nrhs;
#define HDG_BS(B)                                                                                            \
    if (c->bs == B) {                                                                                        \
        hipLaunchKernelGGL((block_apply_fixed_kernel<B>), dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces,   \
                           c->nrhs, c->d_pinv, x, y, c->cg_done);                                            \
        return;                                                                                              \
    }
    HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    hipLaunchKernelGGL(block_apply_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, c->bs, c->nrhs,
                       c->d_pinv, x, y, c->cg_done);
}

static void dot(hdg_ctx* c, const double* x, const double* y, double* out_dev) {
    int64_t n = c->n_faces * c->bs;
    hipLaunchKernelGGL(dot_partial_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, c->nrhs, x, y,
                       c->d_red, c->cg_done);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, c->nrhs, c->d_red,
                       out_dev, c->cg_done);
}

int launch_lincomb(hdg_ctx* c, int64_t n, double a, const double* x, double b, const double* y, double* out) {
    hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, n, a, x, b, y, out);
    return (int)hipGetLastError();
}

int launch_axpy(hdg_ctx* c, int64_t n, double alpha, const double* x, double* y) {
    return launch_lincomb(c, n, alpha, x, 1.0, y, y);
}

int launch_norm2(hdg_ctx* c, int64_t n, const double* x, double* host_out) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, 1, x, x, c->d_red,
                       (const int*)nullptr);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, 1, c->d_red,
                       c->d_scal + 7 * 32, (const int*)nullptr);
    hipError_t e = hipMemcpyAsync(host_out, c->d_scal + 7 * 32, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return (int)e;
    e = hipStreamSynchronize(c->stream);
    *host_out = std::sqrt(*host_out);
    return (int)e;
}

int launch_col_sq(hdg_ctx* c, int64_t n, int R, const double* x, double* host_out, bool bnd_only) {
    if (R < 1 || R > 32) return (int)hipErrorInvalidValue;
    if (bnd_only)
        hipLaunchKernelGGL(bnd_sq_partial_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, R, c->bs,
                           c->d_face_bnd, x, c->d_red);
    else
        hipLaunchKernelGGL(dot_partial_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, R, x, x, c->d_red,
                           (const int*)nullptr);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, R, c->d_red,
                       c->d_scal + 7 * 32, (const int*)nullptr);
    hipError_t e = hipMemcpyAsync(host_out, c->d_scal + 7 * 32, R * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return (int)e;
    return (int)hipStreamSynchronize(c->stream);
}

// Preconditioned CG on the assembled (sign-adjusted) system; all rhs columns iterate
// together with their own scalars.  Convergence is checked on the host every iteration.
int launch_bsr_f32(hdg_ctx* c) {
    if (!c->d_bsr32) return 0;
    c->bsr32_version = c->mat_version;
    const int64_t n = c->n_faces * c->nslot * c->bs * c->bs;
    hipLaunchKernelGGL(to_f32_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, n, c->d_bsr, c->d_bsr32);
    return (int)hipGetLastError();
}

int trace_cg(hdg_ctx* c, double* x, double tol, int* iters, double* relres, bool lowp) {
    const int R = c->nrhs;
    const int64_t n = c->n_faces * c->bs;
    double* rr = c->d_cg_r;
    double* zz = c->d_cg_z;
    double* pp = c->d_cg_p;
    double* qq = c->d_cg_q;
    double* s_rz = c->d_scal;            // [R]
    double* s_rz_new = c->d_scal + 32;   // [R]
    double* s_pq = c->d_scal + 64;       // [R]
    double* s_rr = c->d_scal + 96;       // [R]
    double* s_bb = c->d_scal + 128;      // [R]
    if (c->pinv_version != c->mat_version && launch_block_inverse(c)) return HDG_E_HIP;
    if (lowp && c->bsr32_version != c->mat_version && launch_bsr_f32(c)) return HDG_E_HIP;
    // boundary entries of x are the Dirichlet values (identity rows)
    hipLaunchKernelGGL(copy_bnd_kernel, dim3(nblk(n * R)), dim3(NT), 0, c->stream, c->n_faces, c->bs, R,
                       c->d_face_bnd, c->d_rhs, x);
    spmv(c, x, qq, lowp);
    launch_lincomb(c, n * R, 1.0, c->d_rhs, -1.0, qq, rr);
    precond(c, rr, zz);
    hipMemcpyAsync(pp, zz, n * R * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    dot(c, rr, zz, s_rz);
    dot(c, c->d_rhs, c->d_rhs, s_bb);
    double hb[32];
    hipMemcpyAsync(hb, s_bb, R * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int r = 0; r < R; ++r) hb[r] = std::sqrt(hb[r]) > 0 ? std::sqrt(hb[r]) : 1.0;
    int it = 0;
    double worst = 0.0;
    dot(c, rr, rr, s_rr);   // later iterations get it from the fused update
    double* hrr = c->h_rr;  // pinned: the copy is asynchronous
    for (it = 0; it <= c->krylov_maxit; ++it) {
        if (hipMemcpyAsync(hrr, s_rr, R * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipEventRecord(c->ev_rr, c->stream) != hipSuccess)
            return HDG_E_HIP;
        // the next product (reads p, writes q and p.q only) runs while the host waits for the
        // norms; if they meet the test it is simply not used
        if (it < c->krylov_maxit) spmv(c, pp, qq, lowp, s_pq);
        hipError_t e = hipEventSynchronize(c->ev_rr);
        if (e != hipSuccess) return HDG_E_HIP;
        worst = 0.0;
        bool nonfinite = false;
        for (int r = 0; r < R; ++r) {
            double v = std::sqrt(hrr[r]) / hb[r];
            if (!(v - v == 0.0)) nonfinite = true;   // NaN or inf (std::max would drop a NaN)
            else worst = std::max(worst, v);
        }
        if (nonfinite) {
            worst = std::numeric_limits<double>::quiet_NaN();
            break;
        }
        if (worst <= tol || it == c->krylov_maxit) break;
        hipLaunchKernelGGL(cg_update_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, R, s_rz, s_pq, pp,
                           qq, x, rr, c->d_red, (const int*)nullptr, (int*)nullptr);
        hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, R, c->d_red, s_rr,
                           (const int*)nullptr);
        precond(c, rr, zz, s_rz_new);
        hipLaunchKernelGGL(xpby_cols_kernel, dim3(nblk(n * R)), dim3(NT), 0, c->stream, n, R, s_rz_new, s_rz, zz,
                           pp, (const int*)nullptr);
        std::swap(s_rz, s_rz_new);   // the new r.z becomes the old one (no device copy)
    }
    if (iters) *iters = it;
    if (relres) *relres = worst;
    c->last_iters = it;
    if (!(worst <= tol)) return HDG_E_NOCONV;
    return HDG_OK;
}

namespace {
// ------------------------------------------------------------------ multicolour block SSOR
// The preconditioner works on the block-diagonally scaled matrix  Kt = W K W^T,  W = diag(R_F^{-1}),
// D_F = R_F R_F^T the Cholesky factor of the diagonal block of face F.  Kt has identity diagonal
// blocks, and block SSOR on Kt is block SSOR on K carried over by W (W (D+L) D^{-1} (D+U) W^T =
// (I + Lt)(I + Ut) for the strict block triangles Lt, Ut of Kt), so the iterates are the same; but
// the sweeps need no diagonal block or its inverse and the preconditioner of the transformed CG
// (z = D r) becomes the identity.  Per CG iteration the matrix traffic is one read of the
// off-diagonal blocks of Kt, against four more reads of the diagonal blocks without the scaling.
// The sweeps take the scaled diagonal blocks as the identity and the upper blocks as stored, so K
// must be symmetric to the last bit: every condensation path stores a symmetric K_e.

// R_F^{-1} of each diagonal block, D_F = R_F R_F^T (Cholesky, R_F lower triangular): a group of
// BS lanes per face, lane a holding row a of the block, then row a of R_F^{-1} (64 / BS faces per
// wavefront, the remaining lanes idle).  Right-looking factorisation, then the rows of R_F^{-1} in
// order, Y_a = (e_a - sum_{i<a} R(a,i) Y_i) / R(a,a), each finished row broadcast by shuffles.
// Blocks column-major (entry (r, c) at c BS + r).  A block that is not positive definite gives
// NaN, which the CG reports as not converged.
template <int BS>
__global__ __launch_bounds__(NT) void chol_rinv_kernel(int64_t nf, const double* __restrict__ bsr,
                                                       double* __restrict__ rinv) {
    constexpr int FPW = 64 / BS;
    const int lane = threadIdx.x & 63, fw = min(lane / BS, FPW), a = lane - fw * BS;
    const int64_t F = ((int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * FPW + fw;
    const bool ok = fw < FPW && F < nf;
    const int base = min(lane - a, 64 - BS);
    const double* A = bsr + (size_t)(ok ? F : 0) * 7 * BS * BS + min(a, BS - 1);
    double m[BS];
#pragma unroll
    for (int b = 0; b < BS; ++b) m[b] = A[b * BS];
    // m[j] becomes R(a, j) at step j; ri = 1 / R(a, a).  Lanes a < cc also update their upper
    // entry m[cc], which step cc then sets to zero.
    double ri = 0.0;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const double d = sqrt(__shfl(m[j], base + j, 64));
        const double rd = 1.0 / d;
        const double l = a == j ? d : (a > j ? m[j] * rd : 0.0);
        if (a == j) ri = rd;
        m[j] = l;
#pragma unroll
        for (int cc = j + 1; cc < BS; ++cc) m[cc] -= l * __shfl(l, base + cc, 64);
    }
    double y[BS];
#pragma unroll
    for (int b = 0; b < BS; ++b) y[b] = b == a ? ri : 0.0;
    // row i of R^{-1} is final once steps 0..i-1 have been subtracted; broadcast it to the rows below
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        const double mi = a > i ? m[i] * ri : 0.0;
#pragma unroll
        for (int b = 0; b <= i; ++b) y[b] -= mi * __shfl(y[b], base + i, 64);
    }
    if (ok) {
        double* out = rinv + (size_t)F * BS * BS + a;
#pragma unroll
        for (int b = 0; b < BS; ++b) out[b * BS] = y[b];
    }
}

// Broadcast of lane `src`'s value to the wavefront (src uniform)
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __hiloint2double(hi, lo);
}

// The same factor for blocks of 33..64 unknowns: one face per wavefront, lane a holding row a of
// the block and then of R_F^{-1} as in chol_rinv_kernel, the pivot columns and finished rows
// broadcast by readlane (the source lane is uniform) instead of shuffles.  Lanes past BS repeat
// the last row; nothing reads or stores their values.
template <int BS>
__global__ __launch_bounds__(256) void chol_rinv_wave_kernel(int64_t nf, const double* __restrict__ bsr,
                                                             double* __restrict__ rinv) {
    static_assert(BS > 32 && BS <= 64, "one face per wavefront");
    const int lane = threadIdx.x & 63, a = min(lane, BS - 1);
    const int64_t F = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (F >= nf) return;   // whole wavefronts
    const double* A = bsr + (size_t)F * 7 * BS * BS + a;
    double m[BS];
#pragma unroll
    for (int b = 0; b < BS; ++b) m[b] = A[b * BS];
    double ri = 0.0;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const double d = sqrt(lane_bcast(m[j], j));
        const double rd = 1.0 / d;
        const double l = a == j ? d : (a > j ? m[j] * rd : 0.0);
        if (a == j) ri = rd;
        m[j] = l;
#pragma unroll
        for (int cc = j + 1; cc < BS; ++cc) m[cc] -= l * lane_bcast(l, cc);
    }
    double y[BS];
#pragma unroll
    for (int b = 0; b < BS; ++b) y[b] = b == a ? ri : 0.0;
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        const double mi = a > i ? m[i] * ri : 0.0;
#pragma unroll
        for (int b = 0; b <= i; ++b) y[b] -= mi * lane_bcast(y[b], i);
    }
    if (lane < BS) {
        double* out = rinv + (size_t)F * BS * BS + lane;
#pragma unroll
        for (int b = 0; b < BS; ++b) out[b * BS] = y[b];
    }
}

// The same factor for the other block sizes above 21 (22..32, or above 64): one wavefront per face,
// the block in LDS (column-major), right-looking Cholesky with lane r updating row r of the
// trailing triangle, then lane cc forms column cc of R_F^{-1} in registers by forward
// substitution, x_i = (delta_{i,cc} - sum_{j<i} R(i,j) x_j) / R(i,i): x_j = 0 for j < cc, so the
// fully unrolled sums need no lane-dependent bounds and read R(i, j) as one broadcast per step.
template <int BS>
__global__ __launch_bounds__(64) void chol_rinv_lds_kernel(int64_t nf, const double* __restrict__ bsr,
                                                           double* __restrict__ rinv) {
    __shared__ double M[BS * BS];
    const int lane = threadIdx.x;
    for (int64_t F = blockIdx.x; F < nf; F += gridDim.x) {
        const double* A = bsr + (size_t)F * 7 * BS * BS;
        __syncthreads();   // the previous face's reads of M are done
        for (int i = lane; i < BS * BS; i += 64) M[i] = A[i];
        __syncthreads();
        for (int j = 0; j < BS; ++j) {
            const double d = sqrt(M[j * BS + j]);
            __syncthreads();
            if (lane >= j && lane < BS) M[j * BS + lane] = lane == j ? d : M[j * BS + lane] / d;
            __syncthreads();
            // trailing lower triangle: M(r, c) -= R(r, j) R(c, j) for j < c <= r, r = lane
            if (lane > j && lane < BS) {
                const double lr = M[j * BS + lane];
                for (int c = j + 1; c <= lane; ++c) M[c * BS + lane] -= lr * M[j * BS + c];
            }
            __syncthreads();
        }
        double x[BS];
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            double v = i == lane ? 1.0 : 0.0;
#pragma unroll
            for (int j = 0; j < i; ++j) v -= M[j * BS + i] * x[j];
            x[i] = v / M[i * BS + i];
        }
        if (lane < BS) {
            double* out = rinv + (size_t)F * BS * BS + (size_t)lane * BS;
#pragma unroll
            for (int i = 0; i < BS; ++i) out[i] = x[i];
        }
    }
}

// Off-diagonal blocks of Kt: Kt_{F,s} = R_F^{-1} K_{F,s} R_G^{-T} for the neighbour G of slot s
// (slots 1..6 of the block row), written to block dst[F][s-1] of the sweep order.  A group of BS
// lanes per face as in the factor kernel, one wavefront per workgroup: the group stages K_{F,s}
// and R_G^{-1} in LDS (each lane loads one row of both), then lane a forms
// u = (row a of R_F^{-1}) K_{F,s} and Kt(a, b) = u . (row b of R_G^{-1}).
template <int BS>
__global__ __launch_bounds__(64) void ssor_scale_kernel(int64_t nf, const int32_t* __restrict__ cols,
                                                        const int32_t* __restrict__ dst,
                                                        const double* __restrict__ bsr,
                                                        const double* __restrict__ rinv, double* __restrict__ out) {
    constexpr int FPW = 64 / BS;
    __shared__ double Ks[FPW][BS * BS];
    __shared__ double Rs[FPW][BS * BS];
    const int lane = threadIdx.x, fw = min(lane / BS, FPW), a = lane - fw * BS;
    const int64_t F = (int64_t)blockIdx.x * FPW + fw;
    const bool ok = fw < FPW && F < nf;
    const int g = min(fw, FPW - 1);
    double rf[BS];
    const double* RF = rinv + (size_t)(ok ? F : 0) * BS * BS + a;
#pragma unroll
    for (int i = 0; i < BS; ++i) rf[i] = RF[i * BS];
    for (int s = 1; s < 7; ++s) {
        const int32_t G = ok ? cols[F * 7 + s] : -1;
        const int32_t D = G >= 0 ? dst[F * 6 + s - 1] : -1;   // every neighbour has its sweep block
        if (D >= 0) {
            const double* K = bsr + ((size_t)F * 7 + s) * BS * BS + a;
            const double* RG = rinv + (size_t)G * BS * BS + a;
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                Ks[g][j * BS + a] = K[j * BS];
                Rs[g][j * BS + a] = RG[j * BS];
            }
        }
        __syncthreads();
        if (D >= 0) {
            double u[BS];
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < BS; ++i) acc += rf[i] * Ks[g][j * BS + i];
                u[j] = acc;
            }
            double* O = out + (size_t)D * BS * BS + a;
#pragma unroll
            for (int b = 0; b < BS; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < BS; ++j) acc += u[j] * Rs[g][j * BS + b];
                O[b * BS] = acc;
            }
        }
        __syncthreads();
    }
}

// The same blocks on the FP64 matrix cores, for the larger face blocks: one face per wavefront, its
// six slots in turn, the products as 16x16x4 tiles.  With X(r, c) stored at X[c * BS + r]:
//   U^T  = K_{F,s}^T R_F^{-T}   (rows j, columns a, sum over i),
//   Kt^T = R_G^{-1} U^T        (rows b, columns a, sum over j),
// and Kt(a, b) = Kt^T(b, a) is stored at b * BS + a.  Element v of accumulator tile (mt, nt) of U^T
// is the B operand of k-step 4 mt + v of the second product, so U stays in registers.  Padding
// rows and columns of the operands are zero (the clamped loads only keep the addresses in range).
template <int BS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BS > 32 ? 2 : 1))) void ssor_scale_mfma_kernel(int64_t nf, const int32_t* __restrict__ cols,
                                                              const int32_t* __restrict__ dst,
                                                              const double* __restrict__ bsr,
                                                              const double* __restrict__ rinv,
                                                              double* __restrict__ out) {
    constexpr int MT = (BS + 15) / 16, KS = (BS + 3) / 4;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int64_t F = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (F >= nf) return;   // whole wavefronts
    const double* RF = rinv + (size_t)F * BS * BS;
    for (int s = 1; s < 7; ++s) {
        const int32_t G = __builtin_amdgcn_readfirstlane(cols[F * 7 + s]);
        if (G < 0) continue;
        const int32_t D = __builtin_amdgcn_readfirstlane(dst[F * 6 + s - 1]);
        if (D < 0) continue;
        const double* K = bsr + ((size_t)F * 7 + s) * BS * BS;
        const double* RG = rinv + (size_t)G * BS * BS;
        mf64x4 u[MT][MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < MT; ++nt) u[mt][nt] = mf64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int i = 4 * kk + lg, ic = min(i, BS - 1);
            double bv[MT];
#pragma unroll
            for (int nt = 0; nt < MT; ++nt) {
                const int a = 16 * nt + lr;
                const double t = RF[ic * BS + min(a, BS - 1)];
                bv[nt] = (i < BS && a < BS) ? t : 0.0;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int j = 16 * mt + lr;
                const double t = K[min(j, BS - 1) * BS + ic];
                const double av = j < BS ? t : 0.0;
#pragma unroll
                for (int nt = 0; nt < MT; ++nt)
                    u[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[nt], u[mt][nt], 0, 0, 0);
            }
        }
        // MB row tiles of Kt^T at a time: all of them for two tile rows (more independent MFMA
        // chains), one for three (fewer live accumulators: two wavefronts per SIMD)
        constexpr int MB = MT <= 2 ? MT : 1;
        double* O = out + (size_t)D * BS * BS;
#pragma unroll
        for (int m0 = 0; m0 < MT; m0 += MB) {
            mf64x4 kt[MB][MT];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int na = 0; na < MT; ++na) kt[mb][na] = mf64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (16 * mt + 4 * v >= BS) continue;   // k-steps of padding rows of U^T only
                    const int jc = min(16 * mt + 4 * v + lg, BS - 1);
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) {
                        const double av = RG[jc * BS + min(16 * (m0 + mb) + lr, BS - 1)];
#pragma unroll
                        for (int na = 0; na < MT; ++na)
                            kt[mb][na] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, u[mt][na][v], kt[mb][na], 0, 0, 0);
                    }
                }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int na = 0; na < MT; ++na)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int b = 16 * (m0 + mb) + lg + 4 * v, a = 16 * na + lr;
                        if (b < BS && a < BS) O[b * BS + a] = kt[mb][na][v];
                    }
        }
    }
}

// One sweep of a colour on Kt (unit diagonal blocks): for every face F of colour c (faces of one
// colour share no element, so they are independent), one thread per row a of the face:
//   y_Fa = v_Fa [- t_Fa] - sum over the neighbours G of lower (forward) or higher (backward)
//          colour of (Kt_{F,G} y_G)_a                                   [, q_Fa = t_Fa + y_Fa]
// HAT: the forward sweep of Eisenstat's product, whose right-hand side is p - t and whose output
// is q = t + (I + Lt)^{-1} (p - t).  The blocks of the sweep are stored in its order: those of
// colour-order position P are off[P] .. off[P+1]-1, with neighbours nbr[k]; the faces of one
// colour read one contiguous range.
//
// Fusions of the product sweeps (the CG's other vector work on the same rows):
//   PX (backward sweep of the product, v = p): p_F = r_F + beta p_F first when num is given
//      (beta = num/den, the CG's direction update);
//   C0 (backward sweep of colour 0, the last one): also the forward sweep's colour-0 rows, which
//      have no lower neighbours: u_F = p_F - t_F, q_F = t_F + u_F;
//   with part: partial sums of p.q per workgroup (HAT, and C0 for the colour-0 rows).
struct SweepArgs {
    const int32_t* cfaces;
    const int32_t* off;
    const int32_t* nbr;
    const double* sa;
    const double* v;
    const double* t;
    double* y;
    double* q;
    const double* r;     // PX
    const double* num;   // PX: null, no direction update
    const double* den;
    double* u0;          // C0
    double* part;        // p.q partials (HAT, C0), or null
    const int* done;     // the device-side CG's flag: every launch returns once it is set, or null
    double* xs;          // PX with num, 32 columns: xs += (den / pqp) v before the direction update
    const double* pqp;   // (the previous iteration's solution update), or null
};

template <int BS, bool HAT, bool PX, bool C0>
__global__ __launch_bounds__(NT) void ssor_sweep_kernel(int64_t p0, int64_t nfc, SweepArgs A) {
    if (A.done && *A.done) return;
    const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
    const bool act = gid < nfc * BS;
    double pq = 0.0;
    if (act) {
        const int64_t P = p0 + gid / BS;
        const int a = (int)(gid % BS);
        const int64_t F = A.cfaces[P];
        const int32_t k0 = A.off[P], k1 = A.off[P + 1];
        const int64_t k = F * BS + a;
        double sv = A.v[k];
        if constexpr (PX) {
            if (A.num) {
                const double dd = A.den[0];
                sv = A.r[k] + (dd != 0.0 ? A.num[0] / dd : 0.0) * sv;
                const_cast<double*>(A.v)[k] = sv;
            }
        }
        const double pk = sv;
        double tk = 0.0;
        if constexpr (HAT) {
            tk = A.t[k];
            sv -= tk;
        }
        for (int32_t kb = k0; kb < k1; ++kb) {
            const double* B = A.sa + (size_t)kb * BS * BS + a;
            const double* yv = A.y + (size_t)A.nbr[kb] * BS;
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < BS; ++b) acc += B[b * BS] * yv[b];
            sv -= acc;
        }
        A.y[k] = sv;
        if constexpr (HAT) {
            A.q[k] = tk + sv;
            pq = pk * (tk + sv);
        }
        if constexpr (C0) {
            A.u0[k] = pk - sv;
            A.q[k] = pk;
            pq = pk * pk;
        }
    }
    if constexpr (HAT || C0) {
        if (!A.part) return;
        __shared__ double sh[NT / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pq += __shfl_xor(pq, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = pq;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tsum = 0.0;
            for (int w = 0; w < NT / 64; ++w) tsum += sh[w];
            A.part[blockIdx.x] = tsum;
        }
    }
}

// The sweep of one colour with 32 right-hand sides: one face per wavefront, the sum over the
// face's sweep blocks as 16x16x4 FP64 MFMA tiles (A: the block Kt_{F,G}, B: the neighbour's bs x 32
// vector block), as in the block products of the 32-column CG, then the same row updates and
// fusions as the one-column sweep, per column (PX: p = r + beta_col p, after y += alpha_col p of
// the previous iteration when xs is given).  With part, the p.q sums of the face's rows per
// column go to part[F][32] (a column sum over the faces follows).
template <int BS, bool HAT, bool PX, bool C0>
__global__ __launch_bounds__(256) void ssor_sweep32_kernel(int64_t p0, int64_t nfc, SweepArgs A) {
    if (A.done && *A.done) return;
    constexpr int MT = (BS + 15) / 16, KS = (BS + 3) / 4, R = 32;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int64_t q = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (q >= nfc) return;   // whole wavefronts
    const int64_t P = p0 + q;
    const int64_t F = __builtin_amdgcn_readfirstlane(A.cfaces[P]);
    const int32_t k0 = __builtin_amdgcn_readfirstlane(A.off[P]), k1 = __builtin_amdgcn_readfirstlane(A.off[P + 1]);
    mf64x4 acc[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt][0] = acc[mt][1] = mf64x4{0.0, 0.0, 0.0, 0.0};
    for (int32_t kb = k0; kb < k1; ++kb) {
        const int32_t G = __builtin_amdgcn_readfirstlane(A.nbr[kb]);
        const double* B = A.sa + (size_t)kb * BS * BS;
        const double* yv = A.y + (size_t)G * BS * R;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int b = min(4 * kk + lg, BS - 1);
            const bool bok = 4 * kk + lg < BS;
            double xb[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const double t = yv[b * R + 16 * nt + lr];
                xb[nt] = bok ? t : 0.0;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const double av = B[b * BS + min(16 * mt + lr, BS - 1)];
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb[nt], acc[mt][nt], 0, 0, 0);
            }
        }
    }
    double be[2] = {0.0, 0.0}, al[2] = {0.0, 0.0}, pq[2] = {0.0, 0.0};
    if constexpr (PX) {
        if (A.num)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const double dd = A.den[16 * nt + lr];
                be[nt] = dd != 0.0 ? A.num[16 * nt + lr] / dd : 0.0;
                if (A.xs) {
                    const double pp = A.pqp[16 * nt + lr];
                    al[nt] = pp != 0.0 ? dd / pp : 0.0;
                }
            }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * mt + lg + 4 * v;   // accumulator row of element v of this lane
                if (a >= BS) continue;
                const size_t o = ((size_t)F * BS + a) * R + 16 * nt + lr;
                double sv = A.v[o];
                if constexpr (PX) {
                    if (A.num) {
                        if (A.xs) A.xs[o] += al[nt] * sv;
                        sv = A.r[o] + be[nt] * sv;
                        const_cast<double*>(A.v)[o] = sv;
                    }
                }
                const double pk = sv;
                double tk = 0.0;
                if constexpr (HAT) {
                    tk = A.t[o];
                    sv -= tk;
                }
                sv -= acc[mt][nt][v];
                A.y[o] = sv;
                if constexpr (HAT) {
                    A.q[o] = tk + sv;
                    pq[nt] += pk * (tk + sv);
                }
                if constexpr (C0) {
                    A.u0[o] = pk - sv;
                    A.q[o] = pk;
                    pq[nt] += pk * pk;
                }
            }
    if constexpr (HAT || C0) {
        if (!A.part) return;
        // the four row groups of a column (lanes lr, lr + 16, lr + 32, lr + 48)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            pq[nt] += __shfl_xor(pq[nt], 16, 64);
            pq[nt] += __shfl_xor(pq[nt], 32, 64);
        }
        if (lg == 0) {
            A.part[(size_t)F * R + lr] = pq[0];
            A.part[(size_t)F * R + 16 + lr] = pq[1];
        }
    }
}

// out = x + W^T t with 32 right-hand sides on the matrix cores: one face per wavefront,
// (R_F^{-T} t_F)(a, r) = sum_b R_F^{-1}(b, a) t_F(b, r) as 16x16x4 FP64 tiles (the A operand reads
// R_F^{-1} transposed, the B operands are 16 consecutive right-hand sides of a row of t)
template <int BS>
__global__ __launch_bounds__(256) void rinvt_axpy32_kernel(int64_t nf, const double* __restrict__ rinv,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ t, double* __restrict__ out) {
    constexpr int MT = (BS + 15) / 16, KS = (BS + 3) / 4, R = 32;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int64_t F = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (F >= nf) return;   // whole wavefronts
    const double* Rb = rinv + (size_t)F * BS * BS;
    const double* tv = t + (size_t)F * BS * R;
    mf64x4 acc[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt][0] = acc[mt][1] = mf64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
        const int b = min(4 * kk + lg, BS - 1);
        const bool bok = 4 * kk + lg < BS;
        double xb[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const double v = tv[b * R + 16 * nt + lr];
            xb[nt] = bok ? v : 0.0;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const double av = Rb[min(16 * mt + lr, BS - 1) * BS + b];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb[nt], acc[mt][nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * mt + lg + 4 * v;
                if (a >= BS) continue;
                const size_t o = ((size_t)F * BS + a) * R + 16 * nt + lr;
                out[o] = x[o] + acc[mt][nt][v];
            }
}

// out = x + W^T t  (W^T = diag(R_F^{-T}): row a of R_F^{-T} is column a of R_F^{-1})
template <int BS>
__global__ __launch_bounds__(NT) void rinvt_axpy_kernel(int64_t nf, const double* __restrict__ rinv,
                                                        const double* __restrict__ x, const double* __restrict__ t,
                                                        double* __restrict__ out) {
    const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (gid >= nf * BS) return;
    const int64_t F = gid / BS;
    const int a = (int)(gid % BS);
    const double* Rc = rinv + (size_t)F * BS * BS + (size_t)a * BS;
    const double* tv = t + F * BS;
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < BS; ++b) acc += Rc[b] * tv[b];
    out[gid] = x[gid] + acc;
}
}  // namespace

bool ssor_supported(const hdg_ctx* c) {
    if ((c->nrhs != 1 && c->nrhs != 32) || c->nslot != 7 || c->ncolors == 0 || !c->d_cfaces || !c->d_ssoff)
        return false;
#define HDG_BS(B) \
    if (c->bs == B) return true;
    HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    return false;
}

namespace {
#define HIPCHK_INT(call)                          \
    do {                                          \
        if ((call) != hipSuccess) return HDG_E_HIP; \
    } while (0)

// launch of one colour's sweep with 32 right-hand sides (one face per wavefront, four per workgroup)
template <int BS, bool HAT, bool PX, bool C0>
void sweep32_launch(hdg_ctx* c, int64_t p0, int64_t nfc, const SweepArgs& A) {
    hipLaunchKernelGGL((ssor_sweep32_kernel<BS, HAT, PX, C0>), dim3((unsigned)((nfc + 3) / 4)), dim3(256), 0,
                       c->stream, p0, nfc, A);
}

// one sweep over all colours (forward: colour 0 first; backward: the last colour first)
template <int BS, bool UP, int R = 1>
void ssor_sweep(hdg_ctx* c, const double* v, double* y) {
    SweepArgs A{c->d_cfaces, c->d_ssoff + (UP ? c->n_faces + 1 : 0), c->d_ssnb, c->d_ssA, v, nullptr, y,
                nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < c->ncolors; ++k) {
        const int col = UP ? c->ncolors - 1 - k : k;
        const int64_t p0 = c->color_off[col], nfc = c->color_off[col + 1] - p0;
        if (nfc == 0) continue;
        if constexpr (R == 1)
            hipLaunchKernelGGL((ssor_sweep_kernel<BS, false, false, false>), dim3(nblk(nfc * BS)), dim3(NT), 0,
                               c->stream, p0, nfc, A);
        else
            sweep32_launch<BS, false, false, false>(c, p0, nfc, A);
    }
}

// the product of ssor_product with 32 right-hand sides; p.q per face and column from the launches
// that form q (`part`, n_faces x 32), then summed over the faces.  With xs (and num), the backward
// sweep first adds (den / s_pq) p to xs: the previous iteration's solution update, deferred from
// its CG update so that p is read once
template <int BS>
void ssor_product32(hdg_ctx* c, double* p, const double* r, const double* num, const double* den, double* t,
                    double* u, double* q, double* s_pq, double* part, double* xs) {
    const int nc = c->ncolors;
    SweepArgs B{c->d_cfaces, c->d_ssoff + c->n_faces + 1, c->d_ssnb, c->d_ssA, p, nullptr, t, q, r, num, den,
                u, part, c->cg_done, num ? xs : nullptr, s_pq};
    for (int k = 0; k < nc; ++k) {
        const int col = nc - 1 - k;
        const int64_t p0 = c->color_off[col], nfc = c->color_off[col + 1] - p0;
        if (nfc == 0) continue;
        if (col == 0) sweep32_launch<BS, false, true, true>(c, p0, nfc, B);
        else sweep32_launch<BS, false, true, false>(c, p0, nfc, B);
    }
    SweepArgs H{c->d_cfaces, c->d_ssoff, c->d_ssnb, c->d_ssA, p, t, u, q, nullptr, nullptr, nullptr, nullptr,
                part, c->cg_done};
    for (int col = 1; col < nc; ++col) {
        const int64_t p0 = c->color_off[col], nfc = c->color_off[col + 1] - p0;
        if (nfc == 0) continue;
        sweep32_launch<BS, true, false, false>(c, p0, nfc, H);
    }
    hipLaunchKernelGGL(colsum32_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, c->n_faces, part, c->d_red,
                       (const int*)c->cg_done);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, 32, c->d_red, s_pq,
                       (const int*)c->cg_done);
}

// q = Ahat p = t + Lh^{-1} (p - t), t = Uh^{-1} p, and s_pq = p.q; with num/den first
// p = r + (num/den) p.  The backward sweep's colour-0 launch also forms the forward sweep's
// colour-0 rows; the p.q partials of all launches go to d_red when they fit (else a separate dot).
template <int BS>
void ssor_product(hdg_ctx* c, double* p, const double* r, const double* num, const double* den, double* t,
                  double* u, double* q, double* s_pq) {
    const int nc = c->ncolors;
    int64_t nparts = 0;
    for (int k = 0; k < nc; ++k) nparts += nblk((c->color_off[k + 1] - c->color_off[k]) * BS);
    const bool fuse = nparts <= (int64_t)RED_MAX * 32;
    int64_t po = 0;
    SweepArgs B{c->d_cfaces, c->d_ssoff + c->n_faces + 1, c->d_ssnb, c->d_ssA, p, nullptr, t, q, r, num, den,
                u, nullptr, c->cg_done};
    for (int k = 0; k < nc; ++k) {
        const int col = nc - 1 - k;
        const int64_t p0 = c->color_off[col], nfc = c->color_off[col + 1] - p0;
        if (nfc == 0) continue;
        if (col == 0) {
            B.part = fuse ? c->d_red + po : nullptr;
            po += nblk(nfc * BS);
            hipLaunchKernelGGL((ssor_sweep_kernel<BS, false, true, true>), dim3(nblk(nfc * BS)), dim3(NT), 0,
                               c->stream, p0, nfc, B);
        } else {
            hipLaunchKernelGGL((ssor_sweep_kernel<BS, false, true, false>), dim3(nblk(nfc * BS)), dim3(NT), 0,
                               c->stream, p0, nfc, B);
        }
    }
    SweepArgs H{c->d_cfaces, c->d_ssoff, c->d_ssnb, c->d_ssA, p, t, u, q, nullptr, nullptr, nullptr, nullptr,
                nullptr, c->cg_done};
    for (int col = 1; col < nc; ++col) {
        const int64_t p0 = c->color_off[col], nfc = c->color_off[col + 1] - p0;
        if (nfc == 0) continue;
        H.part = fuse ? c->d_red + po : nullptr;
        po += nblk(nfc * BS);
        hipLaunchKernelGGL((ssor_sweep_kernel<BS, true, false, false>), dim3(nblk(nfc * BS)), dim3(NT), 0,
                           c->stream, p0, nfc, H);
    }
    if (fuse)
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, c->stream, (int)po, c->d_red, s_pq,
                           (const int*)c->cg_done);
    else
        dot(c, p, q, s_pq);
}

// R_F^{-1} and the scaled off-diagonal blocks, when the trace matrix has been assembled since they
// were formed
template <int BS>
hipError_t ssor_prepare(hdg_ctx* c) {
    if (c->ss_version == c->mat_version) return hipSuccess;
    if constexpr (BS <= 21) {
        constexpr int64_t FPB = (64 / BS) * (NT / 64);   // faces per workgroup of the factor kernel
        hipLaunchKernelGGL((chol_rinv_kernel<BS>), dim3((unsigned)((c->n_faces + FPB - 1) / FPB)), dim3(NT), 0,
                           c->stream, c->n_faces, c->d_bsr, c->d_rinv);
    } else if constexpr (BS > 32 && BS <= 64) {
        hipLaunchKernelGGL((chol_rinv_wave_kernel<BS>), dim3((unsigned)((c->n_faces + 3) / 4)), dim3(256), 0,
                           c->stream, c->n_faces, c->d_bsr, c->d_rinv);
    } else {
        hipLaunchKernelGGL((chol_rinv_lds_kernel<BS>), dim3((unsigned)std::min<int64_t>(c->n_faces, 65536)),
                           dim3(64), 0, c->stream, c->n_faces, c->d_bsr, c->d_rinv);
    }
    if constexpr (BS >= 20)   // blocks of 20 and more: matrix cores, a face per wavefront
        hipLaunchKernelGGL((ssor_scale_mfma_kernel<BS>), dim3((unsigned)((c->n_faces + 3) / 4)), dim3(256), 0,
                           c->stream, c->n_faces, c->d_bsr_cols, c->d_ssdst, c->d_bsr, c->d_rinv, c->d_ssA);
    else
        hipLaunchKernelGGL((ssor_scale_kernel<BS>), dim3((unsigned)((c->n_faces + 64 / BS - 1) / (64 / BS))),
                           dim3(64), 0, c->stream, c->n_faces, c->d_bsr_cols, c->d_ssdst, c->d_bsr, c->d_rinv,
                           c->d_ssA);
    c->ss_version = c->mat_version;
    return hipGetLastError();
}

// CG on the transformed system  Ahat y = Lh^{-1} W r0,  Ahat = Lh^{-1} Kt Uh^{-1}  (Lh = I + Lt,
// Uh = I + Ut = Lh^T): the iterates are those of PCG on K with the block SSOR preconditioner
// M = (D + L) D^{-1} (D + U).  Eisenstat's form of the product: t = Uh^{-1} p,
// Ahat p = t + Lh^{-1} (p - t).  The correction of the initial guess x0 is x - x0 = W^T Uh^{-1} y.
// r.r of the transformed residual (the residual of K in the M^{-1} norm) drives the iteration;
// when its relative value drops below the tolerance, the true relative residual |b - K x| / |b|
// is formed and decides (a failed check tightens the estimate's threshold tenfold).
template <int BS, int R>
int cg_ssor(hdg_ctx* c, double* x, double tol, int* iters, double* relres) {
    static_assert(R == 1 || R == 32, "one or 32 right-hand sides");
    const int64_t n = c->n_faces * BS, nR = n * R;
    double* rr = c->d_cg_r;
    double* zz = c->d_cg_z;
    double* pp = c->d_cg_p;
    double* qq = c->d_cg_q;
    double* tt = c->d_ss;
    double* uu = c->d_ss + nR;
    double* yy = c->d_ss + 2 * nR;
    double* s_rz = c->d_scal;            // [R] each
    double* s_rz_new = c->d_scal + 32;
    double* s_pq = c->d_scal + 64;
    double* s_bb = c->d_scal + 128;
    double* s_rr = c->d_scal + 96;
    HIPCHK_INT(ssor_prepare<BS>(c));
    auto wapply = [&](const double* in, double* out) {   // out = W in
        if constexpr (R == 32)   // the block-diagonal product of the 32-column CG (matrix cores)
            launch_spmm32<BS, 1, double>(c, (const int32_t*)nullptr, c->d_rinv, in, out, nullptr);
        else
            hipLaunchKernelGGL((block_apply_fixed_kernel<BS>), dim3(nblk(nR)), dim3(NT), 0, c->stream, c->n_faces,
                               R, c->d_rinv, in, out, (const int*)nullptr);
    };
    auto true_residual = [&](double* hres) -> int {   // x_try = x0 + W^T Uh^{-1} y into zz; |b - K x_try|^2
        ssor_sweep<BS, true, R>(c, yy, tt);
        if constexpr (R == 1)
            hipLaunchKernelGGL((rinvt_axpy_kernel<BS>), dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, c->d_rinv,
                               x, tt, zz);
        else
            hipLaunchKernelGGL((rinvt_axpy32_kernel<BS>), dim3((unsigned)((c->n_faces + 3) / 4)), dim3(256), 0,
                               c->stream, c->n_faces, c->d_rinv, x, tt, zz);
        spmv(c, zz, qq);
        launch_lincomb(c, nR, 1.0, c->d_rhs, -1.0, qq, uu);
        dot(c, uu, uu, s_rr);
        HIPCHK_INT(hipMemcpyAsync(hres, s_rr, R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK_INT(hipStreamSynchronize(c->stream));
        return 0;
    };
    // initial guess: Dirichlet entries are the boundary values (identity rows)
    hipLaunchKernelGGL(copy_bnd_kernel, dim3(nblk(nR)), dim3(NT), 0, c->stream, c->n_faces, BS, R, c->d_face_bnd,
                       c->d_rhs, x);
    spmv(c, x, qq);
    launch_lincomb(c, nR, 1.0, c->d_rhs, -1.0, qq, uu);            // r0 = b - K x0
    wapply(uu, tt);
    ssor_sweep<BS, false, R>(c, tt, rr);                           // rhat = Lh^{-1} W r0
    hipMemsetAsync(yy, 0, nR * sizeof(double), c->stream);
    launch_lincomb(c, nR, 1.0, rr, 0.0, nullptr, pp);
    dot(c, rr, rr, s_rz);
    dot(c, c->d_rhs, c->d_rhs, s_bb);
    // the scale of r.r per column: |Lh^{-1} W b|^2
    wapply(c->d_rhs, tt);
    ssor_sweep<BS, false, R>(c, tt, uu);
    dot(c, uu, uu, s_pq);
    double hb[R], hm[R];
    HIPCHK_INT(hipMemcpyAsync(hb, s_bb, R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK_INT(hipMemcpyAsync(hm, s_pq, R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK_INT(hipStreamSynchronize(c->stream));
    double bnorm[R], bm[R];
    for (int r = 0; r < R; ++r) {
        bnorm[r] = hb[r] > 0 ? std::sqrt(hb[r]) : 1.0;
        bm[r] = hm[r] > 0 ? hm[r] : 1.0;
    }
    double thresh = tol;
    double worst = std::numeric_limits<double>::quiet_NaN();
    int it = 0;
    double* hrz = c->h_rr;   // pinned, 32 values
    // q = Ahat p, p.q (writes t, u, q; with beta also p = r + beta p first, beta = s_rz / s_rz_new
    // after the swap at the end of an iteration)
    auto product = [&](bool beta) {
        if constexpr (R == 1) ssor_product<BS>(c, pp, rr, beta ? s_rz : nullptr, s_rz_new, tt, uu, qq, s_pq);
        else ssor_product32<BS>(c, pp, rr, beta ? s_rz : nullptr, s_rz_new, tt, uu, qq, s_pq, c->d_ss + 3 * nR, yy);
    };
    for (it = 0; it <= c->krylov_maxit; ++it) {
        if (hipMemcpyAsync(hrz, s_rz, R * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipEventRecord(c->ev_rr, c->stream) != hipSuccess)
            return HDG_E_HIP;
        // queue the next product before waiting for r.r (with 32 columns it also applies the
        // previous iteration's y += alpha p; at the iteration limit that update is launched alone)
        if (it < c->krylov_maxit) product(it > 0);
        else if (R == 32 && it > 0)
            hipLaunchKernelGGL(axpy_ratio_cols_kernel, dim3(nblk(nR)), dim3(NT), 0, c->stream, n, R, s_rz_new, s_pq,
                               pp, yy);
        if (hipEventSynchronize(c->ev_rr) != hipSuccess) return HDG_E_HIP;
        double est = 0.0;
        bool nonfinite = false;
        for (int r = 0; r < R; ++r) {
            const double v = std::sqrt(std::fabs(hrz[r]) / bm[r]);
            if (!(v - v == 0.0)) nonfinite = true;
            else est = std::max(est, v);
        }
        if (nonfinite) {
            worst = std::numeric_limits<double>::quiet_NaN();
            break;
        }
        if (est <= thresh || it == c->krylov_maxit) {
            double hres[R];
            if (true_residual(hres)) return HDG_E_HIP;
            worst = 0.0;
            for (int r = 0; r < R; ++r) {
                const double v = std::sqrt(hres[r]) / bnorm[r];
                worst = (v - v == 0.0) ? std::max(worst, v) : std::numeric_limits<double>::quiet_NaN();
                if (!(worst - worst == 0.0)) break;
            }
            if (!(worst - worst == 0.0) || worst <= tol || it == c->krylov_maxit) {
                launch_lincomb(c, nR, 1.0, zz, 0.0, nullptr, x);   // x = x0 + W^T Uh^{-1} y
                break;
            }
            thresh *= 0.1;
            product(false);   // the check overwrote t, u and q: this iteration's product again (p is new)
        }
        if constexpr (R == 1)
            hipLaunchKernelGGL(cg_update_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, R, s_rz, s_pq, pp,
                               qq, yy, rr, c->d_red, (const int*)nullptr, (int*)nullptr);
        else   // y += alpha p in the next product
            hipLaunchKernelGGL(cg_resid_update_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, R, s_rz, s_pq,
                               qq, rr, c->d_red);
        if constexpr (R == 1)
            hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, c->stream, c->red_blocks, c->d_red,
                               s_rz_new);
        else
            hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, R, c->d_red,
                               s_rz_new, (const int*)nullptr);
        std::swap(s_rz, s_rz_new);   // the next product forms p = r + (s_rz / s_rz_new) p
    }
    if (iters) *iters = it;
    if (relres) *relres = worst;
    c->last_iters = it;
    if (!(worst <= tol)) return HDG_E_NOCONV;
    return HDG_OK;
}
}  // namespace

namespace {
__global__ __launch_bounds__(NT) void fill_zero_kernel(int64_t n, double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// device-side test of the SSOR CG's estimate: done = 1 once sqrt(r.r / bm) <= thresh, 2 when
// it is not finite
__global__ void ssor_check_kernel(const double* __restrict__ s_rz, const double* __restrict__ s_bm, double thresh,
                                  int* __restrict__ flags) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || flags[0]) return;
    const double bm = *s_bm > 0.0 ? *s_bm : 1.0;
    const double est = sqrt(fabs(*s_rz) / bm);
    if (!(est - est == 0.0)) flags[0] = 2;
    else if (est <= thresh) flags[0] = 1;
}

// after the iterations: relres = |b - K x| / |b| decides (done = 1 only when it meets tol)
__global__ void ssor_final_kernel(const double* __restrict__ s_rr, const double* __restrict__ s_bb, double tol,
                                  int* __restrict__ flags, double* __restrict__ relres) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double b = sqrt(*s_bb);
    const double v = sqrt(*s_rr) / (b > 0.0 ? b : 1.0);
    *relres = v;
    flags[0] = !(v - v == 0.0) ? 2 : (v <= tol ? 1 : 0);
}

// The SSOR CG of cg_ssor with a fixed number of iterations and the test on the device, for
// capture into a graph (no host synchronisation, no memset): the estimate stops the iterations
// at a tenth of the tolerance (the host version confirms at the tolerance and tightens on a
// failed check), then x = x0 + W^T Uh^{-1} y and its true relative residual, which alone sets
// flags[0] (1 converged, 0 not, 2 non-finite); flags[1] counts the iterations.
template <int BS>
int cg_ssor_device(hdg_ctx* c, double* x, double tol, int nit, int* flags, double* relres_dev) {
    const int64_t n = c->n_faces * BS;
    double* rr = c->d_cg_r;
    double* zz = c->d_cg_z;
    double* pp = c->d_cg_p;
    double* qq = c->d_cg_q;
    double* tt = c->d_ss;
    double* uu = c->d_ss + n;
    double* yy = c->d_ss + 2 * n;
    double* s_rz = c->d_scal;
    double* s_rz_new = c->d_scal + 32;
    double* s_pq = c->d_scal + 64;
    double* s_rr = c->d_scal + 96;
    double* s_bb = c->d_scal + 128;
    double* s_bm = c->d_scal + 192;
    if (ssor_prepare<BS>(c) != hipSuccess) return HDG_E_HIP;
    auto wapply = [&](const double* in, double* out) {   // out = W in
        hipLaunchKernelGGL((block_apply_fixed_kernel<BS>), dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, 1,
                           c->d_rinv, in, out, (const int*)nullptr);
    };
    launch_zero_ints(c, flags, 2);
    hipLaunchKernelGGL(copy_bnd_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, BS, 1, c->d_face_bnd,
                       c->d_rhs, x);
    spmv(c, x, qq);
    launch_lincomb(c, n, 1.0, c->d_rhs, -1.0, qq, uu);             // r0 = b - K x0
    wapply(uu, tt);
    ssor_sweep<BS, false>(c, tt, rr);                              // rhat = Lh^{-1} W r0
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nblk(n)), dim3(NT), 0, c->stream, n, yy);
    launch_lincomb(c, n, 1.0, rr, 0.0, nullptr, pp);
    dot(c, rr, rr, s_rz);
    dot(c, c->d_rhs, c->d_rhs, s_bb);
    wapply(c->d_rhs, tt);
    ssor_sweep<BS, false>(c, tt, uu);
    dot(c, uu, uu, s_bm);                                          // the scale of r.r
    const double thresh = 0.1 * tol;
    hipLaunchKernelGGL(ssor_check_kernel, dim3(1), dim3(64), 0, c->stream, s_rz, s_bm, thresh, flags);
    c->cg_done = flags;   // from here on every launch of the loop returns once the estimate is met
    for (int it = 0; it < nit; ++it) {
        ssor_product<BS>(c, pp, rr, it > 0 ? s_rz : nullptr, s_rz_new, tt, uu, qq, s_pq);
        hipLaunchKernelGGL(cg_update_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, 1, s_rz, s_pq, pp, qq,
                           yy, rr, c->d_red, (const int*)flags, flags + 1);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, c->stream, c->red_blocks, c->d_red,
                           s_rz_new, (const int*)flags);
        hipLaunchKernelGGL(ssor_check_kernel, dim3(1), dim3(64), 0, c->stream, s_rz_new, s_bm, thresh, flags);
        std::swap(s_rz, s_rz_new);
    }
    c->cg_done = nullptr;
    ssor_sweep<BS, true>(c, yy, tt);
    hipLaunchKernelGGL((rinvt_axpy_kernel<BS>), dim3(nblk(n)), dim3(NT), 0, c->stream, c->n_faces, c->d_rinv, x, tt,
                       zz);
    spmv(c, zz, qq);
    launch_lincomb(c, n, 1.0, c->d_rhs, -1.0, qq, uu);
    dot(c, uu, uu, s_rr);
    launch_lincomb(c, n, 1.0, zz, 0.0, nullptr, x);                // x = x0 + W^T Uh^{-1} y
    hipLaunchKernelGGL(ssor_final_kernel, dim3(1), dim3(64), 0, c->stream, s_rr, s_bb, tol, flags, relres_dev);
    return (int)hipGetLastError();
}
}  // namespace

int trace_ssor_alloc(hdg_ctx* c) {
    const size_t nt = (size_t)c->n_faces * c->bs;
    void** bufs[3] = {(void**)&c->d_ss, (void**)&c->d_rinv, (void**)&c->d_ssA};
    // d_ss: t, u, y of the transformed CG, and with 32 right-hand sides the per-face p.q partials
    const size_t sizes[3] = {3 * nt * c->nrhs + (c->nrhs == 32 ? (size_t)c->n_faces * 32 : 0), nt * c->bs,
                             (size_t)std::max<int64_t>(c->ss_nblk, 1) * c->bs * c->bs};
    for (int i = 0; i < 3; ++i) {
        if (*bufs[i]) continue;
        const int e = dev_malloc(c, bufs[i], sizes[i] * sizeof(double));
        if (e) return e;
        c->ss_version = -1;
    }
    return HDG_OK;
}

int trace_cg_ssor(hdg_ctx* c, double* x, double tol, int* iters, double* relres) {
    const int e = trace_ssor_alloc(c);
    if (e) return e;
#define HDG_BS(B)                                                                  \
    if (c->bs == B)                                                                \
        return c->nrhs == 32 ? cg_ssor<B, 32>(c, x, tol, iters, relres) : cg_ssor<B, 1>(c, x, tol, iters, relres);
    HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    return HDG_E_UNSUPPORTED;
}

int trace_cg_ssor_device(hdg_ctx* c, double* x, double tol, int nit, int* flags, double* relres_dev) {
    if (c->nrhs != 1) return HDG_E_UNSUPPORTED;
    if (!c->d_ss || !c->d_rinv || !c->d_ssA) return HDG_E_STATE;   // trace_ssor_alloc first (not under capture)
#define HDG_BS(B) \
    if (c->bs == B) return cg_ssor_device<B>(c, x, tol, nit, flags, relres_dev);
    HDG_BS_CASES(HDG_BS)
#undef HDG_BS
    return HDG_E_UNSUPPORTED;
}
#undef HIPCHK_INT

namespace {
// Device-side convergence test of the captured CG: done = 1 once every column meets the
// tolerance, 2 on a non-finite residual; relres = the largest relative residual.
__global__ void cg_check_kernel(int R, const double* __restrict__ s_rr, const double* __restrict__ s_bb,
                                double tol, int* __restrict__ flags, double* __restrict__ relres) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || flags[0]) return;
    double worst = 0.0;
    bool nonfinite = false;
    for (int r = 0; r < R; ++r) {
        const double b = sqrt(s_bb[r]);
        const double v = sqrt(s_rr[r]) / (b > 0.0 ? b : 1.0);
        if (!(v - v == 0.0)) nonfinite = true;
        else worst = fmax(worst, v);
    }
    *relres = nonfinite ? __builtin_nan("") : worst;
    if (nonfinite) flags[0] = 2;
    else if (worst <= tol) flags[0] = 1;
}

__global__ void zero_ints_kernel(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
}  // namespace

// a fill kernel rather than a memset: it may be captured into a graph
int launch_zero_ints(hdg_ctx* c, int* p, int n) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 63) / 64), dim3(64), 0, c->stream, p, n);
    return (int)hipGetLastError();
}

// The CG of trace_cg with a fixed number of iterations and the convergence test on the device,
// for capture into a graph: every iteration's kernels return at once after the test has passed.
// flags[0] (done: 1 converged, 2 non-finite), flags[1] (iterations) and relres_dev tell the host
// afterwards whether it converged within `nit` iterations.  The arithmetic, and so the iterate,
// is that of trace_cg (FP64 products).
int trace_cg_device(hdg_ctx* c, double* x, double tol, int nit, int* flags, double* relres_dev) {
    const int R = c->nrhs;
    const int64_t n = c->n_faces * c->bs;
    double* rr = c->d_cg_r;
    double* zz = c->d_cg_z;
    double* pp = c->d_cg_p;
    double* qq = c->d_cg_q;
    double* s_rz = c->d_scal;
    double* s_rz_new = c->d_scal + 32;
    double* s_pq = c->d_scal + 64;
    double* s_rr = c->d_scal + 96;
    double* s_bb = c->d_scal + 128;
    double* s_res = relres_dev;
    if (c->pinv_version != c->mat_version && launch_block_inverse(c)) return HDG_E_HIP;
    launch_zero_ints(c, flags, 2);
    hipLaunchKernelGGL(copy_bnd_kernel, dim3(nblk(n * R)), dim3(NT), 0, c->stream, c->n_faces, c->bs, R,
                       c->d_face_bnd, c->d_rhs, x);
    spmv(c, x, qq);
    launch_lincomb(c, n * R, 1.0, c->d_rhs, -1.0, qq, rr);
    precond(c, rr, zz);
    launch_lincomb(c, n * R, 1.0, zz, 0.0, nullptr, pp);
    dot(c, rr, zz, s_rz);
    dot(c, c->d_rhs, c->d_rhs, s_bb);
    dot(c, rr, rr, s_rr);
    hipLaunchKernelGGL(cg_check_kernel, dim3(1), dim3(64), 0, c->stream, R, s_rr, s_bb, tol, flags, s_res);
    c->cg_done = flags;   // from here on every launch of the loop returns once converged
    for (int it = 0; it < nit; ++it) {
        spmv(c, pp, qq, false, s_pq);
        hipLaunchKernelGGL(cg_update_kernel, dim3(c->red_blocks), dim3(NT), 0, c->stream, n, R, s_rz, s_pq, pp,
                           qq, x, rr, c->d_red, (const int*)flags, flags + 1);
        hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, c->stream, c->red_blocks, R, c->d_red, s_rr,
                           (const int*)flags);
        hipLaunchKernelGGL(cg_check_kernel, dim3(1), dim3(64), 0, c->stream, R, s_rr, s_bb, tol, flags, s_res);
        precond(c, rr, zz, s_rz_new);
        hipLaunchKernelGGL(xpby_cols_kernel, dim3(nblk(n * R)), dim3(NT), 0, c->stream, n, R, s_rz_new, s_rz, zz,
                           pp, (const int*)flags);
        std::swap(s_rz, s_rz_new);
    }
    c->cg_done = nullptr;
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Trace solve without any allocation: the CG work vectors (r, z, p, q), the per-workgroup partial
// sums and the device scalars live in this file-scope device array instead of the context's
// buffers.  Each GPU holds its own copy for the life of the process; host code must use the
// address obtained from hipGetSymbolAddress on that device, never the array's name.  Every call on
// one GPU shares it: calls that overlap on a device race.  Nothing in it needs clearing: the CG
// writes every entry it reads (r from the right-hand side, z, p, q from r, the partial sums and
// scalars by their reductions) before reading it.
}  // namespace hdg

static __device__ __align__(256) double scratch[TRACE_STATIC_DOUBLES];

namespace hdg {
namespace {
constexpr int MAX_DEV = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEV] = {};
}  // namespace

int static_scratch_setup() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return HDG_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return HDG_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HDG_E_HIP;
    g_scratch_ptr[dev] = (double*)ptr;
    return HDG_OK;
}

int64_t trace_static_need(const hdg_ctx* c) {
    return 4 * c->n_faces * c->bs * c->nrhs + (int64_t)RED_MAX * 32 + 8 * 32;
}

int trace_cg_static(hdg_ctx* c, double* lambda, int* iters, double* relres) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return HDG_E_HIP;
    double* base;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[dev];
    }
    if (!base) {   // the context was created on another device: set up this one now
        if (static_scratch_setup() != HDG_OK) return HDG_E_HIP;
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[dev];
    }
    const int64_t n = c->n_faces * c->bs * c->nrhs;
    // the context's buffers are swapped out for the call and restored afterwards
    double* saved[6] = {c->d_cg_r, c->d_cg_z, c->d_cg_p, c->d_cg_q, c->d_red, c->d_scal};
    c->d_cg_r = base;
    c->d_cg_z = base + n;
    c->d_cg_p = base + 2 * n;
    c->d_cg_q = base + 3 * n;
    c->d_red = base + 4 * n;
    c->d_scal = base + 4 * n + (int64_t)RED_MAX * 32;
    const int r = trace_cg(c, lambda, c->krylov_tol, iters, relres, c->d_bsr32 != nullptr);
    c->d_cg_r = saved[0];
    c->d_cg_z = saved[1];
    c->d_cg_p = saved[2];
    c->d_cg_q = saved[3];
    c->d_red = saved[4];
    c->d_scal = saved[5];
    return r;
}

}  // namespace hdg
