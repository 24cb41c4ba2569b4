// 16x16x4 matrix-core tiles of gfx950 (one wavefront), FP64 and FP32.
//
// Operand layout: lane l supplies A[l%16][l/16] of the 16x4 A operand and B[l/16][l%16] of the
// 4x16 B operand; the product accumulates into the 16x16 C tile, whose element v (0..3) in
// lane l is C[row][l%16] with row = l/16 + 4 v (FP64 instruction) or 4 (l/16) + v (FP32
// instruction).  Both layouts were checked on gfx950 against a host product.
#pragma once
#include <hip/hip_runtime.h>

namespace hdg {

typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using acc = mf64x4;
    __device__ static __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static __forceinline__ acc mac(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
    using acc = mf32x4;
    __device__ static __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static __forceinline__ acc mac(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Split-BF16 products on the BF16 matrix cores (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation):
// each FP32 operand is split into x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (both
// rounded to nearest even), and a.b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo.lo term and the
// rounding of lo leave a relative error of about 2^-16 per product).  One call covers a k-range of
// 16: lane l supplies A[l%16][4 (l/16) + t] and B[4 (l/16) + t][l%16], t = 0..3; the 16x16 C
// tile has the FP32 layout (element v in lane l is C[4 (l/16) + v][l%16]).  Layout checked on
// gfx950 against a host product.
typedef short bf16x4_bits __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void bf16_split4(const float v[4], bf16x4_bits& hi, bf16x4_bits& lo) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const __bf16 h = (__bf16)v[t];
        const __bf16 l = (__bf16)(v[t] - (float)h);
        hi[t] = __builtin_bit_cast(short, h);
        lo[t] = __builtin_bit_cast(short, l);
    }
}

__device__ __forceinline__ mf32x4 bf16x3_mac16(const float a[4], const float b[4], mf32x4 c) {
    bf16x4_bits ah, al, bh, bl;
    bf16_split4(a, ah, al);
    bf16_split4(b, bh, bl);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);   // small terms first
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
}

}  // namespace hdg
