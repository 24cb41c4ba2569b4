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

}  // namespace hdg
