// Complex products on the matrix cores (shared by the solve sweeps and the factorisation).
//
// Three-multiplication form: with A = Ar + i Ai, B = Br + i Bi,
//   P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi),  AB = (P1 - P2) + i (P3 - P1 - P2),
// three real products where the direct form needs four.  Each is a v_mfma_f32_16x16x4f32
// (complex64) or v_mfma_f64_16x16x4f64 (complex128) over 4 complex k at a time: lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; the 16 x 16 result sits in rows 4(l/16)+v
// (complex64) or l/16+4v (complex128), column l%16 (CAcc::row).
#pragma once

#include "hz_internal.h"

namespace hz {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void mfma_3m(c64 a, c64 b, f32x4& p1, f32x4& p2, f32x4& p3) {
  p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, b.re, p1, 0, 0, 0);
  p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, b.im, p2, 0, 0, 0);
  p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re + a.im, b.re + b.im, p3, 0, 0, 0);
}

// complex accumulator of one 16 x 16 output tile
template <typename T>
struct CAcc;
template <>
struct CAcc<float> {
  f32x4 p1, p2, p3;
  __device__ __forceinline__ void zero() { p1 = p2 = p3 = f32x4{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ void mac(c64 a, c64 b) { mfma_3m(a, b, p1, p2, p3); }
  __device__ __forceinline__ c64 get(int v) const { return cmk(p1[v] - p2[v], p3[v] - p1[v] - p2[v]); }
  static __device__ __forceinline__ int row(int lq, int v) { return 4 * lq + v; }
};
template <>
struct CAcc<double> {
  f64x4 p1, p2, p3;
  __device__ __forceinline__ void zero() { p1 = p2 = p3 = f64x4{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ void mac(c128 a, c128 b) {
    p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, p1, 0, 0, 0);
    p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.im, p2, 0, 0, 0);
    p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re + a.im, b.re + b.im, p3, 0, 0, 0);
  }
  __device__ __forceinline__ c128 get(int v) const { return cmk(p1[v] - p2[v], p3[v] - p1[v] - p2[v]); }
  static __device__ __forceinline__ int row(int lq, int v) { return lq + 4 * v; }
};

}  // namespace hz
