// Multi-RHS complex CSR SpMM  y = alpha A x + beta y_in  on node-major blocks ([n][s]).
// A is complex128 (16 B value + 4 B column per nonzero); x is complex128 or complex64 (the
// preconditioned Krylov vectors of the mixed-precision solve), widened exactly to FP64, so
// every product and sum is FP64 and y is complex128.
//
// Main kernel (9..32 columns): a wavefront owns RW consecutive rows, one after the other.
// Its four 16-lane DPP rows are four groups; a chunk of up to 64 nonzeros of the row is
// loaded one per lane, group g taking the contiguous quarter [g Q, g Q + Q).  Each step t
// broadcasts lane t's column and value to its 16-lane row with the DPP row_newbcast move (a
// VALU op: no LDS traffic), and lane u gathers column(s) u (16 columns) or 2u, 2u+1 (32
// columns) of that x row: one coalesced 128/256/512-byte segment per group.  All Q gathers of
// a chunk are issued before the first use.  Gathers go through a buffer descriptor with
// 32-bit offsets (no 64-bit address arithmetic per step).  Wave-uniform control (row bounds,
// chunk count) stays in scalar registers.  The four group sums are combined with the
// permlane16/32 swaps, the same order in every lane, so results are bitwise reproducible.
// Work items are dealt to the XCDs in contiguous eighths, so rows that share x rows share
// one L2.
//
// Fallback kernel (1..8 columns, or blocks too large for 32-bit offsets): a wavefront per
// row, G = 64/S groups of S column lanes, values broadcast by shuffles.
//
// HBM-bound; algorithmic bytes 20 nnz + 8 (n+1) + n s (sizeof x + 16 (+16 with y_in)).
#include "hz_internal.h"

namespace hz {

namespace {

// ---------------------------------------------------------------- lane moves

// lane L of each 16-lane row to the whole row
template <int L>
__device__ __forceinline__ int row_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + L, 0xF, 0xF, false);
}
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + L, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + L, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// sum over the four 16-lane rows: (r0 + r1) + (r2 + r3), in every lane
__device__ __forceinline__ double sum_rows(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double v2 = __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
  lo = __double2loint(v2);
  hi = __double2hiint(v2);
  a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ int64_t read_lane64(int64_t v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(uint64_t)v, l);
  const int hi = __builtin_amdgcn_readlane((int)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Workgroups are dealt round-robin over the 8 XCDs; this maps the launch index so that each
// XCD takes one contiguous eighth of the work items, in order (a bijection on [0, nb)).
__device__ __forceinline__ int64_t xcd_linear(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
  return x * q + (x < r ? x : r) + k;
}

// CPL consecutive complex entries of x starting at byte offset off (bounds-checked: an
// offset past the buffer reads zeros and touches no memory)
template <typename TX, int CPL, bool PAIR>
struct XLoad {
  cplx<TX> v[CPL];
};
template <typename TX, int CPL, bool PAIR>
__device__ __forceinline__ XLoad<TX, CPL, PAIR> load_x(__amdgpu_buffer_rsrc_t r, int off) {
  XLoad<TX, CPL, PAIR> o;
  if constexpr (sizeof(TX) == 4) {
    if constexpr (CPL == 1) {
      o = __builtin_bit_cast(decltype(o), __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    } else if constexpr (PAIR) {  // 16-byte aligned pair
      o = __builtin_bit_cast(decltype(o), __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    } else {
      auto a = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
      auto b = __builtin_amdgcn_raw_buffer_load_b64(r, off + 8, 0, 0);
      o.v[0] = __builtin_bit_cast(cplx<TX>, a);
      o.v[1] = __builtin_bit_cast(cplx<TX>, b);
    }
  } else {
#pragma unroll
    for (int c = 0; c < CPL; ++c)
      o.v[c] = __builtin_bit_cast(cplx<TX>, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * c, 0, 0));
  }
  return o;
}

template <typename TX, int CPL, bool PAIR>
__global__ __launch_bounds__(256) void k_spmm_dpp(int64_t n, int s, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col, const c128* __restrict__ val,
                                                  const cplx<TX>* __restrict__ x, c128* __restrict__ y, c128 alpha,
                                                  c128 beta, const c128* __restrict__ yin) {
  constexpr int RW = 4;
  constexpr int EB = (int)sizeof(cplx<TX>);
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, u = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t r0 = (xcd_linear(blockIdx.x, gridDim.x) * 4 + wv) * RW;
  if (r0 >= n) return;
  const int nr = (int)min<int64_t>(RW, n - r0);
  const int64_t rpl = rowptr[r0 + (lane < nr ? lane : nr)];
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, (int)((uint64_t)n * (uint64_t)s * EB), 0x00020000);
  const unsigned rs = (unsigned)s * EB;
  const int c0 = u * CPL;
  const unsigned loff = c0 < s ? (unsigned)(c0 * EB) : 0xFFFF0000u;  // lanes past s read nothing used
  for (int rr = 0; rr < nr; ++rr) {
    const int64_t e0 = read_lane64(rpl, rr), e1 = read_lane64(rpl, rr + 1);
    double ar[CPL], ai[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) ar[c] = ai[c] = 0.0;
    for (int64_t base = e0; base < e1; base += 64) {
      const int cnt = __builtin_amdgcn_readfirstlane((int)min<int64_t>(64, e1 - base));
      const int Q = (cnt + 3) >> 2;
      const int k = g * Q + u;
      const bool ok = u < Q && k < cnt;
      const int kk = ok ? k : 0;
      const int mo = (int)((unsigned)col[base + kk] * rs);
      const c128 m0 = val[base + kk];
      const double mr = ok ? m0.re : 0.0, mi = ok ? m0.im : 0.0;
      XLoad<TX, CPL, PAIR> xx[16];
#define HZ_GATHER(T) \
  if (T < Q) xx[T] = load_x<TX, CPL, PAIR>(xr, (int)((unsigned)row_bcast<T>(mo) + loff));
      HZ_GATHER(0) HZ_GATHER(1) HZ_GATHER(2) HZ_GATHER(3) HZ_GATHER(4) HZ_GATHER(5) HZ_GATHER(6) HZ_GATHER(7)
      HZ_GATHER(8) HZ_GATHER(9) HZ_GATHER(10) HZ_GATHER(11) HZ_GATHER(12) HZ_GATHER(13) HZ_GATHER(14) HZ_GATHER(15)
#undef HZ_GATHER
#define HZ_STEP(T)                                                         \
  if (T < Q) {                                                             \
    const double a = row_bcast<T>(mr), b = row_bcast<T>(mi);               \
    _Pragma("unroll") for (int c = 0; c < CPL; ++c) {                      \
      const double xr_ = (double)xx[T].v[c].re, xi_ = (double)xx[T].v[c].im; \
      ar[c] = fma(a, xr_, ar[c]);                                          \
      ar[c] = fma(-b, xi_, ar[c]);                                         \
      ai[c] = fma(a, xi_, ai[c]);                                          \
      ai[c] = fma(b, xr_, ai[c]);                                          \
    }                                                                      \
  }
      HZ_STEP(0) HZ_STEP(1) HZ_STEP(2) HZ_STEP(3) HZ_STEP(4) HZ_STEP(5) HZ_STEP(6) HZ_STEP(7)
      HZ_STEP(8) HZ_STEP(9) HZ_STEP(10) HZ_STEP(11) HZ_STEP(12) HZ_STEP(13) HZ_STEP(14) HZ_STEP(15)
#undef HZ_STEP
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      ar[c] = sum_rows(ar[c]);
      ai[c] = sum_rows(ai[c]);
    }
    if (g == 0) {
      const int64_t row = r0 + rr;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        if (c0 + c >= s) continue;
        c128 r = alpha * cmk(ar[c], ai[c]);
        if (yin) r = r + beta * yin[row * s + c0 + c];
        y[row * s + c0 + c] = r;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m) {
  return __shfl_xor(v, m, 64);
}

template <typename TX, int S>
__global__ __launch_bounds__(256) void k_spmm_rows(int64_t n, int s, const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col, const c128* __restrict__ val,
                                                   const cplx<TX>* __restrict__ x, c128* __restrict__ y, c128 alpha,
                                                   c128 beta, const c128* __restrict__ yin) {
  constexpr int G = 64 / S;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = lane / S;
  const int c = blockIdx.y * S + (lane % S);
  if (row >= n) return;
  const bool act = c < s;
  c128 acc = cmk(0.0, 0.0);
  const int64_t e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int64_t base = e0; base < e1; base += 64) {
    // lanes fetch 64 (column, value) pairs at once; groups read them back by shuffles
    const int cnt = (int)min<int64_t>(64, e1 - base);
    int32_t mj = 0;
    c128 mv = cmk(0.0, 0.0);
    if (lane < cnt) {
      mj = col[base + lane];
      mv = val[base + lane];
    }
    // uniform trip count over the wavefront: every lane takes part in every shuffle.  Steps
    // go in batches of B whose x loads are unconditional (clamped to a valid entry, the
    // coefficient zeroed for padding), so the batch's gathers are in flight together.
    constexpr int B = S < 8 ? S : 8;  // at most 64 / G = S steps per chunk of 64 nonzeros
    const int iters = (cnt + G - 1) / G;
    const int cl = act ? c : 0;
    for (int t0 = 0; t0 < iters; t0 += B) {
      int64_t jj[B];
      c128 aa[B], xx[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = g + (t0 + u) * G;
        const bool ok = k < cnt;
        const int src = ok ? k : 0;
        jj[u] = __shfl(mj, src, 64);
        aa[u] = csel(ok, cmk(__shfl(mv.re, src, 64), __shfl(mv.im, src, 64)), cmk(0.0, 0.0));
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const cplx<TX> v = x[jj[u] * s + cl];
        xx[u] = cmk((double)v.re, (double)v.im);
      }
#pragma unroll
      for (int u = 0; u < B; ++u) cfma(acc, aa[u], xx[u]);
    }
  }
#pragma unroll
  for (int m = S; m < 64; m <<= 1) {
    acc.re += shfl_xor(acc.re, m);
    acc.im += shfl_xor(acc.im, m);
  }
  if (g == 0 && act) {
    c128 r = alpha * acc;
    if (yin) r = r + beta * yin[row * s + c];
    y[row * s + c] = r;
  }
}

}  // namespace

template <typename TX>
void launch_spmm(hipStream_t st, int64_t n, int s, const int64_t* rowptr, const int32_t* col, const c128* val,
                 const cplx<TX>* x, c128* y, c128 alpha, c128 beta, const c128* yin) {
  if (n == 0 || s == 0) return;
  // the main kernel addresses x with 32-bit byte offsets (and marks unused lanes 0xFFFF0000)
  const bool fits32 = (uint64_t)n * (uint64_t)s * sizeof(cplx<TX>) < 0xFFFF0000ull;
  if (s > 8 && s <= 32 && fits32) {
    const unsigned gx = (unsigned)((n + 15) / 16);  // 4 wavefronts x 4 rows
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(gx), dim3(256), 0, st, n, s, rowptr, col, val, x, y, alpha, beta, yin);
    };
    if (s <= 16)
      go(k_spmm_dpp<TX, 1, false>);
    else if (sizeof(TX) == 4 && s % 2 == 0)
      go(k_spmm_dpp<TX, 2, true>);
    else
      go(k_spmm_dpp<TX, 2, false>);
  } else {
    const unsigned gx = (unsigned)((n + 3) / 4);
    auto go = [&](auto kern, int S) {
      hipLaunchKernelGGL(kern, dim3(gx, (unsigned)((s + S - 1) / S)), dim3(256), 0, st, n, s, rowptr, col, val, x, y,
                         alpha, beta, yin);
    };
    if (s == 1)
      go(k_spmm_rows<TX, 1>, 1);
    else if (s == 2)
      go(k_spmm_rows<TX, 2>, 2);
    else if (s <= 4)
      go(k_spmm_rows<TX, 4>, 4);
    else if (s <= 8)
      go(k_spmm_rows<TX, 8>, 8);
    else if (s <= 16)
      go(k_spmm_rows<TX, 16>, 16);
    else
      go(k_spmm_rows<TX, 32>, 32);
  }
  HIP_CHECK(hipGetLastError());
}

template void launch_spmm<double>(hipStream_t, int64_t, int, const int64_t*, const int32_t*, const c128*, const c128*,
                                  c128*, c128, c128, const c128*);
template void launch_spmm<float>(hipStream_t, int64_t, int, const int64_t*, const int32_t*, const c128*, const c64*,
                                 c128*, c128, c128, const c128*);

}  // namespace hz
