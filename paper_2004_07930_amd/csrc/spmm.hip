// Multi-RHS complex CSR SpMM  y = alpha A x + beta y_in  on node-major blocks ([n][s]).
//
// A wavefront owns one row; its 64 lanes are split into G = 64/S groups of S column
// lanes.  Each group walks every G-th nonzero of the row, so a nonzero's value and column
// index are loaded once per group and broadcast to the S lanes, and the S lanes read the
// S contiguous complex entries x[col][0..S) (one coalesced segment).  The G partial sums
// are combined with cross-lane shuffles in a fixed order, so results are bitwise
// reproducible.  HBM-bound: algorithmic bytes 20 nnz + 8 (n+1) + 2 * 16 n s per call (c128).
#include "hz_internal.h"

namespace hz {

namespace {

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m) {
  return __shfl_xor(v, m, 64);
}

template <typename T, int S>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, int s, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, const cplx<T>* __restrict__ val,
                                              const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y, cplx<T> alpha,
                                              cplx<T> beta, const cplx<T>* __restrict__ yin) {
  constexpr int G = 64 / S;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = lane / S;
  const int c = blockIdx.y * S + (lane % S);
  if (row >= n) return;
  const bool act = c < s;
  cplx<T> acc = cmk((T)0, (T)0);
  const int64_t e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int64_t base = e0; base < e1; base += 64) {
    // lanes fetch 64 (column, value) pairs at once; groups read them back by shuffles
    const int cnt = (int)min<int64_t>(64, e1 - base);
    int32_t mj = 0;
    cplx<T> mv = cmk((T)0, (T)0);
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
      cplx<T> aa[B], xx[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = g + (t0 + u) * G;
        const bool ok = k < cnt;
        const int src = ok ? k : 0;
        jj[u] = __shfl(mj, src, 64);
        aa[u] = csel(ok, cmk(__shfl(mv.re, src, 64), __shfl(mv.im, src, 64)), cmk((T)0, (T)0));
      }
#pragma unroll
      for (int u = 0; u < B; ++u) xx[u] = x[jj[u] * s + cl];
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
    cplx<T> r = alpha * acc;
    if (yin) r = r + beta * yin[row * s + c];
    y[row * s + c] = r;
  }
}

}  // namespace

template <typename T>
void launch_spmm(hipStream_t st, int64_t n, int s, const int64_t* rowptr, const int32_t* col, const cplx<T>* val,
                 const cplx<T>* x, cplx<T>* y, cplx<T> alpha, cplx<T> beta, const cplx<T>* yin) {
  if (n == 0 || s == 0) return;
  const unsigned gx = (unsigned)((n + 3) / 4);
  auto go = [&](auto kern, int S) {
    hipLaunchKernelGGL(kern, dim3(gx, (unsigned)((s + S - 1) / S)), dim3(256), 0, st, n, s, rowptr, col, val, x, y,
                       alpha, beta, yin);
  };
  if (s == 1)
    go(k_spmm<T, 1>, 1);
  else if (s == 2)
    go(k_spmm<T, 2>, 2);
  else if (s <= 4)
    go(k_spmm<T, 4>, 4);
  else if (s <= 8)
    go(k_spmm<T, 8>, 8);
  else if (s <= 16)
    go(k_spmm<T, 16>, 16);
  else
    go(k_spmm<T, 32>, 32);
  HIP_CHECK(hipGetLastError());
}

template void launch_spmm<double>(hipStream_t, int64_t, int, const int64_t*, const int32_t*, const c128*, const c128*,
                                  c128*, c128, c128, const c128*);
template void launch_spmm<float>(hipStream_t, int64_t, int, const int64_t*, const int32_t*, const c64*, const c64*,
                                 c64*, c64, c64, const c64*);

}  // namespace hz
