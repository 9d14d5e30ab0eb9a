// Application of the two-level ORAS preconditioner (paper eqs. 2lvl and oras):
//   z = M1^{-1} (v - A q) + q,  q = Z E^{-1} Z^T v,   M1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i
// on a block of s vectors in node-major layout ([n][s], s contiguous per dof).
//
// R_i is a gather by global dof id into the concatenated subdomain vectors (kept in each
// subdomain's elimination order); A_i^{-1} is the multifrontal triangular solve
// L (D (L^T x)) = b, level by level over all subdomains at once; the Boolean partition of
// unity makes sum_i R_i^T D_i a gather from each dof's owner.  No step uses atomics.
#include <cstdlib>
#include <type_traits>

#include "ddm.h"
#include "mfma_cplx.h"
#include "prof.h"

namespace hz {

// q = Z E^{-1} Z^T v and t = v - A q in the coarse precision (complex64 with mixed precision)
void coarse_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* q, c128* t);
void coarse_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c64* q, c64* t);

namespace {

constexpr int kNb = 32;
constexpr int kThreads = 256;

// z = owner's local value (+ add), summed in FP64 and rounded to the output type TZ
template <typename T, typename TQ, typename TZ>
__global__ void k_scatter_owner(int64_t n, int s, const int64_t* __restrict__ own, const cplx<T>* __restrict__ loc,
                                const cplx<TQ>* __restrict__ add, cplx<TZ>* __restrict__ z) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t g = k / s;
  const int c = (int)(k - g * s);
  const cplx<T> v = loc[own[g] * s + c];
  c128 r = cmk((double)v.re, (double)v.im);
  if (add) r = r + cmk((double)add[k].re, (double)add[k].im);
  z[k] = cmk((TZ)r.re, (TZ)r.im);
}

// the smooth partition of unity instead: z = sum over the subdomains holding the dof (in
// subdomain order) of weight x local value, summed in FP64 (+ add)
template <typename T, typename TQ, typename TZ>
__global__ void k_scatter_pou(int64_t n, int s, const int64_t* __restrict__ ptr, const int64_t* __restrict__ pos,
                              const double* __restrict__ wt, const cplx<T>* __restrict__ loc,
                              const cplx<TQ>* __restrict__ add, cplx<TZ>* __restrict__ z) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t g = k / s;
  const int c = (int)(k - g * s);
  c128 r = cmk(0.0, 0.0);
  for (int64_t e = ptr[g]; e < ptr[g + 1]; ++e) {
    const cplx<T> v = loc[pos[e] * s + c];
    r = r + cmk(wt[e] * (double)v.re, wt[e] * (double)v.im);
  }
  if (add) r = r + cmk((double)add[k].re, (double)add[k].im);
  z[k] = cmk((TZ)r.re, (TZ)r.im);
}

// streamed load through a buffer resource (32-bit byte offset; non-temporal)
__device__ __forceinline__ cplx<float> ld_stream_buf(__amdgpu_buffer_rsrc_t r, unsigned off, const cplx<float>*) {
  return __builtin_bit_cast(cplx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 2));
}
__device__ __forceinline__ cplx<double> ld_stream_buf(__amdgpu_buffer_rsrc_t r, unsigned off, const cplx<double>*) {
  return __builtin_bit_cast(cplx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 2));
}

// Forward, step 1 of a level: work block w = [b_p; 0] + extend-add of the children's
// contributions, through the inverse maps (own, child 0, child 1: a fixed order).  One block
// per 64-row tile of a front (the forward worklist: tiles of one front on one XCD).

// streamed load (the factor is read once per sweep): non-temporal hint
__device__ __forceinline__ cplx<float> ld_stream(const cplx<float>* p) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 v = __builtin_nontemporal_load(reinterpret_cast<const f2*>(p));
  return cmk(v.x, v.y);
}
__device__ __forceinline__ cplx<double> ld_stream(const cplx<double>* p) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
  return cmk(v.x, v.y);
}

// Forward, step 1: the work block of a front, w = [b_p; 0] + the children's update rows, in a
// fixed order (own, child 0, child 1).  b_p is read from the global right-hand side through
// the local-to-global map of the front's pivots (rounded to the factor precision), so no
// local copy of the right-hand side is made.
template <typename T, typename TS>
__global__ __launch_bounds__(256) void k_fwd_assemble(const int32_t* __restrict__ work, const FrontDesc* __restrict__ fr,
                                                      const int32_t* __restrict__ imap,
                                                      const int32_t* __restrict__ gidx,
                                                      const cplx<TS>* __restrict__ src, cplx<T>* __restrict__ wbuf,
                                                      int s, int pivots_only) {
  const int fid = work[2 * blockIdx.x];
  if (fid < 0) return;  // padding entry of the XCD-interleaved worklist (block-uniform)
  const int64_t i0 = work[2 * blockIdx.x + 1];
  const FrontDesc F = fr[fid];
  const int64_t f = F.p + F.r;
  const int64_t iend = pivots_only ? F.p : f;  // the matrix-core sweeps form update rows themselves
  if (i0 >= iend) return;
  const int64_t tot = (min<int64_t>(iend, i0 + 64) - i0) * s;
  const cplx<T>* w0 = nullptr;
  const cplx<T>* w1 = nullptr;
  if (F.child0 >= 0) {
    const FrontDesc C = fr[F.child0];
    w0 = wbuf + (C.w_off + C.p) * s;
  }
  if (F.child1 >= 0) {
    const FrontDesc C = fr[F.child1];
    w1 = wbuf + (C.w_off + C.p) * s;
  }
  const int32_t* m0 = imap + F.imap_off;
  const int32_t* m1 = m0 + f;
  // four elements per thread and pass: their index loads go out together, then their
  // gathers, then the sums (in the order own, child 0, child 1) and the stores
  constexpr int U = 4;
  const cplx<T> zero = cmk((T)0, (T)0);
  for (int64_t kb = threadIdx.x; kb < tot; kb += U * (int64_t)blockDim.x) {
    int64_t ii[U];
    int cc[U];
    int32_t g[U], q0[U], q1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = kb + u * (int64_t)blockDim.x;
      const int kk = k < tot ? (int)k : 0;  // past the tile: the tile's first element, not stored
      ii[u] = i0 + kk / s;                  // a tile holds at most 64 s elements: 32-bit division
      cc[u] = kk - (kk / s) * s;
      g[u] = ii[u] < F.p ? gidx[F.vec_off + F.pos0 + ii[u]] : 0;
      q0[u] = w0 ? m0[ii[u]] : -1;
      q1[u] = w1 ? m1[ii[u]] : -1;
    }
    cplx<T> b[U], x0[U], x1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ii[u] < F.p) {
        const cplx<TS> bs = src[(int64_t)g[u] * s + cc[u]];
        b[u] = cmk((T)bs.re, (T)bs.im);
      } else {
        b[u] = zero;
      }
      x0[u] = q0[u] >= 0 ? w0[(int64_t)q0[u] * s + cc[u]] : zero;
      x1[u] = q1[u] >= 0 ? w1[(int64_t)q1[u] * s + cc[u]] : zero;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cplx<T> v = b[u];
      if (q0[u] >= 0) v = v + x0[u];
      if (q1[u] >= 0) v = v + x1[u];
      if (kb + u * (int64_t)blockDim.x < tot) wbuf[(F.w_off + ii[u]) * s + cc[u]] = v;
    }
  }
}

// Forward, step 2: rows [i0, i0 + 64) of  [y; c] = [F_top w_p; w_r - F_bot w_p].
// F_top = L11^{-1} is unit lower triangular, so a tile of top rows stops at its diagonal.
// The pivot rows are stored divided by their pivots (y_p / d), what the backward sweep uses.
template <typename T, int S>
__global__ __launch_bounds__(256) void k_fwd_gemm(const int32_t* __restrict__ work, const FrontDesc* __restrict__ fr,
                                                  const cplx<T>* __restrict__ L, const cplx<T>* __restrict__ dinv,
                                                  cplx<T>* __restrict__ wbuf, cplx<T>* __restrict__ bout, int s) {
  constexpr int RT = 64, JC = 32, NA = (S + 3) / 4;
  __shared__ cplx<T> Ft[JC][RT + 1];
  __shared__ cplx<T> Wt[JC][S];
  const int fid = work[2 * blockIdx.x];
  if (fid < 0) return;  // padding entry of the XCD-interleaved worklist (block-uniform)
  const int64_t i0 = work[2 * blockIdx.x + 1];
  const FrontDesc F = fr[fid];
  const int64_t f = F.p + F.r;
  const int64_t jend = i0 < F.p ? min<int64_t>(F.p, i0 + RT) : F.p;
  const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const cplx<T>* Lf = L + F.L_off;
  const cplx<T>* wp = wbuf + F.w_off * s;
  cplx<T> acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = cmk((T)0, (T)0);
  for (int64_t j = 0; j < jend; j += JC) {
    const int jn = (int)min<int64_t>(JC, jend - j);
    __syncthreads();
    for (int e = threadIdx.x; e < JC * RT; e += 256) {
      const int jj = e / RT, rr = e - (e / RT) * RT;
      Ft[jj][rr] = (jj < jn && i0 + rr < f) ? Lf[(j + jj) * F.ld + i0 + rr] : cmk((T)0, (T)0);
    }
    for (int e = threadIdx.x; e < JC * S; e += 256) {
      const int jj = e / S, c = e - (e / S) * S;
      Wt[jj][c] = (jj < jn && c < s) ? wp[(j + jj) * s + c] : cmk((T)0, (T)0);
    }
    __syncthreads();
    if (cg < S) {
      for (int jj = 0; jj < jn; ++jj) {
        const cplx<T> a = Ft[jj][r];
#pragma unroll
        for (int q = 0; q < NA; ++q)
          if (cg + 4 * q < S) cfma(acc[q], a, Wt[jj][cg + 4 * q]);
      }
    }
  }
  const int64_t i = i0 + r;
  if (i < f) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int c = cg + 4 * q;
      if (c >= s) continue;
      if (i < F.p) {  // pivot rows leave y_p / d for the backward sweep
        const int64_t pos = F.vec_off + F.pos0 + i;
        bout[pos * s + c] = acc[q] * dinv[pos];
      } else {
        cplx<T>* w = &wbuf[(F.w_off + i) * s + c];
        *w = *w - acc[q];
      }
    }
  }
}

// Backward: columns [j0, j0 + 32) of  x_p = F^T u,  u = [y_p / d; -x_r]  (rows from j0 on;
// F_top is unit lower so rows above a column contribute nothing; the forward sweep stored y_p / d).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_bwd_gemm(const int32_t* __restrict__ work, const FrontDesc* __restrict__ fr,
                                                  const cplx<T>* __restrict__ L, const int32_t* __restrict__ urows,
                                                  const cplx<T>* __restrict__ bout,
                                                  cplx<T>* __restrict__ bin, int s) {
  constexpr int CT = 32, RC = 64, NB = (S + 7) / 8;
  __shared__ cplx<T> Ft[RC][CT + 1];
  __shared__ cplx<T> Ut[RC][S];
  const int fid = work[2 * blockIdx.x];
  if (fid < 0) return;  // padding entry of the XCD-interleaved worklist (block-uniform)
  const int64_t j0 = work[2 * blockIdx.x + 1];
  const FrontDesc F = fr[fid];
  const int64_t f = F.p + F.r;
  const int nj = (int)min<int64_t>(CT, F.p - j0);
  const int jj = threadIdx.x & 31, cgp = threadIdx.x >> 5;
  const cplx<T>* Lf = L + F.L_off;
  cplx<T> acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = cmk((T)0, (T)0);
  for (int64_t i = j0; i < f; i += RC) {
    const int rn = (int)min<int64_t>(RC, f - i);
    __syncthreads();
    for (int e = threadIdx.x; e < RC * CT; e += 256) {
      const int cc = e / RC, rr = e - (e / RC) * RC;
      Ft[rr][cc] = (rr < rn && cc < nj) ? Lf[(j0 + cc) * F.ld + i + rr] : cmk((T)0, (T)0);
    }
    for (int e = threadIdx.x; e < RC * S; e += 256) {
      const int rr = e / S, c = e - (e / S) * S;
      cplx<T> v = cmk((T)0, (T)0);
      if (rr < rn && c < s) {
        const int64_t row = i + rr;
        if (row < F.p) {
          const int64_t pos = F.vec_off + F.pos0 + row;
          v = bout[pos * s + c];  // y_p / d, left so by the forward sweep
        } else {
          const int64_t pos = F.vec_off + urows[F.rows_off + (row - F.p)];
          const cplx<T> x = bin[pos * s + c];
          v = cmk(-x.re, -x.im);
        }
      }
      Ut[rr][c] = v;
    }
    __syncthreads();
    if (cgp < S) {
      for (int rr = 0; rr < rn; ++rr) {
        const cplx<T> a = Ft[rr][jj];
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (cgp + 8 * q < S) cfma(acc[q], a, Ut[rr][cgp + 8 * q]);
      }
    }
  }
  if (jj < nj) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int c = cgp + 8 * q;
      if (c < s) bin[(F.vec_off + F.pos0 + j0 + jj) * s + c] = acc[q];
    }
  }
}

// ---- sweeps on the matrix cores (blocks of 16 or 32 columns): complex products in the
// three-multiplication form, CAcc (mfma_cplx.h)

// Forward rows [i0, i0 + 64 MT) (the k_fwd_gemm product on a wider tile): wavefront wv owns
// MT tiles of 16 rows, NG groups of 16 columns.  Each thread stages a fixed share of the next
// chunk in registers (loads from a clamped, always valid index, so they issue back to back)
// while the current chunk is multiplied out of LDS; the bounds predicate is applied when the
// registers are written to LDS, so the loads stay in flight across the products.
// The pivot rows of w, which every row tile multiplies, are read from the pass k_fwd_assemble
// made of them; the update rows of w = [b_p; 0] + the children's update contributions are
// formed in the epilogue, where each is read once, in the order of k_fwd_assemble (own,
// child 0, child 1).
template <typename T, int NG, int MT, int JC>
__global__ __launch_bounds__(256) void k_fwd_mfma(const int32_t* __restrict__ work, const FrontDesc* __restrict__ fr,
                                                  const cplx<T>* __restrict__ L, const int32_t* __restrict__ imap,
                                                  const cplx<T>* __restrict__ dinv, cplx<T>* __restrict__ wbuf,
                                                  cplx<T>* __restrict__ bout, int s) {
  constexpr int RT = 64 * MT, SC = 16 * NG;
  constexpr int NF = JC * RT / 256, NW = JC * SC / 256;
  // unpadded tile (20 KB for complex64, 64-row tiles: eight blocks per CU); a complex64 row's
  // 16-entry halves swap on odd columns, so the four columns a wavefront's products read at
  // once fall on the two halves of the LDS banks
  __shared__ cplx<T> Ft[JC][RT];
  __shared__ cplx<T> Wt[JC][SC];
  constexpr int SW = sizeof(cplx<T>) == 8 ? 16 : 0;
  const int fid = work[2 * blockIdx.x];
  if (fid < 0) return;  // padding entry of the XCD-interleaved worklist (block-uniform)
  const int64_t i0 = work[2 * blockIdx.x + 1];
  const FrontDesc F = fr[fid];
  const int64_t f = F.p + F.r;
  const int64_t jend = i0 < F.p ? min<int64_t>(F.p, i0 + RT) : F.p;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, l = tid & 63;
  const int lr = l & 15, lq = l >> 4;
  const cplx<T>* Lf = L + F.L_off;
  const cplx<T>* wp = wbuf + F.w_off * s;          // the assembled work block
  const int32_t* m0 = imap + F.imap_off;           // parent row -> child row (or -1), per child
  const int32_t* m1 = m0 + f;
  const cplx<T>* w0 = nullptr;  // the children's update rows (only children that have some)
  const cplx<T>* w1 = nullptr;
  if (F.child0 >= 0) {
    const FrontDesc C = fr[F.child0];
    if (C.r > 0) w0 = wbuf + (C.w_off + C.p) * s;
  }
  if (F.child1 >= 0) {
    const FrontDesc C = fr[F.child1];
    if (C.r > 0) w1 = wbuf + (C.w_off + C.p) * s;
  }
  const cplx<T> zero = cmk((T)0, (T)0);
  cplx<T> rf[NF], rb[NW];
  auto fetch = [&](int64_t j) {
    const int jn = (int)min<int64_t>(JC, jend - j);
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int e = tid + 256 * u, jj = e / RT, rr = e - (e / RT) * RT;  // element e of [JC][RT]
      rf[u] = ld_stream(&Lf[(jj < jn && i0 + rr < f) ? (j + jj) * F.ld + i0 + rr : 0]);
    }
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      const int e = tid + 256 * u, jj = e / SC, c = e - (e / SC) * SC;
      const bool ok = jj < jn && c < s;
      const int64_t row = ok ? j + jj : 0, cc = ok ? c : 0;
      rb[u] = wp[row * s + cc];
    }
  };
  CAcc<T> acc[MT][NG];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[m][g].zero();
  fetch(0);
  for (int64_t j = 0; j < jend; j += JC) {
    const int jn = (int)min<int64_t>(JC, jend - j);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int e = tid + 256 * u, jj = e / RT, rr = e - (e / RT) * RT;
      Ft[jj][rr ^ (SW * (jj & 1))] = csel(jj < jn && i0 + rr < f, rf[u], zero);
    }
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      const int e = tid + 256 * u, jj = e / SC, c = e - (e / SC) * SC;
      Wt[jj][c] = csel(jj < jn && c < s, rb[u], zero);
    }
    __syncthreads();
    if (j + JC < jend) fetch(j + JC);
    // four complex columns per step; columns past jn are zero in LDS, so the step count may
    // be rounded up to a multiple of 2
    const int steps = (((jn + 3) >> 2) + 1) & ~1;
#pragma unroll 2
    for (int t = 0; t < steps; ++t) {
      const int kc = 4 * t + lq;
      cplx<T> wb[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) wb[g] = Wt[kc][16 * g + lr];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const cplx<T> av = Ft[kc][(16 * (wv * MT + m) + lr) ^ (SW * (kc & 1))];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[m][g].mac(av, wb[g]);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int c = 16 * g + lr;
      if (c >= s) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + 16 * (wv * MT + m) + CAcc<T>::row(lq, v);
        if (i >= f) continue;
        const cplx<T> val = acc[m][g].get(v);
        if (i < F.p) {  // y_p / d for the backward sweep
          const int64_t pos = F.vec_off + F.pos0 + i;
          bout[pos * s + c] = val * dinv[pos];
        } else {  // update row: (0 + child 0 + child 1) - F_bot w_p
          cplx<T> wr = zero;
          if (w0) {
            const int32_t q = m0[i];
            if (q >= 0) wr = wr + w0[(int64_t)q * s + c];
          }
          if (w1) {
            const int32_t q = m1[i];
            if (q >= 0) wr = wr + w1[(int64_t)q * s + c];
          }
          wbuf[(F.w_off + i) * s + c] = wr - val;
        }
      }
    }
}

// Backward pivot columns [j0, j0 + 64 NT) (the k_bwd_gemm product on a wider tile):
// wavefront wv owns NT tiles of 16 columns; rows from j0 in chunks of 32, staged as in the
// forward kernel.  u rows below the pivot block are gathered through the update-row map;
// the row indices are loaded first, so the factor loads stay in flight while the dependent
// gathers wait for them.
template <typename T, int NG, int NT, int RC>
__global__ __launch_bounds__(256) void k_bwd_mfma(const int32_t* __restrict__ work, const FrontDesc* __restrict__ fr,
                                                  const cplx<T>* __restrict__ L, const int32_t* __restrict__ urows,
                                                  const cplx<T>* __restrict__ bout,
                                                  cplx<T>* __restrict__ bin, int s) {
  constexpr int CT = 64 * NT, SC = 16 * NG;
  constexpr int NF = RC * CT / 256, NU = RC * SC / 256;
  // unpadded tile with an XOR swizzle of the column by the row (sw): the 32 rows of one column
  // that consecutive lanes store fall on distinct banks, and so do the entries the products
  // read (complex64: the two rows a half-wavefront reads at once use the two halves of the banks)
  __shared__ cplx<T> Ft[RC][CT];
  __shared__ cplx<T> Ut[RC][SC];
  auto sw = [](int r) { return sizeof(cplx<T>) == 8 ? (((r & 1) << 4) | ((r >> 1) & 15)) : (r & 15); };
  const int fid = work[2 * blockIdx.x];
  if (fid < 0) return;  // padding entry of the XCD-interleaved worklist (block-uniform)
  const int64_t j0 = work[2 * blockIdx.x + 1];
  const FrontDesc F = fr[fid];
  const int64_t f = F.p + F.r;
  const int nj = (int)min<int64_t>(CT, F.p - j0);
  const int tid = threadIdx.x;
  const int wv = tid >> 6, l = tid & 63;
  const int lr = l & 15, lq = l >> 4;
  // the tile's columns of the front's panel as a buffer (byte offsets fit 32 bits: a panel is
  // ld p entries, far below 4 GB)
  const __amdgpu_buffer_rsrc_t Lr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(L + F.L_off + j0 * F.ld), (short)0, (int)((int64_t)F.ld * nj * (int64_t)sizeof(cplx<T>)), 0x00020000);
  const int64_t pbase = F.vec_off + F.pos0;  // first pivot position: a valid clamp target
  const cplx<T> zero = cmk((T)0, (T)0);
  cplx<T> rf[NF], rx[NU];
  auto fetch = [&](int64_t i) {
    const int rn = (int)min<int64_t>(RC, f - i);
    // update-row indices from a clamped (valid) index; a front without update rows reads
    // none (its map may be empty), a block-uniform test
    int32_t ui[NU];
    if (F.r > 0) {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int rr = (tid + 256 * u) / SC;
        const int64_t row = i + rr;
        ui[u] = urows[F.rows_off + ((rr < rn && row >= F.p) ? row - F.p : 0)];
      }
    } else {
#pragma unroll
      for (int u = 0; u < NU; ++u) ui[u] = 0;
    }
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int e = tid + 256 * u, cc = e / RC, rr = e - (e / RC) * RC;  // element e of [CT][RC]
      const unsigned off = (rr < rn && cc < nj) ? (unsigned)(cc * F.ld + (int)i + rr) * (unsigned)sizeof(cplx<T>) : 0u;
      rf[u] = ld_stream_buf(Lr, off, (const cplx<T>*)nullptr);
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + 256 * u, rr = e / SC, c = e - (e / SC) * SC;
      const int64_t row = i + rr;
      const bool ok = rr < rn && c < s;
      const bool piv = row < F.p;
      const int64_t pos = piv ? pbase + row : F.vec_off + ui[u];
      rx[u] = (piv ? bout : bin)[(ok ? pos : pbase) * s + (ok ? c : 0)];
    }
  };
  CAcc<T> acc[NT][NG];
#pragma unroll
  for (int m = 0; m < NT; ++m)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[m][g].zero();
  fetch(j0);
  for (int64_t i = j0; i < f; i += RC) {
    const int rn = (int)min<int64_t>(RC, f - i);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int e = tid + 256 * u, cc = e / RC, rr = e - (e / RC) * RC;
      Ft[rr][cc ^ sw(rr)] = csel(rr < rn && cc < nj, rf[u], zero);
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + 256 * u, rr = e / SC, c = e - (e / SC) * SC;
      const bool ok = rr < rn && c < s;
      const bool piv = i + rr < F.p;
      const cplx<T> x = rx[u];
      Ut[rr][c] = csel(ok, csel(piv, x, cmk(-x.re, -x.im)), zero);  // [y_p / d; -x_r]
    }
    __syncthreads();
    if (i + RC < f) fetch(i + RC);
    const int steps = (((rn + 3) >> 2) + 1) & ~1;
#pragma unroll 2
    for (int t = 0; t < steps; ++t) {
      const int rr = 4 * t + lq;
      cplx<T> ub[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) ub[g] = Ut[rr][16 * g + lr];
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        const cplx<T> av = Ft[rr][(16 * (wv * NT + m) + lr) ^ sw(rr)];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[m][g].mac(av, ub[g]);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < NT; ++m)
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int c = 16 * g + lr;
      if (c >= s) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = 16 * (wv * NT + m) + CAcc<T>::row(lq, v);
        if (jj < nj) bin[(F.vec_off + F.pos0 + j0 + jj) * s + c] = acc[m][g].get(v);
      }
    }
}

// Matrix-core sweeps serve blocks of at least 8 columns (both precisions in the three-product
// form); narrower blocks stay on the vector-unit kernels.
template <typename T, int S>
constexpr bool use_mfma() {
  return S >= 8;
}

template <typename T, typename TS>
void fwd_assemble(Ctx* ctx, Ddm& d, size_t lv, int s, const cplx<TS>* src, cplx<T>* wbuf, bool pivots_only) {
  const unsigned nb = (unsigned)(d.fwd_off[lv + 1] - d.fwd_off[lv]);  // 64-row tiles of the level
  hipLaunchKernelGGL((k_fwd_assemble<T, TS>), dim3(nb), dim3(256), 0, ctx->stream,
                     d.d_fwd_work.ptr() + 2 * d.fwd_off[lv], d.d_fronts.ptr(), d.d_imap.ptr(), d.d_gidx.ptr(), src,
                     wbuf, s, pivots_only ? 1 : 0);
}

// Vector-unit sweeps (complex128, and complex64 blocks narrower than 8 columns).
template <typename T, int S, typename TS>
void sweep_valu(Ctx* ctx, Ddm& d, int s, const cplx<TS>* src, cplx<T>* bin, cplx<T>* bout, cplx<T>* wbuf) {
  hipStream_t st = ctx->stream;
  const cplx<T>* L = d.d_factor.as<cplx<T>>();
  const double esz = (double)sizeof(cplx<T>);
  for (size_t lv = 0; lv < d.levels.size(); ++lv) {
    fwd_assemble<T, TS>(ctx, d, lv, s, src, wbuf, false);
    const Level& Lv = d.levels[lv];
    // algorithmic traffic: the level's stored factor once, its work rows read and written once
    ProfScope ps(ctx, HZ_K_ORAS_FWD, esz * ((double)Lv.useful + 2.0 * (double)Lv.sum_f * s),
                 8.0 * (double)Lv.useful * s);
    hipLaunchKernelGGL((k_fwd_gemm<T, S>), dim3((unsigned)(d.fwd_off[lv + 1] - d.fwd_off[lv])), dim3(256), 0, st,
                       d.d_fwd_work.ptr() + 2 * d.fwd_off[lv], d.d_fronts.ptr(), L, d.d_dinv.as<cplx<T>>(), wbuf,
                       bout, s);
  }
  for (size_t lv = d.levels.size(); lv-- > 0;) {
    const Level& Lv = d.levels[lv];
    ProfScope ps(ctx, HZ_K_ORAS_BWD, esz * ((double)Lv.useful + (double)(Lv.sum_f + Lv.sum_p) * s),
                 8.0 * (double)Lv.useful * s);
    hipLaunchKernelGGL((k_bwd_gemm<T, S>), dim3((unsigned)(d.bwd_off[lv + 1] - d.bwd_off[lv])), dim3(256), 0, st,
                       d.d_bwd_work.ptr() + 2 * d.bwd_off[lv], d.d_fronts.ptr(), L, d.d_urows.ptr(), bout, bin, s);
  }
  HIP_CHECK(hipGetLastError());
}

// Matrix-core sweeps (8..32 columns; complex64 or complex128).  The tile of each level and direction is one
// of two sizes; the first apply for a column-group width times both on every level (all tile
// sizes give bit-identical results, and every timed launch is repeated exactly as the real
// one: a forward level re-assembles the pivot rows of its work block before each try) and
// keeps the faster one.
template <typename T, int S, typename TS>
void sweep_mfma(Ctx* ctx, Ddm& d, int s, const cplx<TS>* src, cplx<T>* bin, cplx<T>* bout, cplx<T>* wbuf) {
  constexpr int NG = (S + 15) / 16;
  hipStream_t st = ctx->stream;
  const cplx<T>* L = d.d_factor.as<cplx<T>>();
  const double esz = (double)sizeof(cplx<T>);
  const size_t nl = d.levels.size();
  const int gi = NG - 1;
  const bool tune = d.tile_fwd[gi].size() != nl;
  auto fwd = [&](size_t lv, int t) {
    const dim3 grid((unsigned)(d.fwdm_off[t][lv + 1] - d.fwdm_off[t][lv]));
    const int32_t* wl = d.d_fwdm_work[t].ptr() + 2 * d.fwdm_off[t][lv];
    if (t == 0)
      hipLaunchKernelGGL((k_fwd_mfma<T, NG, kFwdRowsMfma[0] / 64, 32>), grid, dim3(256), 0, st, wl, d.d_fronts.ptr(), L,
                         d.d_imap.ptr(), d.d_dinv.as<cplx<T>>(), wbuf, bout, s);
    else
      hipLaunchKernelGGL((k_fwd_mfma<T, NG, kFwdRowsMfma[1] / 64, 32>), grid, dim3(256), 0, st, wl, d.d_fronts.ptr(), L,
                         d.d_imap.ptr(), d.d_dinv.as<cplx<T>>(), wbuf, bout, s);
  };
  auto bwd = [&](size_t lv, int t) {
    const dim3 grid((unsigned)(d.bwdm_off[t][lv + 1] - d.bwdm_off[t][lv]));
    const int32_t* wl = d.d_bwdm_work[t].ptr() + 2 * d.bwdm_off[t][lv];
    if (t == 0)
      hipLaunchKernelGGL((k_bwd_mfma<T, NG, kBwdColsMfma[0] / 64, 32>), grid, dim3(256), 0, st, wl, d.d_fronts.ptr(), L,
                         d.d_urows.ptr(), bout, bin, s);
    else
      hipLaunchKernelGGL((k_bwd_mfma<T, NG, kBwdColsMfma[1] / 64, 32>), grid, dim3(256), 0, st, wl, d.d_fronts.ptr(), L,
                         d.d_urows.ptr(), bout, bin, s);
  };
  if (!tune) {
    for (size_t lv = 0; lv < nl; ++lv) {
      fwd_assemble<T, TS>(ctx, d, lv, s, src, wbuf, true);
      const Level& Lv = d.levels[lv];
      // algorithmic traffic: the level's stored factor once, its work rows read and written once
      ProfScope ps(ctx, HZ_K_ORAS_FWD, esz * ((double)Lv.useful + 2.0 * (double)Lv.sum_f * s),
                   8.0 * (double)Lv.useful * s);
      fwd(lv, d.tile_fwd[gi][lv]);
    }
    for (size_t lv = nl; lv-- > 0;) {
      const Level& Lv = d.levels[lv];
      ProfScope ps(ctx, HZ_K_ORAS_BWD, esz * ((double)Lv.useful + (double)(Lv.sum_f + Lv.sum_p) * s),
                   8.0 * (double)Lv.useful * s);
      bwd(lv, d.tile_bwd[gi][lv]);
    }
    HIP_CHECK(hipGetLastError());
    return;
  }
  // tuning apply: both tile sizes on every level, each run twice and timed the second time
  // (the first launch of a kernel carries one-time costs); the last try leaves the result
  std::vector<hipEvent_t> ev(8 * nl);
  for (auto& e : ev) HIP_CHECK(hipEventCreate(&e));
  auto at = [&](int dir, size_t lv, int t, int edge) -> hipEvent_t& { return ev[((dir * nl + lv) * 2 + t) * 2 + edge]; };
  for (size_t lv = 0; lv < nl; ++lv)
    for (int rep = 0; rep < 2; ++rep)
      for (int t = 0; t < 2; ++t) {
        fwd_assemble<T, TS>(ctx, d, lv, s, src, wbuf, true);
        if (rep) HIP_CHECK(hipEventRecord(at(0, lv, t, 0), st));
        fwd(lv, t);
        if (rep) HIP_CHECK(hipEventRecord(at(0, lv, t, 1), st));
      }
  for (size_t lv = nl; lv-- > 0;)
    for (int rep = 0; rep < 2; ++rep)
      for (int t = 0; t < 2; ++t) {
        if (rep) HIP_CHECK(hipEventRecord(at(1, lv, t, 0), st));
        bwd(lv, t);
        if (rep) HIP_CHECK(hipEventRecord(at(1, lv, t, 1), st));
      }
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<uint8_t> cf(nl), cb(nl);
  for (int dir = 0; dir < 2; ++dir)
    for (size_t lv = 0; lv < nl; ++lv) {
      float ms[2];
      for (int t = 0; t < 2; ++t) HIP_CHECK(hipEventElapsedTime(&ms[t], at(dir, lv, t, 0), at(dir, lv, t, 1)));
      const uint8_t pick = ms[1] < 0.97f * ms[0] ? 1 : 0;  // the smaller tile unless clearly slower
      (dir == 0 ? cf : cb)[lv] = pick;
    }
  for (auto& e : ev) HIP_CHECK(hipEventDestroy(e));
  d.tile_fwd[gi] = cf;
  d.tile_bwd[gi] = cb;
}

// src: the global right-hand side (the forward sweep reads its pivot rows through the
// local-to-global map); bin: the local solution, written by the backward sweep
template <typename T, int S, typename TS>
void sweep(Ctx* ctx, Ddm& d, int s, const cplx<TS>* src, cplx<T>* bin, cplx<T>* bout, cplx<T>* wbuf) {
  if constexpr (use_mfma<T, S>())
    sweep_mfma<T, S, TS>(ctx, d, s, src, bin, bout, wbuf);
  else
    sweep_valu<T, S, TS>(ctx, d, s, src, bin, bout, wbuf);
}

template <typename T, typename TS, typename TQ, typename TZ>
void one_level(Ctx* ctx, Ddm& d, int s, const cplx<TS>* v, const cplx<TQ>* add, cplx<TZ>* z, DevBuf& bin, DevBuf& bout,
               DevBuf& wbuf) {
  hipStream_t st = ctx->stream;
  const int64_t nl = d.n_local_total;
  const int64_t n = d.op->mesh->n;
  auto ensure = [&](DevBuf& b, int64_t elems) {
    const size_t need = (size_t)std::max<int64_t>(1, elems) * sizeof(cplx<T>);
    if (b.bytes < need) {
      b.release();
      b.alloc(ctx, need);
    }
  };
  ensure(bin, nl * s);
  ensure(bout, nl * s);
  if (!d.icc) ensure(wbuf, d.w_total * s);
  cplx<T>* bi = bin.as<cplx<T>>();
  cplx<T>* bo = bout.as<cplx<T>>();
  cplx<T>* wb = wbuf.as<cplx<T>>();
  if (s > 32)
    fail(HZ_ERR_ARG, "preconditioner: at most 32 columns per block");
  else if (d.icc)
    icc_apply(ctx, d, s, v, bi, bo);  // incomplete factors: the local solutions straight into bi
  else if (s <= 1)
    sweep<T, 1, TS>(ctx, d, s, v, bi, bo, wb);
  else if (s <= 2)
    sweep<T, 2, TS>(ctx, d, s, v, bi, bo, wb);
  else if (s <= 4)
    sweep<T, 4, TS>(ctx, d, s, v, bi, bo, wb);
  else if (s <= 8)
    sweep<T, 8, TS>(ctx, d, s, v, bi, bo, wb);
  else if (s <= 16)
    sweep<T, 16, TS>(ctx, d, s, v, bi, bo, wb);
  else
    sweep<T, 32, TS>(ctx, d, s, v, bi, bo, wb);
  if (d.pou == HZ_POU_SMOOTH)
    hipLaunchKernelGGL((k_scatter_pou<T, TQ, TZ>), dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, st, n, s,
                       d.d_pou_ptr.ptr(), d.d_pou_pos.ptr(), d.d_pou_w.ptr(), bi, add, z);
  else
    hipLaunchKernelGGL((k_scatter_owner<T, TQ, TZ>), dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, st, n, s,
                       d.d_own_src.ptr(), bi, add, z);
  HIP_CHECK(hipGetLastError());
}

}  // namespace

void precond_release_workspace(Ddm& d) { d.pw = PrecondWork(); }

namespace {

template <typename TZ>
void precond_apply_t(Ctx* ctx, Ddm& d, int s, const c128* v, cplx<TZ>* z) {
  PrecondWork& w = ctx->shared_pw ? *ctx->shared_pw : d.pw;
  const int64_t n = d.op->mesh->n;
  const bool mixed = d.precision == HZ_PREC_MIXED;
  if (d.coarse) {  // q and t in the coarse precision
    const size_t need = (size_t)(n * s) * (mixed ? sizeof(c64) : sizeof(c128));
    if (w.q.bytes < need) {
      w.q.release();
      w.t.release();
      w.q.alloc(ctx, need);
      w.t.alloc(ctx, need);
    }
    if (mixed) {
      coarse_apply(ctx, d, s, v, w.q.as<c64>(), w.t.as<c64>());
      one_level<float, float, float, TZ>(ctx, d, s, w.t.as<c64>(), w.q.as<c64>(), z, w.bin, w.bout, w.wbuf);
    } else {
      coarse_apply(ctx, d, s, v, w.q.as<c128>(), w.t.as<c128>());
      one_level<double, double, double, TZ>(ctx, d, s, w.t.as<c128>(), w.q.as<c128>(), z, w.bin, w.bout, w.wbuf);
    }
  } else if (mixed) {
    one_level<float, double, float, TZ>(ctx, d, s, v, (const c64*)nullptr, z, w.bin, w.bout, w.wbuf);
  } else {
    one_level<double, double, double, TZ>(ctx, d, s, v, (const c128*)nullptr, z, w.bin, w.bout, w.wbuf);
  }
}

}  // namespace

void precond_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* z) { precond_apply_t<double>(ctx, d, s, v, z); }

void precond_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c64* z) {
  HZ_REQUIRE(d.precision == HZ_PREC_MIXED, HZ_ERR_STATE, "preconditioner: complex64 output needs mixed precision");
  precond_apply_t<float>(ctx, d, s, v, z);
}

}  // namespace hz
