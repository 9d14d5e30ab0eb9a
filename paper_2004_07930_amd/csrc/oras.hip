// Application of the two-level ORAS preconditioner (paper eqs. 2lvl and oras):
//   z = M1^{-1} (v - A q) + q,  q = Z E^{-1} Z^T v,   M1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i
// on a block of s vectors in node-major layout ([n][s], s contiguous per dof).
//
// R_i is a gather by global dof id into the concatenated subdomain vectors (kept in each
// subdomain's elimination order); A_i^{-1} is the multifrontal triangular solve
// L (D (L^T x)) = b, level by level over all subdomains at once; the Boolean partition of
// unity makes sum_i R_i^T D_i a gather from each dof's owner.  No step uses atomics.
#include <cstdlib>

#include "ddm.h"

namespace hz {

void coarse_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* q, c128* t);

namespace {

constexpr int kNb = 32;
constexpr int kThreads = 256;

template <typename T>
__global__ void k_gather_local(int64_t nloc, int s, const int32_t* __restrict__ gidx, const c128* __restrict__ src,
                               cplx<T>* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nloc * s) return;
  const int64_t q = k / s;
  const int c = (int)(k - q * s);
  const c128 v = src[(int64_t)gidx[q] * s + c];
  dst[k] = cmk((T)v.re, (T)v.im);
}

template <typename T>
__global__ void k_scatter_owner(int64_t n, int s, const int64_t* __restrict__ own, const cplx<T>* __restrict__ loc,
                                const c128* __restrict__ add, c128* __restrict__ z) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t g = k / s;
  const int c = (int)(k - g * s);
  const cplx<T> v = loc[own[g] * s + c];
  c128 r = cmk((double)v.re, (double)v.im);
  if (add) r = r + add[k];
  z[k] = r;
}

// Forward multifrontal sweep of one level: one block per front.
// bloc: concatenated local vectors [pos][s]; cbuf: per-front r x s contributions.
template <typename T, int S>
__global__ __launch_bounds__(kThreads) void k_fwd(const int32_t* __restrict__ lf, const FrontDesc* __restrict__ fr,
                                                  const cplx<T>* __restrict__ L, const int32_t* __restrict__ emap,
                                                  cplx<T>* __restrict__ bloc, cplx<T>* __restrict__ cbuf, int s) {
  __shared__ cplx<T> yk[kNb][S];
  const FrontDesc F = fr[lf[blockIdx.x]];
  const int64_t f = F.p + F.r;
  cplx<T>* bp = bloc + (F.vec_off + F.pos0) * s;  // pivot rows
  cplx<T>* cb = cbuf + F.cvec_off * s;            // update rows
  for (int64_t k = threadIdx.x; k < (int64_t)F.r * s; k += kThreads) cb[k] = cmk((T)0, (T)0);
  __syncthreads();
  for (int slot = 0; slot < 2; ++slot) {
    const int c = slot == 0 ? F.child0 : F.child1;
    if (c < 0) continue;
    const FrontDesc C = fr[c];
    const cplx<T>* cc = cbuf + C.cvec_off * s;
    for (int64_t k = threadIdx.x; k < (int64_t)C.r * s; k += kThreads) {
      const int64_t i = k / s;
      const int col = (int)(k - i * s);
      const int64_t t = emap[C.emap_off + i];
      cplx<T>* dst = t < F.p ? &bp[t * s + col] : &cb[(t - F.p) * s + col];
      *dst = *dst + cc[k];
    }
    __syncthreads();
  }
  const cplx<T>* Lf = L + F.L_off;
  for (int kb = 0; kb < F.p; kb += kNb) {
    const int nb = min(kNb, F.p - kb);
    // y_k = inv(L_kk) b_k ; inverse stored transposed in the block's strict upper part
    const cplx<T>* blk = Lf + (int64_t)kb * f + kb;
    for (int k = threadIdx.x; k < nb * s; k += kThreads) {
      const int i = k / s, col = k - (k / s) * s;
      cplx<T> acc = bp[(int64_t)(kb + i) * s + col];
      for (int l = 0; l < i; ++l) cfma(acc, blk[(int64_t)i * f + l], bp[(int64_t)(kb + l) * s + col]);
      yk[i][col] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb * s; k += kThreads) {
      const int i = k / s, col = k - (k / s) * s;
      bp[(int64_t)(kb + i) * s + col] = yk[i][col];
    }
    // rows below: b_i -= L[i][kb:kb+nb] y_k
    for (int64_t i = kb + nb + threadIdx.x; i < f; i += kThreads) {
      cplx<T> acc[S];
#pragma unroll
      for (int col = 0; col < S; ++col) acc[col] = cmk((T)0, (T)0);
      for (int l = 0; l < nb; ++l) {
        const cplx<T> a = Lf[(int64_t)(kb + l) * f + i];
#pragma unroll
        for (int col = 0; col < S; ++col) cfma(acc[col], a, yk[l][col]);
      }
      cplx<T>* dst = i < F.p ? &bp[i * s] : &cb[(i - F.p) * s];
#pragma unroll
      for (int col = 0; col < S; ++col)
        if (col < s) dst[col] = dst[col] - acc[col];
    }
    __syncthreads();
  }
}

// Backward sweep of one level: x_k = inv(L_kk)^T (z_k / d_k - L[below, k]^T x_below),
// blocks from the last to the first; rows >= p read the ancestors' solutions.
template <typename T, int S>
__global__ __launch_bounds__(kThreads) void k_bwd(const int32_t* __restrict__ lf, const FrontDesc* __restrict__ fr,
                                                  const cplx<T>* __restrict__ L, const int32_t* __restrict__ urows,
                                                  cplx<T>* __restrict__ bloc, int s) {
  constexpr int kRows = 64;
  __shared__ cplx<T> Lt[kRows][kNb + 1];
  __shared__ cplx<T> Xt[kRows][S];
  __shared__ cplx<T> W[kNb][S];
  const FrontDesc F = fr[lf[blockIdx.x]];
  const int64_t f = F.p + F.r;
  cplx<T>* bv = bloc + F.vec_off * s;
  cplx<T>* bp = bv + (int64_t)F.pos0 * s;
  const cplx<T>* Lf = L + F.L_off;
  const int nblk = (F.p + kNb - 1) / kNb;
  // each thread owns (j, col) pairs of the 32 x S accumulator
  for (int b = nblk - 1; b >= 0; --b) {
    const int kb = b * kNb;
    const int nb = min(kNb, F.p - kb);
    cplx<T> acc[(kNb * S + kThreads - 1) / kThreads];
#pragma unroll
    for (int a = 0; a < (kNb * S + kThreads - 1) / kThreads; ++a) acc[a] = cmk((T)0, (T)0);
    for (int64_t i0 = kb + nb; i0 < f; i0 += kRows) {
      const int rows = (int)min<int64_t>(kRows, f - i0);
      __syncthreads();
      for (int t = threadIdx.x; t < kRows * kNb; t += kThreads) {
        const int l = t / kRows, r = t - (t / kRows) * kRows;
        Lt[r][l] = (r < rows && l < nb) ? Lf[(int64_t)(kb + l) * f + i0 + r] : cmk((T)0, (T)0);
      }
      for (int t = threadIdx.x; t < kRows * S; t += kThreads) {
        const int r = t / S, col = t - (t / S) * S;
        cplx<T> x = cmk((T)0, (T)0);
        if (r < rows && col < s) {
          const int64_t i = i0 + r;
          const int64_t pos = i < F.p ? F.pos0 + i : urows[F.rows_off + (i - F.p)];
          x = bv[pos * s + col];
        }
        Xt[r][col] = x;
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < (kNb * S + kThreads - 1) / kThreads; ++a) {
        const int t = threadIdx.x + a * kThreads;
        if (t < kNb * S) {
          const int j = t / S, col = t - (t / S) * S;
          for (int r = 0; r < rows; ++r) cfma(acc[a], Lt[r][j], Xt[r][col]);
        }
      }
    }
    __syncthreads();
    const cplx<T>* blk = Lf + (int64_t)kb * f + kb;
#pragma unroll
    for (int a = 0; a < (kNb * S + kThreads - 1) / kThreads; ++a) {
      const int t = threadIdx.x + a * kThreads;
      if (t < kNb * S) {
        const int j = t / S, col = t - (t / S) * S;
        if (j < nb && col < s) {
          const cplx<T> dj = blk[(int64_t)j * f + j];
          W[j][col] = cdiv(bp[(int64_t)(kb + j) * s + col], dj) - acc[a];
        } else {
          W[j][col] = cmk((T)0, (T)0);
        }
      }
    }
    __syncthreads();
    // x_k = inv(L_kk)^T w : x[l] = w[l] + sum_{m > l} X[m][l] w[m], X[m][l] at blk[m*f + l]
    for (int t = threadIdx.x; t < nb * s; t += kThreads) {
      const int l = t / s, col = t - (t / s) * s;
      cplx<T> x = W[l][col];
      for (int m = l + 1; m < nb; ++m) cfma(x, blk[(int64_t)m * f + l], W[m][col]);
      bp[(int64_t)(kb + l) * s + col] = x;
    }
    __syncthreads();
  }
}

template <typename T>
struct Work {
  DevBuf bloc, cbuf;
  DevBuf t, q;
  int s = 0;
};

template <typename T, int S>
void sweep(Ctx* ctx, Ddm& d, int s, cplx<T>* bloc, cplx<T>* cbuf) {
  hipStream_t st = ctx->stream;
  const cplx<T>* L = d.d_factor.as<cplx<T>>();
  for (size_t lv = 0; lv < d.levels.size(); ++lv) {
    const int nf = (int)d.levels[lv].fronts.size();
    hipLaunchKernelGGL((k_fwd<T, S>), dim3(nf), dim3(kThreads), 0, st, d.d_level_fronts.ptr() + d.level_off[lv],
                       d.d_fronts.ptr(), L, d.d_emap.ptr(), bloc, cbuf, s);
  }
  for (size_t lv = d.levels.size(); lv-- > 0;) {
    const int nf = (int)d.levels[lv].fronts.size();
    hipLaunchKernelGGL((k_bwd<T, S>), dim3(nf), dim3(kThreads), 0, st, d.d_level_fronts.ptr() + d.level_off[lv],
                       d.d_fronts.ptr(), L, d.d_urows.ptr(), bloc, s);
  }
  HIP_CHECK(hipGetLastError());
}

template <typename T>
void one_level(Ctx* ctx, Ddm& d, int s, const c128* v, const c128* add, c128* z, DevBuf& bloc, DevBuf& cbuf) {
  hipStream_t st = ctx->stream;
  const int64_t nl = d.n_local_total;
  const int64_t n = d.op->mesh->n;
  if (bloc.bytes < (size_t)(nl * s) * sizeof(cplx<T>)) {
    bloc.release();
    bloc.alloc(ctx, (size_t)(nl * s) * sizeof(cplx<T>));
  }
  if (cbuf.bytes < (size_t)(std::max<int64_t>(1, d.cvec_total) * s) * sizeof(cplx<T>)) {
    cbuf.release();
    cbuf.alloc(ctx, (size_t)(std::max<int64_t>(1, d.cvec_total) * s) * sizeof(cplx<T>));
  }
  cplx<T>* bl = bloc.as<cplx<T>>();
  cplx<T>* cb = cbuf.as<cplx<T>>();
  hipLaunchKernelGGL(k_gather_local<T>, dim3((unsigned)((nl * s + 255) / 256)), dim3(256), 0, st, nl, s,
                     d.d_gidx.ptr(), v, bl);
  if (s <= 1)
    sweep<T, 1>(ctx, d, s, bl, cb);
  else if (s <= 2)
    sweep<T, 2>(ctx, d, s, bl, cb);
  else if (s <= 4)
    sweep<T, 4>(ctx, d, s, bl, cb);
  else if (s <= 8)
    sweep<T, 8>(ctx, d, s, bl, cb);
  else if (s <= 16)
    sweep<T, 16>(ctx, d, s, bl, cb);
  else if (s <= 32)
    sweep<T, 32>(ctx, d, s, bl, cb);
  else
    fail(HZ_ERR_ARG, "preconditioner: at most 32 columns per block");
  hipLaunchKernelGGL(k_scatter_owner<T>, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, st, n, s,
                     d.d_own_src.ptr(), bl, add, z);
  HIP_CHECK(hipGetLastError());
}

}  // namespace

struct PrecondWork {
  DevBuf bloc, cbuf, q, t;
};
static std::map<const Ddm*, std::unique_ptr<PrecondWork>> g_work;
static std::mutex g_work_mu;

static PrecondWork& work_for(const Ddm& d) {
  std::lock_guard<std::mutex> lk(g_work_mu);
  auto& w = g_work[&d];
  if (!w) w = std::make_unique<PrecondWork>();
  return *w;
}

void precond_release_workspace(Ddm& d) {
  std::lock_guard<std::mutex> lk(g_work_mu);
  g_work.erase(&d);
}

void precond_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* z) {
  PrecondWork& w = work_for(d);
  const int64_t n = d.op->mesh->n;
  const c128* rhs = v;
  const c128* add = nullptr;
  if (d.coarse) {
    const size_t need = (size_t)(n * s) * sizeof(c128);
    if (w.q.bytes < need) {
      w.q.release();
      w.t.release();
      w.q.alloc(ctx, need);
      w.t.alloc(ctx, need);
    }
    coarse_apply(ctx, d, s, v, w.q.as<c128>(), w.t.as<c128>());
    rhs = w.t.as<c128>();
    add = w.q.as<c128>();
  }
  if (d.precision == HZ_PREC_MIXED)
    one_level<float>(ctx, d, s, rhs, add, z, w.bloc, w.cbuf);
  else
    one_level<double>(ctx, d, s, rhs, add, z, w.bloc, w.cbuf);
}

}  // namespace hz
