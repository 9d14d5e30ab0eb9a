// Batched multifrontal LDL^T of all local ORAS operators (complex symmetric: A_i = L D L^T
// with a plain transpose, no conjugation), level by level over the elimination trees of
// every subdomain at once.  The paper factors each fine local matrix with a complete
// Cholesky-type direct solver (section "Numerical results", the local solver comparison);
// here the factorisation is a supernodal LDL^T on nested-dissection order with static
// pivoting (tiny pivots replaced by a threshold, counted).
//
// Per level: scatter the original entries into the fronts, extend-add the children's
// update blocks (one child slot per launch, so every sum has a fixed order), then for each
// panel of kNb pivot columns: factor the diagonal block, solve the panel rows below it,
// and apply the rank-kNb update to the trailing lower triangle (L region and Schur block) on
// the matrix cores.
// Finally each kNb x kNb diagonal block gets its inverse unit-lower factor stored
// transposed in its (otherwise unused) strict upper triangle, for the triangular solves.
#include <cmath>
#include <cstdlib>

#include "ddm.h"
#include "mfma_cplx.h"

namespace hz {

namespace {

constexpr int kNb = 32;     // panel width
constexpr int kTile = 64;   // trailing-update tile

template <typename T>
__device__ __forceinline__ cplx<T> ld_front(const cplx<T>* L, const cplx<T>* U, const FrontDesc& F, int64_t i,
                                            int64_t j) {
  return j < F.p ? L[F.L_off + j * F.ld + i] : U[F.U_off + (j - F.p) * F.r + (i - F.p)];
}
template <typename T>
__device__ __forceinline__ cplx<T>* at_front(cplx<T>* L, cplx<T>* U, const FrontDesc& F, int64_t i, int64_t j) {
  return j < F.p ? &L[F.L_off + j * F.ld + i] : &U[F.U_off + (j - F.p) * F.r + (i - F.p)];
}

template <typename T>
__global__ void k_scatter_orig(const int32_t* __restrict__ lf, int nf, const FrontDesc* __restrict__ fr,
                               const int64_t* __restrict__ osrc, const int64_t* __restrict__ odst,
                               const c128* __restrict__ lval, cplx<T>* __restrict__ L) {
  const FrontDesc F = fr[lf[blockIdx.x]];
  for (int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < F.orig_cnt; k += (int64_t)gridDim.y * blockDim.x) {
    const c128 v = lval[osrc[F.orig_off + k]];
    L[F.L_off + odst[F.orig_off + k]] = cmk((T)v.re, (T)v.im);
  }
}

// zero the update blocks of a level's fronts (the arena is shared over lifetimes)
template <typename T>
__global__ void k_zero_update(const int32_t* __restrict__ lf, const FrontDesc* __restrict__ fr, cplx<T>* __restrict__ U) {
  const FrontDesc F = fr[lf[blockIdx.x]];
  const int64_t tot = (int64_t)F.r * F.r;
  for (int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.y * blockDim.x)
    U[F.U_off + k] = cmk((T)0, (T)0);
}

// add child `slot`'s update block into its parent (the fronts in lf are parents)
template <typename T>
__global__ void k_extend_add(const int32_t* __restrict__ lf, int nf, const FrontDesc* __restrict__ fr, int slot,
                             const int32_t* __restrict__ emap, cplx<T>* __restrict__ L, cplx<T>* __restrict__ U) {
  const FrontDesc P = fr[lf[blockIdx.x]];
  const int c = slot == 0 ? P.child0 : P.child1;
  if (c < 0) return;
  const FrontDesc C = fr[c];
  const int64_t rc = C.r;
  const int64_t total = rc * rc;
  for (int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.y * blockDim.x) {
    const int64_t j = k / rc, i = k - j * rc;
    if (i < j) continue;
    const cplx<T> v = U[C.U_off + j * rc + i];
    const int64_t pi = emap[C.emap_off + i], pj = emap[C.emap_off + j];
    cplx<T>* dst = at_front(L, U, P, pi, pj);
    *dst = *dst + v;
  }
}

// unblocked LDL^T of the diagonal block [k0, k0+nb) of every active front (one block each)
template <typename T>
__global__ __launch_bounds__(256) void k_diag_block(const int32_t* __restrict__ lf, const FrontDesc* __restrict__ fr,
                                                    int k0, cplx<T>* __restrict__ L, const double* __restrict__ tau_sub,
                                                    const int32_t* __restrict__ front_sub,
                                                    unsigned long long* __restrict__ npiv) {
  __shared__ cplx<T> A[kNb][kNb + 1];
  const int fid = lf[blockIdx.x];
  const FrontDesc F = fr[fid];
  const int nb = min(kNb, F.p - k0);
  const int64_t ld = F.ld;
  cplx<T>* base = L + F.L_off + (int64_t)k0 * ld + k0;
  for (int t = threadIdx.x; t < kNb * kNb; t += blockDim.x) {
    const int j = t / kNb, i = t % kNb;
    A[i][j] = (i < nb && j < nb && i >= j) ? base[(int64_t)j * ld + i] : cmk((T)0, (T)0);
  }
  __syncthreads();
  const T tau = (T)tau_sub[front_sub[fid]];
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) {
      cplx<T> d = A[j][j];
      const T ad = sqrt(d.re * d.re + d.im * d.im);
      if (!(ad >= tau)) {
        d = ad > (T)0 ? cmk(d.re * (tau / ad), d.im * (tau / ad)) : cmk(tau, (T)0);
        atomicAdd(npiv, 1ull);
        A[j][j] = d;
      }
    }
    __syncthreads();
    const cplx<T> d = A[j][j];
    // a_ik -= a_ij a_kj / d for i >= k > j
    for (int t = threadIdx.x; t < kNb * kNb; t += blockDim.x) {
      const int k = t / kNb, i = t % kNb;
      if (k > j && i >= k && i < nb) {
        const cplx<T> lij = cdiv(A[i][j], d);
        cfms(A[i][k], lij, A[k][j]);
      }
    }
    __syncthreads();
    for (int i = j + 1 + (int)threadIdx.x; i < nb; i += blockDim.x) A[i][j] = cdiv(A[i][j], d);
    __syncthreads();
  }
  for (int t = threadIdx.x; t < kNb * kNb; t += blockDim.x) {
    const int j = t / kNb, i = t % kNb;
    if (i < nb && j < nb && i >= j) base[(int64_t)j * ld + i] = A[i][j];
  }
}

// rows below the diagonal block: L[i, panel] = F[i, panel] L_kk^{-T} D^{-1}
template <typename T>
__global__ __launch_bounds__(256) void k_panel_rows(const int32_t* __restrict__ lf, const FrontDesc* __restrict__ fr,
                                                    int k0, cplx<T>* __restrict__ L) {
  __shared__ cplx<T> Lkk[kNb][kNb + 1];
  const FrontDesc F = fr[lf[blockIdx.x]];
  const int nb = min(kNb, F.p - k0);
  const int64_t f = F.p + F.r;
  const int64_t r0 = k0 + nb;
  const int64_t rows = f - r0;
  const int64_t chunk = (int64_t)blockIdx.y * blockDim.x;
  if (chunk >= rows) return;
  const int64_t ld = F.ld;
  cplx<T>* col0 = L + F.L_off + (int64_t)k0 * ld;
  for (int t = threadIdx.x; t < kNb * kNb; t += blockDim.x) {
    const int j = t / kNb, i = t % kNb;
    Lkk[i][j] = (i < nb && j < nb && i >= j) ? col0[(int64_t)j * ld + k0 + i] : cmk((T)0, (T)0);
  }
  __syncthreads();
  for (int64_t i = r0 + chunk + threadIdx.x; i < f; i += (int64_t)gridDim.y * blockDim.x) {
    cplx<T> y[kNb];
#pragma unroll
    for (int j = 0; j < kNb; ++j) y[j] = j < nb ? col0[(int64_t)j * ld + i] : cmk((T)0, (T)0);
#pragma unroll
    for (int j = 0; j < kNb; ++j) {
#pragma unroll
      for (int l = 0; l < j; ++l) cfms(y[j], y[l], Lkk[j][l]);
    }
#pragma unroll
    for (int j = 0; j < kNb; ++j)
      if (j < nb) col0[(int64_t)j * ld + i] = cdiv(y[j], Lkk[j][j]);
  }
}

// trailing update: F[i][j] -= sum_l L[i][l] d_l L[j][l] for i >= j >= k0 + nb, one lower 64 x 64
// tile of the trailing region per block, on the matrix cores (CAcc: the three-product form,
// complex64 on v_mfma_f32_16x16x4f32, complex128 on v_mfma_f64_16x16x4f64).  The panel's rows
// of the tile (As) and its d-scaled rows of the tile's columns (Bs) are staged in LDS; each
// wavefront forms one 32 x 32 quarter of the tile as 2 x 2 matrix-core tiles over the panel's
// nb <= 32 columns (entries past nb are zero).
template <typename T>
__global__ __launch_bounds__(256) void k_trailing(const int32_t* __restrict__ lf, const FrontDesc* __restrict__ fr,
                                                  int k0, cplx<T>* __restrict__ L, cplx<T>* __restrict__ U) {
  __shared__ cplx<T> As[kNb][kTile + 1];  // As[l][r] = L[i0 + r][k0 + l]
  __shared__ cplx<T> Bs[kNb][kTile + 1];  // Bs[l][r] = d_l L[j0 + r][k0 + l]
  const FrontDesc F = fr[lf[blockIdx.x]];
  const int nb = min(kNb, F.p - k0);
  const int64_t f = F.p + F.r;
  const int64_t c0 = k0 + nb;
  const int64_t nrem = f - c0;
  if (nrem <= 0) return;
  const int64_t nt = (nrem + kTile - 1) / kTile;
  const int64_t tid = blockIdx.y;
  if (tid >= nt * (nt + 1) / 2) return;
  // triangular tile index -> (ti, tj), ti >= tj
  int64_t ti = (int64_t)((sqrt(8.0 * (double)tid + 1.0) - 1.0) / 2.0);
  while (ti * (ti + 1) / 2 > tid) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= tid) ++ti;
  const int64_t tj = tid - ti * (ti + 1) / 2;
  const int64_t i0 = c0 + ti * kTile, j0 = c0 + tj * kTile;
  const int64_t ld = F.ld;
  const cplx<T>* pan = L + F.L_off + (int64_t)k0 * ld;
  const cplx<T>* dg = pan + k0;  // diagonal entries at pan[l*ld + k0 + l]
  for (int t = threadIdx.x; t < kNb * kTile; t += blockDim.x) {
    const int l = t / kTile, r = t % kTile;
    cplx<T> a = cmk((T)0, (T)0), b = cmk((T)0, (T)0);
    if (l < nb) {
      if (i0 + r < f) a = pan[(int64_t)l * ld + i0 + r];
      if (j0 + r < f) b = pan[(int64_t)l * ld + j0 + r] * dg[(int64_t)l * ld + l];
    }
    As[l][r] = a;
    Bs[l][r] = b;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, lr = ln & 15, lq = ln >> 4;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;  // this wavefront's quarter of the tile
  CAcc<T> acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 2; ++g) acc[m][g].zero();
#pragma unroll 2
  for (int k = 0; k < kNb; k += 4) {
    const int kk = k + lq;
    cplx<T> a[2], b[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) a[m] = As[kk][wr + 16 * m + lr];  // A[i][k]
#pragma unroll
    for (int g = 0; g < 2; ++g) b[g] = Bs[kk][wc + 16 * g + lr];  // B[k][j]
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int g = 0; g < 2; ++g) acc[m][g].mac(a[m], b[g]);
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int64_t j = j0 + wc + 16 * g + lr;
      if (j >= f) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wr + 16 * m + CAcc<T>::row(lq, v);
        if (i >= f || i < j) continue;
        cplx<T>* dst = at_front(L, U, F, i, j);
        *dst = *dst - acc[m][g].get(v);
      }
    }
}

// ---- partitioned inverse: [L11; L21] -> [L11^{-1}; L21 L11^{-1}] (unit diagonal kept)
//
// With F = [L11^{-1}; L21 L11^{-1}] the multifrontal solves need no sequential
// substitution: forward  [y; c] = [F_top w_p; w_r - F_bot w_p]
//              backward x_p = F^T [z_p / d; -x_r].
// Column blocks are transformed from the right: with K the already transformed columns
// right of block J and L_JJ the unit-lower diagonal block,
//   M[:, J] = ([E_J; L21[:, J]] - M[:, K] L11[K, J]) L_JJ^{-1}.
// Each front's pivots D are first moved to a compact inverse-pivot array.

template <typename T>
__global__ void k_extract_dinv(int nf, const FrontDesc* __restrict__ fr, cplx<T>* __restrict__ L,
                               cplx<T>* __restrict__ dinv) {
  const FrontDesc F = fr[blockIdx.x];
  for (int j = threadIdx.x; j < F.p; j += blockDim.x) {
    cplx<T>* dg = L + F.L_off + (int64_t)j * F.ld + j;
    dinv[F.vec_off + F.pos0 + j] = cdiv(cmk((T)1, (T)0), *dg);
  }
}

// copy L11[j0:p, J] of every active front into a compact panel buffer (ld = p - j0)
template <typename T>
__global__ void k_inv_copy(const int32_t* __restrict__ act, const FrontDesc* __restrict__ fr,
                           const int64_t* __restrict__ poff, int t, cplx<T>* __restrict__ L, cplx<T>* __restrict__ P) {
  const int fid = act[blockIdx.x];
  const FrontDesc F = fr[fid];
  const int nblk = (F.p + kNb - 1) / kNb;
  const int J = nblk - 1 - t;
  const int j0 = J * kNb;
  const int nbJ = min(kNb, F.p - j0);
  const int64_t rows = F.p - j0;
  cplx<T>* dst = P + poff[blockIdx.x];
  for (int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < rows * nbJ; k += (int64_t)gridDim.y * blockDim.x) {
    const int64_t jj = k / rows, r = k - jj * rows;
    dst[jj * rows + r] = L[F.L_off + (int64_t)(j0 + jj) * F.ld + j0 + r];
  }
}

// one block per (active front, 64-row tile of rows >= j0): new column block J
template <typename T>
__global__ __launch_bounds__(256) void k_inv_block(const int32_t* __restrict__ act, const FrontDesc* __restrict__ fr,
                                                   const int64_t* __restrict__ poff, int t,
                                                   cplx<T>* __restrict__ L, const cplx<T>* __restrict__ P) {
  constexpr int RT = 64, KC = 32;
  __shared__ cplx<T> Lt[KC][kNb + 1];     // L11[k, J] chunk
  __shared__ cplx<T> Mt[KC][RT + 1];      // M[rows, k] chunk
  __shared__ cplx<T> Rr[RT][kNb + 1];     // result rows
  __shared__ cplx<T> Ljj[kNb][kNb + 1];
  const int fid = act[blockIdx.x];
  const FrontDesc F = fr[fid];
  const int nblk = (F.p + kNb - 1) / kNb;
  const int J = nblk - 1 - t;
  const int j0 = J * kNb;
  const int nbJ = min(kNb, F.p - j0);
  const int64_t f = F.p + F.r;
  const int64_t i0 = j0 + (int64_t)blockIdx.y * RT;
  if (i0 >= f) return;
  const int64_t prow = F.p - j0;  // ld of the panel copy
  const cplx<T>* Pp = P + poff[blockIdx.x];
  cplx<T>* Lf = L + F.L_off;
  for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
    const int a = e / kNb, b = e % kNb;  // Ljj[a][b] = L11[j0 + a][j0 + b]
    Ljj[a][b] = (a < nbJ && b < nbJ) ? Pp[(int64_t)b * prow + a] : cmk((T)0, (T)0);
  }
  const int r = threadIdx.x & 63;
  const int64_t i = i0 + r;
  // GEMM over the transformed columns K = [j0 + nbJ, kend) on the matrix cores: wavefront wv
  // forms rows [16 wv, 16 wv + 16) of the tile, both 16-column halves of the block
  const int wv = threadIdx.x >> 6, lr = threadIdx.x & 15, lq = (threadIdx.x >> 4) & 3;
  CAcc<T> acc[2];
  acc[0].zero();
  acc[1].zero();
  const int64_t k1 = j0 + nbJ;
  const int64_t kend = i0 < F.p ? min<int64_t>(F.p, i0 + RT) : F.p;
  for (int64_t kc = k1; kc < kend; kc += KC) {
    const int kn = (int)min<int64_t>(KC, kend - kc);
    __syncthreads();
    for (int e = threadIdx.x; e < KC * kNb; e += 256) {
      const int k = e / kNb, jj = e % kNb;
      Lt[k][jj] = (k < kn && jj < nbJ) ? Pp[(int64_t)jj * prow + (kc + k - j0)] : cmk((T)0, (T)0);
    }
    for (int e = threadIdx.x; e < KC * RT; e += 256) {
      const int k = e / RT, rr = e % RT;
      Mt[k][rr] = (k < kn && i0 + rr < f) ? Lf[(kc + k) * F.ld + i0 + rr] : cmk((T)0, (T)0);
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < KC; k += 4) {  // entries past kn are zero
      const cplx<T> a = Mt[k + lq][16 * wv + lr];  // A[i][k]
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h].mac(a, Lt[k + lq][16 * h + lr]);  // B[k][j]
    }
  }
  // R = base - acc ; base = e_J on the top block, L21[i, J] below
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v) Rr[16 * wv + CAcc<T>::row(lq, v)][16 * h + lr] = acc[h].get(v);
  __syncthreads();
  for (int jj = 0; jj < nbJ; ++jj) {
    if (threadIdx.x >= RT) break;
    cplx<T> base = cmk((T)0, (T)0);
    if (i < f) {
      if (i < F.p)
        base = cmk((T)(i == j0 + jj ? 1 : 0), (T)0);
      else
        base = Lf[(int64_t)(j0 + jj) * F.ld + i];
    }
    Rr[r][jj] = base - Rr[r][jj];
  }
  __syncthreads();
  // x L_JJ = R  (unit lower L_JJ):  x_jj = R_jj - sum_{l > jj} x_l L_JJ[l][jj]
  if (threadIdx.x < RT && i < f) {
    for (int jj = nbJ - 1; jj >= 0; --jj) {
      cplx<T> x = Rr[r][jj];
      for (int l = jj + 1; l < nbJ; ++l) cfms(x, Rr[r][l], Ljj[l][jj]);
      Rr[r][jj] = x;
    }
    for (int jj = 0; jj < nbJ; ++jj) Lf[(int64_t)(j0 + jj) * F.ld + i] = Rr[r][jj];
  }
}

// max |a_ij| of each subdomain's local operator (deterministic: one block per subdomain)
__global__ void k_sub_norm(const int64_t* __restrict__ csr_off, const c128* __restrict__ lval, double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t a = csr_off[blockIdx.x], b = csr_off[blockIdx.x + 1];
  double m = 0;
  for (int64_t k = a + threadIdx.x; k < b; k += blockDim.x) {
    const c128 v = lval[k];
    m = fmax(m, sqrt(v.re * v.re + v.im * v.im));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_scale(double* x, int n, double s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= s;
}

template <typename T>
void factor_typed(Ctx* ctx, Ddm& d) {
  hipStream_t st = ctx->stream;
  try {
    d.d_factor.alloc(ctx, std::max<int64_t>(1, d.factor_entries) * sizeof(cplx<T>));
  } catch (const Error& e) {
    fail(e.code, std::string("factor array (") + std::to_string(d.factor_entries) + " entries): " + e.what());
  }
  try {
    d.d_update.alloc(ctx, std::max<int64_t>(1, d.update_entries) * sizeof(cplx<T>));
  } catch (const Error& e) {
    fail(e.code, std::string("update arena (") + std::to_string(d.update_entries) + " entries): " + e.what());
  }
  HIP_CHECK(hipMemsetAsync(d.d_factor.p, 0, d.d_factor.bytes, st));
  cplx<T>* L = d.d_factor.as<cplx<T>>();
  cplx<T>* U = d.d_update.as<cplx<T>>();
  // static pivot threshold per subdomain
  const char* e = std::getenv("HZ_PIVOT_EPS");
  const double eps = e ? std::atof(e) : (sizeof(T) == 8 ? 1e-12 : 1e-6);
  DevArray<int64_t> d_csroff;
  DevArray<double> d_tau;
  DevArray<int32_t> d_fsub;
  {
    std::vector<int64_t> co;
    for (auto& S : d.subs) co.push_back(S.csr_off);
    co.push_back(d.subs.back().csr_off + (int64_t)d.subs.back().col.size());
    d_csroff.upload(ctx, co);
    d_tau.alloc(ctx, d.n_sub);
    hipLaunchKernelGGL(k_sub_norm, dim3(d.n_sub), dim3(256), 0, st, d_csroff.ptr(), d.d_lval.ptr(), d_tau.ptr());
    hipLaunchKernelGGL(k_scale, dim3((d.n_sub + 255) / 256), dim3(256), 0, st, d_tau.ptr(), d.n_sub, eps);
    std::vector<int32_t> fs(d.fronts.size());
    for (size_t i = 0; i < d.fronts.size(); ++i) fs[i] = d.fronts[i].sub;
    d_fsub.upload(ctx, fs);
  }
  d.d_npiv.alloc(ctx, 1);
  HIP_CHECK(hipMemsetAsync(d.d_npiv.ptr(), 0, sizeof(unsigned long long), st));
  const FrontDesc* fr = d.d_fronts.ptr();
  const size_t nlev = d.levels.size();
  const size_t ngroups = d.fgroup_off.size() - 1;
  for (size_t gl = 0; gl < ngroups * nlev; ++gl) {
    const size_t lv = gl % nlev;
    const int nf = (int)(d.flf_off[gl + 1] - d.flf_off[gl]);
    if (nf == 0) continue;
    const int32_t* lfh = d.flf.data() + d.flf_off[gl];  // host copy: p descending
    const int32_t* lf = d.d_flf.ptr() + d.flf_off[gl];
    int64_t max_orig = 1, max_child_u = 1, lv_max_r = 0, lv_max_p = 0;
    for (int k = 0; k < nf; ++k) {
      const int32_t fi = lfh[k];
      lv_max_r = std::max(lv_max_r, d.fronts[fi].r);
      lv_max_p = std::max(lv_max_p, d.fronts[fi].p);
      max_orig = std::max(max_orig, d.fronts[fi].orig_cnt);
      for (int k = 0; k < d.fronts[fi].nchild; ++k)
        max_child_u = std::max(max_child_u, d.fronts[d.fronts[fi].child[k]].r * d.fronts[d.fronts[fi].child[k]].r);
    }
    const unsigned gy_o = (unsigned)std::min<int64_t>((max_orig + 255) / 256, 1024);
    if (lv_max_r > 0) {
      const unsigned gy_z = (unsigned)std::min<int64_t>((lv_max_r * lv_max_r + 255) / 256, 4096);
      hipLaunchKernelGGL(k_zero_update<T>, dim3(nf, gy_z), dim3(256), 0, st, lf, fr, U);
    }
    hipLaunchKernelGGL(k_scatter_orig<T>, dim3(nf, gy_o), dim3(256), 0, st, lf, nf, fr, d.d_orig_src.ptr(),
                       d.d_orig_dst.ptr(), d.d_lval.ptr(), L);
    HIP_CHECK(hipGetLastError());
    if (lv > 0) {
      const unsigned gy_e = (unsigned)std::min<int64_t>((max_child_u + 255) / 256, 4096);
      for (int slot = 0; slot < 2; ++slot) {
        hipLaunchKernelGGL(k_extend_add<T>, dim3(nf, gy_e), dim3(256), 0, st, lf, nf, fr, slot, d.d_emap.ptr(), L, U);
        HIP_CHECK(hipGetLastError());
      }
    }
    for (int64_t k0 = 0; k0 < lv_max_p; k0 += kNb) {
      int cnt = 0;  // fronts sorted by p descending: active prefix
      int64_t max_f = 0;
      while (cnt < nf && d.fronts[lfh[cnt]].p > k0) {
        max_f = std::max(max_f, d.fronts[lfh[cnt]].f());
        ++cnt;
      }
      hipLaunchKernelGGL(k_diag_block<T>, dim3(cnt), dim3(256), 0, st, lf, fr, (int)k0, L, d_tau.ptr(), d_fsub.ptr(),
                         d.d_npiv.ptr());
      HIP_CHECK(hipGetLastError());
      const int64_t rows = max_f - k0;
      const unsigned gy_r = (unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + 255) / 256, 64));
      hipLaunchKernelGGL(k_panel_rows<T>, dim3(cnt, gy_r), dim3(256), 0, st, lf, fr, (int)k0, L);
      HIP_CHECK(hipGetLastError());
      const int64_t nrem = max_f - k0 - 1;
      const int64_t nt = std::max<int64_t>(1, (nrem + kTile - 1) / kTile);
      const int64_t tiles = nt * (nt + 1) / 2;
      HZ_REQUIRE(tiles < 65536, HZ_ERR_STATE, "factor: front too large for the tile grid");
      hipLaunchKernelGGL(k_trailing<T>, dim3(cnt, (unsigned)tiles), dim3(256), 0, st, lf, fr, (int)k0, L, U);
      HIP_CHECK(hipGetLastError());
    }
  }
  // the update workspace is only needed during the factorisation
  d.d_update.release();
  // partitioned inverse of every front, all fronts at once, column blocks from the right
  {
    const int nfr = (int)d.fronts.size();
    d.d_dinv.alloc(ctx, (size_t)std::max<int64_t>(1, d.n_local_total) * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_extract_dinv<T>, dim3(nfr), dim3(256), 0, st, nfr, fr, L, d.d_dinv.as<cplx<T>>());
    HIP_CHECK(hipGetLastError());
    std::vector<int32_t> order(nfr);
    for (int i = 0; i < nfr; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d.fronts[a].p > d.fronts[b].p; });
    // panel copies: front fi needs (p - j0) * nbJ <= p * kNb entries
    std::vector<int64_t> poff(nfr);
    int64_t tot = 0;
    for (int k = 0; k < nfr; ++k) {
      poff[k] = tot;
      tot += d.fronts[order[k]].p * kNb;
    }
    DevArray<int32_t> d_act;
    DevArray<int64_t> d_poff;
    d_act.upload(ctx, order);
    d_poff.upload(ctx, poff);
    DevBuf panel;
    panel.alloc(ctx, (size_t)std::max<int64_t>(1, tot) * sizeof(cplx<T>));
    const int64_t maxp = d.fronts[order[0]].p;
    const int tmax = (int)((maxp + kNb - 1) / kNb);
    for (int t = 0; t < tmax; ++t) {
      int cnt = 0;
      int64_t maxrows = 0;
      while (cnt < nfr && (d.fronts[order[cnt]].p + kNb - 1) / kNb > t) {
        const Front& Fr = d.fronts[order[cnt]];
        const int64_t j0 = ((Fr.p + kNb - 1) / kNb - 1 - t) * kNb;
        maxrows = std::max(maxrows, Fr.f() - j0);
        ++cnt;
      }
      hipLaunchKernelGGL(k_inv_copy<T>, dim3(cnt, 8), dim3(256), 0, st, d_act.ptr(), fr, d_poff.ptr(), t, L,
                         panel.as<cplx<T>>());
      const unsigned gy = (unsigned)((maxrows + 63) / 64);
      hipLaunchKernelGGL(k_inv_block<T>, dim3(cnt, gy), dim3(256), 0, st, d_act.ptr(), fr, d_poff.ptr(), t, L,
                         panel.as<cplx<T>>());
      HIP_CHECK(hipGetLastError());
    }
    HIP_CHECK(hipStreamSynchronize(st));
  }
  {
    unsigned long long np = 0;
    HIP_CHECK(hipMemcpyAsync(&np, d.d_npiv.ptr(), sizeof(np), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    d.static_pivots = (int64_t)np;
  }
}

}  // namespace

void factor_all(Ctx* ctx, Ddm& d) {
  if (d.precision == HZ_PREC_MIXED)
    factor_typed<float>(ctx, d);
  else
    factor_typed<double>(ctx, d);
}

}  // namespace hz
