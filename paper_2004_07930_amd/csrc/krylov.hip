// Block FGMRES(m) in FP64 on the GPU: classical Gram-Schmidt twice (CGS2) as tall-skinny
// products, CholQR2 block normalisation, Householder QR of the block Hessenberg matrix and
// the least-squares update in one workgroup.
//
// The paper solves A u = b with GMRES preconditioned by the two-level ORAS operator and
// stops on ||A u - b|| / ||b|| <= eps (sections "Tetrahedral finite element method" and
// "Domain decomposition preconditioner").  The flexible variant is used because the
// preconditioner may run in single precision; x0 = 0; all columns of a block share one
// Arnoldi process; convergence is confirmed on the explicit FP64 residual.
//
// Vectors are node-major blocks [n][s] (s contiguous per dof).  Every reduction goes
// through per-chunk partial sums reduced in a fixed order, so results are reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ddm.h"
#include "krylov.h"

namespace hz {

namespace {

constexpr int kChunkRows = 4096;  // rows per partial-sum chunk
constexpr int kJT = 64;           // basis columns per gram tile

__global__ void k_to_node(int64_t n, int s, const c128* __restrict__ src, c128* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t i = k / s;
  const int c = (int)(k - i * s);
  dst[k] = src[(int64_t)c * n + i];
}
__global__ void k_from_node(int64_t n, int s, const c128* __restrict__ src, c128* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int c = (int)(k / n);
  const int64_t i = k - (int64_t)c * n;
  dst[k] = src[i * s + c];
}

// partials[chunk][J][c] = sum_{rows in chunk} conj(V_J[row]) W[row][c],
// V_J = column (J mod s) of block (J / s), blocks spaced by ldv elements.
template <int S>
__global__ __launch_bounds__(256) void k_gram(int64_t n, int s, int Jtot, const c128* __restrict__ V, int64_t ldv,
                                              const c128* __restrict__ W, c128* __restrict__ part) {
  constexpr int R = 16;  // rows staged per step
  __shared__ c128 Vt[R][kJT];
  __shared__ c128 Wt[R][S];
  const int64_t r0 = (int64_t)blockIdx.x * kChunkRows;
  const int64_t r1 = min<int64_t>(n, r0 + kChunkRows);
  const int J0 = blockIdx.y * kJT;
  const int jj = threadIdx.x & 63;
  const int cg = threadIdx.x >> 6;  // 4 column groups
  constexpr int NC = (S + 3) / 4;
  c128 acc[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) acc[a] = cmk(0.0, 0.0);
  for (int64_t rb = r0; rb < r1; rb += R) {
    __syncthreads();
    for (int t = threadIdx.x; t < R * kJT; t += 256) {
      const int r = t / kJT, j = t - (t / kJT) * kJT;
      const int64_t row = rb + r;
      const int J = J0 + j;
      c128 v = cmk(0.0, 0.0);
      if (row < r1 && J < Jtot) {
        const int b = J / s, jc = J - (J / s) * s;
        v = V[(int64_t)b * ldv + row * s + jc];
      }
      Vt[r][j] = v;
    }
    for (int t = threadIdx.x; t < R * S; t += 256) {
      const int r = t / S, c = t - (t / S) * S;
      const int64_t row = rb + r;
      Wt[r][c] = (row < r1 && c < s) ? W[row * s + c] : cmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
      const c128 v = Vt[r][jj];
#pragma unroll
      for (int a = 0; a < NC; ++a) cfma_conj(acc[a], v, Wt[r][cg + 4 * a]);
    }
  }
  const int J = J0 + jj;
  if (J < Jtot)
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const int c = cg + 4 * a;
      if (c < s) part[((int64_t)blockIdx.x * Jtot + J) * s + c] = acc[a];
    }
}

__global__ void k_reduce_part(int nchunk, int64_t m, const c128* __restrict__ part, c128* __restrict__ out, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  c128 s = cmk(0.0, 0.0);
  for (int k = 0; k < nchunk; ++k) s = s + part[(int64_t)k * m + e];
  out[e] = accumulate ? out[e] + s : s;
}

// Y[row][c] = Yin[row][c] + beta * sum_J V_J[row] H[J][c]
template <int S>
__global__ __launch_bounds__(256) void k_block_axpy(int64_t n, int s, int Jtot, const c128* __restrict__ V, int64_t ldv,
                                                    const c128* __restrict__ H, double beta,
                                                    const c128* __restrict__ Yin, c128* __restrict__ Y) {
  constexpr int RPB = 256 / S;  // rows per block
  __shared__ c128 Ht[kJT][S];
  const int c = threadIdx.x % S;
  const int64_t row = (int64_t)blockIdx.x * RPB + threadIdx.x / S;
  c128 acc = cmk(0.0, 0.0);
  for (int J0 = 0; J0 < Jtot; J0 += kJT) {
    __syncthreads();
    for (int t = threadIdx.x; t < kJT * S; t += 256) {
      const int j = t / S, cc = t - (t / S) * S;
      Ht[j][cc] = (J0 + j < Jtot && cc < s) ? H[(int64_t)(J0 + j) * s + cc] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (row < n && c < s) {
      const int jn = min(kJT, Jtot - J0);
      for (int j = 0; j < jn; ++j) {
        const int J = J0 + j;
        const int b = J / s, jc = J - (J / s) * s;
        cfma(acc, V[(int64_t)b * ldv + row * s + jc], Ht[j][c]);
      }
    }
  }
  if (row < n && c < s) {
    const int64_t k = row * s + c;
    Y[k] = (Yin ? Yin[k] : cmk(0.0, 0.0)) + cmk(beta * acc.re, beta * acc.im);
  }
}

// out[row][c] = sum_k W[row][k] M[k][c]  (M s x s upper triangular, row-major)
__global__ void k_right_mult(int64_t n, int s, const c128* __restrict__ W, const c128* __restrict__ M,
                             c128* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t row = k / s;
  const int c = (int)(k - row * s);
  c128 acc = cmk(0.0, 0.0);
  for (int l = 0; l <= c; ++l) cfma(acc, W[row * s + l], M[l * s + c]);
  out[k] = acc;
}

// Cholesky G = R^H R (upper R, real positive diagonal), Rinv = R^{-1}; Racc = R * Racc.
// flag[0] = 1 on breakdown (non-positive pivot).
__global__ void k_chol_small(int s, const c128* __restrict__ G, c128* __restrict__ R, c128* __restrict__ Rinv,
                             c128* __restrict__ Racc, int* __restrict__ flag) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < s * s; ++i) R[i] = cmk(0.0, 0.0);
  for (int k = 0; k < s; ++k) {
    double d = G[k * s + k].re;
    for (int l = 0; l < k; ++l) d -= R[l * s + k].re * R[l * s + k].re + R[l * s + k].im * R[l * s + k].im;
    const double scale = fabs(G[k * s + k].re) + 1e-300;
    if (!(d > 1e-28 * scale) || !isfinite(d)) {
      flag[0] = 1;
      d = fmax(d, 1e-28 * scale);
    }
    const double rk = sqrt(d);
    R[k * s + k] = cmk(rk, 0.0);
    for (int j = k + 1; j < s; ++j) {
      c128 v = G[k * s + j];
      for (int l = 0; l < k; ++l) {
        // v -= conj(R[l][k]) R[l][j]
        const c128 a = R[l * s + k], b = R[l * s + j];
        v.re -= a.re * b.re + a.im * b.im;
        v.im -= a.re * b.im - a.im * b.re;
      }
      R[k * s + j] = cmk(v.re / rk, v.im / rk);
    }
  }
  for (int i = 0; i < s * s; ++i) Rinv[i] = cmk(0.0, 0.0);
  for (int c = 0; c < s; ++c) {
    // solve R x = e_c (upper): back substitution
    for (int i = c; i >= 0; --i) {
      c128 v = cmk(i == c ? 1.0 : 0.0, 0.0);
      for (int l = i + 1; l <= c; ++l) cfms(v, R[i * s + l], Rinv[l * s + c]);
      Rinv[i * s + c] = cmk(v.re / R[i * s + i].re, v.im / R[i * s + i].re);
    }
  }
  if (Racc) {
    // Racc <- R * Racc (both upper)
    c128 tmp[32 * 32];
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        c128 v = cmk(0.0, 0.0);
        for (int l = i; l <= j; ++l) cfma(v, R[i * s + l], Racc[l * s + j]);
        tmp[i * s + j] = v;
      }
    for (int i = 0; i < s * s; ++i) Racc[i] = tmp[i];
  }
}

__global__ void k_set_identity(int s, c128* M) {
  for (int i = threadIdx.x; i < s * s; i += blockDim.x) M[i] = cmk((i / s) == (i % s) ? 1.0 : 0.0, 0.0);
}

// ---------------------------------------------------------------- least squares (one block)
// State: Hc (rows x s, row-major, the new block column), Rm (column-major, ld = ldr),
// refl[step][2s][s] reflector vectors (v[0] = 1) and tau[step][s], G (ldg x s row-major).
__global__ __launch_bounds__(256) void k_lsq_step(int s, int jj, c128* __restrict__ Hc, c128* __restrict__ Rm,
                                                  int64_t ldr, c128* __restrict__ refl, c128* __restrict__ tau,
                                                  c128* __restrict__ G, double* __restrict__ res) {
  const int c = threadIdx.x;
  const int s2 = 2 * s;
  __shared__ c128 beta_tau[2];
  // 1. previous reflectors, in order
  for (int i = 0; i < jj; ++i) {
    const c128* Vi = refl + (int64_t)i * s2 * s;
    const c128* ti = tau + (int64_t)i * s;
    for (int k = 0; k < s; ++k) {
      if (c < s) {
        c128 w = cmk(0.0, 0.0);
        for (int r = k; r < s2; ++r) cfma_conj(w, Vi[r * s + k], Hc[(int64_t)(i * s + r) * s + c]);
        const c128 ct = conj(ti[k]) * w;
        for (int r = k; r < s2; ++r) cfms(Hc[(int64_t)(i * s + r) * s + c], Vi[r * s + k], ct);
      }
    }
  }
  __syncthreads();
  // 2. new reflectors on rows [jj s, jj s + 2s)
  c128* Vn = refl + (int64_t)jj * s2 * s;
  c128* tn = tau + (int64_t)jj * s;
  const int64_t base = (int64_t)jj * s;
  for (int k = 0; k < s; ++k) {
    if (c == 0) {
      const c128 alpha = Hc[(base + k) * s + k];
      double xn = 0;
      for (int r = k + 1; r < s2; ++r) {
        const c128 x = Hc[(base + r) * s + k];
        xn += x.re * x.re + x.im * x.im;
      }
      c128 t = cmk(0.0, 0.0), beta = alpha;
      for (int r = 0; r < s2; ++r) Vn[r * s + k] = cmk(0.0, 0.0);
      Vn[k * s + k] = cmk(1.0, 0.0);
      if (xn > 0 || alpha.im != 0) {
        const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn);
        const double b = alpha.re >= 0 ? -nrm : nrm;
        t = cmk((b - alpha.re) / b, -alpha.im / b);
        const c128 sc = cdiv(cmk(1.0, 0.0), cmk(alpha.re - b, alpha.im));
        for (int r = k + 1; r < s2; ++r) Vn[r * s + k] = Hc[(base + r) * s + k] * sc;
        beta = cmk(b, 0.0);
      }
      tn[k] = t;
      Hc[(base + k) * s + k] = beta;
      for (int r = k + 1; r < s2; ++r) Hc[(base + r) * s + k] = cmk(0.0, 0.0);
    }
    __syncthreads();
    if (c > k && c < s) {
      c128 w = cmk(0.0, 0.0);
      for (int r = k; r < s2; ++r) cfma_conj(w, Vn[r * s + k], Hc[(base + r) * s + c]);
      const c128 ct = conj(tn[k]) * w;
      for (int r = k; r < s2; ++r) cfms(Hc[(base + r) * s + c], Vn[r * s + k], ct);
    }
    __syncthreads();
  }
  // 3. R column block jj: rows 0 .. (jj+1)s-1
  const int64_t rows = (int64_t)(jj + 1) * s;
  for (int64_t t = threadIdx.x; t < rows * s; t += blockDim.x) {
    const int64_t r = t / s;
    const int cc = (int)(t - r * s);
    Rm[(base + cc) * ldr + r] = Hc[r * s + cc];
  }
  // 4. apply the new reflectors to G rows [jj s, jj s + 2s)
  for (int k = 0; k < s; ++k) {
    if (c < s) {
      c128 w = cmk(0.0, 0.0);
      for (int r = k; r < s2; ++r) cfma_conj(w, Vn[r * s + k], G[(base + r) * s + c]);
      const c128 ct = conj(tn[k]) * w;
      for (int r = k; r < s2; ++r) cfms(G[(base + r) * s + c], Vn[r * s + k], ct);
    }
  }
  __syncthreads();
  if (c < s) {
    double q = 0;
    for (int r = 0; r < s; ++r) {
      const c128 g = G[(base + s + r) * s + c];
      q += g.re * g.re + g.im * g.im;
    }
    res[c] = sqrt(q);
  }
  (void)beta_tau;
}

// Y = Rm[0:J, 0:J]^{-1} G[0:J]  (back substitution, one thread per column)
__global__ void k_lsq_solve(int s, int J, const c128* __restrict__ Rm, int64_t ldr, const c128* __restrict__ G,
                            c128* __restrict__ Y) {
  const int c = threadIdx.x;
  if (c >= s) return;
  for (int i = J - 1; i >= 0; --i) {
    c128 v = G[(int64_t)i * s + c];
    for (int l = i + 1; l < J; ++l) cfms(v, Rm[(int64_t)l * ldr + i], Y[(int64_t)l * s + c]);
    Y[(int64_t)i * s + c] = cdiv(v, Rm[(int64_t)i * ldr + i]);
  }
}

// squared column norms, partial sums per chunk
__global__ void k_colnorm_part(int64_t n, int s, const c128* __restrict__ X, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t r0 = (int64_t)blockIdx.x * kChunkRows;
  const int64_t r1 = min<int64_t>(n, r0 + kChunkRows);
  for (int c = 0; c < s; ++c) {
    double q = 0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const c128 v = X[r * s + c];
      q += v.re * v.re + v.im * v.im;
    }
    red[threadIdx.x] = q;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
      if (threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * s + c] = red[0];
    __syncthreads();
  }
}
__global__ void k_colnorm_reduce(int nchunk, int s, const double* __restrict__ part, double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= s) return;
  double q = 0;
  for (int k = 0; k < nchunk; ++k) q += part[(int64_t)k * s + c];
  out[c] = sqrt(q);
}

}  // namespace

// ---------------------------------------------------------------- host helpers

KrylovKernels::KrylovKernels(Ctx* c, int64_t n_, int s_) : ctx(c), n(n_), s(s_) {
  nchunk = (int)((n + kChunkRows - 1) / kChunkRows);
}

void KrylovKernels::to_node(const c128* src, c128* dst) {
  hipLaunchKernelGGL(k_to_node, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, src, dst);
}
void KrylovKernels::from_node(const c128* src, c128* dst) {
  hipLaunchKernelGGL(k_from_node, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, src, dst);
}

template <int S>
static void gram_t(KrylovKernels& k, int Jtot, const c128* V, int64_t ldv, const c128* W, c128* part) {
  hipLaunchKernelGGL(k_gram<S>, dim3((unsigned)k.nchunk, (unsigned)((Jtot + kJT - 1) / kJT)), dim3(256), 0,
                     k.ctx->stream, k.n, k.s, Jtot, V, ldv, W, part);
}

void KrylovKernels::gram(int nblk, const c128* V, int64_t ldv, const c128* W, c128* part, c128* H, bool accumulate,
                         c128* H2) {
  const int Jtot = nblk * s;
  if (s <= 4)
    gram_t<4>(*this, Jtot, V, ldv, W, part);
  else if (s <= 8)
    gram_t<8>(*this, Jtot, V, ldv, W, part);
  else if (s <= 16)
    gram_t<16>(*this, Jtot, V, ldv, W, part);
  else
    gram_t<32>(*this, Jtot, V, ldv, W, part);
  const int64_t m = (int64_t)Jtot * s;
  hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, ctx->stream, nchunk, m, part, H,
                     accumulate ? 1 : 0);
  if (H2)
    hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, ctx->stream, nchunk, m, part, H2, 1);
  HIP_CHECK(hipGetLastError());
}

template <int S>
static void axpy_t(KrylovKernels& k, int Jtot, const c128* V, int64_t ldv, const c128* H, double beta, const c128* Yin,
                   c128* Y) {
  constexpr int RPB = 256 / S;
  hipLaunchKernelGGL(k_block_axpy<S>, dim3((unsigned)((k.n + RPB - 1) / RPB)), dim3(256), 0, k.ctx->stream, k.n, k.s,
                     Jtot, V, ldv, H, beta, Yin, Y);
}

void KrylovKernels::block_axpy(int nblk, const c128* V, int64_t ldv, const c128* H, double beta, const c128* Yin,
                               c128* Y) {
  const int Jtot = nblk * s;
  if (s == 1)
    axpy_t<1>(*this, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s == 2)
    axpy_t<2>(*this, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s <= 4)
    axpy_t<4>(*this, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s <= 8)
    axpy_t<8>(*this, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s <= 16)
    axpy_t<16>(*this, Jtot, V, ldv, H, beta, Yin, Y);
  else
    axpy_t<32>(*this, Jtot, V, ldv, H, beta, Yin, Y);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::cholqr_pass(const c128* W, c128* out, c128* part, c128* G, c128* R, c128* Rinv, c128* Racc,
                                int* flag) {
  gram(1, W, n * s, W, part, G, false);
  hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, ctx->stream, s, G, R, Rinv, Racc, flag);
  hipLaunchKernelGGL(k_right_mult, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, W, Rinv, out);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::identity(c128* M) {
  hipLaunchKernelGGL(k_set_identity, dim3(1), dim3(256), 0, ctx->stream, s, M);
}

void KrylovKernels::lsq_step(int jj, c128* Hc, c128* Rm, int64_t ldr, c128* refl, c128* tau, c128* G, double* res) {
  hipLaunchKernelGGL(k_lsq_step, dim3(1), dim3(64), 0, ctx->stream, s, jj, Hc, Rm, ldr, refl, tau, G, res);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::lsq_solve(int J, const c128* Rm, int64_t ldr, const c128* G, c128* Y) {
  hipLaunchKernelGGL(k_lsq_solve, dim3(1), dim3(64), 0, ctx->stream, s, J, Rm, ldr, G, Y);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::colnorms(const c128* X, double* part, double* out) {
  hipLaunchKernelGGL(k_colnorm_part, dim3((unsigned)nchunk), dim3(256), 0, ctx->stream, n, s, X, part);
  hipLaunchKernelGGL(k_colnorm_reduce, dim3(1), dim3(64), 0, ctx->stream, nchunk, s, part, out);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hz
