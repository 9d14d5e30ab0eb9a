// Block FGMRES(m) in FP64 on the GPU: classical Gram-Schmidt as tall-skinny products (with
// delayed reorthogonalisation for 16- and 32-column blocks, twice (CGS2) with CholQR2 block
// normalisation otherwise), Householder QR of the block Hessenberg matrix and
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
#include "prof.h"

namespace hz {

namespace {

constexpr int kChunkRows = 4096;  // rows per partial-sum chunk
constexpr int kJT = 64;           // basis columns per gram tile

template <typename T>
__global__ void k_to_node(int64_t n, int s, const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst) {
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
                                              const c128* __restrict__ W, c128* __restrict__ part, int64_t rpc) {
  constexpr int R = 16;  // rows staged per step
  __shared__ c128 Vt[R][kJT];
  __shared__ c128 Wt[R][S];
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = min<int64_t>(n, r0 + rpc);
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

// ---- FP64 matrix-core variants for blocks of 16 or 32 columns
//
// v_mfma_f64_16x16x4f64, lane l: A[l%16][l/16], B[l/16][l%16], D[l/16 + 4v][l%16] in
// register v.  A complex product is a real one over twice the k range; here the k index is
// ordered so that one complex element held by a lane feeds two consecutive steps (its real
// part, then its imaginary part), the right operand supplying the matching signs:
//   conj(a) b :  (a_re, [b_re, b_im]) then (a_im, [ b_im, -b_re])
//        a  b :  (a_re, [b_re, b_im]) then (a_im, [-b_im,  b_re])
// Both kernels load the operands of the next step before issuing this step's products, so
// that memory latency overlaps the matrix-core work of the same wavefront.
typedef double f64x4 __attribute__((ext_vector_type(4)));
#define HZ_MFMA64 __builtin_amdgcn_mfma_f64_16x16x4f64

// Partial sums of H = V^H W over one chunk of rows.  The left operand is Jtot basis columns
// in blocks of S = 16 NCT (block b < nvb at V + b ldv, block nvb at Vx); the right operand is
// NRB blocks of S columns (W0, then W1), so H has NRB S columns.  A wavefront holds GJ tiles
// of 16 basis columns; the block's 4 wavefronts take interleaved groups of 4 rows (lane l
// reads row 4 (wave) + l/16 of each group of 16, column l%16: 256 contiguous bytes per row),
// RG groups per step, and are summed through LDS in a fixed order.  Two wavefronts per SIMD
// (register budget 256): with one, the loads of the next step do not cover the memory latency.
// M3: three real products per complex one (where the matrix cores bound the kernel):
//   P1 = a_re b_re, P2 = a_im b_im, P3 = (a_re + a_im)(b_im - b_re);
//   conj(a) b = (P1 + P2) + i (P3 + P1 - P2)
template <int NCT, int NRB, int GJ, int RG, bool M3 = false>
__global__ __launch_bounds__(256, 2) void k_gram_mfma(int64_t n, int Jtot, const c128* __restrict__ V, int64_t ldv,
                                                   int nvb, const c128* __restrict__ Vx, const c128* __restrict__ W0,
                                                   const c128* __restrict__ W1, c128* __restrict__ part, int64_t rpc,
                                                   int jbase) {
  constexpr int S = 16 * NCT, NC = NRB * NCT, SO = NRB * S;
  __shared__ c128 red[GJ * 16][SO];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, lc = l & 15, q = l >> 4;
  // the basis groups of one row chunk run one after another on one XCD (blocks are dealt to
  // the 8 XCDs in turn), so the chunk's right-operand rows they all read are shared in its L2
  int bx = blockIdx.x, by = blockIdx.y;
  if (NRB == 2) {
    const int64_t nb = (int64_t)gridDim.x * gridDim.y, b = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
    const int64_t qd = nb / 8, rm = nb % 8, x = b % 8, k = b / 8;
    const int64_t lg = x * qd + (x < rm ? x : rm) + k;
    bx = (int)(lg / gridDim.y);
    by = (int)(lg % gridDim.y);
  }
  const int64_t r0 = (int64_t)bx * rpc;
  const int64_t r1 = min<int64_t>(n, r0 + rpc);
  const int J0 = jbase + by * GJ * 16;
  f64x4 hre[GJ][NC], him[GJ][NC], h3[GJ][NC];
  const c128* vp[GJ];
  const c128* wp[NC];
  bool jv[GJ];
#pragma unroll
  for (int g = 0; g < GJ; ++g) {
    const int J = J0 + 16 * g;
    jv[g] = J < Jtot;
    const int b = J / S, jc = J - (J / S) * S;
    vp[g] = jv[g] ? (b < nvb ? V + (int64_t)b * ldv : Vx) + jc + lc : V;
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) hre[g][ct] = him[g][ct] = h3[g][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int ct = 0; ct < NC; ++ct) wp[ct] = (ct < NCT ? W0 : W1) + 16 * (ct % NCT) + lc;
  auto load = [&](int64_t rb, c128 (&w)[RG][NC], c128 (&a)[RG][GJ]) {
#pragma unroll
    for (int u = 0; u < RG; ++u) {
      const int64_t r = rb + 16 * u + q;
      const bool ok = r < r1;
#pragma unroll
      for (int ct = 0; ct < NC; ++ct) w[u][ct] = ok ? wp[ct][r * S] : cmk(0.0, 0.0);
#pragma unroll
      for (int g = 0; g < GJ; ++g) a[u][g] = (ok && jv[g]) ? vp[g][r * S] : cmk(0.0, 0.0);
    }
  };
  c128 wc[RG][NC], ac[RG][GJ];
  int64_t rb = r0 + 4 * wv;
  load(rb, wc, ac);
  for (; rb < r1; rb += 16 * RG) {
    c128 wn[RG][NC], an[RG][GJ];
    load(rb + 16 * RG, wn, an);
#pragma unroll
    for (int u = 0; u < RG; ++u) {
      if constexpr (M3) {  // hre = P1, him = P2, h3 = P3
        double sa[GJ], sw[NC];
#pragma unroll
        for (int g = 0; g < GJ; ++g) sa[g] = ac[u][g].re + ac[u][g].im;
#pragma unroll
        for (int ct = 0; ct < NC; ++ct) sw[ct] = wc[u][ct].im - wc[u][ct].re;
#pragma unroll
        for (int g = 0; g < GJ; ++g)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) {
            hre[g][ct] = HZ_MFMA64(ac[u][g].re, wc[u][ct].re, hre[g][ct], 0, 0, 0);
            him[g][ct] = HZ_MFMA64(ac[u][g].im, wc[u][ct].im, him[g][ct], 0, 0, 0);
            h3[g][ct] = HZ_MFMA64(sa[g], sw[ct], h3[g][ct], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int g = 0; g < GJ; ++g)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) {
            hre[g][ct] = HZ_MFMA64(ac[u][g].re, wc[u][ct].re, hre[g][ct], 0, 0, 0);
            him[g][ct] = HZ_MFMA64(ac[u][g].re, wc[u][ct].im, him[g][ct], 0, 0, 0);
          }
#pragma unroll
        for (int g = 0; g < GJ; ++g)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) {
            hre[g][ct] = HZ_MFMA64(ac[u][g].im, wc[u][ct].im, hre[g][ct], 0, 0, 0);
            him[g][ct] = HZ_MFMA64(ac[u][g].im, -wc[u][ct].re, him[g][ct], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int u = 0; u < RG; ++u) {
#pragma unroll
      for (int ct = 0; ct < NC; ++ct) wc[u][ct] = wn[u][ct];
#pragma unroll
      for (int g = 0; g < GJ; ++g) ac[u][g] = an[u][g];
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int g = 0; g < GJ; ++g)
#pragma unroll
        for (int ct = 0; ct < NC; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            c128& d = red[16 * g + q + 4 * v][16 * ct + lc];
            const c128 x = M3 ? cmk(hre[g][ct][v] + him[g][ct][v], h3[g][ct][v] + hre[g][ct][v] - him[g][ct][v])
                              : cmk(hre[g][ct][v], him[g][ct][v]);
            d = w == 0 ? x : d + x;
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < GJ * 16 * SO; e += 256) {
    const int j = e / SO, c = e - (e / SO) * SO;
    if (J0 + j < Jtot) part[((int64_t)bx * Jtot + J0 + j) * SO + c] = red[j][c];
  }
}

// Y = Yin + beta V H.  V is Jtot basis columns in blocks of S = 16 NCT (block b < nvb at
// V + b ldv, block nvb at Vx, block nvb + 1 at Vx2); Y is NRB blocks of S columns (Y0, Y1, each
// with its own Yin, which may be null or equal to its Y), H has NRB S columns.  A Y block may
// also be one of the V blocks: every row of Y is written by the wavefront that read that row
// of every V block, after its last read.  A wavefront holds RT tiles of
// 16 rows; the basis columns go 16 at a time, lane l taking columns 4 (l/16) .. 4 (l/16) + 3
// of row l%16 of each tile (64 contiguous bytes) for eight consecutive k steps.
// M3: three real products per complex one (where the matrix cores bound the kernel):
//   P1 = a_re b_re, P2 = a_im b_im, P3 = (a_re + a_im)(b_re + b_im);  a b = (P1 - P2) + i (P3 - P1 - P2)
// Three wavefronts per SIMD (register budget 168); two with four column tiles or with two row
// tiles of the split form.
template <typename TV, int NCT, int NRB, int RT, bool M3 = false>
__global__ __launch_bounds__(256, (NCT * NRB > 2 || (NRB == 2 && RT > 1)) ? 2 : 3) void k_axpy_mfma(int64_t n, int Jtot, const cplx<TV>* V, int64_t ldv, int nvb,
                                                      const cplx<TV>* Vx, const cplx<TV>* Vx2,
                                                      const c128* __restrict__ H, double beta, const c128* Yin0,
                                                      c128* Y0, const c128* Yin1, c128* Y1) {
  constexpr int S = 16 * NCT, NC = NRB * NCT, SH = NRB * S;
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, lc = l & 15, q = l >> 4;
  const int64_t rbase = ((int64_t)blockIdx.x * 4 + wv) * (16 * RT);
  f64x4 cre[RT][NC], cim[RT][NC], c3[RT][NC];
  int64_t row[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    row[t] = rbase + 16 * t + lc;
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) cre[t][ct] = cim[t][ct] = c3[t][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  auto load = [&](int J, c128 (&h)[4][NC], c128 (&a)[RT][4]) {
    const bool jok = J < Jtot;
    const int b = J / S, jc = J - (J / S) * S;
    const cplx<TV>* vb = (b < nvb ? V + (int64_t)b * ldv : b == nvb ? Vx : Vx2) + jc + 4 * q;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int ct = 0; ct < NC; ++ct)
        h[k][ct] = jok ? H[(int64_t)(J + 4 * q + k) * SH + 16 * ct + lc] : cmk(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const cplx<TV> v = (jok && row[t] < n) ? vb[row[t] * S + k] : cmk((TV)0, (TV)0);
        a[t][k] = cmk((double)v.re, (double)v.im);
      }
  };
  c128 hc[4][NC], ac[RT][4];
  load(0, hc, ac);
  for (int J = 0; J < Jtot; J += 16) {
    c128 hn[4][NC], an[RT][4];
    load(J + 16, hn, an);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (M3) {  // cre = P1, cim = P2, c3 = P3
        double sa[RT], sh[NC];
#pragma unroll
        for (int t = 0; t < RT; ++t) sa[t] = ac[t][k].re + ac[t][k].im;
#pragma unroll
        for (int ct = 0; ct < NC; ++ct) sh[ct] = hc[k][ct].re + hc[k][ct].im;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) {
            cre[t][ct] = HZ_MFMA64(ac[t][k].re, hc[k][ct].re, cre[t][ct], 0, 0, 0);
            cim[t][ct] = HZ_MFMA64(ac[t][k].im, hc[k][ct].im, cim[t][ct], 0, 0, 0);
            c3[t][ct] = HZ_MFMA64(sa[t], sh[ct], c3[t][ct], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) {
            cre[t][ct] = HZ_MFMA64(ac[t][k].re, hc[k][ct].re, cre[t][ct], 0, 0, 0);
            cim[t][ct] = HZ_MFMA64(ac[t][k].re, hc[k][ct].im, cim[t][ct], 0, 0, 0);
          }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) {
            cre[t][ct] = HZ_MFMA64(ac[t][k].im, -hc[k][ct].im, cre[t][ct], 0, 0, 0);
            cim[t][ct] = HZ_MFMA64(ac[t][k].im, hc[k][ct].re, cim[t][ct], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int ct = 0; ct < NC; ++ct) hc[k][ct] = hn[k][ct];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int k = 0; k < 4; ++k) ac[t][k] = an[t][k];
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) {
      const c128* yin = ct < NCT ? Yin0 : Yin1;
      c128* y = ct < NCT ? Y0 : Y1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = rbase + 16 * t + q + 4 * v;
        if (r >= n) continue;
        const int64_t k = r * S + 16 * (ct % NCT) + lc;
        const double pr = M3 ? cre[t][ct][v] - cim[t][ct][v] : cre[t][ct][v];
        const double pi = M3 ? c3[t][ct][v] - cre[t][ct][v] - cim[t][ct][v] : cim[t][ct][v];
        y[k] = (yin ? yin[k] : cmk(0.0, 0.0)) + cmk(beta * pr, beta * pi);
      }
    }
}

// out[e] (+)= sum over chunks of part[chunk][e]: 4 groups of 64 threads take every fourth
// chunk, then the group sums are added in a fixed order
__global__ __launch_bounds__(256) void k_reduce_part(int nchunk, int64_t m, const c128* __restrict__ part,
                                                     c128* __restrict__ out, int accumulate) {
  __shared__ c128 red[4][64];
  const int g = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  c128 s = cmk(0.0, 0.0);
  if (e < m)
    for (int k = g; k < nchunk; k += 4) s = s + part[(int64_t)k * m + e];
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && e < m) {
    const int i = threadIdx.x;
    const c128 t = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
    out[e] = accumulate ? out[e] + t : t;
  }
}

// Y[row][c] = Yin[row][c] + beta * sum_J V_J[row] H[J][c]
// 64 rows per block; V tiles (64 rows x 32 basis columns) staged through LDS with
// coalesced loads, H chunk (32 x s) in LDS; thread = (row, group of s/4 columns).
template <typename TV, int S>
__global__ __launch_bounds__(256) void k_block_axpy(int64_t n, int s, int Jtot, const cplx<TV>* __restrict__ V, int64_t ldv,
                                                    const c128* __restrict__ H, double beta,
                                                    const c128* __restrict__ Yin, c128* __restrict__ Y) {
  constexpr int RB = 64, JC = 32, NC = (S + 3) / 4;
  __shared__ c128 Vt[JC][RB + 1];  // [basis column][row]: conflict-free reads along rows
  __shared__ c128 Ht[JC][S];
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
  c128 acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = cmk(0.0, 0.0);
  for (int J0 = 0; J0 < Jtot; J0 += JC) {
    const int jn = min(JC, Jtot - J0);
    __syncthreads();
    for (int e = threadIdx.x; e < RB * JC; e += 256) {
      const int rr = e / JC, jj = e - (e / JC) * JC;
      const int64_t row = r0 + rr;
      c128 v = cmk(0.0, 0.0);
      if (jj < jn && row < n) {
        const int J = J0 + jj;
        const int b = J / s, jc = J - (J / s) * s;
        const cplx<TV> w = V[(int64_t)b * ldv + row * s + jc];
        v = cmk((double)w.re, (double)w.im);
      }
      Vt[jj][rr] = v;
    }
    for (int e = threadIdx.x; e < JC * S; e += 256) {
      const int jj = e / S, c = e - (e / S) * S;
      Ht[jj][c] = (jj < jn && c < s) ? H[(int64_t)(J0 + jj) * s + c] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (cg < S) {
      for (int jj = 0; jj < jn; ++jj) {
        const c128 v = Vt[jj][r];
#pragma unroll
        for (int q = 0; q < NC; ++q)
          if (cg + 4 * q < S) cfma(acc[q], v, Ht[jj][cg + 4 * q]);
      }
    }
  }
  const int64_t row = r0 + r;
  if (row < n) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = cg + 4 * q;
      if (c < s) {
        const int64_t k = row * s + c;
        Y[k] = (Yin ? Yin[k] : cmk(0.0, 0.0)) + cmk(beta * acc[q].re, beta * acc[q].im);
      }
    }
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
// flag[0] = 1 on breakdown (a pivot below 1e-14 of its diagonal entry).  One block, s <= 32.
__global__ __launch_bounds__(256) void k_chol_small(int s, const c128* __restrict__ G, c128* __restrict__ R,
                                                    c128* __restrict__ Rinv, c128* __restrict__ Racc,
                                                    int* __restrict__ flag) {
  __shared__ c128 A[32][33];
  __shared__ c128 Rs[32][33];
  __shared__ c128 Xs[32][33];
  const int t = threadIdx.x;
  for (int e = t; e < 32 * 32; e += 256) {
    const int i = e / 32, j = e % 32;
    A[i][j] = (i < s && j < s) ? G[i * s + j] : cmk(0.0, 0.0);
    Rs[i][j] = cmk(0.0, 0.0);
    Xs[i][j] = cmk(0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < s; ++k) {
    if (t == 0) {
      double d = A[k][k].re;
      const double scale = fabs(G[k * s + k].re) + 1e-300;
      // breakdown: the column's part orthogonal to the ones before it is below 1e-7 of its
      // norm (d / G_kk < 1e-14), where CholQR can no longer recover orthogonality
      if (!(d > 1e-14 * scale) || !isfinite(d)) {
        flag[0] = 1;
        d = fmax(d, 1e-14 * scale);
      }
      Rs[k][k] = cmk(sqrt(d), 0.0);
    }
    __syncthreads();
    const double rk = Rs[k][k].re;
    for (int j = k + 1 + t; j < s; j += 256) Rs[k][j] = cmk(A[k][j].re / rk, A[k][j].im / rk);
    __syncthreads();
    // A[i][j] -= conj(R[k][i]) R[k][j] for k < i <= j
    for (int e = t; e < s * s; e += 256) {
      const int i = e / s, j = e % s;
      if (i > k && j >= i) cfma_conj(A[i][j], cmk(-Rs[k][i].re, -Rs[k][i].im), Rs[k][j]);
    }
    __syncthreads();
  }
  // Rinv: column c by thread c (back substitution)
  if (t < s) {
    const int c = t;
    for (int i = c; i >= 0; --i) {
      c128 v = cmk(i == c ? 1.0 : 0.0, 0.0);
      for (int l = i + 1; l <= c; ++l) cfms(v, Rs[i][l], Xs[l][c]);
      Xs[i][c] = cmk(v.re / Rs[i][i].re, v.im / Rs[i][i].re);
    }
  }
  __syncthreads();
  for (int e = t; e < s * s; e += 256) {
    const int i = e / s, j = e % s;
    R[e] = Rs[i][j];
    Rinv[e] = Xs[i][j];
  }
  if (Racc) {
    // Racc <- R * Racc (both upper); read all of Racc before anyone writes
    c128 v[4];
    int cnt = 0;
    for (int e = t; e < s * s; e += 256, ++cnt) {
      const int i = e / s, j = e % s;
      c128 acc = cmk(0.0, 0.0);
      for (int l = i; l <= j; ++l) cfma(acc, Rs[i][l], Racc[l * s + j]);
      v[cnt] = acc;
    }
    __syncthreads();
    cnt = 0;
    for (int e = t; e < s * s; e += 256, ++cnt) Racc[e] = v[cnt];
  }
}

// Delayed reorthogonalisation (DCGS2, one pass over the basis per product): the block Vt
// that was projected once at the previous step is projected again and normalised in the
// same pass that projects the new product W once.  With V = [V_0 .. V_{j-1}] orthonormal and
// G = [V, Vt]^H [Vt, W] ((nb + s) x 2s, nb = j s; a = V^H Vt, c = V^H W, b = Vt^H Vt,
// d = Vt^H W):
//   R^H R = b - a^H a (Cholesky of the Gram matrix of Vt - V a), v_j = (Vt - V a) Ri, Ri = R^{-1},
//   h = v_j^H W = R^{-H} (d - a^H c), W' = W - V c - v_j h.
// The next block is Vt' = W' D, D = diag(1 / R_kk): each column then carries the scale of a
// normalised step instead of the product of every earlier step's scale (which underflows once
// a column has converged).  A diagonal keeps the products as well conditioned as W' itself;
// scaling by Ri would multiply the cancellation in W' by the condition number of R again.
// One product writes both: [v_j, Vt'] = [V, Vt, W] C with T = Ri h,
//   C = [[-a Ri, (a T - c) D], [Ri, -T D], [0, D]].
// Vt = V a + v_j R completes the Hessenberg column of the previous step, whose block was
// scaled by Rprev^{-1} (Hp: += a Rprev on rows < nb, R Rprev on rows nb .. nb + s); the new
// column (Hn) holds c, h until the next step adds its own part; Rprev becomes D^{-1}.
// Finishing (C null): G = [V, Vt]^H Vt ((nb + s) x s, V = [V_0 .. V_j]): Hn += a Rprev on rows
// < nb and R Rprev on rows nb .. nb + s.  flag[0] = 1 when a pivot of R^H R falls below 1e-14 of
// its diagonal entry of b (a numerically dependent block), as in CholQR.
// One block of 1024 threads; S (the block size) a power of two <= 32, a template parameter
// so that the loops over a row of the Gram block unroll and their loads issue together.
template <int S>
__global__ __launch_bounds__(1024) void k_dcgs_coef(int nb, const c128* __restrict__ G, c128* __restrict__ C,
                                                    c128* __restrict__ Hp, c128* __restrict__ Hn,
                                                    c128* __restrict__ Rprev, int* __restrict__ flag) {
  constexpr int s = S;
  __shared__ c128 A[32][33];   // b - a^H a, eliminated in place
  __shared__ c128 Rs[32][33];  // R
  __shared__ c128 Xs[32][33];  // Ri
  __shared__ c128 Qs[32][33];  // d - a^H c, then h
  __shared__ c128 Ts[32][33];  // T = Ri h
  __shared__ c128 Ps[32][33];  // Rprev
  __shared__ c128 red[1024];
  const int t = threadIdx.x;
  const bool fused = C != nullptr;
  const int so = fused ? 2 * s : s;
  const int ss = s * s, ng = 1024 / ss;
  auto Gat = [&](int i, int c) { return G[(int64_t)i * so + c]; };
  if (t < ss) Ps[t / s][t % s] = Rprev[t];
  // P = b - a^H a and Q = d - a^H c: ng groups of threads take every ng-th basis row, then
  // the group sums are added in a fixed order
  for (int pass = 0; pass < (fused ? 2 : 1); ++pass) {
    const int e = t % ss, g = t / ss, k = e / s, l = e % s;
    c128 acc = cmk(0.0, 0.0);
    if (g < ng) {
#pragma unroll 4
      for (int i = g; i < nb; i += ng) cfma_conj(acc, Gat(i, k), Gat(i, pass * s + l));
    }
    red[t] = acc;
    __syncthreads();
    if (t < ss) {
      c128 sum = red[t];
      for (int q = 1; q < ng; ++q) sum = sum + red[q * ss + t];
      const c128 v = Gat(nb + k, pass * s + l) - sum;
      if (pass == 0) {
        A[k][l] = v;
        Rs[k][l] = cmk(0.0, 0.0);
        Xs[k][l] = cmk(0.0, 0.0);
      } else {
        Qs[k][l] = v;
      }
    }
    __syncthreads();
  }
  // a pivot below 1e-14 of its diagonal entry of b is a numerically dependent direction: its
  // row of R (and of Ri, and its scaling) is zero, so that the column this call completes gets
  // no subdiagonal part from it and nothing overflows (clamping it instead made Ri grow by
  // 1e7 per dependent direction)
  for (int k = 0; k < s; ++k) {
    if (t == 0) {
      const double d = A[k][k].re;
      const double scale = fabs(Gat(nb + k, k).re);
      const bool dep = !(d > 1e-14 * scale) || !isfinite(d);
      if (dep) flag[0] = 1;
      Rs[k][k] = cmk(dep ? 0.0 : sqrt(d), 0.0);
    }
    __syncthreads();
    const double rk = Rs[k][k].re;
    if (t > k && t < s) Rs[k][t] = rk > 0.0 ? cmk(A[k][t].re / rk, A[k][t].im / rk) : cmk(0.0, 0.0);
    __syncthreads();
    if (t < ss) {
      const int i = t / s, j = t % s;
      if (i > k && j >= i) cfma_conj(A[i][j], cmk(-Rs[k][i].re, -Rs[k][i].im), Rs[k][j]);
    }
    __syncthreads();
  }
  if (t < s) {  // Ri: column c by thread c (back substitution; dependent rows stay zero)
    const int c = t;
    for (int i = c; i >= 0; --i) {
      c128 v = cmk(i == c ? 1.0 : 0.0, 0.0);
      for (int l = i + 1; l <= c; ++l) cfms(v, Rs[i][l], Xs[l][c]);
      const double ri = Rs[i][i].re;
      Xs[i][c] = ri > 0.0 ? cmk(v.re / ri, v.im / ri) : cmk(0.0, 0.0);
    }
  }
  __syncthreads();
  c128* Hc = fused ? Hp : Hn;  // the column this call completes
  for (int e = t; e < nb * s; e += 1024) {  // rows < nb: += a Rprev (Rprev upper triangular)
    const int i = e / s, l = e % s;
    c128 v = Hc[e];
    for (int m = 0; m <= l; ++m) cfma(v, Gat(i, m), Ps[m][l]);
    Hc[e] = v;
  }
  if (t < ss) {  // subdiagonal block R Rprev
    const int k = t / s, l = t % s;
    c128 v = cmk(0.0, 0.0);
    for (int m = k; m <= l; ++m) cfma(v, Rs[k][m], Ps[m][l]);
    Hc[(int64_t)nb * s + t] = v;
  }
  if (!fused) return;
  c128 hv = cmk(0.0, 0.0);
  if (t < ss) {  // h = Ri^H Q (Ri upper triangular)
    const int k = t / s, l = t % s;
    for (int m = 0; m <= k; ++m) cfma_conj(hv, Xs[m][k], Qs[m][l]);
  }
  __syncthreads();
  if (t < ss) Qs[t / s][t % s] = hv;
  __syncthreads();
  c128 tv = cmk(0.0, 0.0);
  if (t < ss) {  // T = Ri h
    const int k = t / s, l = t % s;
    for (int m = k; m < s; ++m) cfma(tv, Xs[k][m], Qs[m][l]);
    Ts[k][l] = tv;
  }
  __syncthreads();
  for (int e = t; e < nb * s; e += 1024) {
    const int i = e / s, l = e % s;
    c128 x = cmk(0.0, 0.0), y = cmk(0.0, 0.0) - Gat(i, s + l);
#pragma unroll 4
    for (int m = 0; m < s; ++m) {
      const c128 am = Gat(i, m);
      if (m <= l) cfms(x, am, Xs[m][l]);
      cfma(y, am, Ts[m][l]);
    }
    const double dl = Rs[l][l].re > 0.0 ? 1.0 / Rs[l][l].re : 0.0;
    C[(int64_t)i * 2 * s + l] = x;
    C[(int64_t)i * 2 * s + s + l] = cmk(y.re * dl, y.im * dl);
    Hn[e] = Gat(i, s + l);
  }
  if (t < ss) {
    const int k = t / s, l = t % s;
    const double dl = Rs[l][l].re > 0.0 ? 1.0 / Rs[l][l].re : 0.0;
    C[(int64_t)(nb + k) * 2 * s + l] = Xs[k][l];
    C[(int64_t)(nb + k) * 2 * s + s + l] = cmk(-Ts[k][l].re * dl, -Ts[k][l].im * dl);
    C[(int64_t)(nb + s + k) * 2 * s + l] = cmk(0.0, 0.0);
    C[(int64_t)(nb + s + k) * 2 * s + s + l] = cmk(k == l ? dl : 0.0, 0.0);
    Hn[(int64_t)nb * s + t] = Qs[k][l];
    Rprev[t] = k == l ? Rs[k][k] : cmk(0.0, 0.0);
  }
}

// per-block counts of non-finite entries, summed in integers (exact, order-free)
__global__ __launch_bounds__(256) void k_count_nonfinite(const c128* __restrict__ x, int64_t m,
                                                         unsigned long long* __restrict__ count) {
  __shared__ unsigned int red[256];
  unsigned int c = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    c += (isfinite(x[k].re) && isfinite(x[k].im)) ? 0u : 1u;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0]) atomicAdd(count, (unsigned long long)red[0]);
}

__global__ void k_set_identity(int s, c128* M) {
  for (int i = threadIdx.x; i < s * s; i += blockDim.x) M[i] = cmk((i / s) == (i % s) ? 1.0 : 0.0, 0.0);
}

// ---------------------------------------------------------------- least squares (one block)
// State: Hc (rows x s, row-major, the new block column), Rm (column-major, ld = ldr),
// refl[step][2s][s] reflector vectors (v[0] = 1) and tau[step][s], G (ldg x s row-major).
// Each column of the block is handled by a group of L lanes of one wavefront; dot
// products reduce with cross-lane shuffles in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// sum over aligned groups of L lanes, the same value in every lane of a group: partner lanes
// are paired symmetrically at each step (xor 1, xor 2 by quad permutes, then the half-row and
// row mirrors on DPP; xor 16 and 32 by shuffles), and a + b == b + a exactly
template <int L>
__device__ __forceinline__ double group_sum_t(double v) {
  if constexpr (L >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (L >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (L >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
  if constexpr (L >= 16) v += dpp_move<0x140>(v); // row_mirror
  if constexpr (L >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
template <int L>
__device__ __forceinline__ c128 group_sum_t(c128 v) {
  return cmk(group_sum_t<L>(v.re), group_sum_t<L>(v.im));
}

// apply H^H = I - conj(tau) v v^H (v on rows [r0 + k, r0 + 2s), v[k] = 1) to column c of X
template <int L>
__device__ __forceinline__ void apply_refl(c128* X, int s, int r0, int k, const c128* V, c128 tau, int c, int lane) {
  const int s2 = 2 * s;
  c128 w = cmk(0.0, 0.0);
  for (int r = k + lane; r < s2; r += L) cfma_conj(w, V[r * s + k], X[(int64_t)(r0 + r) * s + c]);
  w = group_sum_t<L>(w);
  const c128 ct = conj(tau) * w;
  for (int r = k + lane; r < s2; r += L) cfms(X[(int64_t)(r0 + r) * s + c], V[r * s + k], ct);
}

// One step of the block Hessenberg QR (s <= 32, 256 threads, L lanes per column).
// A block i of s Householder reflectors P_k = I - conj(tau_k) v_k v_k^H, applied in the order
// k = 0 .. s-1, is the single update X <- X - V T^H V^H X, with V = [v_0 .. v_{s-1}] (2s x s,
// unit lower trapezoidal) and T the upper triangular factor of P_0^H .. P_{s-1}^H = I - V T V^H
// (T[k][k] = tau_k, T[0:k, k] = -tau_k T[0:k, 0:k] V[:, 0:k]^H v_k).  Each block's T is formed
// once, when its reflectors are made, and kept beside them.

// X (2s x s, in LDS through row(r)) <- X - V T^H V^H X; V, T and the work blocks in LDS
template <typename RowFn>
__device__ __forceinline__ void wy_apply(int s, RowFn row, const c128 (*Vs)[32], const c128 (*Ts)[32], c128 (*W1)[32],
                                         c128 (*W2)[32]) {
  const int s2 = 2 * s;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {  // W1 = V^H X
    const int a = e / s, c = e - (e / s) * s;
    c128 w = cmk(0.0, 0.0);
    for (int r = a; r < s2; ++r) cfma_conj(w, Vs[r][a], row(r)[c]);
    W1[a][c] = w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {  // W2 = T^H W1
    const int a = e / s, c = e - (e / s) * s;
    c128 w = cmk(0.0, 0.0);
    for (int b = 0; b <= a; ++b) cfma_conj(w, Ts[b][a], W1[b][c]);
    W2[a][c] = w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s2 * s; e += blockDim.x) {  // X -= V W2
    const int r = e / s, c = e - (e / s) * s;
    c128 x = row(r)[c];
    const int am = r < s ? r : s - 1;
    for (int a = 0; a <= am; ++a) cfms(x, Vs[r][a], W2[a][c]);
    row(r)[c] = x;
  }
  __syncthreads();
}

// L lanes per column (L = min(64, 256 / s rounded up to a power of two)); s <= 32
template <int L>
__global__ __launch_bounds__(256) void k_lsq_step(int s, int jj, c128* __restrict__ Hc, c128* __restrict__ Rm,
                                                  int64_t ldr, c128* __restrict__ refl, c128* __restrict__ tau,
                                                  c128* __restrict__ tmat, c128* __restrict__ G,
                                                  double* __restrict__ res) {
  const int c = threadIdx.x / L, lane = threadIdx.x % L;
  const bool act = c < s;
  const int s2 = 2 * s;
  const int64_t base = (int64_t)jj * s;
  __shared__ c128 win[2 * 32 * 32];  // [half][row][column]
  __shared__ c128 Vs[64][32];
  __shared__ c128 Ts[32][32];
  __shared__ c128 W1[32][32];
  __shared__ c128 W2[32][32];
  // 1. previous blocks of reflectors, in order, on the new column block.  Block i touches rows
  //    [i s, i s + 2s) only, so the column block streams through an LDS window of 2s rows (two
  //    halves used as a ring): after block i its first s rows are final and go back to memory,
  //    and rows [(i+2)s, (i+3)s) come in.
  if (jj > 0) {
    int ha = 0;
    auto row = [&](int r) -> c128* { return &win[((r < s ? ha : 1 - ha) * 32 + (r < s ? r : r - s)) * 32]; };
    for (int e = threadIdx.x; e < s2 * s; e += blockDim.x) row(e / s)[e % s] = Hc[e];
    for (int i = 0; i < jj; ++i) {
      const c128* Vi = refl + (int64_t)i * s2 * s;
      const c128* Ti = tmat + (int64_t)i * s * s;
      for (int e = threadIdx.x; e < s2 * s; e += blockDim.x) Vs[e / s][e % s] = Vi[e];
      for (int e = threadIdx.x; e < s * s; e += blockDim.x) Ts[e / s][e % s] = Ti[e];
      __syncthreads();
      wy_apply(s, row, Vs, Ts, W1, W2);
      // rows [i s, i s + s) are final; rows [(i+2)s, (i+3)s) take their place in the ring
      for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        c128& x = row(e / s)[e % s];
        Hc[(int64_t)i * s * s + e] = x;
        x = Hc[(int64_t)(i + 2) * s * s + e];
      }
      __syncthreads();
      ha = 1 - ha;
    }
    for (int e = threadIdx.x; e < s2 * s; e += blockDim.x)  // the window holds rows [jj s, jj s + 2s)
      Hc[(int64_t)jj * s * s + e] = row(e / s)[e % s];
  }
  __syncthreads();
  // 2. new reflectors on rows [jj s, jj s + 2s)
  c128* Vn = refl + (int64_t)jj * s2 * s;
  c128* tn = tau + (int64_t)jj * s;
  for (int k = 0; k < s; ++k) {
    if (c == k) {
      const c128 alpha = Hc[(base + k) * s + k];
      double xn = 0;
      for (int r = k + 1 + lane; r < s2; r += L) {
        const c128 x = Hc[(base + r) * s + k];
        xn += x.re * x.re + x.im * x.im;
      }
      xn = group_sum_t<L>(xn);
      c128 t = cmk(0.0, 0.0), beta = alpha, sc = cmk(0.0, 0.0);
      const bool refl_needed = xn > 0 || alpha.im != 0;
      if (refl_needed) {
        const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn);
        const double b = alpha.re >= 0 ? -nrm : nrm;
        t = cmk((b - alpha.re) / b, -alpha.im / b);
        sc = cdiv(cmk(1.0, 0.0), cmk(alpha.re - b, alpha.im));
        beta = cmk(b, 0.0);
      }
      for (int r = lane; r < s2; r += L) {
        c128 v = cmk(0.0, 0.0);
        if (r == k) v = cmk(1.0, 0.0);
        else if (r > k && refl_needed) v = Hc[(base + r) * s + k] * sc;
        Vn[r * s + k] = v;
        Vs[r][k] = v;
      }
      if (lane == 0) {
        tn[k] = t;
        Ts[k][k] = t;
        Hc[(base + k) * s + k] = beta;
      }
      for (int r = k + 1 + lane; r < s2; r += L) Hc[(base + r) * s + k] = cmk(0.0, 0.0);
    }
    __syncthreads();
    if (act && c > k) apply_refl<L>(Hc, s, (int)base, k, Vn, tn[k], c, lane);
    __syncthreads();
  }
  // the block's T: W1 = V^H V, then column k of T from the columns before it
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
    const int a = e / s, k = e - (e / s) * s;
    c128 w = cmk(0.0, 0.0);
    if (a < k)
      for (int r = k; r < s2; ++r) cfma_conj(w, Vs[r][a], Vs[r][k]);
    W1[a][k] = w;
    if (a > k) Ts[a][k] = cmk(0.0, 0.0);
  }
  __syncthreads();
  for (int k = 1; k < s; ++k) {
    for (int a = threadIdx.x; a < k; a += blockDim.x) {
      c128 w = cmk(0.0, 0.0);
      for (int b = a; b < k; ++b) cfma(w, Ts[a][b], W1[b][k]);
      W2[a][0] = cmk(0.0, 0.0) - Ts[k][k] * w;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < k; a += blockDim.x) Ts[a][k] = W2[a][0];
    __syncthreads();
  }
  c128* Tn = tmat + (int64_t)jj * s * s;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) Tn[e] = Ts[e / s][e % s];
  // 3. R column block jj: rows 0 .. (jj+1)s-1
  const int64_t rows = (int64_t)(jj + 1) * s;
  for (int64_t e = threadIdx.x; e < rows * s; e += blockDim.x) {
    const int64_t r = e / s;
    const int cc = (int)(e - r * s);
    Rm[(base + cc) * ldr + r] = Hc[r * s + cc];
  }
  // 4. the new block of reflectors on G rows [jj s, jj s + 2s); residual estimates
  {
    auto grow = [&](int r) -> c128* { return &win[r * 32]; };
    for (int e = threadIdx.x; e < s2 * s; e += blockDim.x) grow(e / s)[e % s] = G[base * s + e];
    __syncthreads();
    wy_apply(s, grow, Vs, Ts, W1, W2);
    for (int e = threadIdx.x; e < s2 * s; e += blockDim.x) G[base * s + e] = grow(e / s)[e % s];
    if (act) {
      double q = 0;
      for (int r = lane; r < s; r += L) {
        const c128 g = grow(s + r)[c];
        q += g.re * g.re + g.im * g.im;
      }
      q = group_sum_t<L>(q);
      if (lane == 0) res[c] = sqrt(q);
    }
  }
}

// Y = Rm[0:J, 0:J]^{-1} G[0:J]: back substitution by blocks of 16 rows, one workgroup of NT
// threads, Y kept in global memory (any J s).  Per block: the block's rows go to LDS, one
// thread per column solves the 16 x 16 triangle there, and every entry above is updated by the
// solved block.  The order of operations per entry is fixed.  Rm is column-major with leading
// dimension ldr; G and Y are [J][s] (Y may not alias G).
template <int NT>
__global__ __launch_bounds__(NT) void k_lsq_solve(int s, int J, const c128* __restrict__ Rm, int64_t ldr,
                                                  const c128* __restrict__ G, c128* __restrict__ Y) {
  constexpr int B = 16;
  __shared__ c128 Yb[B][32];
  __shared__ c128 Rb[B][B];
  const int tot = J * s;
  for (int e = threadIdx.x; e < tot; e += NT) Y[e] = G[e];
  __syncthreads();
  for (int i0 = ((J - 1) / B) * B; i0 >= 0; i0 -= B) {
    const int nb = min(B, J - i0);
    for (int e = threadIdx.x; e < B * s; e += NT) Yb[e / s][e % s] = e < nb * s ? Y[(int64_t)i0 * s + e] : cmk(0.0, 0.0);
    for (int e = threadIdx.x; e < nb * nb; e += NT) Rb[e % nb][e / nb] = Rm[(int64_t)(i0 + e / nb) * ldr + i0 + e % nb];
    __syncthreads();
    if (threadIdx.x < s) {  // the block's columns are independent: one thread per column
      const int c = threadIdx.x;
      for (int i = nb - 1; i >= 0; --i) {
        const c128 yi = cdiv(Yb[i][c], Rb[i][i]);
        Yb[i][c] = yi;
        for (int r = 0; r < i; ++r) cfms(Yb[r][c], Rb[r][i], yi);
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nb * s; e += NT) Y[(int64_t)i0 * s + e] = Yb[e / s][e % s];
    // rows above the block: y_r -= sum_k R[r][i0 + k] y_{i0 + k}, k ascending
    for (int e = threadIdx.x; e < i0 * s; e += NT) {
      const int r = e / s, c = e - r * s;
      c128 y = Y[e];
#pragma unroll 1
      for (int k0 = 0; k0 < B; k0 += 4) {
        c128 rv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) rv[k] = k0 + k < nb ? Rm[(int64_t)(i0 + k0 + k) * ldr + r] : cmk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) cfms(y, rv[k], Yb[k0 + k][c]);
      }
      Y[e] = y;
    }
    __syncthreads();
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
  hipLaunchKernelGGL(k_to_node<double>, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, src,
                     dst);
}
void KrylovKernels::to_node(const c64* src, c64* dst) {
  hipLaunchKernelGGL(k_to_node<float>, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, src,
                     dst);
}
void KrylovKernels::from_node(const c128* src, c128* dst) {
  hipLaunchKernelGGL(k_from_node, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, src, dst);
}

template <int S>
static void gram_t(KrylovKernels& k, int Jtot, const c128* V, int64_t ldv, const c128* W, c128* part, int nch,
                   int64_t rpc) {
  hipLaunchKernelGGL(k_gram<S>, dim3((unsigned)nch, (unsigned)((Jtot + kJT - 1) / kJT)), dim3(256), 0, k.ctx->stream,
                     k.n, k.s, Jtot, V, ldv, W, part, rpc);
}

void KrylovKernels::gram(int nblk, const c128* V, int64_t ldv, const c128* W, c128* part, c128* H, bool accumulate,
                         c128* H2) {
  gram_ext(nblk, V, ldv, nblk, nullptr, W, nullptr, part, H, accumulate, H2);
}

void KrylovKernels::gram_ext(int nblk, const c128* V, int64_t ldv, int nvb, const c128* Vx, const c128* W0,
                             const c128* W1, c128* part, c128* H, bool accumulate, c128* H2) {
  const int Jtot = nblk * s;
  const int nrb = W1 ? 2 : 1;
  const bool mfma = s == 16 || s == 32;
  HZ_REQUIRE((nvb == nblk && nrb == 1) || s == 16 || s == 32, HZ_ERR_STATE, "gram: split operands need 16 or 32 columns");
  // about 2048 blocks in total: fewer, longer row chunks when there are many basis tiles
  // (never more chunks than `nchunk`: the partial-sum workspace is sized for nchunk)
  const int jper = s == 16 ? (nrb == 2 ? 48 : 64) : s == 32 ? 32 : kJT;
  const int jtiles = (Jtot + jper - 1) / jper;
  int nch = std::min(nchunk, std::max(16, 2048 / jtiles));
  int64_t rpc = ((n + nch - 1) / nch + 15) / 16 * 16;
  nch = (int)((n + rpc - 1) / rpc);
  HZ_REQUIRE(nch >= 1 && nch <= nchunk, HZ_ERR_STATE, "gram: chunk count exceeds the partial-sum workspace");
  {
    // algorithmic traffic: the Jtot basis columns and W once; 8 flops per complex multiply-add
    // (the scope times the partial-product kernel alone, not the reduction below)
    ProfScope ps(ctx, HZ_K_CGS_GRAM, (double)n * (Jtot + nrb * s) * sizeof(c128), 8.0 * n * Jtot * nrb * s);
    if (mfma && s == 16) {
      // groups of 4 basis blocks, then one launch sized for the remaining 1..3 (so that no
      // block multiplies zero padding: the single block of CholQR and of the first step)
      const int full = nblk / 4, rem = nblk % 4;
      auto go = [&](auto kern, dim3 grid, int jbase) {
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, ctx->stream, n, Jtot, V, ldv, nvb, Vx, W0, W1, part, rpc, jbase);
      };
      const dim3 g1((unsigned)nch, 1);
      if (nrb == 1) {
        if (full > 0) go(k_gram_mfma<1, 1, 4, 2>, dim3((unsigned)nch, (unsigned)full), 0);
        if (rem == 1) go(k_gram_mfma<1, 1, 1, 2>, g1, 64 * full);
        if (rem == 2) go(k_gram_mfma<1, 1, 2, 2>, g1, 64 * full);
        if (rem == 3) go(k_gram_mfma<1, 1, 3, 2>, g1, 64 * full);
      } else {
        // 32 right-hand columns, 3M form: groups of 3 basis blocks fit two wavefronts per SIMD
        const int f3 = nblk / 3, r3 = nblk % 3;
        if (f3 > 0) go(k_gram_mfma<1, 2, 3, 2, true>, dim3((unsigned)nch, (unsigned)f3), 0);
        if (r3 == 1) go(k_gram_mfma<1, 2, 1, 2, true>, g1, 48 * f3);
        if (r3 == 2) go(k_gram_mfma<1, 2, 2, 2, true>, g1, 48 * f3);
      }
    } else if (mfma && nrb == 1) {
      const dim3 grid((unsigned)nch, (unsigned)jtiles);
      hipLaunchKernelGGL((k_gram_mfma<2, 1, 2, 2>), grid, dim3(256), 0, ctx->stream, n, Jtot, V, ldv, nvb, Vx, W0,
                         (const c128*)nullptr, part, rpc, 0);
    } else if (mfma) {  // 32 columns, right operand [W0, W1]: one basis block per group (the
      // 3M form does not fit two wavefronts per SIMD at this width)
      const dim3 grid((unsigned)nch, (unsigned)nblk);
      hipLaunchKernelGGL((k_gram_mfma<2, 2, 2, 2>), grid, dim3(256), 0, ctx->stream, n, Jtot, V, ldv, nvb, Vx, W0, W1,
                         part, rpc, 0);
    } else if (s <= 4) {
      gram_t<4>(*this, Jtot, V, ldv, W0, part, nch, rpc);
    } else if (s <= 8) {
      gram_t<8>(*this, Jtot, V, ldv, W0, part, nch, rpc);
    } else if (s <= 16) {
      gram_t<16>(*this, Jtot, V, ldv, W0, part, nch, rpc);
    } else {
      gram_t<32>(*this, Jtot, V, ldv, W0, part, nch, rpc);
    }
  }
  const int64_t m = (int64_t)Jtot * nrb * s;
  hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((m + 63) / 64)), dim3(256), 0, ctx->stream, nch, m, part, H,
                     accumulate ? 1 : 0);
  if (H2)
    hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((m + 63) / 64)), dim3(256), 0, ctx->stream, nch, m, part, H2, 1);
  HIP_CHECK(hipGetLastError());
}

template <typename TV, int S>
static void axpy_t(KrylovKernels& k, int Jtot, const cplx<TV>* V, int64_t ldv, const c128* H, double beta,
                   const c128* Yin, c128* Y) {
  hipLaunchKernelGGL((k_block_axpy<TV, S>), dim3((unsigned)((k.n + 63) / 64)), dim3(256), 0, k.ctx->stream, k.n, k.s,
                     Jtot, V, ldv, H, beta, Yin, Y);
}

template <typename TV>
static void block_axpy_t(KrylovKernels& k, int nblk, const cplx<TV>* V, int64_t ldv, const c128* H, double beta,
                         const c128* Yin, c128* Y) {
  const int64_t n = k.n;
  const int s = k.s;
  const int Jtot = nblk * s;
  ProfScope ps(k.ctx, HZ_K_CGS_UPDATE, (double)n * Jtot * sizeof(cplx<TV>) + (double)n * (Yin ? 2 : 1) * s * sizeof(c128),
               8.0 * n * Jtot * s);
  hipStream_t st = k.ctx->stream;
  const cplx<TV>* none = nullptr;
  if (s == 16)  // 4 wavefronts x 2 tiles of 16 rows per block
    hipLaunchKernelGGL((k_axpy_mfma<TV, 1, 1, 2>), dim3((unsigned)((n + 127) / 128)), dim3(256), 0, st, n, Jtot, V, ldv,
                       nblk, none, none, H, beta, Yin, Y, (const c128*)nullptr, (c128*)nullptr);
  else if (s == 32)  // 4 wavefronts x 1 tile of 16 rows per block
    hipLaunchKernelGGL((k_axpy_mfma<TV, 2, 1, 1>), dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, n, Jtot, V, ldv,
                       nblk, none, none, H, beta, Yin, Y, (const c128*)nullptr, (c128*)nullptr);
  else if (s == 1)
    axpy_t<TV, 1>(k, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s == 2)
    axpy_t<TV, 2>(k, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s <= 4)
    axpy_t<TV, 4>(k, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s <= 8)
    axpy_t<TV, 8>(k, Jtot, V, ldv, H, beta, Yin, Y);
  else if (s <= 16)
    axpy_t<TV, 16>(k, Jtot, V, ldv, H, beta, Yin, Y);
  else
    axpy_t<TV, 32>(k, Jtot, V, ldv, H, beta, Yin, Y);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::block_axpy(int nblk, const c128* V, int64_t ldv, const c128* H, double beta, const c128* Yin,
                               c128* Y) {
  block_axpy_t<double>(*this, nblk, V, ldv, H, beta, Yin, Y);
}

void KrylovKernels::block_axpy(int nblk, const c64* V, int64_t ldv, const c128* H, double beta, const c128* Yin,
                               c128* Y) {
  block_axpy_t<float>(*this, nblk, V, ldv, H, beta, Yin, Y);
}

void KrylovKernels::update_split(int nvb, const c128* V, int64_t ldv, const c128* Vx, const c128* Vx2, const c128* C,
                                 c128* Y0, c128* Y1) {
  HZ_REQUIRE(s == 16 || s == 32, HZ_ERR_STATE, "update_split: needs 16 or 32 columns");
  const int Jtot = (nvb + 2) * s;
  // algorithmic traffic: the Jtot basis columns once, Y0 and Y1 written once
  ProfScope ps(ctx, HZ_K_CGS_UPDATE, (double)n * (Jtot + 2 * s) * sizeof(c128), 8.0 * n * Jtot * 2 * s);
  if (s == 16)  // 4 wavefronts x 2 tiles of 16 rows per block: each coefficient load feeds both tiles
    hipLaunchKernelGGL((k_axpy_mfma<double, 1, 2, 2, true>), dim3((unsigned)((n + 127) / 128)), dim3(256), 0,
                       ctx->stream, n, Jtot, V, ldv, nvb, Vx, Vx2, C, 1.0, (const c128*)nullptr, Y0,
                       (const c128*)nullptr, Y1);
  else  // 4 wavefronts x 1 tile; direct form: the 3M form spills at four column tiles
    hipLaunchKernelGGL((k_axpy_mfma<double, 2, 2, 1>), dim3((unsigned)((n + 63) / 64)), dim3(256), 0, ctx->stream, n,
                       Jtot, V, ldv, nvb, Vx, Vx2, C, 1.0, (const c128*)nullptr, Y0, (const c128*)nullptr, Y1);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::dcgs_coef(int nb, const c128* G, c128* C, c128* Hp, c128* Hn, c128* Rprev, int* flag) {
  HZ_REQUIRE(s == 1 || s == 2 || s == 4 || s == 8 || s == 16 || s == 32, HZ_ERR_STATE,
             "dcgs_coef: block size must be a power of two");
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(1), dim3(1024), 0, ctx->stream, nb, G, C, Hp, Hn, Rprev, flag); };
  switch (s) {
    case 1: go(k_dcgs_coef<1>); break;
    case 2: go(k_dcgs_coef<2>); break;
    case 4: go(k_dcgs_coef<4>); break;
    case 8: go(k_dcgs_coef<8>); break;
    case 16: go(k_dcgs_coef<16>); break;
    default: go(k_dcgs_coef<32>); break;
  }
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::cholqr_pass(const c128* W, c128* out, c128* part, c128* G, c128* R, c128* Rinv, c128* Racc,
                                int* flag) {
  gram(1, W, n * s, W, part, G, false);
  hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(256), 0, ctx->stream, s, G, R, Rinv, Racc, flag);
  if (s == 16 || s == 32)  // Rinv is stored whole (zero below the diagonal): a one-block update
    block_axpy(1, W, n * s, Rinv, 1.0, nullptr, out);
  else
    hipLaunchKernelGGL(k_right_mult, dim3((unsigned)((n * s + 255) / 256)), dim3(256), 0, ctx->stream, n, s, W, Rinv,
                       out);
  HIP_CHECK(hipGetLastError());
}

int64_t count_nonfinite(Ctx* ctx, const c128* x, int64_t m) {
  if (m <= 0) return 0;
  DevArray<unsigned long long> cnt;
  cnt.alloc(ctx, 1);
  cnt.zero(ctx);
  const unsigned grid = (unsigned)std::min<int64_t>(2048, (m + 255) / 256);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(grid), dim3(256), 0, ctx->stream, x, m, cnt.ptr());
  HIP_CHECK(hipGetLastError());
  unsigned long long h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, cnt.ptr(), sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  return (int64_t)h;
}

void KrylovKernels::identity(c128* M) {
  hipLaunchKernelGGL(k_set_identity, dim3(1), dim3(256), 0, ctx->stream, s, M);
}

void KrylovKernels::lsq_step(int jj, c128* Hc, c128* Rm, int64_t ldr, c128* refl, c128* tau, c128* tmat, c128* G,
                             double* res, hipStream_t stream) {
  int sp = 1;
  while (sp < s) sp <<= 1;
  const int L = std::min(64, 256 / sp);
  hipStream_t st = stream ? stream : ctx->stream;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(1), dim3(256), 0, st, s, jj, Hc, Rm, ldr, refl, tau, tmat, G, res);
  };
  if (L == 64)
    go(k_lsq_step<64>);
  else if (L == 32)
    go(k_lsq_step<32>);
  else if (L == 16)
    go(k_lsq_step<16>);
  else
    go(k_lsq_step<8>);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::lsq_solve(int J, const c128* Rm, int64_t ldr, const c128* G, c128* Y) {
  hipLaunchKernelGGL((k_lsq_solve<1024>), dim3(1), dim3(1024), 0, ctx->stream, s, J, Rm, ldr, G, Y);
  HIP_CHECK(hipGetLastError());
}

void KrylovKernels::colnorms(const c128* X, double* part, double* out) {
  hipLaunchKernelGGL(k_colnorm_part, dim3((unsigned)nchunk), dim3(256), 0, ctx->stream, n, s, X, part);
  hipLaunchKernelGGL(k_colnorm_reduce, dim3(1), dim3(64), 0, ctx->stream, nchunk, s, part, out);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hz
