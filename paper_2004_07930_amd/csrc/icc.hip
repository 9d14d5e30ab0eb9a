// Incomplete LDL^T local solver: the approximate local solver of the paper's numerical section
// (its comparison of complete and incomplete Cholesky for the local matrices of eq. (oras)).
// The paper names no variant; the reading taken is level 0 without fill: A_i ~ L D L^T with L
// unit lower triangular on the strict lower pattern of A_i (transpose, not conjugate, since
// A_i is complex symmetric), in the local order of A_i, no shift and no pivoting.  A variant
// keeps L on the lower pattern of A_i^2 instead (rows joined through one neighbour).
//
// Set-up: the host lists each row's strict lower entries and both substitutions' dependency
// levels (a row's level is one more than the deepest row it reads); the numeric factorisation
// runs on the GPU level by level, one thread per row: the row's entries in ascending column
// order, each from the sparse product of the row so far with the (finished) row of its column,
// then the pivot.  It is done in FP64 and the factors are stored in the preconditioner
// precision.
// Apply: gather R_i v for every subdomain, forward substitution with L (one launch per level,
// every subdomain's rows of that level together), then x_i = d_i^{-1} y_i minus the rows of L^T
// (one launch per backward level), and a store into the local vectors in elimination order,
// where the owner (or partition-of-unity) gather of the one-level preconditioner reads them.
#include <chrono>
#include <cmath>

#include "ddm.h"

namespace hz {

namespace {

// One thread per row of a level.  l_ij = (a_ij - sum_k l_ik d_k l_jk) / d_j over the columns k
// < j that rows i and j share (a merge of two ascending lists), then
// d_i = a_ii - sum_k l_ik^2 d_k.  Rows of earlier levels are final.
__global__ __launch_bounds__(256) void k_icc_factor(int nrows, const int32_t* __restrict__ rows,
                                                    const int64_t* __restrict__ lp, const int32_t* __restrict__ lc,
                                                    const int64_t* __restrict__ src, const int64_t* __restrict__ dsrc,
                                                    const c128* __restrict__ a, c128* L, c128* dg,
                                                    int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const int32_t i = rows[t];
  const int64_t b0 = lp[i], b1 = lp[i + 1];
  for (int64_t k = b0; k < b1; ++k) {
    const int32_t j = lc[k];
    const int64_t sk = src[k];
    c128 acc = cmk(0.0, 0.0);
    if (sk >= 0) acc = a[sk];  // a fill position starts from zero
    int64_t x = b0, y = lp[j];
    const int64_t ye = lp[j + 1];
    while (x < k && y < ye) {
      const int32_t cx = lc[x], cy = lc[y];
      if (cx == cy) {
        acc = acc - (L[x] * dg[cx]) * L[y];
        ++x;
        ++y;
      } else if (cx < cy) {
        ++x;
      } else {
        ++y;
      }
    }
    L[k] = cdiv(acc, dg[j]);
  }
  c128 acc = a[dsrc[i]];
  for (int64_t x = b0; x < b1; ++x) acc = acc - (L[x] * L[x]) * dg[lc[x]];
  const bool ok = (acc.re != 0.0 || acc.im != 0.0) && isfinite(acc.re) && isfinite(acc.im);
  if (!ok) *bad = 1;
  dg[i] = acc;
}

template <typename T>
__global__ void k_icc_store_factors(int64_t nnz, int64_t n, const c128* __restrict__ Lw, const c128* __restrict__ dg,
                                    cplx<T>* __restrict__ L, cplx<T>* __restrict__ dinv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) L[k] = cmk((T)Lw[k].re, (T)Lw[k].im);
  if (k < n) {
    const c128 r = cdiv(cmk(1.0, 0.0), dg[k]);
    dinv[k] = cmk((T)r.re, (T)r.im);
  }
}

// y[r][c] = v[g(r)][c]: every subdomain's restriction R_i v, rows in local order
template <typename T, typename TS>
__global__ void k_icc_gather(int64_t nl, int s, const int32_t* __restrict__ g, const cplx<TS>* __restrict__ v,
                             cplx<T>* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nl * s) return;
  const int64_t r = k / s;
  const int c = (int)(k - r * s);
  const cplx<TS> t = v[(int64_t)g[r] * s + c];
  y[k] = cmk((T)t.re, (T)t.im);
}

// forward substitution, one level: y_i -= sum_j l_ij y_j (unit diagonal), in place
template <typename T>
__global__ __launch_bounds__(256) void k_icc_fwd(int cnt, int s, const int32_t* __restrict__ rows,
                                                 const int64_t* __restrict__ lp, const int32_t* __restrict__ lc,
                                                 const cplx<T>* __restrict__ L, cplx<T>* y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)cnt * s) return;
  const int64_t t = k / s;
  const int c = (int)(k - t * s);
  const int64_t i = rows[t];
  cplx<T> acc = y[i * s + c];
  for (int64_t e = lp[i]; e < lp[i + 1]; ++e) cfms(acc, L[e], y[(int64_t)lc[e] * s + c]);
  y[i * s + c] = acc;
}

// scaling and backward substitution, one level: x_i = d_i^{-1} y_i - sum_j l_ji x_j over the
// later rows j that hold column i, in place
template <typename T>
__global__ __launch_bounds__(256) void k_icc_bwd(int cnt, int s, const int32_t* __restrict__ rows,
                                                 const int64_t* __restrict__ up, const int32_t* __restrict__ ur,
                                                 const int64_t* __restrict__ uk, const cplx<T>* __restrict__ L,
                                                 const cplx<T>* __restrict__ dinv, cplx<T>* y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)cnt * s) return;
  const int64_t t = k / s;
  const int c = (int)(k - t * s);
  const int64_t i = rows[t];
  cplx<T> acc = y[i * s + c] * dinv[i];
  for (int64_t e = up[i]; e < up[i + 1]; ++e) cfms(acc, L[uk[e]], y[(int64_t)ur[e] * s + c]);
  y[i * s + c] = acc;
}

// the local solutions into the local vectors (elimination order)
template <typename T>
__global__ void k_icc_store(int64_t nl, int s, const int64_t* __restrict__ out, const cplx<T>* __restrict__ y,
                            cplx<T>* __restrict__ z) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nl * s) return;
  const int64_t r = k / s;
  const int c = (int)(k - r * s);
  z[out[r] * s + c] = y[k];
}

inline unsigned blocks_for(int64_t work) { return (unsigned)std::max<int64_t>(1, (work + 255) / 256); }

// rows grouped by level (counting sort, ascending row within a level)
void group_by_level(const std::vector<int32_t>& lev, int32_t nlev, std::vector<int64_t>& off,
                    std::vector<int32_t>& rows) {
  off.assign((size_t)nlev + 1, 0);
  for (int32_t v : lev) ++off[(size_t)v + 1];
  for (int32_t l = 0; l < nlev; ++l) off[(size_t)l + 1] += off[(size_t)l];
  rows.assign(lev.size(), 0);
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  for (size_t r = 0; r < lev.size(); ++r) rows[(size_t)pos[(size_t)lev[r]]++] = (int32_t)r;
}

template <typename T, typename TS>
void apply_t(Ctx* ctx, Ddm& d, int s, const cplx<TS>* v, cplx<T>* out, cplx<T>* y) {
  HZ_REQUIRE(d.icc, HZ_ERR_STATE, "incomplete factors missing");
  const IccFactor& F = *d.icc;
  hipStream_t st = ctx->stream;
  const int64_t nl = d.n_local_total;
  const cplx<T>* L = F.d_L.as<cplx<T>>();
  const cplx<T>* dinv = F.d_dinv.as<cplx<T>>();
  hipLaunchKernelGGL((k_icc_gather<T, TS>), dim3(blocks_for(nl * s)), dim3(256), 0, st, nl, s, F.d_g.ptr(), v, y);
  for (int32_t l = 0; l < F.n_fwd; ++l) {
    const int cnt = (int)(F.fwd_off[(size_t)l + 1] - F.fwd_off[(size_t)l]);
    hipLaunchKernelGGL((k_icc_fwd<T>), dim3(blocks_for((int64_t)cnt * s)), dim3(256), 0, st, cnt, s,
                       F.d_fwd_rows.ptr() + F.fwd_off[(size_t)l], F.d_lp.ptr(), F.d_lc.ptr(), L, y);
  }
  for (int32_t l = 0; l < F.n_bwd; ++l) {
    const int cnt = (int)(F.bwd_off[(size_t)l + 1] - F.bwd_off[(size_t)l]);
    hipLaunchKernelGGL((k_icc_bwd<T>), dim3(blocks_for((int64_t)cnt * s)), dim3(256), 0, st, cnt, s,
                       F.d_bwd_rows.ptr() + F.bwd_off[(size_t)l], F.d_up.ptr(), F.d_ur.ptr(), F.d_uk.ptr(), L, dinv,
                       y);
  }
  hipLaunchKernelGGL((k_icc_store<T>), dim3(blocks_for(nl * s)), dim3(256), 0, st, nl, s, F.d_out.ptr(), y, out);
  HIP_CHECK(hipGetLastError());
}

}  // namespace

void icc_setup(Ctx* ctx, Ddm& d) {
  HZ_REQUIRE(d.d_lval.ptr() != nullptr, HZ_ERR_STATE, "incomplete factorisation: local operator values missing");
  const int64_t nl = d.n_local_total;
  HZ_REQUIRE(nl < (int64_t)INT32_MAX, HZ_ERR_ARG, "incomplete factorisation: over 2^31 local rows");
  auto F = std::make_unique<IccFactor>();
  // strict lower rows (columns ascending) with the index of each value in the local operator
  // (-1 for a fill position, whose value in A_i is zero), and each row's diagonal entry; with
  // the square pattern a row also holds every earlier column joined to it through one
  // neighbour (the lower pattern of A_i^2).  One subdomain per task of parallel_for (which runs
  // serially for fewer than 4096 tasks, so for any realistic subdomain count).
  const bool square = d.local_solver == HZ_LOCAL_ICC_A2;
  const int64_t ns = (int64_t)d.subs.size();
  std::vector<std::vector<int32_t>> scol((size_t)ns);
  std::vector<std::vector<int64_t>> ssrc((size_t)ns), sptr((size_t)ns);
  std::vector<int64_t> dsrc((size_t)nl, -1);
  parallel_for(ns, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t i = b; i < e; ++i) {
      const Subdomain& S = d.subs[(size_t)i];
      auto& C = scol[(size_t)i];
      auto& R = ssrc[(size_t)i];
      auto& P = sptr[(size_t)i];
      P.assign((size_t)S.n + 1, 0);
      std::vector<int32_t> mark(square ? (size_t)S.n : 0, -1);
      for (int64_t l = 0; l < S.n; ++l) {
        row.clear();
        for (int64_t k = S.rowptr[l]; k < S.rowptr[l + 1]; ++k) {
          const int32_t c = S.col[k];
          if (c < l) {
            row.emplace_back(c, S.csr_off + k);
            if (square) mark[(size_t)c] = (int32_t)l;
          } else if (c == l) {
            dsrc[(size_t)(S.vec_off + l)] = S.csr_off + k;
          }
        }
        if (square)
          for (int64_t k = S.rowptr[l]; k < S.rowptr[l + 1]; ++k) {
            const int32_t j = S.col[k];
            for (int64_t kk = S.rowptr[j]; kk < S.rowptr[j + 1]; ++kk) {
              const int32_t c = S.col[kk];
              if (c < l && mark[(size_t)c] != (int32_t)l) {
                mark[(size_t)c] = (int32_t)l;
                row.emplace_back(c, -1);
              }
            }
          }
        std::sort(row.begin(), row.end());
        for (const auto& pr : row) {
          C.push_back(pr.first);
          R.push_back(pr.second);
        }
        P[(size_t)l + 1] = (int64_t)C.size();
      }
    }
  });
  std::vector<int64_t> lp((size_t)nl + 1, 0);
  {
    int64_t base = 0, rows = 0;
    for (int64_t i = 0; i < ns; ++i) {
      const Subdomain& S = d.subs[(size_t)i];
      HZ_REQUIRE(S.vec_off == rows, HZ_ERR_STATE, "incomplete factorisation: local vectors not contiguous");
      for (int64_t l = 0; l < S.n; ++l) lp[(size_t)(S.vec_off + l)] = base + sptr[(size_t)i][(size_t)l];
      base += (int64_t)scol[(size_t)i].size();
      rows += S.n;
    }
    HZ_REQUIRE(rows == nl, HZ_ERR_STATE, "incomplete factorisation: row count");
    lp[(size_t)nl] = base;
  }
  const int64_t nnz = lp[(size_t)nl];
  std::vector<int32_t> lc((size_t)nnz);
  std::vector<int64_t> src((size_t)nnz);
  parallel_for(ns, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      const Subdomain& S = d.subs[(size_t)i];
      const int64_t o = lp[(size_t)S.vec_off];
      const auto& C = scol[(size_t)i];
      for (size_t q = 0; q < C.size(); ++q) {
        lc[(size_t)o + q] = (int32_t)(S.vec_off + C[q]);
        src[(size_t)o + q] = ssrc[(size_t)i][q];
      }
      std::vector<int32_t>().swap(scol[(size_t)i]);
      std::vector<int64_t>().swap(ssrc[(size_t)i]);
    }
  });
  for (int64_t r = 0; r < nl; ++r)
    HZ_REQUIRE(dsrc[(size_t)r] >= 0, HZ_ERR_STATE, "incomplete factorisation: row without diagonal");
  // the same entries by column: the rows of L^T (rows ascending within a column)
  std::vector<int64_t> up((size_t)nl + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) ++up[(size_t)lc[(size_t)e] + 1];
  for (int64_t r = 0; r < nl; ++r) up[(size_t)r + 1] += up[(size_t)r];
  std::vector<int32_t> ur((size_t)nnz);
  std::vector<int64_t> uk((size_t)nnz);
  {
    std::vector<int64_t> pos(up.begin(), up.end() - 1);
    for (int64_t r = 0; r < nl; ++r)
      for (int64_t e = lp[(size_t)r]; e < lp[(size_t)r + 1]; ++e) {
        const int64_t q = pos[(size_t)lc[(size_t)e]]++;
        ur[(size_t)q] = (int32_t)r;
        uk[(size_t)q] = e;
      }
  }
  // dependency levels: forward (and factorisation) from the columns a row reads, backward from
  // the later rows that read it
  std::vector<int32_t> flev((size_t)nl, 0), blev((size_t)nl, 0);
  int32_t nf = 0, nb = 0;
  for (int64_t r = 0; r < nl; ++r) {
    int32_t m = -1;
    for (int64_t e = lp[(size_t)r]; e < lp[(size_t)r + 1]; ++e) m = std::max(m, flev[(size_t)lc[(size_t)e]]);
    flev[(size_t)r] = m + 1;
    nf = std::max(nf, m + 2);
  }
  for (int64_t r = nl; r-- > 0;) {
    int32_t m = -1;
    for (int64_t e = up[(size_t)r]; e < up[(size_t)r + 1]; ++e) m = std::max(m, blev[(size_t)ur[(size_t)e]]);
    blev[(size_t)r] = m + 1;
    nb = std::max(nb, m + 2);
  }
  std::vector<int32_t> frows, brows;
  group_by_level(flev, nf, F->fwd_off, frows);
  group_by_level(blev, nb, F->bwd_off, brows);
  F->n_fwd = nf;
  F->n_bwd = nb;
  F->nnz = nnz;
  // row -> global dof, row -> local vector position (elimination order)
  std::vector<int32_t> g((size_t)nl);
  std::vector<int64_t> out((size_t)nl);
  for (const Subdomain& S : d.subs)
    for (int64_t l = 0; l < S.n; ++l) {
      g[(size_t)(S.vec_off + l)] = S.gdofs[(size_t)l];
      out[(size_t)(S.vec_off + l)] = S.vec_off + S.ipos[(size_t)l];
    }
  F->d_lp.upload(ctx, lp);
  F->d_lc.upload(ctx, lc);
  F->d_up.upload(ctx, up);
  F->d_ur.upload(ctx, ur);
  F->d_uk.upload(ctx, uk);
  F->d_fwd_rows.upload(ctx, frows);
  F->d_bwd_rows.upload(ctx, brows);
  F->d_g.upload(ctx, g);
  F->d_out.upload(ctx, out);
  // numeric factorisation in FP64, level by level
  hipStream_t st = ctx->stream;
  const auto t0 = std::chrono::steady_clock::now();
  {
    DevArray<int64_t> d_src, d_dsrc;
    d_src.upload(ctx, src);
    d_dsrc.upload(ctx, dsrc);
    DevArray<c128> Lw, dg;
    Lw.alloc(ctx, (size_t)std::max<int64_t>(1, nnz));
    dg.alloc(ctx, (size_t)std::max<int64_t>(1, nl));
    DevArray<int> bad;
    bad.alloc(ctx, 1);
    HIP_CHECK(hipMemsetAsync(bad.ptr(), 0, sizeof(int), st));
    for (int32_t l = 0; l < nf; ++l) {
      const int cnt = (int)(F->fwd_off[(size_t)l + 1] - F->fwd_off[(size_t)l]);
      hipLaunchKernelGGL(k_icc_factor, dim3(blocks_for(cnt)), dim3(256), 0, st, cnt,
                         F->d_fwd_rows.ptr() + F->fwd_off[(size_t)l], F->d_lp.ptr(), F->d_lc.ptr(), d_src.ptr(),
                         d_dsrc.ptr(), d.d_lval.ptr(), Lw.ptr(), dg.ptr(), bad.ptr());
    }
    HIP_CHECK(hipGetLastError());
    int hbad = 0;
    HIP_CHECK(hipMemcpyAsync(&hbad, bad.ptr(), sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    HZ_REQUIRE(hbad == 0, HZ_ERR_SINGULAR, "incomplete factorisation: zero or non-finite pivot");
    const bool single = d.precision == HZ_PREC_MIXED;
    const size_t esz = single ? sizeof(c64) : sizeof(c128);
    F->d_L.alloc(ctx, (size_t)std::max<int64_t>(1, nnz) * esz);
    F->d_dinv.alloc(ctx, (size_t)std::max<int64_t>(1, nl) * esz);
    const unsigned nblk = blocks_for(std::max(nnz, nl));
    if (single)
      hipLaunchKernelGGL((k_icc_store_factors<float>), dim3(nblk), dim3(256), 0, st, nnz, nl, Lw.ptr(), dg.ptr(),
                         F->d_L.as<c64>(), F->d_dinv.as<c64>());
    else
      hipLaunchKernelGGL((k_icc_store_factors<double>), dim3(nblk), dim3(256), 0, st, nnz, nl, Lw.ptr(), dg.ptr(),
                         F->d_L.as<c128>(), F->d_dinv.as<c128>());
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
  }
  d.factor_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  d.factor_flops = 0;
  d.icc = std::move(F);
}

void icc_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* out, c128* y) { apply_t<double, double>(ctx, d, s, v, out, y); }
void icc_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c64* out, c64* y) { apply_t<float, double>(ctx, d, s, v, out, y); }
void icc_apply(Ctx* ctx, Ddm& d, int s, const c64* v, c64* out, c64* y) { apply_t<float, float>(ctx, d, s, v, out, y); }

}  // namespace hz
