// Block FGMRES(m) driver (host control flow, all arithmetic in krylov.hip / spmm.hip /
// oras.hip kernels).  One Arnoldi process per right-hand-side block:
//   cycle:  R = B - A X ; [V_1, S] = CholQR2(R) ; G = [S; 0]
//   step j: Z_j = M^{-1} V_j ; W = A Z_j ; two passes of H = V^H W, W -= V H (CGS2) ;
//           [V_{j+1}, H_{j+1,j}] = CholQR2(W) ; Householder update of the block Hessenberg
//           QR applied to G ; per-column residual estimate |G_{j+1}| / |b|
//   end:    Y = R^{-1} G ; X += Z Y ; explicit residual decides restart.
#include <algorithm>
#include <cmath>

#include "krylov.h"
#include "prof.h"

namespace hz {

void fgmres(Ctx* ctx, Ddm& d, int s, const c128* B, c128* X, const SolveOptions& o, std::vector<ColInfo>& info) {
  const Operator& op = *d.op;
  const int64_t n = op.mesh->n;
  hipStream_t st = ctx->stream;
  HZ_REQUIRE(s >= 1 && s <= 32, HZ_ERR_ARG, "fgmres: block size must be 1..32");
  int m = std::max(1, o.restart);
  if (o.fixed_iters > 0) m = std::max(m, o.fixed_iters);
  {  // cap the restart length by free device memory: (2m + 4) n s 16 bytes
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const double per = (double)n * s * sizeof(c128);
    const int mcap = (int)std::floor((0.8 * (double)fr / per - 4.0) / 2.0);
    HZ_REQUIRE(mcap >= 1, HZ_ERR_OOM, "fgmres: not enough device memory for one Krylov step");
    if (o.fixed_iters > 0) HZ_REQUIRE(mcap >= o.fixed_iters, HZ_ERR_OOM, "fgmres: fixed_iters exceeds memory");
    m = std::min(m, mcap);
  }
  KrylovKernels K(ctx, n, s);
  const int64_t ns = n * s;
  const int64_t ldr = (int64_t)(m + 1) * s;
  DevArray<c128> V, Zb, W, Wt, R, part, Hc, Hp, Rm, refl, tau, G, Y, Gs, Rs, Ri, Racc;
  DevArray<double> res, npart, nrm;
  DevArray<int> flag;
  V.alloc(ctx, (m + 1) * ns);
  Zb.alloc(ctx, m * ns);
  W.alloc(ctx, ns);
  Wt.alloc(ctx, ns);
  R.alloc(ctx, ns);
  part.alloc(ctx, (int64_t)K.nchunk * (m + 1) * s * s);
  Hc.alloc(ctx, (int64_t)(m + 2) * s * s);
  Hp.alloc(ctx, (int64_t)(m + 1) * s * s);
  Rm.alloc(ctx, (int64_t)m * s * ldr);
  refl.alloc(ctx, (int64_t)m * 2 * s * s);
  tau.alloc(ctx, (int64_t)m * s);
  G.alloc(ctx, ldr * s);
  Y.alloc(ctx, (int64_t)m * s * s);
  Gs.alloc(ctx, s * s);
  Rs.alloc(ctx, s * s);
  Ri.alloc(ctx, s * s);
  Racc.alloc(ctx, s * s);
  res.alloc(ctx, s);
  npart.alloc(ctx, (int64_t)K.nchunk * s);
  nrm.alloc(ctx, s);
  flag.alloc(ctx, 1);
  HIP_CHECK(hipMemsetAsync(flag.ptr(), 0, sizeof(int), st));

  std::vector<double> bnorm(s), est(s), rel(s);
  K.colnorms(B, npart.ptr(), nrm.ptr());
  HIP_CHECK(hipMemcpyAsync(bnorm.data(), nrm.ptr(), s * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int c = 0; c < s; ++c) {
    HZ_REQUIRE(std::isfinite(bnorm[c]), HZ_ERR_ARG, "hz_solve: non-finite right-hand side");
    HZ_REQUIRE(bnorm[c] > 0, HZ_ERR_ARG, "hz_solve: zero right-hand side column (solve it separately: x = 0)");
  }
  HIP_CHECK(hipMemsetAsync(X, 0, ns * sizeof(c128), st));

  auto cholqr2 = [&](const c128* in, c128* out) {
    K.identity(Racc.ptr());
    K.cholqr_pass(in, Wt.ptr(), part.ptr(), Gs.ptr(), Rs.ptr(), Ri.ptr(), Racc.ptr(), flag.ptr());
    K.cholqr_pass(Wt.ptr(), out, part.ptr(), Gs.ptr(), Rs.ptr(), Ri.ptr(), Racc.ptr(), flag.ptr());
  };
  const c128 one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0), mone = cmk(-1.0, 0.0);
  const double nnz = (double)op.nnz();
  // y = alpha A x + beta yin ; algorithmic traffic: CSR once (16 B value + 4 B column per
  // nonzero, 8 B row pointer per row), x once, y written once (+ yin read once)
  auto spmm = [&](const c128* x, c128* y, c128 alpha, c128 beta, const c128* yin) {
    const double vec = (double)n * s * sizeof(c128);
    ProfScope ps(ctx, HZ_K_SPMM, 20.0 * nnz + 8.0 * (n + 1) + (yin ? 3.0 : 2.0) * vec, 8.0 * nnz * s);
    launch_spmm<double>(st, n, s, op.mesh->d_rowptr.ptr(), op.mesh->d_col.ptr(), op.d_val.ptr(), x, y, alpha, beta,
                        yin);
  };
  int total = 0, restarts = 0;
  for (;;) {
    // R = B - A X
    if (total == 0)
      HIP_CHECK(hipMemcpyAsync(R.ptr(), B, ns * sizeof(c128), hipMemcpyDeviceToDevice, st));
    else
      spmm(X, R.ptr(), mone, one, B);
    cholqr2(R.ptr(), V.ptr());
    HIP_CHECK(hipMemsetAsync(G.ptr(), 0, ldr * s * sizeof(c128), st));
    HIP_CHECK(hipMemcpyAsync(G.ptr(), Racc.ptr(), s * s * sizeof(c128), hipMemcpyDeviceToDevice, st));
    int jj = 0;
    for (;; ++jj) {
      c128* Vj = V.ptr() + jj * ns;
      c128* Zj = Zb.ptr() + jj * ns;
      precond_apply(ctx, d, s, Vj, Zj);
      spmm(Zj, W.ptr(), one, zero, nullptr);
      // CGS2
      K.gram(jj + 1, V.ptr(), ns, W.ptr(), part.ptr(), Hc.ptr(), false);
      K.block_axpy(jj + 1, V.ptr(), ns, Hc.ptr(), -1.0, W.ptr(), W.ptr());
      K.gram(jj + 1, V.ptr(), ns, W.ptr(), part.ptr(), Hp.ptr(), false, Hc.ptr());
      K.block_axpy(jj + 1, V.ptr(), ns, Hp.ptr(), -1.0, W.ptr(), W.ptr());
      // V_{j+1} R = W
      cholqr2(W.ptr(), V.ptr() + (jj + 1) * ns);
      HIP_CHECK(hipMemcpyAsync(Hc.ptr() + (int64_t)(jj + 1) * s * s, Racc.ptr(), s * s * sizeof(c128),
                               hipMemcpyDeviceToDevice, st));
      K.lsq_step(jj, Hc.ptr(), Rm.ptr(), ldr, refl.ptr(), tau.ptr(), G.ptr(), res.ptr());
      HIP_CHECK(hipMemcpyAsync(est.data(), res.ptr(), s * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      ++total;
      bool conv = true;
      for (int c = 0; c < s; ++c) conv = conv && (est[c] / bnorm[c] <= o.tol);
      if (o.fixed_iters > 0) {
        if (jj + 1 >= o.fixed_iters) break;
      } else if (conv || total >= o.max_iter || jj + 1 >= m) {
        break;
      }
    }
    const int J = (jj + 1) * s;
    K.lsq_solve(J, Rm.ptr(), ldr, G.ptr(), Y.ptr());
    K.block_axpy(jj + 1, Zb.ptr(), ns, Y.ptr(), 1.0, X, X);
    spmm(X, R.ptr(), mone, one, B);
    K.colnorms(R.ptr(), npart.ptr(), nrm.ptr());
    std::vector<double> rn(s);
    HIP_CHECK(hipMemcpyAsync(rn.data(), nrm.ptr(), s * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    bool conv = true;
    for (int c = 0; c < s; ++c) {
      rel[c] = rn[c] / bnorm[c];
      conv = conv && rel[c] <= o.tol;
    }
    if (o.fixed_iters > 0 || conv || total >= o.max_iter) {
      info.assign(s, ColInfo{});
      for (int c = 0; c < s; ++c) {
        info[c].iters = total;
        info[c].restarts = restarts;
        info[c].rel_residual = rel[c];
        info[c].status = (o.fixed_iters > 0 || rel[c] <= o.tol) ? HZ_OK : HZ_ERR_NOT_CONVERGED;
      }
      return;
    }
    ++restarts;
  }
}

}  // namespace hz
