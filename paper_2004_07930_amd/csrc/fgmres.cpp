// Block FGMRES(m) as a resumable job (host control flow; all arithmetic in krylov.hip /
// spmm.hip / oras.hip kernels).  One Arnoldi process per right-hand-side block:
//   cycle:  R = B - A X ; [V_1, S] = CholQR2(R) ; G = [S; 0]
//   step j: Z_j = M^{-1} V~_j (stored in complex64 with the mixed-precision preconditioner:
//           the flexible method multiplies and combines exactly the stored Z_j) ; W = A Z_j ;
//           orthogonalisation of W against the basis ; Householder update of the block
//           Hessenberg QR applied to G ; per-column residual estimate |G_{j+1}| / |b|
//   end:    Y = R^{-1} G ; X += Z Y ; explicit residual decides restart.
// Orthogonalisation, 16 or 32 columns: delayed reorthogonalisation (DCGS2).  W is projected once
// (W' = W - V V^H W); W' scaled by diag(R_j)^{-1} (R_j: the triangular factor that normalised
// V_j; the scale of each step's block then does not compound) is the block V~_{j+1} that the
// next step preconditions, and that step projects it again and normalises it (V_{j+1}) in the
// same passes over the basis that project its own product.  So each step reads the basis twice (one Gram product, one
// update) instead of four times, and column j of the Hessenberg matrix is complete one step
// later: the convergence test of column j runs at step j + 1, and the step known to be the
// cycle's last finishes its own column with one more Gram product.  The flexible method
// accepts Z_j = M^{-1} V~_j: A Z = V H holds for any Z, and x = Z y.
// Other widths: two passes of H = V^H W, W -= V H (CGS2), then [V_{j+1}, H_{j+1,j}] = CholQR2(W).
// hz_solve drives a job step by step; the serving scheduler interleaves many jobs and
// packs their Z_j = M^{-1} V~_j and W = A Z_j products into shared launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <type_traits>

#include "krylov.h"
#include "prof.h"

namespace hz {

// workspace layout of a job: every array at a 256-byte boundary
int64_t FgmresJob::carve(char* base) {
  const int64_t ns = n * s;
  int64_t off = 0;
  auto take = [&](auto& arr, int64_t count) {
    using T = std::remove_pointer_t<decltype(arr.p)>;
    arr.p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (std::max<int64_t>(1, count) * (int64_t)sizeof(T) + 255) / 256 * 256;
  };
  take(V, (m + 1) * ns);
  if (z32)
    take(Zs, m * ns);
  else
    take(Zb, m * ns);
  take(W, ns);
  take(Wt, ns);
  take(R, ns);
  take(part, (int64_t)K.nchunk * (m + 2) * s * s * (dcgs ? 2 : 1));
  take(Hc, (int64_t)(m + 2) * s * s);
  if (dcgs) {
    take(Hc2, (int64_t)(m + 2) * s * s);
    take(Gm, (int64_t)(m + 2) * s * 2 * s);
    take(Cm, (int64_t)(m + 2) * s * 2 * s);
    take(Rprev, (int64_t)s * s);
  } else {
    take(Hp, (int64_t)(m + 1) * s * s);
  }
  take(Rm, (int64_t)m * s * ldr);
  take(refl, (int64_t)m * 2 * s * s);
  take(tau, (int64_t)m * s);
  take(tmat, (int64_t)m * s * s);
  take(G, ldr * s);
  take(Y, (int64_t)m * s * s);
  take(Gs, s * s);
  take(Rs, s * s);
  take(Ri, s * s);
  take(Racc, s * s);
  take(res, s);
  take(npart, (int64_t)K.nchunk * s);
  take(nrm, s);
  take(flag, 2);
  return off;
}

int64_t FgmresJob::bytes_needed(int64_t n, int s, int m, bool z32) {
  // the same layout as carve(): 26 arrays, each padded to 256 bytes
  const int64_t ns = n * s;
  const int nchunk = (int)((n + 4095) / 4096);
  const int64_t ldr = (int64_t)(m + 1) * s;
  const int64_t pw = delayed(s) ? 2 : 1;                  // Gram products of width 2s
  int64_t e = ((int64_t)m + 4) * ns;                      // V, W, Wt, R
  e += (int64_t)nchunk * (m + 2) * s * s * pw;            // partial sums
  e += (int64_t)(2 * m + 3) * s * s + (int64_t)m * s * ldr + 3 * (int64_t)m * s * s + ldr * s + 8 * s * s;
  if (delayed(s)) e += (int64_t)(m + 3) * s * s + 2 * (int64_t)(m + 2) * s * 2 * s;  // Hc2, Rprev, Gm, Cm
  return e * (int64_t)sizeof(c128) + (int64_t)m * ns * (int64_t)(z32 ? sizeof(c64) : sizeof(c128)) + 26 * 256;
}

int FgmresJob::restart_fit(Ctx* ctx, int64_t n, int s, int want, int fixed, bool z32, int64_t extra) {
  int m = std::max(1, want);
  if (fixed > 0) m = std::max(m, fixed);
  size_t fr = 0, tot = 0;
  HIP_CHECK(hipMemGetInfo(&fr, &tot));
  // the context's cached workspace is free for the next job
  const double cached = (ctx->krylov_busy ? 0.0 : (double)ctx->krylov_ws.bytes) + (double)ctx->krylov_io.bytes;
  const double avail = 0.8 * ((double)fr + cached);
  const int floor_m = fixed > 0 ? m : std::min(m, kMinRestart);
  for (int k = m; k >= floor_m; --k)
    if ((double)(bytes_needed(n, s, k, z32) + extra) <= avail) return k;
  return 0;
}

void krylov_cache_release(Ctx* ctx) {
  if (!ctx->krylov_busy) ctx->krylov_ws.release();
  ctx->krylov_io.release();
}

FgmresJob::FgmresJob(Ctx* c, std::shared_ptr<Ddm> dd, int s_, const c128* B_, c128* X_, const SolveOptions& o_, int m_,
                     bool use_cache)
    : ctx(c),
      d(std::move(dd)),
      s(s_),
      B(B_),
      X(X_),
      o(o_),
      m(m_),
      n(d->op->mesh->n),
      K(c, d->op->mesh->n, s_),
      z32(d->precision == HZ_PREC_MIXED),
      dcgs(delayed(s_)) {
  HZ_REQUIRE(s >= 1 && s <= 32, HZ_ERR_ARG, "fgmres: block size must be 1..32");
  ldr = (int64_t)(m + 1) * s;
  const int64_t total = carve(nullptr);
  char* base = nullptr;
  if (use_cache && !ctx->krylov_busy) {
    if ((int64_t)ctx->krylov_ws.bytes < total) {
      ctx->krylov_ws.release();
      ctx->krylov_ws.alloc(ctx, (size_t)total);
    }
    base = ctx->krylov_ws.as<char>();
    ctx->krylov_busy = true;
    ws_cached = true;
  } else {
    ws_own.alloc(ctx, (size_t)total);
    base = ws_own.as<char>();
  }
  carve(base);
  bnorm.assign(s, 0.0);
  est.alloc(s);
  hflags.alloc(2);
  rel.assign(s, 0.0);
  if (dcgs) {
    HIP_CHECK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  }
}

FgmresJob::~FgmresJob() {
  if (ws_cached) {  // the workspace stays with the context; the stream orders its next use
    if (side) (void)hipStreamSynchronize(side);
    ctx->krylov_busy = false;
  }
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
  }
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
}

void FgmresJob::spmm(const c128* x, c128* y, c128 alpha, c128 beta, const c128* yin) {
  const Operator& op = *d->op;
  const double nnz = (double)op.nnz();
  // algorithmic traffic: CSR once (16 B value + 4 B column per nonzero, 8 B row pointer per
  // row), x once, y written once (+ yin read once)
  const double vec = (double)n * s * sizeof(c128);
  ProfScope ps(ctx, HZ_K_SPMM, 20.0 * nnz + 8.0 * (n + 1) + (yin ? 3.0 : 2.0) * vec, 8.0 * nnz * s);
  launch_spmm<double>(ctx->stream, n, s, op.mesh->d_rowptr.ptr(), op.mesh->d_col.ptr(), op.d_val.ptr(), x, y, alpha,
                      beta, yin);
}

void FgmresJob::spmm_z(const c64* z, c128* w) {
  const Operator& op = *d->op;
  const double nnz = (double)op.nnz();
  const double vec = (double)n * s;
  ProfScope ps(ctx, HZ_K_SPMM, 20.0 * nnz + 8.0 * (n + 1) + vec * (sizeof(c64) + sizeof(c128)), 8.0 * nnz * s);
  launch_spmm<float>(ctx->stream, n, s, op.mesh->d_rowptr.ptr(), op.mesh->d_col.ptr(), op.d_val.ptr(), z, w,
                     cmk(1.0, 0.0), cmk(0.0, 0.0), nullptr);
}

void FgmresJob::matvec() {
  if (z32) {
    precond_apply(ctx, *d, s, v_cur(), z32_cur());
    spmm_z(z32_cur(), w_cur());
  } else {
    precond_apply(ctx, *d, s, v_cur(), z_cur());
    spmm(z_cur(), w_cur(), cmk(1.0, 0.0), cmk(0.0, 0.0), nullptr);
  }
}

void FgmresJob::cholqr2(const c128* in, c128* out) {
  K.identity(Racc.ptr());
  K.cholqr_pass(in, Wt.ptr(), part.ptr(), Gs.ptr(), Rs.ptr(), Ri.ptr(), Racc.ptr(), flag.ptr());
  K.cholqr_pass(Wt.ptr(), out, part.ptr(), Gs.ptr(), Rs.ptr(), Ri.ptr(), Racc.ptr(), flag.ptr());
}

void FgmresJob::start() {
  hipStream_t st = ctx->stream;
  HIP_CHECK(hipMemsetAsync(flag.ptr(), 0, 2 * sizeof(int), st));
  K.colnorms(B, npart.ptr(), nrm.ptr());
  HIP_CHECK(hipMemcpyAsync(bnorm.data(), nrm.ptr(), s * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int c = 0; c < s; ++c) {
    HZ_REQUIRE(std::isfinite(bnorm[c]), HZ_ERR_ARG, "hz_solve: non-finite right-hand side");
    HZ_REQUIRE(bnorm[c] > 0, HZ_ERR_ARG, "hz_solve: zero right-hand side column (solve it separately: x = 0)");
  }
  HIP_CHECK(hipMemsetAsync(X, 0, n * s * sizeof(c128), st));
  total = 0;
  base = 0;
  restarts = 0;
  start_cycle();
  HIP_CHECK(hipMemcpyAsync(hflags.p, flag.ptr(), sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  HZ_REQUIRE(hflags[0] == 0, HZ_ERR_ARG,
             "hz_solve: the right-hand-side block is numerically rank deficient (dependent columns): "
             "solve such columns in separate blocks");
}

void FgmresJob::start_cycle() {
  hipStream_t st = ctx->stream;
  const c128 one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  HIP_CHECK(hipMemsetAsync(flag.ptr(), 0, 2 * sizeof(int), st));
  if (total == 0)
    HIP_CHECK(hipMemcpyAsync(R.ptr(), B, n * s * sizeof(c128), hipMemcpyDeviceToDevice, st));
  else
    spmm(X, R.ptr(), mone, one, B);
  cholqr2(R.ptr(), V.ptr());
  HIP_CHECK(hipMemsetAsync(G.ptr(), 0, ldr * s * sizeof(c128), st));
  HIP_CHECK(hipMemcpyAsync(G.ptr(), Racc.ptr(), s * s * sizeof(c128), hipMemcpyDeviceToDevice, st));
  jj = 0;
  base = total;
}

// delayed reorthogonalisation: step j >= 1 preconditions V~_j, the once-projected product of
// step j - 1, kept in W (j even) or Wt (j odd); A Z_j goes to the other one and is projected
// in place, becoming V~_{j+1}
c128* FgmresJob::v_cur() {
  if (dcgs && jj > 0) return (jj & 1) ? Wt.ptr() : W.ptr();
  return V.ptr() + jj * n * s;
}
c128* FgmresJob::h_col(int j) { return (dcgs && (j & 1)) ? Hc2.ptr() : Hc.ptr(); }
c128* FgmresJob::z_cur() { return z32 ? nullptr : Zb.ptr() + jj * n * s; }
c64* FgmresJob::z32_cur() { return z32 ? Zs.ptr() + jj * n * s : nullptr; }
c128* FgmresJob::w_cur() { return (dcgs && !(jj & 1)) ? Wt.ptr() : W.ptr(); }

void FgmresJob::after_matvec() {
  hipStream_t st = ctx->stream;
  const int64_t ns = n * s;
  last = jj + 1 >= m || (o.fixed_iters > 0 ? jj + 1 >= o.fixed_iters : base + jj + 1 >= o.max_iter);
  if (!dcgs) {
    // CGS2
    K.gram(jj + 1, V.ptr(), ns, W.ptr(), part.ptr(), Hc.ptr(), false);
    K.block_axpy(jj + 1, V.ptr(), ns, Hc.ptr(), -1.0, W.ptr(), W.ptr());
    K.gram(jj + 1, V.ptr(), ns, W.ptr(), part.ptr(), Hp.ptr(), false, Hc.ptr());
    K.block_axpy(jj + 1, V.ptr(), ns, Hp.ptr(), -1.0, W.ptr(), W.ptr());
    // V_{j+1} R = W
    cholqr2(W.ptr(), V.ptr() + (jj + 1) * ns);
    HIP_CHECK(hipMemcpyAsync(Hc.ptr() + (int64_t)(jj + 1) * s * s, Racc.ptr(), s * s * sizeof(c128),
                             hipMemcpyDeviceToDevice, st));
    K.lsq_step(jj, Hc.ptr(), Rm.ptr(), ldr, refl.ptr(), tau.ptr(), tmat.ptr(), G.ptr(), res.ptr());
  } else {
    c128* w = w_cur();
    c128* hn = h_col(jj);
    if (jj == 0) {  // V_0 is final (CholQR2 of the residual): one projection, V~_1 = W'
      K.identity(Rprev.ptr());
      K.gram(1, V.ptr(), ns, w, part.ptr(), hn, false);
      K.block_axpy(1, V.ptr(), ns, hn, -1.0, w, w);
    } else {
      // [V_<j, V~_j]^H [V~_j, W], the coefficients, then V_j and V~_{j+1} = W' diag(R_j)^{-1} in
      // one update (written over W)
      c128* vt = v_cur();
      c128* hp = h_col(jj - 1);
      K.gram_ext(jj + 1, V.ptr(), ns, jj, vt, vt, w, part.ptr(), Gm.ptr(), false);
      K.dcgs_coef(jj * s, Gm.ptr(), Cm.ptr(), hp, hn, Rprev.ptr(), flag.ptr());
      // column j - 1 is complete: its least-squares step runs beside the update
      HIP_CHECK(hipEventRecord(ev_fork, st));
      HIP_CHECK(hipStreamWaitEvent(side, ev_fork, 0));
      K.lsq_step(jj - 1, hp, Rm.ptr(), ldr, refl.ptr(), tau.ptr(), tmat.ptr(), G.ptr(), res.ptr(), side);
      HIP_CHECK(hipEventRecord(ev_join, side));
      K.update_split(jj, V.ptr(), ns, vt, w, Cm.ptr(), V.ptr() + jj * ns, w);
      HIP_CHECK(hipStreamWaitEvent(st, ev_join, 0));
    }
    if (last) {  // finish column j: [V_<=j, V~_{j+1}]^H V~_{j+1}
      K.gram_ext(jj + 2, V.ptr(), ns, jj + 1, w, w, nullptr, part.ptr(), Gm.ptr(), false);
      K.dcgs_coef((jj + 1) * s, Gm.ptr(), nullptr, nullptr, hn, Rprev.ptr(), flag.ptr() + 1);
      K.lsq_step(jj, hn, Rm.ptr(), ldr, refl.ptr(), tau.ptr(), tmat.ptr(), G.ptr(), res.ptr());
    }
  }
  HIP_CHECK(hipMemcpyAsync(est.p, res.ptr(), s * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipMemcpyAsync(hflags.p, flag.ptr(), 2 * sizeof(int), hipMemcpyDeviceToHost, st));
}

bool FgmresJob::cycle_done() {
  // the caller has synchronised the stream since after_matvec()
  // a breakdown (a new block numerically dependent on the basis: the Krylov space is exhausted
  // for some column) ends the cycle at the column whose subdiagonal block it gives: with CGS2
  // and the finishing pass that is column j; with the delayed form's step j it is column j - 1,
  // and column j (built from the dependent block) is dropped
  const bool brk = hflags[0] != 0, brk_fin = hflags[1] != 0;
  // Hessenberg columns complete in this cycle (the estimate refers to the last of them)
  const int done = !dcgs ? jj + 1 : brk ? jj : last ? jj + 1 : jj;
  total = base + done;
  bool conv = done > 0;
  for (int c = 0; c < s; ++c) conv = conv && (est[c] / bnorm[c] <= o.tol);
  const bool end = brk || brk_fin || last || (o.fixed_iters <= 0 && conv);
  if (end)
    ncols = done;
  else
    ++jj;
  return end;
}

void FgmresJob::trace_step() const {
  // est[] refers to the latest completed Hessenberg column (one step late in the delayed form)
  double mx = 0;
  for (int c = 0; c < s; ++c) mx = std::max(mx, est[c] / bnorm[c]);
  std::fprintf(stderr, "hz: step  n=%lld s=%d m=%d cycle-step=%d completed=%d est max rel residual %.3e%s\n",
               (long long)n, s, m, jj, total, mx, (hflags[0] || hflags[1]) ? " (breakdown)" : "");
}

bool FgmresJob::end_cycle() {
  hipStream_t st = ctx->stream;
  const c128 one = cmk(1.0, 0.0), mone = cmk(-1.0, 0.0);
  const int J = ncols * s;
  K.lsq_solve(J, Rm.ptr(), ldr, G.ptr(), Y.ptr());
  if (z32)
    K.block_axpy(ncols, Zs.ptr(), n * s, Y.ptr(), 1.0, X, X);
  else
    K.block_axpy(ncols, Zb.ptr(), n * s, Y.ptr(), 1.0, X, X);
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
  if (!(o.fixed_iters > 0 || conv || total >= o.max_iter)) {
    ++restarts;
    start_cycle();
    HIP_CHECK(hipMemcpyAsync(hflags.p, flag.ptr(), sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (hflags[0] == 0) return false;
    // the new residual block is numerically rank deficient: no further cycle can start, and
    // the columns are reported as they stand
  }
  if (ctx->trace) {
    double mx = 0;
    for (int c = 0; c < s; ++c) mx = std::max(mx, rel[c]);
    std::fprintf(stderr, "hz: cycle end  n=%lld s=%d m=%d iters=%d restarts=%d explicit max rel residual %.3e\n",
                 (long long)n, s, m, total, restarts, mx);
  }
  info.assign(s, ColInfo{});
  for (int c = 0; c < s; ++c) {
    info[c].m = m;
    info[c].block = s;
    info[c].iters = total;
    info[c].restarts = restarts;
    info[c].rel_residual = rel[c];
    info[c].status = (o.fixed_iters > 0 || rel[c] <= o.tol) ? HZ_OK : HZ_ERR_NOT_CONVERGED;
  }
  return true;
}

void fgmres(Ctx* ctx, std::shared_ptr<Ddm> d, int s, const c128* B, c128* X, const SolveOptions& o, int m,
            std::vector<ColInfo>& info) {
  FgmresJob job(ctx, d, s, B, X, o, m, /*use_cache=*/true);
  job.start();
  // each cycle completes at least one column with at most one step more than it completes
  const int limit = 2 * (o.fixed_iters > 0 ? o.fixed_iters : o.max_iter) + 1;
  for (int it = 0;; ++it) {
    HZ_REQUIRE(it <= limit, HZ_ERR_STATE, "fgmres: iteration bookkeeping error");
    job.matvec();
    job.after_matvec();
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    const bool cyc = job.cycle_done();
    if (ctx->trace) job.trace_step();
    if (cyc && job.end_cycle()) break;
  }
  info = job.info;
}

}  // namespace hz
