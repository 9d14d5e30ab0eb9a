// Host-side launchers of the FP64 Krylov kernels (krylov.hip) and the block FGMRES driver.
#pragma once

#include "ddm.h"

namespace hz {

struct KrylovKernels {
  Ctx* ctx;
  int64_t n;
  int s;
  int nchunk;
  KrylovKernels(Ctx* c, int64_t n_, int s_);
  void to_node(const c128* src, c128* dst);
  void to_node(const c64* src, c64* dst);
  void from_node(const c128* src, c128* dst);
  // H[J][c] (+)= sum_rows conj(V_J) W   for J < nblk * s ; partial buffer >= nchunk * nblk * s * s;
  // if H2 is given the same sums are also added into it
  void gram(int nblk, const c128* V, int64_t ldv, const c128* W, c128* part, c128* H, bool accumulate,
            c128* H2 = nullptr);
  // the same with the basis blocks b < nvb at V + b ldv and block nvb at Vx (Jtot = (nblk) s
  // columns in all), and a right operand of two blocks [W0, W1] when W1 is given (H then has
  // 2s columns); split operands need s = 16 or 32
  void gram_ext(int nblk, const c128* V, int64_t ldv, int nvb, const c128* Vx, const c128* W0, const c128* W1,
                c128* part, c128* H, bool accumulate, c128* H2 = nullptr);
  // [Y0, Y1] = [V_0 .. V_{nvb-1}, Vx, Vx2] C, C ((nvb + 2) s x 2s); Y1 may be Vx2; s = 16 or 32
  void update_split(int nvb, const c128* V, int64_t ldv, const c128* Vx, const c128* Vx2, const c128* C, c128* Y0,
                    c128* Y1);
  // delayed-reorthogonalisation coefficients (k_dcgs_coef): C null finishes a column; Rprev is
  // the triangular factor that scaled the block being completed (updated by the fused form)
  void dcgs_coef(int nb, const c128* G, c128* C, c128* Hp, c128* Hn, c128* Rprev, int* flag);
  // Y = Yin + beta * sum_J V_J H[J][:]
  void block_axpy(int nblk, const c128* V, int64_t ldv, const c128* H, double beta, const c128* Yin, c128* Y);
  // the same with complex64 basis blocks (widened exactly)
  void block_axpy(int nblk, const c64* V, int64_t ldv, const c128* H, double beta, const c128* Yin, c128* Y);
  // one CholQR pass: G = W^H W = R^H R, out = W R^{-1}, Racc = R Racc
  void cholqr_pass(const c128* W, c128* out, c128* part, c128* G, c128* R, c128* Rinv, c128* Racc, int* flag);
  void identity(c128* M);
  // block Hessenberg QR step jj: refl/tau/tmat hold each block's reflectors and its T factor
  // (on `stream` when given, else the context's stream)
  void lsq_step(int jj, c128* Hc, c128* Rm, int64_t ldr, c128* refl, c128* tau, c128* tmat, c128* G, double* res,
                hipStream_t stream = nullptr);
  void lsq_solve(int J, const c128* Rm, int64_t ldr, const c128* G, c128* Y);
  void colnorms(const c128* X, double* part, double* out);
};

// number of entries of a complex128 array with a non-finite real or imaginary part
int64_t count_nonfinite(Ctx* ctx, const c128* x, int64_t m);

struct SolveOptions {
  double tol = 1e-6;
  int max_iter = 500;
  int restart = 40;
  int fixed_iters = 0;
};

struct ColInfo {
  int iters = 0, restarts = 0, status = 0;
  double rel_residual = 0;
  int m = 0, block = 0;  // restart length and Arnoldi block width the column ran with
};

// A view of one array carved out of a job's workspace buffer (the DevArray interface minus
// ownership).
template <typename T>
struct Carved {
  T* p = nullptr;
  T* ptr() const { return p; }
};

// One block FGMRES(m) solve as a resumable state machine.  Driver protocol:
//   start();  loop { matvec() (Z = M^{-1} v_cur(), W = A Z);  after_matvec();
//                    synchronise;  if (cycle_done() && end_cycle()) finished; }
// B and X are node-major [n][s] device blocks owned by the caller.
struct FgmresJob {
  Ctx* ctx;
  std::shared_ptr<Ddm> d;
  int s;
  const c128* B;
  c128* X;
  SolveOptions o;
  int m;
  int64_t n, ldr = 0;
  KrylovKernels K;
  bool z32;   // preconditioned blocks kept in complex64 (mixed-precision preconditioner)
  bool dcgs;  // delayed reorthogonalisation (16 or 32 columns); CGS2 + CholQR2 otherwise
  // every device array of the job lives in one workspace buffer: the context's cached one
  // (hz_solve: kept between solves, so repeated solves allocate nothing) or the job's own
  Carved<c128> V, Zb, W, Wt, R, part, Hc, Hp, Hc2, Gm, Cm, Rprev, Rm, refl, tau, tmat, G, Y, Gs, Rs, Ri, Racc;
  Carved<c64> Zs;
  Carved<double> res, npart, nrm;
  Carved<int> flag;
  DevBuf ws_own;
  bool ws_cached = false;
  std::vector<double> bnorm, rel;
  HostPinned<double> est;  // per-column residual estimates of the latest least-squares step
  int total = 0, restarts = 0, jj = 0;
  int base = 0;        // Hessenberg columns completed before this cycle
  int ncols = 0;       // columns of this cycle that end_cycle() combines
  bool last = false;   // this step is the cycle's last (restart length, fixed count, max_iter)
  // host copies of the breakdown flags (a numerically dependent block): [0] CholQR, or the
  // delayed form's step (column j - 1); [1] the delayed form's finishing pass (column j)
  HostPinned<int> hflags;
  std::vector<ColInfo> info;

  // delayed form: the least-squares step of column j - 1 runs on a second stream (default
  // priority) beside the update of the same step, which does not depend on it
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  FgmresJob(Ctx* c, std::shared_ptr<Ddm> dd, int s_, const c128* B_, c128* X_, const SolveOptions& o_, int m_,
            bool use_cache = false);
  ~FgmresJob();
  FgmresJob(const FgmresJob&) = delete;
  FgmresJob& operator=(const FgmresJob&) = delete;
  static int64_t bytes_needed(int64_t n, int s, int m, bool z32);
  static bool delayed(int s) { return s == 16 || s == 32; }
  // largest restart length <= want (>= fixed) whose Krylov memory for an s-column block, plus
  // `extra` bytes, fits in 80% of the free device memory; 0 if not even kMinRestart (or fixed) fits
  static int restart_fit(Ctx* ctx, int64_t n, int s, int want, int fixed, bool z32, int64_t extra = 0);
  // carves the workspace of an (n, s, m) job from base (null: only sizes it); returns its bytes
  int64_t carve(char* base);
  static constexpr int kMinRestart = 8;
  void start();                 // norms of B (synchronises), X = 0, first cycle
  c128* v_cur();                // block to precondition this step
  c128* z_cur();                // where M^{-1} v goes (kept for the update of X); FP64 jobs
  c64* z32_cur();               // the same for jobs that keep Z in complex64
  c128* w_cur();                // where A z goes
  void matvec();                // z_cur() = M^{-1} v_cur(), w_cur() = A z_cur()
  void spmm_z(const c64* z, c128* w);  // w = A z, z complex64 widened exactly
  void after_matvec();          // orthogonalisation, least-squares step; estimates copied to host (async)
  bool cycle_done();            // after a synchronisation: end of this cycle?
  bool end_cycle();             // X update and explicit residual (synchronises); true when finished
  void trace_step() const;      // one stderr line: step, completed columns, largest estimate
  void spmm(const c128* x, c128* y, c128 alpha, c128 beta, const c128* yin);

 private:
  void start_cycle();
  void cholqr2(const c128* in, c128* out);
  c128* h_col(int j);  // Hessenberg column buffer of step j (two alternate with delayed reorthogonalisation)
};

// Solve A X = B for a node-major block B [n][s] (device, c128) with restart length m.  X
// (device) receives the solution.  Returns per-column info; status HZ_ERR_NOT_CONVERGED if
// max_iter is hit.
void fgmres(Ctx* ctx, std::shared_ptr<Ddm> d, int s, const c128* B, c128* X, const SolveOptions& o, int m,
            std::vector<ColInfo>& info);
// drops the context's cached Krylov workspace (before set-up and serving, which size their
// memory by what is free)
void krylov_cache_release(Ctx* ctx);

}  // namespace hz
