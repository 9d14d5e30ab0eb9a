/*
 * hz.h -- C ABI of libhz, an MI355X (gfx950) solver for the frequency-domain Helmholtz
 * equation discretised with continuous P3 Lagrange elements on tetrahedra and solved by
 * block FGMRES with a two-level optimized restricted additive Schwarz (ORAS)
 * preconditioner, for many source right-hand sides at once.
 *
 * Method: Dolean, Jolivet, Operto, Tournier, "Large-scale frequency-domain seismic wave
 * modeling on h-adaptive tetrahedral meshes with iterative solver and multi-level
 * domain-decomposition preconditioners" (arXiv 2004.07930).  Each entry point below names
 * the passage of that paper that defines what it computes.
 *
 * General conventions
 *  - C11, no C++ types cross the ABI.  Complex numbers are interleaved (re, im) pairs of
 *    double (complex128) unless stated otherwise.
 *  - The caller owns every pointer it passes.  The library copies inputs before returning
 *    and keeps no caller pointer, except serving requests, whose rhs / x / info buffers
 *    must stay valid until the ticket completes.
 *  - Handles (mesh, operator, ddm) are owned by the library and reference counted: an
 *    operator pins its mesh, a ddm pins its operator.  0 is never a valid handle.
 *  - Every function returns an hz_status; nothing throws or aborts across the ABI.
 *    hz_last_error() holds a message for the last failure on the context.  After
 *    HZ_ERR_HIP the context is poisoned and only hz_finalize is valid.
 *  - Non-serving calls on one context must be serialised by the caller.  All GPU work of
 *    a context runs on the stream given at hz_init (NULL = the null stream).
 *  - Multi-RHS blocks are laid out [n_rhs][n_dofs] (each right-hand side contiguous).
 *    *_mem arguments say whether a pointer is host (HZ_MEM_HOST) or device memory
 *    (HZ_MEM_DEVICE) of the context's GPU.
 */
#ifndef HZ_H_
#define HZ_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HZ_ABI_VERSION 4

typedef enum {
  HZ_OK = 0,
  HZ_ERR_ARG = -1,            /* invalid argument (null pointer, bad size, NaN input ...) */
  HZ_ERR_OOM = -2,            /* device allocation failed or over the memory budget      */
  HZ_ERR_HIP = -3,            /* a HIP runtime call failed; the context is poisoned      */
  HZ_ERR_NOT_CONVERGED = -4,  /* max_iter reached; x holds the best iterate              */
  HZ_ERR_SINGULAR = -5,       /* a local or coarse factorisation met a zero pivot        */
  HZ_ERR_BUSY = -6,           /* serving: request can never be admitted                  */
  HZ_ERR_STATE = -7,          /* call not valid in the current state                      */
  HZ_ERR_ABI = -8             /* struct_size / ABI version mismatch                       */
} hz_status;

typedef struct hz_ctx hz_ctx;
typedef uint64_t hz_handle;

enum { HZ_BC_NONE = 0, HZ_BC_IMPEDANCE = 1, HZ_BC_DIRICHLET = 2 };
enum { HZ_PREC_C128 = 0, HZ_PREC_MIXED = 1 };
enum { HZ_MEM_HOST = 0, HZ_MEM_DEVICE = 1 };
enum { HZ_POU_BOOLEAN = 0, HZ_POU_SMOOTH = 1 };
/* local solver of the one-level preconditioner (hz_ddm_opts.local_solver) */
enum { HZ_LOCAL_EXACT = 0, HZ_LOCAL_ICC = 1, HZ_LOCAL_ICC_A2 = 2 };

typedef struct {
  size_t struct_size;  /* sizeof(hz_init_opts)                                        */
  int device;          /* HIP device ordinal                                           */
  size_t hbm_budget;   /* bytes the serving admission may use; 0 = 90% of free memory  */
  /* Optional device allocator, both or neither (NULL = hipMalloc / hipFree).  alloc returns
   * NULL on failure (reported as HZ_ERR_OOM).  Every call passes `stream`; memory handed to
   * free may still be read by work already queued on that stream, so the allocator must
   * reuse it only in that stream's order (as a stream-ordered caching allocator such as
   * PyTorch's does for the stream it is given).  Called from the caller's thread and, while
   * serving, from the library's scheduler thread. */
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* alloc_user;
  void* stream;        /* hipStream_t for all GPU work; NULL = null stream              */
} hz_init_opts;

/* Create a context on one GPU.  Builds the P3 reference tables on the device. */
hz_status hz_init(hz_ctx** out, const hz_init_opts* opts);
/* Destroy a context and everything it owns (waits for its GPU work). */
void hz_finalize(hz_ctx* ctx);
/* Message of the last failure on ctx (valid until the next call on ctx). */
const char* hz_last_error(const hz_ctx* ctx);
/* Drop the caller's reference to a handle.  Also drops the Krylov workspace that hz_solve
 * keeps with the context between calls (so that repeated solves allocate nothing). */
hz_status hz_release(hz_ctx* ctx, hz_handle h);

/*
 * hz_mesh -- ingest a tetrahedral mesh and number its P3 degrees of freedom.
 * Paper: section "Tetrahedral finite element method" (Lagrange P3 elements on a
 * tetrahedral mesh of the domain).
 *   tets    [n_tets][4] int32, 0-based vertex ids (any orientation)
 *   coords  [n_verts][3] float64, z pointing down
 *   face_bc nullable [n_tets][4] int8: tag of the face opposite local vertex v, read only
 *           on boundary faces (faces of one tet): HZ_BC_IMPEDANCE (first-order absorbing)
 *           or HZ_BC_DIRICHLET (free surface).  NULL = impedance everywhere.
 * Dof numbering: every node gets an integer key -- vertex g: (g,-1,-1,0); edge lo<hi:
 * (lo,hi,-1,0) at 2/3 lo + 1/3 hi and (lo,hi,-1,1) at 1/3 lo + 2/3 hi; face a<b<c:
 * (a,b,c,0) -- and its id is the rank of the key in ascending lexicographic order.
 * Also builds the CSR pattern of the global operator (columns ascending).
 * Errors: HZ_ERR_ARG on null pointers, out-of-range vertex ids or degenerate tets.
 */
hz_status hz_mesh(hz_ctx* ctx, int64_t n_tets, const int32_t* tets, int64_t n_verts,
                  const double* coords, const int8_t* face_bc, hz_handle* mesh, int64_t* n_dofs);

/*
 * hz_assemble -- element matrices and the global sparse operator A of eq. (2).
 * Paper: eq. (1) (Helmholtz with k = omega / c, c complex in viscous media) and the
 * boundary conditions stated after eq. (2).
 *   velocity [n_tets] m/s (any consistent length unit), > 0, constant per tet
 *   Q        nullable [n_tets] quality factors > 0: c = v (1 + i / (2 Q))
 *   freq_hz  frequency f, omega = 2 pi f
 * A = K - k^2 M + i k M_G (exp(+i omega t) convention; complex symmetric), Dirichlet dofs
 * are identity rows/columns kept in the pattern.  Values are FP64 on the device, with a
 * complex64 copy.  Errors: HZ_ERR_ARG on non-positive / non-finite coefficients.
 */
hz_status hz_assemble(hz_ctx* ctx, hz_handle mesh, const double* velocity, const double* Q,
                      double freq_hz, hz_handle* op);

typedef struct {
  int64_t n_tets;
  const int32_t* tets;   /* [n_tets][4] */
  int64_t n_verts;
  const double* coords;  /* [n_verts][3] */
} hz_coarse_mesh;

/*
 * hz_setup_ddm -- overlapping decomposition, local Robin operators, their LDL^T factors
 * and the coarse space.  Paper: eqs. (2lvl) and (oras) and the text around them.
 *   partition [n_tets] int32 in [0, n_sub): non-overlapping subdomain of each tet
 *   overlap   number of tet layers added (vertex adjacency), >= 0
 *   coarse    NULL = one-level ORAS; else a P1 coarse mesh covering the fine one
 *   precision HZ_PREC_C128 (factors, ORAS and coarse solve in complex128) or
 *             HZ_PREC_MIXED (complex64 factors, ORAS and coarse solve; FGMRES in FP64)
 * Errors: HZ_ERR_ARG (bad partition, fine node outside the coarse mesh), HZ_ERR_OOM.
 * Tiny pivots are replaced by a threshold (static pivoting) and counted (hz_ddm_stats).
 */
hz_status hz_setup_ddm(hz_ctx* ctx, hz_handle op, const int32_t* partition, int32_t n_sub,
                       int32_t overlap, const hz_coarse_mesh* coarse, int precision, hz_handle* ddm);

/*
 * hz_setup_ddm_ex -- hz_setup_ddm with options.  Paper: eq. (oras), D_i "local diagonal
 * matrices representing the partition of unity" (no construction is given).
 *   opts->precision  as in hz_setup_ddm
 *   opts->pou        HZ_POU_BOOLEAN: each dof belongs to the lowest subdomain id whose
 *                    non-overlapping tets hold it (D_i = 0 or 1; hz_setup_ddm's choice);
 *                    HZ_POU_SMOOTH: a dof's raw weight in subdomain i is 1 - l / (overlap + 1),
 *                    l its layer in i (0 on the non-overlapping tets, k on the tets the k-th
 *                    overlap step added; the smallest over the tets holding it), divided by the
 *                    sum of its raw weights over the subdomains holding it (subdomain order).
 *   opts->local_solver  HZ_LOCAL_EXACT: A_i^{-1} of eq. (oras) by the multifrontal LDL^T factors
 *                    (hz_setup_ddm's choice).  HZ_LOCAL_ICC: by an incomplete factorisation,
 *                    the approximate local solver of the paper's numerical section (which names
 *                    no variant; read here as level 0, no fill): A_i ~ L D L^T (transpose, not
 *                    conjugate), L unit lower triangular on the strict lower pattern of A_i in
 *                    its local order (ascending global dof), no shift or pivoting.  The factors
 *                    are computed in FP64 on the GPU and stored in the preconditioner precision;
 *                    the solve is forward substitution, scaling by D^{-1} and backward
 *                    substitution, one launch per dependency level.  The multifrontal factors
 *                    are then not built (hz_ddm_stats still reports their symbolic size).
 *                    HZ_LOCAL_ICC_A2: the same factorisation on the lower pattern of A_i^2
 *                    (every pair of local dofs joined through one neighbour; entries of A_i
 *                    absent there start from zero).  It stores about 11 times the entries of
 *                    level 0 (P3 on tets).  Memory per stored entry: on the device the value
 *                    (8 or 16 bytes) and 16 bytes of column, row and position indices, plus 24
 *                    bytes during set-up (its source index and FP64 working value); on the
 *                    host up to 36 bytes during set-up.
 * Errors: as hz_setup_ddm; HZ_ERR_ABI on struct_size; HZ_ERR_ARG on an unknown pou or local
 * solver or an overlap above 250; HZ_ERR_SINGULAR when the incomplete factorisation meets a
 * zero or non-finite pivot.
 */
typedef struct {
  size_t struct_size;  /* sizeof(hz_ddm_opts) */
  int precision;       /* HZ_PREC_C128 or HZ_PREC_MIXED */
  int pou;             /* HZ_POU_BOOLEAN or HZ_POU_SMOOTH */
  int local_solver;    /* HZ_LOCAL_EXACT, HZ_LOCAL_ICC or HZ_LOCAL_ICC_A2 */
} hz_ddm_opts;
hz_status hz_setup_ddm_ex(hz_ctx* ctx, hz_handle op, const int32_t* partition, int32_t n_sub,
                          int32_t overlap, const hz_coarse_mesh* coarse, const hz_ddm_opts* opts,
                          hz_handle* ddm);

typedef struct {
  int32_t iters;        /* inner FGMRES iterations done for this column's block */
  int32_t restarts;
  double rel_residual;  /* explicit ||b - A x|| / ||b|| in FP64 */
  int32_t status;       /* HZ_OK or HZ_ERR_NOT_CONVERGED */
  int32_t restart_len;  /* restart length m the column's block ran with */
  int32_t block;        /* width of the column's Arnoldi block */
} hz_col_info;

typedef struct {
  size_t struct_size;   /* sizeof(hz_solve_opts) */
  double tol;           /* per-column relative residual target (paper: backward error) */
  int32_t max_iter;     /* total inner iterations allowed */
  int32_t restart;      /* FGMRES restart length m (0 = default 40) */
  int32_t fixed_iters;  /* > 0: run exactly this many steps in one cycle, ignore tol */
  int32_t block;        /* right-hand sides per Arnoldi block (0 = automatic, max 32) */
} hz_solve_opts;

/*
 * hz_solve -- right-preconditioned block FGMRES(m) with two-level ORAS, x0 = 0.
 * Paper: section "Domain decomposition preconditioner" (GMRES with M^{-1}, eq. 2lvl) and
 * the stopping test ||A u - b|| / ||b|| <= eps of the FE section.  Blocks of 16 or 32
 * columns are orthogonalised by classical Gram-Schmidt with delayed reorthogonalisation (one
 * Gram product and one update over the basis per step; each column of the Hessenberg matrix
 * is complete one step later), other widths by classical Gram-Schmidt applied twice with
 * CholQR2 block normalisation; Householder least squares; all FP64.
 *   rhs [n_rhs][n_dofs] complex128, x same layout (may not alias rhs)
 * Memory: the Krylov basis of a block of s columns at restart m takes about
 * (m + 1) n s complex128 entries plus m n s preconditioned entries (complex64 with
 * HZ_PREC_MIXED).  With block = 0 the block is the widest of min(n_rhs, 32) columns and its
 * successive halvings whose basis at the requested m fits in 80% of the free device memory;
 * only if one column does not fit is m shortened, down to 8 at the least (below that:
 * HZ_ERR_OOM).  An explicit block keeps its width and shortens m the same way.  The
 * m and width used are reported per column (hz_col_info.restart_len, .block).  With
 * fixed_iters, m is at least fixed_iters and is never shortened (HZ_ERR_OOM instead).
 * Setting the environment variable HZ_TRACE=1 before hz_init prints one line per Arnoldi
 * step (largest residual estimate) and per restart cycle (explicit residuals) to stderr.
 * Returns HZ_ERR_NOT_CONVERGED (x = best iterate, info filled) when max_iter is hit;
 * HZ_ERR_ARG for a non-finite entry in rhs, a zero column, a block whose columns are
 * numerically dependent (CholQR pivot below 1e-14 of its diagonal entry: solve such columns
 * in separate blocks), a negative or non-finite tol, n_rhs < 1 or null x / info (x is then
 * not written).  A step whose new block becomes dependent (every direction of some column
 * exhausted) ends its restart cycle there; a residual block that is dependent at a restart
 * ends the solve with the columns' status as they stand.
 */
hz_status hz_solve(hz_ctx* ctx, hz_handle ddm, int64_t n_rhs, const void* rhs, int rhs_mem,
                   double tol, int32_t max_iter, void* x, int x_mem, hz_col_info* info);
hz_status hz_solve_ex(hz_ctx* ctx, hz_handle ddm, int64_t n_rhs, const void* rhs, int rhs_mem,
                      const hz_solve_opts* opts, void* x, int x_mem, hz_col_info* info);

/*
 * hz_point_sources -- load vectors of point sources: rhs[s][j] = amp_s phi_j(x_s), zero on
 * Dirichlet dofs, the containing tet being the lowest id whose barycentrics are all
 * >= -1e-12.  Paper: the point source of section "Numerical results".
 *   xyz [n_src][3]; amp nullable [n_src] complex128 (NULL = 1); rhs [n_src][n_dofs] c128
 * Errors: HZ_ERR_ARG if a source lies outside the mesh.
 */
hz_status hz_point_sources(hz_ctx* ctx, hz_handle mesh, int64_t n_src, const double* xyz,
                           const double* amp, void* rhs, int rhs_mem);

/*
 * Building blocks exposed for parity tests and measurement (same kernels as hz_solve).
 * hz_spmm:        y = A x for a block (FP64 operator), Paper eq. (2).
 * hz_spmm_c64x:   the same product for a complex64 block x, as the mixed-precision solve
 *                 applies it to its complex64 preconditioned vectors: x is widened exactly
 *                 and every product and sum is FP64; y is complex128.
 * hz_precond:     z = M^{-1} v (eq. 2lvl; eq. oras without a coarse space), in the ddm's
 *                 precision, FP64 in and out.
 * Blocks are [n_rhs][n_dofs], complex128 except the x of hz_spmm_c64x.  Host inputs are
 * checked for non-finite values (HZ_ERR_ARG).
 */
hz_status hz_spmm(hz_ctx* ctx, hz_handle op, int64_t n_rhs, const void* x, int x_mem, void* y, int y_mem);
hz_status hz_spmm_c64x(hz_ctx* ctx, hz_handle op, int64_t n_rhs, const void* x, int x_mem, void* y, int y_mem);
hz_status hz_precond(hz_ctx* ctx, hz_handle ddm, int64_t n_rhs, const void* v, int v_mem, void* z, int z_mem);

/*
 * hz_spmm_noalloc -- y = A x like hz_spmm, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * It calls no device allocator: its node-major staging copies of x and y live in a
 * library-owned scratch array of 2^23 complex128 entries (128 MiB) that every GPU the library
 * runs on holds from hz_init until the process ends.
 *   x, y  device pointers of the context's GPU, [n_rhs][n_dofs] complex128 (y may not alias x)
 * Limit: n_dofs <= 2^22 (one column's two copies); columns are processed in chunks of
 * min(32, 2^22 / n_dofs).  x is not checked for non-finite values.
 * The scratch array is shared by every call on the same GPU and keeps the last call's
 * contents: calls that overlap on one GPU (from several contexts, streams or threads) race
 * and must be serialised by the caller.  Synchronises the context stream before returning.
 * Errors: HZ_ERR_ARG (null pointers, n_rhs < 1, n_dofs over the limit, unknown operator).
 */
hz_status hz_spmm_noalloc(hz_ctx* ctx, hz_handle op, int64_t n_rhs, const void* x, void* y);

typedef struct {
  int64_t n_dofs, nnz, n_sub;
  int64_t local_dofs_total;   /* sum of overlapped subdomain sizes */
  int64_t factor_entries;     /* stored entries of all L factors (diagonal blocks and column padding to 16 included;
                                 with HZ_LOCAL_ICC the symbolic size of the exact factors, not allocated) */
  int64_t n_fronts, n_levels, max_front;
  int64_t n_coarse;
  int64_t static_pivots;      /* pivots replaced by the static threshold */
  int64_t update_entries;     /* peak entries of the Schur-update arena during the factorisation */
  int64_t factor_useful;      /* stored factor nonzeros: sum over fronts of p(p+1)/2 + r p */
  int64_t device_bytes;       /* device memory held by the ddm (operator excluded) */
  double setup_seconds;
  double factor_seconds;      /* numeric factorisation (GPU), part of setup_seconds */
  double factor_flops;        /* its algorithmic real flops: 8 per complex multiply-add of the
                                 diagonal blocks, panel solves, trailing updates and the
                                 partitioned inverse (direct complex form); 0 with HZ_LOCAL_ICC */
  int64_t local_solver;       /* HZ_LOCAL_EXACT, HZ_LOCAL_ICC or HZ_LOCAL_ICC_A2 */
  int64_t icc_entries;        /* incomplete factors: stored entries of L (strict lower) and D; else 0 */
  int64_t icc_levels;         /* incomplete factors: dependency levels of the forward substitution */
} hz_ddm_stats;
hz_status hz_ddm_stats_get(hz_ctx* ctx, hz_handle ddm, hz_ddm_stats* out);

/*
 * Per elimination level of the multifrontal solves (level 0 holds the leaves of every
 * subdomain's nested-dissection tree; each sweep direction makes one launch per level).
 * hz_ddm_levels writes min(max_levels, L) entries to out and L to *n_levels; out may be
 * null when max_levels is 0.  Errors: HZ_ERR_ARG (null n_levels, or null out with
 * max_levels > 0).
 */
typedef struct {
  int64_t n_fronts;
  int64_t max_pivots;     /* largest pivot block p */
  int64_t max_front;      /* largest front order f = p + r */
  int64_t sum_pivots;     /* sum of p */
  int64_t sum_front;      /* sum of f */
  int64_t factor_useful;  /* stored factor nonzeros: sum of p(p+1)/2 + r p */
  int32_t fwd_tile_rows;  /* complex64 blocks of up to 16 columns: forward tile rows and */
  int32_t bwd_tile_cols;  /* backward tile columns picked by timing (0 until the first apply) */
} hz_ddm_level;
hz_status hz_ddm_levels(hz_ctx* ctx, hz_handle ddm, hz_ddm_level* out, int32_t max_levels, int32_t* n_levels);

/*
 * Live kernel accounting for measurement (not needed to solve).  While enabled, the
 * library brackets every launch of the kernel classes below with HIP events on the
 * context stream and records the launch's algorithmic bytes and flops (the minimum
 * traffic / arithmetic of the operation, not counter readings).
 *   HZ_K_SPMM        multi-RHS operator product (FP64 CSR)
 *   HZ_K_ORAS_FWD    forward multifrontal sweep, one launch per tree level
 *   HZ_K_ORAS_BWD    backward multifrontal sweep, one launch per tree level
 *   HZ_K_CGS_GRAM    V^H W partial products of classical Gram-Schmidt (both forms)
 *   HZ_K_CGS_UPDATE  W -= V H, the delayed form's [v_j, next block] update, X += Z Y
 * hz_profile_enable(ctx, 1) clears and starts recording, (ctx, 0) stops.
 * hz_profile_get synchronises the stream and returns the totals of one class.
 */
enum { HZ_K_SPMM = 0, HZ_K_ORAS_FWD = 1, HZ_K_ORAS_BWD = 2, HZ_K_CGS_GRAM = 3, HZ_K_CGS_UPDATE = 4, HZ_K_COUNT = 5 };
typedef struct {
  int64_t launches;
  double seconds;  /* sum of event-timed launch durations */
  double bytes;    /* sum of algorithmic bytes */
  double flops;    /* sum of algorithmic flops */
} hz_kernel_stat;
hz_status hz_profile_enable(hz_ctx* ctx, int on);
hz_status hz_profile_get(hz_ctx* ctx, int kernel_class, hz_kernel_stat* out);

/* serving: continuous batching of solve requests (thread-safe) */
typedef struct {
  size_t struct_size;
  hz_handle ddm;
  int64_t n_rhs;
  const void* rhs;   /* [n_rhs][n_dofs] complex128 */
  void* x;           /* [n_rhs][n_dofs] complex128 */
  int mem;           /* HZ_MEM_HOST or HZ_MEM_DEVICE, for both rhs and x */
  double tol;
  int32_t max_iter;
  hz_col_info* info; /* [n_rhs] */
} hz_request;

typedef struct {
  double p50_s, p99_s, sources_per_s;
  int64_t completed, rejected;
  int64_t parts_done;   /* request parts finished so far (progress of long requests) */
  int64_t steps;        /* block Arnoldi steps taken so far, summed over the parts */
  int64_t active_parts; /* parts running now */
} hz_serve_stats;

/*
 * Serving many source right-hand sides per frequency (paper: introduction and conclusion,
 * the multi-RHS use of the solver) as a stream of requests on resident ddms.
 * hz_serve_start: starts the scheduler thread, which owns the context stream until
 *   hz_serve_stop; other calls on the context return HZ_ERR_STATE meanwhile.  max_slots
 *   >= 1 bounds the parts (blocks of at most 32 sources) running at once.
 * hz_serve_submit: queues a request (FIFO) and returns its ticket.  Each request is solved
 *   like hz_solve (x0 = 0, per-column relative residual req->tol, req->max_iter inner
 *   iterations, 0 = 500) in parts of w sources with restart length m, both chosen at
 *   submission from hbm_budget minus the resident objects (the ddms, operators and meshes,
 *   and the packing buffers hz_serve_start allocates for the largest operator): for each w in
 *   min(n_rhs, 32) and its halvings, the longest m up to 40 with which one part fits alone;
 *   the widest w whose m reaches 20, else the w with the longest m.  Its parts are admitted in
 *   order when a slot is free and their memory fits; each part stages its own columns of a
 *   host rhs / x (no copy of the whole request is held on the device) through a page-locked
 *   host buffer that hz_serve_start allocates for one part of the largest operator.
 *   rhs / x / info (info nullable, [n_rhs]) stay caller-owned and must stay valid until the
 *   ticket completes; req->mem says whether rhs and x are host or device.
 *   Errors: HZ_ERR_ARG (unknown ddm, n_rhs < 1, null buffers, bad mem), HZ_ERR_ABI
 *   (struct_size), HZ_ERR_BUSY (fits at no restart length >= 8: never admissible),
 *   HZ_ERR_STATE (not serving, or the scheduler failed).
 * hz_serve_poll: *done = 1 once the ticket completed.  hz_serve_wait: blocks until then,
 *   returns the request's status in *status (nullable; HZ_OK, HZ_ERR_NOT_CONVERGED,
 *   HZ_ERR_OOM when the allocator could not give one part its memory even with nothing else
 *   running, or HZ_ERR_ARG when a part's block is dependent or has a zero column; x is then
 *   undefined) and retires the ticket.  A part whose allocation fails
 *   while others run waits for their memory.  Both: HZ_ERR_ARG for an unknown ticket.
 * hz_serve_stats_get: p50 / p99 of the submit-to-completion latency of completed requests,
 *   sources per second from the first submission to the last completion, counts.
 * hz_serve_stop: lets every queued and running request finish, then joins the scheduler.
 *   HZ_ERR_HIP if the scheduler met a GPU failure (the context is then poisoned).
 */
hz_status hz_serve_start(hz_ctx* ctx, int32_t max_slots);
hz_status hz_serve_submit(hz_ctx* ctx, const hz_request* req, uint64_t* ticket);
hz_status hz_serve_poll(hz_ctx* ctx, uint64_t ticket, int* done);
hz_status hz_serve_wait(hz_ctx* ctx, uint64_t ticket, int32_t* status);
hz_status hz_serve_stats_get(hz_ctx* ctx, hz_serve_stats* out);
hz_status hz_serve_stop(hz_ctx* ctx);

/* introspection for bit-exact parity tests (host output buffers) */
hz_status hz_get_dofmap(hz_ctx* ctx, hz_handle mesh, int32_t* tet_dofs /*[n_tets][20]*/);
hz_status hz_get_csr_size(hz_ctx* ctx, hz_handle op, int64_t* n, int64_t* nnz);
hz_status hz_get_csr(hz_ctx* ctx, hz_handle op, int64_t* rowptr, int32_t* col, double* val /*c128*/);
hz_status hz_get_subdomain_size(hz_ctx* ctx, hz_handle ddm, int32_t i, int64_t* n_i, int64_t* nnz_i);
hz_status hz_get_subdomain(hz_ctx* ctx, hz_handle ddm, int32_t i, int32_t* gdofs, uint8_t* owned,
                           int64_t* rowptr, int32_t* col, double* val /*c128, nullable*/);
/* partition-of-unity weights D_i of subdomain i, aligned with its sorted dofs (0/1 for the
 * Boolean partition) */
hz_status hz_get_pou(hz_ctx* ctx, hz_handle ddm, int32_t i, double* weights);
hz_status hz_get_coarse_size(hz_ctx* ctx, hz_handle ddm, int64_t* n_c, int64_t* nnz);
hz_status hz_get_coarse(hz_ctx* ctx, hz_handle ddm, int64_t* rowptr, int32_t* col, double* val /*Z, real*/);

#ifdef __cplusplus
}
#endif
#endif /* HZ_H_ */
