// Two-level ORAS preconditioner data (host + device), see ddm.cpp / factor.hip / oras.hip.
#pragma once

#include "hz_internal.h"

namespace hz {

// One supernode of a subdomain's elimination tree (multifrontal LDL^T).
// Its dense front has f = p + r rows: the p pivots (contiguous elimination positions
// [pos0, pos0 + p) of the subdomain) then the r update rows (later positions, ascending).
// Storage: L block f x p column-major in the factor array at L_off, leading dimension ld =
// f rounded up to 16 entries (so column segments start on cache-line boundaries); the diagonal
// holds D, below it L (unit diagonal implied).  The r x r update (Schur) block lives in a
// workspace at U_off (ld = r) until the parent has absorbed it.
struct Front {
  int32_t sub = 0;
  int32_t level = 0;       // height in the tree: leaves 0
  int32_t parent = -1;     // global front id
  int32_t nchild = 0;
  int32_t child[2] = {-1, -1};
  int64_t p = 0, r = 0;
  int64_t pos0 = 0;        // first pivot position (subdomain-local elimination order)
  int64_t L_off = 0;       // factor array offset (elements)
  int64_t U_off = 0;       // update workspace offset (elements)
  int64_t rows_off = 0;    // offset of the r update-row positions in Ddm::urows
  int64_t emap_off = 0;    // offset of the r extend-add targets in the parent's front
  int64_t orig_off = 0, orig_cnt = 0;  // original-entry scatter list
  int64_t f() const { return p + r; }
  int64_t ld() const { return (f() + 15) / 16 * 16; }
};

// device-side compact description of a front (used by kernels)
struct FrontDesc {
  int64_t L_off, U_off, rows_off, emap_off, orig_off, orig_cnt;
  int64_t vec_off;   // offset of the subdomain's local vector (concatenated over subdomains)
  int64_t w_off;     // offset (rows) of this front's f x s work block in the solve workspace
  int64_t imap_off;  // offset of the inverse extend-add maps: 2 x f entries (child slot 0, 1)
  int32_t p, r;
  int32_t parent;    // global front id or -1
  int32_t child0, child1;
  int32_t pos0;
  int32_t ld;        // leading dimension of the L block (f rounded up to 16)
};

struct Subdomain {
  int64_t n = 0;                  // overlapped local dofs
  std::vector<int32_t> gdofs;     // R_i: sorted global dofs
  std::vector<uint8_t> owned;     // D_i (Boolean)
  std::vector<int32_t> perm;      // elimination position -> local id (index into gdofs)
  std::vector<int32_t> ipos;      // local id -> elimination position
  std::vector<int64_t> rowptr;    // local CSR pattern (local ids)
  std::vector<int32_t> col;
  RowIncidence inc;               // element incidences of the local rows (set-up only)
  std::vector<int32_t> tsel;      // the overlapped set's tets (global ids, ascending; set-up only)
  std::vector<uint8_t> robin;     // Robin faces (bitmask) of each of those tets (set-up only)
  std::vector<uint8_t> dir;       // local Dirichlet flags
  std::vector<uint8_t> layer;     // overlap layer of each local dof (smallest over its tets)
  std::vector<double> pouw;       // smooth partition of unity: weight of each local dof
  int64_t vec_off = 0;            // offset in the concatenated local vector
  int64_t csr_off = 0;            // offset of its nnz in the concatenated local CSR values
  int64_t row_off = 0;            // offset of its rows in the concatenated rowptr
  std::vector<int32_t> fronts;    // global front ids (post-order)
};

struct Level {
  std::vector<int32_t> fronts;    // global front ids, sorted by p descending
  int64_t max_p = 0, max_f = 0, max_r = 0;
  int64_t useful = 0;             // stored factor nonzeros of the level: sum p(p+1)/2 + r p
  int64_t sum_f = 0, sum_p = 0;
};

struct CoarseSpace {
  int64_t nc = 0;
  std::vector<int64_t> zptr;      // Z CSR (n x nc)
  std::vector<int32_t> zcol;
  std::vector<double> zval;
  std::vector<int64_t> ztptr;     // Z^T CSR (nc x n)
  std::vector<int32_t> ztcol;
  std::vector<double> ztval;
  std::vector<int64_t> azptr;     // pattern of A Z (n x nc)
  std::vector<int32_t> azcol;
  DevArray<int64_t> d_zptr, d_ztptr, d_azptr;
  DevArray<int32_t> d_zcol, d_ztcol, d_azcol;
  DevArray<double> d_zval, d_ztval;
  DevArray<c128> d_az;            // A Z values (FP64)
  DevArray<c64> d_az32;
  DevArray<c128> d_E;             // E = Z^T A Z, then its LU factors (column-major nc x nc)
  DevArray<c64> d_E32;
  DevArray<int32_t> d_piv;        // LU row pivots
  DevBuf w_y, w_y2, w_part;       // apply workspace (restricted vector, product, K-chunk partials)
};

// Incomplete LDL^T of every local operator (level 0: L keeps the strict lower pattern of A_i,
// in the local order of A_i), the paper's approximate local solver in place of the exact
// factors.  Rows are numbered over the concatenated subdomains (row r = vec_off + local id).
struct IccFactor {
  int64_t nnz = 0;                       // stored strict-lower entries
  int32_t n_fwd = 0, n_bwd = 0;          // dependency levels of the two substitutions
  std::vector<int64_t> fwd_off, bwd_off;  // rows of each level in d_fwd_rows / d_bwd_rows
  DevArray<int64_t> d_lp;                // strict lower rows: pointers (absolute)
  DevArray<int32_t> d_lc;                // their columns (concatenated row numbers, ascending)
  DevArray<int64_t> d_up;                // the same entries by column (rows of L^T)
  DevArray<int32_t> d_ur;                // row of each such entry
  DevArray<int64_t> d_uk;                // its position in the strict lower rows
  DevArray<int32_t> d_fwd_rows, d_bwd_rows;
  DevArray<int32_t> d_g;                 // row -> global dof
  DevArray<int64_t> d_out;               // row -> local vector position (elimination order)
  DevBuf d_L;                            // L values in the factor precision
  DevBuf d_dinv;                         // 1 / d per row, factor precision
  size_t bytes() const {
    return d_lp.bytes() + d_lc.bytes() + d_up.bytes() + d_ur.bytes() + d_uk.bytes() + d_fwd_rows.bytes() +
           d_bwd_rows.bytes() + d_g.bytes() + d_out.bytes() + d_L.bytes + d_dinv.bytes;
  }
};

// solve workspace of the preconditioner, grown on demand and kept with its ddm
struct PrecondWork {
  DevBuf bin, bout, wbuf, q, t;
};

// tile sizes the matrix-core solve sweeps choose from (per tree level): forward
// rows per block, backward pivot columns per block
constexpr int kFwdRowsMfma[2] = {64, 128};
constexpr int kBwdColsMfma[2] = {64, 128};

struct Ddm {
  std::shared_ptr<Operator> op;
  int precision = HZ_PREC_C128;
  int pou = HZ_POU_BOOLEAN;
  int local_solver = HZ_LOCAL_EXACT;
  int32_t n_sub = 0, overlap = 0;
  std::vector<Subdomain> subs;
  std::vector<Front> fronts;
  std::vector<Level> levels;
  int64_t n_local_total = 0;      // sum of n_i
  int64_t factor_entries = 0, update_entries = 0, urows_total = 0, orig_total = 0;  // update: per group
  int64_t max_front = 0;
  int64_t static_pivots = 0;
  double setup_seconds = 0;
  double factor_seconds = 0;  // numeric factorisation (wall clock, synchronised)
  double factor_flops = 0;    // its algorithmic real flops (8 per complex multiply-add)
  std::unique_ptr<CoarseSpace> coarse;
  std::unique_ptr<IccFactor> icc;  // HZ_LOCAL_ICC: replaces the multifrontal factors

  // host index arrays
  std::vector<int32_t> urows;     // update-row positions per front (subdomain-local)
  std::vector<int32_t> emap;      // extend-add targets per front
  std::vector<int64_t> orig_src;  // concatenated local CSR index of each original entry
  std::vector<int64_t> orig_dst;  // front-relative flat index (L region)
  std::vector<int32_t> gidx;      // concatenated local vector position -> global dof
  std::vector<int64_t> own_src;   // global dof -> concatenated local vector position of its owner

  // device arrays
  DevArray<FrontDesc> d_fronts;
  DevArray<int32_t> d_urows, d_emap, d_gidx;
  DevArray<int64_t> d_orig_src, d_orig_dst, d_own_src;
  DevArray<int64_t> d_lrowptr;
  DevArray<int32_t> d_lcol;

  DevArray<uint8_t> d_ldir;
  DevArray<c128> d_lval;          // local operator values (FP64), concatenated
  DevArray<int32_t> d_level_fronts;  // fronts of every level, concatenated
  std::vector<int64_t> level_off;    // offsets into d_level_fronts
  // numeric factorisation in groups of consecutive subdomains (the update arena holds one
  // group's Schur blocks at a time): group g is subdomains [fgroup_off[g], fgroup_off[g+1]);
  // flf lists the fronts of each (group, level) by p descending, at flf_off[g * levels + lv]
  std::vector<int32_t> fgroup_off;
  std::vector<int32_t> flf;
  std::vector<int64_t> flf_off;
  DevArray<int32_t> d_flf;
  DevBuf d_factor;                // c128 or c64 L blocks
  DevBuf d_update;                // update workspace
  DevBuf d_dinv;                  // inverse pivots per local position (factor precision)
  DevArray<unsigned long long> d_npiv;  // static pivot counter
  int64_t w_total = 0;            // solve workspace rows (sum of f over fronts)
  int64_t factor_useful = 0;      // stored nonzeros: sum p(p+1)/2 + r p
  // solve worklists per level: forward (front, 64-row tile start), backward (front, 32-column
  // start); the matrix-core sweeps have their own for each tile size they can pick
  // (kFwdRowsMfma[t] rows, kBwdColsMfma[t] columns)
  std::vector<int64_t> fwd_off, bwd_off, fwdm_off[2], bwdm_off[2];
  DevArray<int32_t> d_fwd_work, d_bwd_work, d_fwdm_work[2], d_bwdm_work[2];  // pairs
  // tile choice per level of the matrix-core sweeps, picked by timing on the first apply
  // (index 0: blocks of up to 16 columns, 1: up to 32); empty until tuned
  std::vector<uint8_t> tile_fwd[2], tile_bwd[2];
  DevArray<int32_t> d_imap;
  // smooth partition of unity: per global dof, its (local vector position, weight) pairs in
  // subdomain order
  DevArray<int64_t> d_pou_ptr, d_pou_pos;
  DevArray<double> d_pou_w;
  PrecondWork pw;  // solve workspace (precond_apply)
  int64_t device_bytes() const;
};

// ddm.cpp
std::shared_ptr<Ddm> build_ddm(Ctx* ctx, std::shared_ptr<Operator> op, const int32_t* partition, int32_t n_sub,
                               int32_t overlap, const hz_coarse_mesh* coarse, int precision, int pou,
                               int local_solver);
// factor.hip
void factor_all(Ctx* ctx, Ddm& d);
// icc.hip: the incomplete factors of every local operator (in place of factor_all), and their
// solve for a block in node-major layout: out (local vectors, elimination order) from the
// global block v; y is a work block of n_local_total x s entries
void icc_setup(Ctx* ctx, Ddm& d);
void icc_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* out, c128* y);
void icc_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c64* out, c64* y);
void icc_apply(Ctx* ctx, Ddm& d, int s, const c64* v, c64* out, c64* y);
// coarse.hip
void coarse_setup(Ctx* ctx, Ddm& d);
// oras.hip: z = M^{-1} v for a block in node-major layout [n][s] (c128 in/out)
struct OrasWork;
void precond_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* z);
// the same, z rounded to complex64 (mixed precision only): the flexible Krylov solve keeps
// its preconditioned vectors in complex64 and multiplies exactly what it stored
void precond_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c64* z);
void precond_release_workspace(Ddm& d);

}  // namespace hz
