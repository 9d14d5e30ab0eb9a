// Batched P3 element matrices and deterministic CSR assembly (gfx950).
//
// Element matrix of tet e (paper eq. 1 discretised with P3 Lagrange elements, absorbing
// boundary on impedance faces):
//   A_e = |T| sum_{a<=b} G_ab S'_ab - k_e^2 |T| Mhat + i k_e sum_f |f| Fhat_f
// with G_ab = grad l_a . grad l_b and S'_ab the combined reference stiffness tables.
// The kernel writes, per tet, the packed lower triangle of the volume part (210 complex)
// and, for each of the 4 faces, i k_e |f| Fhat_f packed over the face's 10 nodes
// (55 complex).  Which faces count (physical impedance, Robin on subdomain cuts) is decided
// by the gather maps, so one element buffer serves the global and all local operators.
//
// CSR values are gathered, never scattered: entry e sums its contributions in the fixed
// order of its gather list (ascending tet, volume before faces), so the result is
// bit-reproducible and exactly symmetric (entries (i,j) and (j,i) read the same packed
// values in the same order).
#include "hz_internal.h"

namespace hz {

__constant__ double c_S[10][kElemVol];
__constant__ double c_M[kElemVol];
__constant__ double c_F[4][kFaceEnt];

void p3_upload_tables(Ctx* ctx) {
  const P3Tables& t = p3_tables();
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_S), t.S, sizeof(t.S)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_M), t.M, sizeof(t.M)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_F), t.F, sizeof(t.F)));
}

namespace {

constexpr int kTetsPerBlock = 32;
constexpr int kElemThreads = 256;

struct TetGeo {
  double G[10];
  double vol;
  double area[4];
  double kre, kim;
};

__global__ __launch_bounds__(kElemThreads) void k_element(int64_t T, const int32_t* __restrict__ tets,
                                                          const double* __restrict__ coords,
                                                          const double* __restrict__ vel, const double* __restrict__ Q,
                                                          double omega, c128* __restrict__ kout, c128* __restrict__ elem) {
  __shared__ TetGeo geo[kTetsPerBlock];
  const int64_t t0 = (int64_t)blockIdx.x * kTetsPerBlock;
  const int nt = (int)min<int64_t>(kTetsPerBlock, T - t0);
  if (threadIdx.x < nt) {
    const int64_t t = t0 + threadIdx.x;
    double P[4][3];
    for (int v = 0; v < 4; ++v) {
      const int64_t g = tets[4 * t + v];
      for (int d = 0; d < 3; ++d) P[v][d] = coords[3 * g + d];
    }
    // J columns = p_c - p_0 ; grad l_c (c=1..3) = rows of J^{-1}
    double J[3][3];
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) J[d][c] = P[c + 1][d] - P[0][d];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    double gr[4][3];
    // inverse via adjugate: Jinv[r][c] = cof[c][r] / det
    gr[1][0] = c00 * id;
    gr[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    gr[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    gr[2][0] = c01 * id;
    gr[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    gr[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    gr[3][0] = c02 * id;
    gr[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    gr[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    for (int d = 0; d < 3; ++d) gr[0][d] = -(gr[1][d] + gr[2][d] + gr[3][d]);
    TetGeo& g = geo[threadIdx.x];
    int p = 0;
    for (int a = 0; a < 4; ++a)
      for (int b = a; b < 4; ++b, ++p) g.G[p] = gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2];
    g.vol = fabs(det) / 6.0;
    for (int f = 0; f < 4; ++f) {
      int a = f == 0 ? 1 : 0, b = f <= 1 ? 2 : 1, c = f <= 2 ? 3 : 2;
      double e1[3], e2[3];
      for (int d = 0; d < 3; ++d) {
        e1[d] = P[b][d] - P[a][d];
        e2[d] = P[c][d] - P[a][d];
      }
      const double x = e1[1] * e2[2] - e1[2] * e2[1], y = e1[2] * e2[0] - e1[0] * e2[2],
                   z = e1[0] * e2[1] - e1[1] * e2[0];
      g.area[f] = 0.5 * sqrt(x * x + y * y + z * z);
    }
    // k = omega / (v (1 + i/(2Q)))
    c128 c = cmk(vel[t], 0.0);
    if (Q) c = cmk(vel[t], vel[t] / (2.0 * Q[t]));
    c128 k = cdiv(cmk(omega, 0.0), c);
    g.kre = k.re;
    g.kim = k.im;
    kout[t] = k;
  }
  __syncthreads();
  const int total = nt * kElemStride;
  c128* out = elem + t0 * kElemStride;
  for (int idx = threadIdx.x; idx < total; idx += kElemThreads) {
    const int lt = idx / kElemStride;
    const int ent = idx - lt * kElemStride;
    const TetGeo& g = geo[lt];
    c128 v;
    if (ent < kElemVol) {
      double kst = 0.0;
#pragma unroll
      for (int p = 0; p < 10; ++p) kst = fma(g.G[p], c_S[p][ent], kst);
      kst *= g.vol;
      const double m = g.vol * c_M[ent];
      // -k^2 m  with k = kre + i kim
      const double k2re = g.kre * g.kre - g.kim * g.kim, k2im = 2.0 * g.kre * g.kim;
      v = cmk(kst - k2re * m, -k2im * m);
    } else {
      const int fe = ent - kElemVol;
      const int f = fe / kFaceEnt;
      const double s = g.area[f] * c_F[f][fe - f * kFaceEnt];
      // i k s
      v = cmk(-g.kim * s, g.kre * s);
    }
    out[idx] = v;
  }
}

// position of each element node on each face (-1: not on it)
struct FacePos {
  int8_t p[4][20];
};

// one wavefront per row, its entries 64 at a time (lane: one entry); for each element
// incidence of the row (ascending tet) and each node j of that tet, the lane holding column
// j's dof adds the element entry, then the Robin face entries, in the order of the host's
// former gather lists
__global__ __launch_bounds__(256) void k_incidence_fill(int64_t n_rows, const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, const int32_t* __restrict__ gdofs,
                                                        const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
                                                        const int32_t* __restrict__ tsel, const uint8_t* __restrict__ robin,
                                                        const int32_t* __restrict__ tet_dofs, const c128* __restrict__ elem,
                                                        const uint8_t* __restrict__ dir, c128* __restrict__ val,
                                                        c64* __restrict__ val32, FacePos fp) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  const bool drow = dir && dir[row];
  const int64_t k0 = inc_ptr[row], k1 = inc_ptr[row + 1];
  for (int64_t base = rowptr[row]; base < rowptr[row + 1]; base += 64) {
    const int64_t e = base + lane;
    const bool mine = e < rowptr[row + 1];
    const int32_t c = mine ? col[e] : -1;
    const int32_t gc = mine ? (gdofs ? gdofs[c] : c) : -1;
    c128 s = cmk(0.0, 0.0);
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t qi = inc[k];
      const int32_t q = qi / 20, i = qi - (qi / 20) * 20;
      const int64_t t = tsel ? (int64_t)tsel[q] : (int64_t)q;
      const uint8_t rm = robin ? robin[q] : (uint8_t)0;
      const c128* et = elem + t * kElemStride;
      for (int j = 0; j < 20; ++j) {
        if (tet_dofs[t * 20 + j] != gc) continue;
        const int pij = i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
        s = s + et[pij];
        for (int f = 0; f < 4; ++f) {
          const int fi = fp.p[f][i], fj = fp.p[f][j];
          if (((rm >> f) & 1) && fi >= 0 && fj >= 0) {
            const int pf = fi >= fj ? fi * (fi + 1) / 2 + fj : fj * (fj + 1) / 2 + fi;
            s = s + et[kElemVol + f * kFaceEnt + pf];
          }
        }
      }
    }
    if (!mine) continue;
    if (drow || (dir && dir[c])) s = cmk(c == row ? 1.0 : 0.0, 0.0);
    val[e] = s;
    if (val32) val32[e] = cmk((float)s.re, (float)s.im);
  }
}

// ---- point sources
__device__ void tet_barycentrics(const int32_t* tets, const double* coords, int64_t t, const double x[3],
                                 double lam[4]) {
  double P[4][3];
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) P[v][d] = coords[3 * (int64_t)tets[4 * t + v] + d];
  double J[3][3];
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) J[d][c] = P[c + 1][d] - P[0][d];
  const double r[3] = {x[0] - P[0][0], x[1] - P[0][1], x[2] - P[0][2]};
  // Cramer's rule
  auto det3 = [](const double a[3], const double b[3], const double c[3]) {
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
  };
  double c0[3] = {J[0][0], J[1][0], J[2][0]}, c1[3] = {J[0][1], J[1][1], J[2][1]}, c2[3] = {J[0][2], J[1][2], J[2][2]};
  // det of matrix with columns c0,c1,c2 == det3 of its transpose rows
  const double D = det3(c0, c1, c2);
  lam[1] = det3(r, c1, c2) / D;
  lam[2] = det3(c0, r, c2) / D;
  lam[3] = det3(c0, c1, r) / D;
  lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
}

__global__ void k_locate(int64_t T, int64_t ns, const int32_t* tets, const double* coords, const double* xyz,
                         unsigned long long* best) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  for (int64_t s = 0; s < ns; ++s) {
    double lam[4];
    const double x[3] = {xyz[3 * s], xyz[3 * s + 1], xyz[3 * s + 2]};
    tet_barycentrics(tets, coords, t, x, lam);
    if (lam[0] >= -1e-12 && lam[1] >= -1e-12 && lam[2] >= -1e-12 && lam[3] >= -1e-12)
      atomicMin(&best[s], (unsigned long long)t);
  }
}

__device__ void p3_basis(const double l[4], double phi[20]) {
  const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int a = 0; a < 4; ++a) phi[a] = 0.5 * l[a] * (3 * l[a] - 1) * (3 * l[a] - 2);
  for (int e = 0; e < 6; ++e) {
    const int a = E[e][0], b = E[e][1];
    phi[4 + 2 * e] = 4.5 * l[a] * l[b] * (3 * l[a] - 1);
    phi[5 + 2 * e] = 4.5 * l[a] * l[b] * (3 * l[b] - 1);
  }
  for (int f = 0; f < 4; ++f) {
    double p = 27.0;
    for (int v = 0; v < 4; ++v)
      if (v != f) p *= l[v];
    phi[16 + f] = p;
  }
}

// one thread per source: zero-filled rhs rows get the 20 basis values of the located tet
__global__ void k_point_load(int64_t ns, int64_t n, const int32_t* tets, const double* coords, const int32_t* tet_dofs,
                             const uint8_t* dir, const double* xyz, const double* amp,
                             const unsigned long long* best, c128* rhs) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const int64_t t = (int64_t)best[s];
  double lam[4], phi[20];
  const double x[3] = {xyz[3 * s], xyz[3 * s + 1], xyz[3 * s + 2]};
  tet_barycentrics(tets, coords, t, x, lam);
  p3_basis(lam, phi);
  const c128 a = amp ? cmk(amp[2 * s], amp[2 * s + 1]) : cmk(1.0, 0.0);
  for (int l = 0; l < 20; ++l) {
    const int32_t g = tet_dofs[20 * t + l];
    if (dir[g]) continue;
    rhs[s * n + g] = rhs[s * n + g] + a * cmk(phi[l], 0.0);
  }
}

}  // namespace

void launch_element_matrices(Ctx* ctx, const Mesh& m, Operator& op, const double* d_vel, const double* d_q) {
  const int64_t blocks = (m.T + kTetsPerBlock - 1) / kTetsPerBlock;
  hipLaunchKernelGGL(k_element, dim3((unsigned)blocks), dim3(kElemThreads), 0, ctx->stream, m.T, m.d_tets.ptr(),
                     m.d_coords.ptr(), d_vel, d_q, 2.0 * M_PI * op.freq, op.d_k.ptr(), op.d_elem.ptr());
  HIP_CHECK(hipGetLastError());
}

void launch_incidence_fill(hipStream_t st, int64_t n_rows, const int64_t* d_rowptr, const int32_t* d_col,
                           const int32_t* d_gdofs, const int64_t* d_inc_ptr, const int32_t* d_inc,
                           const int32_t* d_tsel, const uint8_t* d_robin, const int32_t* d_tet_dofs,
                           const c128* d_elem, const uint8_t* d_dir, c128* d_val, c64* d_val32) {
  if (n_rows == 0) return;
  const P3Tables& tab = p3_tables();
  FacePos fp;
  for (int f = 0; f < 4; ++f) {
    for (int i = 0; i < 20; ++i) fp.p[f][i] = -1;
    for (int a = 0; a < 10; ++a) fp.p[f][tab.face_nodes[f][a]] = (int8_t)a;
  }
  const int64_t blocks = (n_rows + 3) / 4;
  hipLaunchKernelGGL(k_incidence_fill, dim3((unsigned)blocks), dim3(256), 0, st, n_rows, d_rowptr, d_col, d_gdofs,
                     d_inc_ptr, d_inc, d_tsel, d_robin, d_tet_dofs, d_elem, d_dir, d_val, d_val32, fp);
  HIP_CHECK(hipGetLastError());
}

void launch_point_sources(Ctx* ctx, const Mesh& m, int64_t ns, const double* d_xyz, const double* d_amp,
                          unsigned long long* d_best, c128* d_rhs) {
  HIP_CHECK(hipMemsetAsync(d_best, 0xff, ns * sizeof(unsigned long long), ctx->stream));
  HIP_CHECK(hipMemsetAsync(d_rhs, 0, ns * m.n * sizeof(c128), ctx->stream));
  hipLaunchKernelGGL(k_locate, dim3((unsigned)((m.T + 255) / 256)), dim3(256), 0, ctx->stream, m.T, ns,
                     m.d_tets.ptr(), m.d_coords.ptr(), d_xyz, d_best);
  HIP_CHECK(hipGetLastError());
  std::vector<unsigned long long> best(ns);
  HIP_CHECK(hipMemcpyAsync(best.data(), d_best, ns * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  for (int64_t s = 0; s < ns; ++s) HZ_REQUIRE(best[s] < (unsigned long long)m.T, HZ_ERR_ARG, "hz_point_sources: source outside the mesh");
  hipLaunchKernelGGL(k_point_load, dim3((unsigned)((ns + 63) / 64)), dim3(64), 0, ctx->stream, ns, m.n, m.d_tets.ptr(),
                     m.d_coords.ptr(), m.d_tet_dofs.ptr(), m.d_dirichlet.ptr(), d_xyz, d_amp, d_best, d_rhs);
  HIP_CHECK(hipGetLastError());
}

}  // namespace hz
