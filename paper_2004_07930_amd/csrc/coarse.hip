// Coarse space of the two-level preconditioner (paper eq. 2lvl):
//   Q = Z E^{-1} Z^T,  E = Z^T A Z,
// with Z the P1 interpolation from a coarse tetrahedral mesh: Z[j, c] is the barycentric
// coordinate of coarse vertex c at fine node j, taken in the lowest-id coarse tet that
// contains the node (|lambda| <= 1e-12 dropped, Dirichlet rows zero).  The paper solves
// the coarse problem with 10 inner GMRES iterations; here E is factored by LU with partial
// pivoting on the GPU and its inverse is formed once (same bytes per apply as two
// triangular solves, but one fully parallel product).
#include <algorithm>
#include <cmath>

#include "ddm.h"
#include "mfma_cplx.h"

namespace hz {

// ---------------------------------------------------------------- host: Z by point location

void build_coarse_host(const Mesh& m, const hz_coarse_mesh* cm, CoarseSpace& cs) {
  HZ_REQUIRE(cm->n_tets > 0 && cm->n_verts >= 4 && cm->tets && cm->coords, HZ_ERR_ARG, "coarse mesh: empty");
  const int64_t CT = cm->n_tets, CV = cm->n_verts;
  for (int64_t k = 0; k < 4 * CT; ++k)
    HZ_REQUIRE(cm->tets[k] >= 0 && cm->tets[k] < CV, HZ_ERR_ARG, "coarse mesh: vertex id out of range");
  cs.nc = CV;
  // per coarse tet: p0 and J^{-1}
  std::vector<double> Jinv(9 * CT), p0(3 * CT), lo(3 * CT), hi(3 * CT);
  double gmin[3] = {INFINITY, INFINITY, INFINITY}, gmax[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t t = 0; t < CT; ++t) {
    double P[4][3];
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) P[v][d] = cm->coords[3 * (int64_t)cm->tets[4 * t + v] + d];
    double J[3][3];
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) J[d][c] = P[c + 1][d] - P[0][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    HZ_REQUIRE(det != 0 && std::isfinite(det), HZ_ERR_ARG, "coarse mesh: degenerate tet");
    double* I = &Jinv[9 * t];
    I[0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    I[1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    I[2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    I[3] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    I[4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    I[5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    I[6] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    I[7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    I[8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int d = 0; d < 3; ++d) {
      p0[3 * t + d] = P[0][d];
      lo[3 * t + d] = std::min(std::min(P[0][d], P[1][d]), std::min(P[2][d], P[3][d]));
      hi[3 * t + d] = std::max(std::max(P[0][d], P[1][d]), std::max(P[2][d], P[3][d]));
      gmin[d] = std::min(gmin[d], lo[3 * t + d]);
      gmax[d] = std::max(gmax[d], hi[3 * t + d]);
    }
  }
  // uniform bucket grid over the coarse tets' bounding boxes (candidates kept in id order)
  const int nb = std::max(1, (int)std::cbrt((double)CT));
  double cell[3];
  for (int d = 0; d < 3; ++d) cell[d] = (gmax[d] - gmin[d]) / nb + 1e-300;
  auto cidx = [&](double x, int d) {
    int64_t k = (int64_t)std::floor((x - gmin[d]) / cell[d]);
    return (int)std::min<int64_t>(std::max<int64_t>(k, 0), nb - 1);
  };
  std::vector<std::vector<int32_t>> bucket((size_t)nb * nb * nb);
  for (int64_t t = 0; t < CT; ++t) {
    int a0[3], a1[3];
    for (int d = 0; d < 3; ++d) {
      const double pad = 1e-9 * (gmax[d] - gmin[d]);
      a0[d] = cidx(lo[3 * t + d] - pad, d);
      a1[d] = cidx(hi[3 * t + d] + pad, d);
    }
    for (int x = a0[0]; x <= a1[0]; ++x)
      for (int y = a0[1]; y <= a1[1]; ++y)
        for (int z = a0[2]; z <= a1[2]; ++z) bucket[((size_t)z * nb + y) * nb + x].push_back((int32_t)t);
  }
  cs.zptr.assign(m.n + 1, 0);
  std::vector<std::array<std::pair<int32_t, double>, 4>> rowv(m.n);
  std::vector<int8_t> rown(m.n, 0);
  std::vector<uint8_t> bad(m.n, 0);
  parallel_for(m.n, [&](int64_t a, int64_t b) {
    for (int64_t j = a; j < b; ++j) {
      if (m.dirichlet[j]) continue;
      const double* x = &m.dof_xyz[3 * j];
      const auto& cand = bucket[((size_t)cidx(x[2], 2) * nb + cidx(x[1], 1)) * nb + cidx(x[0], 0)];
      bool found = false;
      for (int32_t t : cand) {
        const double* I = &Jinv[9 * t];
        const double r[3] = {x[0] - p0[3 * t], x[1] - p0[3 * t + 1], x[2] - p0[3 * t + 2]};
        double lam[4];
        for (int k = 0; k < 3; ++k) lam[k + 1] = I[3 * k] * r[0] + I[3 * k + 1] * r[1] + I[3 * k + 2] * r[2];
        lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
        if (lam[0] >= -1e-12 && lam[1] >= -1e-12 && lam[2] >= -1e-12 && lam[3] >= -1e-12) {
          // columns sorted ascending, duplicates impossible (distinct vertices)
          int cnt = 0;
          std::pair<int32_t, double> e[4];
          for (int v = 0; v < 4; ++v)
            if (std::fabs(lam[v]) > 1e-12) e[cnt++] = {cm->tets[4 * t + v], lam[v]};
          std::sort(e, e + cnt);
          for (int k = 0; k < cnt; ++k) rowv[j][k] = e[k];
          rown[j] = (int8_t)cnt;
          found = true;
          break;
        }
      }
      if (!found) bad[j] = 1;
    }
  });
  for (int64_t j = 0; j < m.n; ++j) HZ_REQUIRE(!bad[j], HZ_ERR_ARG, "coarse mesh does not cover fine node");
  for (int64_t j = 0; j < m.n; ++j) cs.zptr[j + 1] = cs.zptr[j] + rown[j];
  cs.zcol.resize(cs.zptr[m.n]);
  cs.zval.resize(cs.zptr[m.n]);
  for (int64_t j = 0; j < m.n; ++j)
    for (int k = 0; k < rown[j]; ++k) {
      cs.zcol[cs.zptr[j] + k] = rowv[j][k].first;
      cs.zval[cs.zptr[j] + k] = rowv[j][k].second;
    }
  // Z^T
  cs.ztptr.assign(CV + 1, 0);
  for (int32_t c : cs.zcol) cs.ztptr[c + 1]++;
  for (int64_t c = 0; c < CV; ++c) cs.ztptr[c + 1] += cs.ztptr[c];
  cs.ztcol.resize(cs.zcol.size());
  cs.ztval.resize(cs.zcol.size());
  {
    std::vector<int64_t> fill(cs.ztptr.begin(), cs.ztptr.end() - 1);
    for (int64_t j = 0; j < m.n; ++j)
      for (int64_t k = cs.zptr[j]; k < cs.zptr[j + 1]; ++k) {
        const int64_t pos = fill[cs.zcol[k]]++;
        cs.ztcol[pos] = (int32_t)j;
        cs.ztval[pos] = cs.zval[k];
      }
  }
  // pattern of A Z
  cs.azptr.assign(m.n + 1, 0);
  std::vector<std::vector<int32_t>> rows(m.n);
  parallel_for(m.n, [&](int64_t a, int64_t b) {
    std::vector<int32_t> buf;
    for (int64_t i = a; i < b; ++i) {
      buf.clear();
      for (int64_t k = m.rowptr[i]; k < m.rowptr[i + 1]; ++k) {
        const int32_t j = m.col[k];
        for (int64_t q = cs.zptr[j]; q < cs.zptr[j + 1]; ++q) buf.push_back(cs.zcol[q]);
      }
      std::sort(buf.begin(), buf.end());
      buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
      rows[i] = buf;
    }
  });
  for (int64_t i = 0; i < m.n; ++i) cs.azptr[i + 1] = cs.azptr[i] + (int64_t)rows[i].size();
  cs.azcol.resize(cs.azptr[m.n]);
  for (int64_t i = 0; i < m.n; ++i) std::copy(rows[i].begin(), rows[i].end(), cs.azcol.begin() + cs.azptr[i]);
}

namespace {

// AZ[i, c] = sum_k A[i, j_k] Z[j_k, c]  (one thread per AZ entry, fixed order over k)
__global__ void k_az(int64_t n, const int64_t* __restrict__ arow, const int32_t* __restrict__ acol,
                     const c128* __restrict__ aval, const int64_t* __restrict__ zptr, const int32_t* __restrict__ zcol,
                     const double* __restrict__ zval, const int64_t* __restrict__ azptr,
                     const int32_t* __restrict__ azcol, const int32_t* __restrict__ azrow, int64_t nnz_az,
                     c128* __restrict__ az, c64* __restrict__ az32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz_az) return;
  const int64_t i = azrow[e];
  const int32_t c = azcol[e];
  c128 s = cmk(0.0, 0.0);
  for (int64_t k = arow[i]; k < arow[i + 1]; ++k) {
    const int32_t j = acol[k];
    for (int64_t q = zptr[j]; q < zptr[j + 1]; ++q)
      if (zcol[q] == c) s = s + aval[k] * cmk(zval[q], 0.0);
  }
  az[e] = s;
  az32[e] = cmk((float)s.re, (float)s.im);
}

// Er[c, :] = sum_{i in supp Z[:, c]} Z[i, c] AZ[i, :]: one block owns row c of the zeroed
// row-major buffer Er and adds the fine rows in a fixed order (the entries of one AZ row
// have distinct columns, so the lanes never collide)
__global__ __launch_bounds__(64) void k_ztaz(int64_t nc, const int64_t* __restrict__ ztptr,
                                             const int32_t* __restrict__ ztcol, const double* __restrict__ ztval,
                                             const int64_t* __restrict__ azptr, const int32_t* __restrict__ azcol,
                                             const c128* __restrict__ az, c128* __restrict__ Er) {
  const int64_t c = blockIdx.x;
  c128* row = Er + c * nc;
  for (int64_t k = ztptr[c]; k < ztptr[c + 1]; ++k) {
    const int64_t i = ztcol[k];
    const double z = ztval[k];
    for (int64_t q = azptr[i] + threadIdx.x; q < azptr[i + 1]; q += blockDim.x) {
      const int32_t d = azcol[q];
      row[d] = row[d] + az[q] * cmk(z, 0.0);
    }
    __syncthreads();
  }
}

// column-major E from the row-major Er
__global__ void k_to_colmajor(int64_t nc, const c128* __restrict__ Er, c128* __restrict__ E) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc * nc) return;
  const int64_t c = k / nc, d = k - c * nc;
  E[c + d * nc] = Er[k];
}

// ---- LU with partial pivoting, blocked right looking: panels of kLuNb columns.  Per panel:
// k_lu_panel factors it (one block, column by column), k_lu_swaps applies its row
// interchanges to the other columns, k_lu_trsm forms U12 = L11^{-1} A12 and k_lu_gemm updates
// the trailing matrix A22 -= L21 U12 on the matrix cores (three-product form, CAcc).
constexpr int kLuNb = 32, kLuTile = 64;

// panel columns [k0, k0 + nb) over rows [k0, nc): pivot = the largest |re| + |im| in the
// column (the lowest row among equals), rows swapped within the panel, multipliers below the
// diagonal, rank-1 update of the panel's later columns
template <typename T>
__global__ __launch_bounds__(1024) void k_lu_panel(int64_t nc, int64_t k0, int nb, cplx<T>* A, int32_t* piv) {
  __shared__ T bv[1024];
  __shared__ int64_t bi[1024];
  const int t = threadIdx.x;
  for (int jj = 0; jj < nb; ++jj) {
    const int64_t k = k0 + jj;
    T best = -1;
    int64_t arg = k;
    for (int64_t i = k + t; i < nc; i += 1024) {
      const cplx<T> v = A[i + k * nc];
      const T a = fabs(v.re) + fabs(v.im);
      if (a > best) {
        best = a;
        arg = i;
      }
    }
    bv[t] = best;
    bi[t] = arg;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (t < h) {
        const T o = bv[t + h];
        const int64_t oi = bi[t + h];
        if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
          bv[t] = o;
          bi[t] = oi;
        }
      }
      __syncthreads();
    }
    const int64_t p = bi[0];
    if (t == 0) piv[k] = (int32_t)p;
    if (p != k)
      for (int64_t j = k0 + t; j < k0 + nb; j += 1024) {
        const cplx<T> x = A[k + j * nc];
        A[k + j * nc] = A[p + j * nc];
        A[p + j * nc] = x;
      }
    __syncthreads();
    const cplx<T> d = A[k + k * nc];
    for (int64_t i = k + 1 + t; i < nc; i += 1024) A[i + k * nc] = cdiv(A[i + k * nc], d);
    __syncthreads();
    const int64_t mr = nc - k - 1, mcol = k0 + nb - k - 1;
    for (int64_t e = t; e < mr * mcol; e += 1024) {
      const int64_t i = k + 1 + e % mr, j = k + 1 + e / mr;
      cfms(A[i + j * nc], A[i + k * nc], A[k + j * nc]);
    }
    __syncthreads();
  }
}

// the panel's interchanges, in order, on every column outside it
template <typename T>
__global__ void k_lu_swaps(int64_t nc, int64_t k0, int nb, cplx<T>* A, const int32_t* __restrict__ piv) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc - nb) return;
  if (j >= k0) j += nb;
  for (int jj = 0; jj < nb; ++jj) {
    const int64_t k = k0 + jj, p = piv[k];
    if (p != k) {
      const cplx<T> x = A[k + j * nc];
      A[k + j * nc] = A[p + j * nc];
      A[p + j * nc] = x;
    }
  }
}

// U12 = L11^{-1} A12 (L11 unit lower), one column per thread
template <typename T>
__global__ void k_lu_trsm(int64_t nc, int64_t k0, int nb, cplx<T>* A) {
  const int64_t j = k0 + nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  cplx<T>* c = A + j * nc + k0;
  const cplx<T>* L = A + k0 * nc + k0;
  for (int r = 1; r < nb; ++r) {
    cplx<T> x = c[r];
    for (int q = 0; q < r; ++q) cfms(x, L[r + (int64_t)q * nc], c[q]);
    c[r] = x;
  }
}

// A22 -= L21 U12 over 64 x 64 tiles, k = nb <= kLuNb: each wavefront a 32 x 32 quarter
template <typename T>
__global__ __launch_bounds__(256) void k_lu_gemm(int64_t nc, int64_t k0, int nb, cplx<T>* A) {
  __shared__ cplx<T> As[kLuNb][kLuTile + 1];  // As[l][r] = L21[i0 + r][l]
  __shared__ cplx<T> Bs[kLuNb][kLuTile + 1];  // Bs[l][c] = U12[l][j0 + c]
  const int64_t c0 = k0 + nb;
  const int64_t i0 = c0 + (int64_t)blockIdx.x * kLuTile, j0 = c0 + (int64_t)blockIdx.y * kLuTile;
  for (int e = threadIdx.x; e < kLuNb * kLuTile; e += 256) {
    const int l = e / kLuTile, r = e % kLuTile;
    cplx<T> a = cmk((T)0, (T)0), b = cmk((T)0, (T)0);
    if (l < nb) {
      if (i0 + r < nc) a = A[i0 + r + (k0 + l) * nc];
      if (j0 + r < nc) b = A[k0 + l + (j0 + r) * nc];
    }
    As[l][r] = a;
    Bs[l][r] = b;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, lr = ln & 15, lq = ln >> 4;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;
  CAcc<T> acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int g = 0; g < 2; ++g) acc[m][g].zero();
#pragma unroll 2
  for (int k = 0; k < kLuNb; k += 4) {
    const int kk = k + lq;
    cplx<T> a[2], b[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) a[m] = As[kk][wr + 16 * m + lr];
#pragma unroll
    for (int g = 0; g < 2; ++g) b[g] = Bs[kk][wc + 16 * g + lr];
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
      if (j >= nc) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wr + 16 * m + CAcc<T>::row(lq, v);
        if (i < nc) A[i + j * nc] = A[i + j * nc] - acc[m][g].get(v);
      }
    }
}

// X = E^{-1}: block j solves L U x = P e_j in place in column j of X, rows in parallel
template <typename T>
__global__ __launch_bounds__(256) void k_lu_inverse(int64_t nc, const cplx<T>* LU, const int32_t* piv, cplx<T>* X) {
  const int64_t j = blockIdx.x;
  cplx<T>* x = X + j * nc;
  for (int64_t i = threadIdx.x; i < nc; i += blockDim.x) x[i] = cmk((T)(i == j ? 1 : 0), (T)0);
  __syncthreads();
  if (threadIdx.x == 0)
    for (int64_t k = 0; k < nc; ++k) {
      const int64_t p = piv[k];
      if (p != k) {
        const cplx<T> t = x[k];
        x[k] = x[p];
        x[p] = t;
      }
    }
  __syncthreads();
  for (int64_t k = 0; k < nc; ++k) {
    const cplx<T> xk = x[k];
    __syncthreads();
    if (xk.re != (T)0 || xk.im != (T)0)
      for (int64_t i = k + 1 + threadIdx.x; i < nc; i += blockDim.x) cfms(x[i], LU[i + k * nc], xk);
    __syncthreads();
  }
  for (int64_t k = nc - 1; k >= 0; --k) {
    const cplx<T> xk = cdiv(x[k], LU[k + k * nc]);
    __syncthreads();
    if (threadIdx.x == 0) x[k] = xk;
    for (int64_t i = threadIdx.x; i < k; i += blockDim.x) cfms(x[i], LU[i + k * nc], xk);
    __syncthreads();
  }
}

__global__ void k_c128_to_c64(int64_t n, const c128* a, c64* b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = cmk((float)a[i].re, (float)a[i].im);
}

template <typename T>
void lu_and_inverse(Ctx* ctx, int64_t nc, cplx<T>* E, int32_t* piv, cplx<T>* Einv) {
  hipStream_t st = ctx->stream;
  for (int64_t k0 = 0; k0 < nc; k0 += kLuNb) {
    const int nb = (int)std::min<int64_t>(kLuNb, nc - k0);
    hipLaunchKernelGGL(k_lu_panel<T>, dim3(1), dim3(1024), 0, st, nc, k0, nb, E, piv);
    if (nc > nb)
      hipLaunchKernelGGL(k_lu_swaps<T>, dim3((unsigned)((nc - nb + 255) / 256)), dim3(256), 0, st, nc, k0, nb, E,
                         (const int32_t*)piv);
    const int64_t m = nc - k0 - nb;
    if (m > 0) {
      hipLaunchKernelGGL(k_lu_trsm<T>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, nc, k0, nb, E);
      const unsigned t = (unsigned)((m + kLuTile - 1) / kLuTile);
      hipLaunchKernelGGL(k_lu_gemm<T>, dim3(t, t), dim3(256), 0, st, nc, k0, nb, E);
    }
  }
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_lu_inverse<T>, dim3((unsigned)nc), dim3(256), 0, st, nc, E, piv, Einv);
  HIP_CHECK(hipGetLastError());
}

// y[c][col] = sum_{i in Z^T row c} Z[i,c] v[i][col]  (fixed-order partial sums per column).
// A coarse row holds thousands of fine dofs: 1024 threads per row keep enough gathers in flight.
template <typename T>
__global__ __launch_bounds__(1024) void k_restrict(int64_t nc, int s, const int64_t* __restrict__ ztptr,
                                                   const int32_t* __restrict__ ztcol, const double* __restrict__ ztval,
                                                   const c128* __restrict__ v, cplx<T>* __restrict__ y) {
  __shared__ c128 part[1024];
  const int64_t c = blockIdx.x;
  const int groups = 1024 / s;
  const int g = threadIdx.x / s, col = threadIdx.x - (threadIdx.x / s) * s;
  c128 acc = cmk(0.0, 0.0);
  if (g < groups)
    for (int64_t k = ztptr[c] + g; k < ztptr[c + 1]; k += groups)
      acc = acc + v[(int64_t)ztcol[k] * s + col] * cmk(ztval[k], 0.0);
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < s) {
    c128 t = cmk(0.0, 0.0);
    for (int q = 0; q < groups; ++q) t = t + part[q * s + threadIdx.x];
    y[c * s + threadIdx.x] = cmk((T)t.re, (T)t.im);
  }
}

// partial products of y2 = Einv y over K chunks: part[kc][i][col] (64 rows x all columns
// per block, K chunk blockIdx.y)
template <typename T>
__global__ __launch_bounds__(256) void k_dense_apply(int64_t nc, int s, int64_t kchunk, const cplx<T>* __restrict__ Ei,
                                                     const cplx<T>* __restrict__ y, cplx<T>* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int cg = threadIdx.x >> 6;  // 4 column groups
  const int64_t k0 = (int64_t)blockIdx.y * kchunk, k1 = min<int64_t>(nc, k0 + kchunk);
  if (i >= nc) return;
  for (int col = cg; col < s; col += 4) {
    cplx<T> acc = cmk((T)0, (T)0);
    for (int64_t k = k0; k < k1; ++k) cfma(acc, Ei[i + k * nc], y[k * s + col]);
    part[((int64_t)blockIdx.y * nc + i) * s + col] = acc;
  }
}

template <typename T>
__global__ void k_dense_reduce(int nk, int64_t m, const cplx<T>* __restrict__ part, cplx<T>* __restrict__ y2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  cplx<T> a = cmk((T)0, (T)0);
  for (int k = 0; k < nk; ++k) a = a + part[(int64_t)k * m + e];
  y2[e] = a;
}

// lane L of each 16-lane row of a wavefront, in every lane of that row (DPP row broadcast)
template <int L>
__device__ __forceinline__ int row_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + L, 0xF, 0xF, false);
}
template <int L>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(row_bcast<L>(__float_as_int(v)));
}
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
  return __hiloint2double(row_bcast<L>(__double2hiint(v)), row_bcast<L>(__double2loint(v)));
}
// out[j] = lane B + j of the row, j < N
template <int B, int N, typename V>
__device__ __forceinline__ void row_lanes(V v, V* out) {
  if constexpr (N > 0) {
    out[0] = row_bcast<B>(v);
    row_lanes<B + 1, N - 1>(v, out + 1);
  }
}

// q = Z y2 ; t = v - AZ y2 (v - AZ y2 formed in FP64, both stored in the coarse precision T:
// the one-level apply reads t in T and the owner gather adds q).  One 16-lane row of a
// wavefront per fine row: lane u loads entry u of the row's Z part (rows hold at most 4) and
// of its first 16 AZ entries (rows hold about 5) once, the row's lanes receive each entry by
// a DPP broadcast, and lane u forms columns u, u + 16, ...  Entries are taken in batches
// (Z: 4, AZ: 8) whose gathers of y2 go out together; past the row an entry has weight zero
// and gathers from coarse row 0.  Longer rows continue with direct loads.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong(int64_t n, int s, const int64_t* __restrict__ zptr,
                                                 const int32_t* __restrict__ zcol, const double* __restrict__ zval,
                                                 const int64_t* __restrict__ azptr, const int32_t* __restrict__ azcol,
                                                 const cplx<T>* __restrict__ az, const cplx<T>* __restrict__ y2,
                                                 const c128* __restrict__ v, cplx<T>* __restrict__ q,
                                                 cplx<T>* __restrict__ t) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int u = threadIdx.x & 15;
  if (i >= n) return;  // the 16 lanes of a fine row leave together
  const int64_t z0 = zptr[i], z1 = zptr[i + 1], a0 = azptr[i], a1 = azptr[i + 1];
  int32_t zc = 0, ac = 0;
  T zw = 0, ar = 0, ai = 0;
  if (u < 4 && z0 + u < z1) {
    zc = zcol[z0 + u];
    zw = (T)zval[z0 + u];
  }
  if (a0 + u < a1) {
    ac = azcol[a0 + u];
    const cplx<T> x = az[a0 + u];
    ar = x.re;
    ai = x.im;
  }
  for (int c0 = 0; c0 < s; c0 += 16) {
    const int col = c0 + u;
    const int cl = col < s ? col : s - 1;  // lanes past the last column repeat it, store nothing
    const c128 vk = v[i * s + cl];
    cplx<T> qa = cmk((T)0, (T)0), ta = cmk((T)0, (T)0);
    {
      int32_t jc[4];
      T w[4];
      cplx<T> y[4];
      row_lanes<0, 4>(zc, jc);
      row_lanes<0, 4>(zw, w);
#pragma unroll
      for (int e = 0; e < 4; ++e) y[e] = y2[(int64_t)jc[e] * s + cl];
#pragma unroll
      for (int e = 0; e < 4; ++e) cfma(qa, cmk(w[e], (T)0), y[e]);
    }
    {
      int32_t jc[8];
      T wr[8], wi[8];
      cplx<T> y[8];
      row_lanes<0, 8>(ac, jc);
      row_lanes<0, 8>(ar, wr);
      row_lanes<0, 8>(ai, wi);
#pragma unroll
      for (int e = 0; e < 8; ++e) y[e] = y2[(int64_t)jc[e] * s + cl];
#pragma unroll
      for (int e = 0; e < 8; ++e) cfma(ta, cmk(wr[e], wi[e]), y[e]);
    }
    if (a1 - a0 > 8) {  // the same for every lane of the row
      int32_t jc[8];
      T wr[8], wi[8];
      cplx<T> y[8];
      row_lanes<8, 8>(ac, jc);
      row_lanes<8, 8>(ar, wr);
      row_lanes<8, 8>(ai, wi);
#pragma unroll
      for (int e = 0; e < 8; ++e) y[e] = y2[(int64_t)jc[e] * s + cl];
#pragma unroll
      for (int e = 0; e < 8; ++e) cfma(ta, cmk(wr[e], wi[e]), y[e]);
    }
    for (int64_t e = z0 + 4; e < z1; e += 4) {
      int32_t jc[4];
      T zv[4];
      cplx<T> yv[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const bool ok = e + w < z1;
        jc[w] = zcol[ok ? e + w : e];
        zv[w] = ok ? (T)zval[e + w] : (T)0;
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) yv[w] = y2[(int64_t)jc[w] * s + cl];
#pragma unroll
      for (int w = 0; w < 4; ++w) cfma(qa, cmk(zv[w], (T)0), yv[w]);
    }
    for (int64_t e = a0 + 16; e < a1; e += 8) {
      int32_t jc[8];
      cplx<T> av[8], yv[8];
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const bool ok = e + w < a1;
        jc[w] = azcol[ok ? e + w : e];
        const cplx<T> x = az[ok ? e + w : e];
        av[w] = csel(ok, x, cmk((T)0, (T)0));
      }
#pragma unroll
      for (int w = 0; w < 8; ++w) yv[w] = y2[(int64_t)jc[w] * s + cl];
#pragma unroll
      for (int w = 0; w < 8; ++w) cfma(ta, av[w], yv[w]);
    }
    if (col < s) {
      q[i * s + col] = qa;
      const c128 r = vk - cmk((double)ta.re, (double)ta.im);
      t[i * s + col] = cmk((T)r.re, (T)r.im);
    }
  }
}

}  // namespace

void coarse_setup(Ctx* ctx, Ddm& d) {
  CoarseSpace& cs = *d.coarse;
  const Mesh& m = *d.op->mesh;
  hipStream_t st = ctx->stream;
  cs.d_zptr.upload(ctx, cs.zptr);
  cs.d_zcol.upload(ctx, cs.zcol);
  cs.d_zval.upload(ctx, cs.zval);
  cs.d_ztptr.upload(ctx, cs.ztptr);
  cs.d_ztcol.upload(ctx, cs.ztcol);
  cs.d_ztval.upload(ctx, cs.ztval);
  cs.d_azptr.upload(ctx, cs.azptr);
  cs.d_azcol.upload(ctx, cs.azcol);
  const int64_t nnz_az = (int64_t)cs.azcol.size();
  {
    std::vector<int32_t> azrow(nnz_az);
    for (int64_t i = 0; i < m.n; ++i)
      for (int64_t e = cs.azptr[i]; e < cs.azptr[i + 1]; ++e) azrow[e] = (int32_t)i;
    DevArray<int32_t> d_azrow;
    d_azrow.upload(ctx, azrow);
    cs.d_az.alloc(ctx, std::max<int64_t>(1, nnz_az));
    cs.d_az32.alloc(ctx, std::max<int64_t>(1, nnz_az));
    hipLaunchKernelGGL(k_az, dim3((unsigned)((nnz_az + 255) / 256)), dim3(256), 0, st, m.n, d.op->mesh->d_rowptr.ptr(),
                       d.op->mesh->d_col.ptr(), d.op->d_val.ptr(), cs.d_zptr.ptr(), cs.d_zcol.ptr(), cs.d_zval.ptr(),
                       cs.d_azptr.ptr(), cs.d_azcol.ptr(), d_azrow.ptr(), nnz_az, cs.d_az.ptr(), cs.d_az32.ptr());
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
  }
  const int64_t nc = cs.nc;
  HZ_REQUIRE(nc >= 1 && nc <= 65535, HZ_ERR_ARG, "coarse space: 1 to 65535 coarse vertices");
  DevArray<c128> E;
  E.alloc(ctx, nc * nc);
  {
    DevArray<c128> Er;
    Er.alloc(ctx, nc * nc);
    Er.zero(ctx);
    hipLaunchKernelGGL(k_ztaz, dim3((unsigned)nc), dim3(64), 0, st, nc, cs.d_ztptr.ptr(), cs.d_ztcol.ptr(),
                       cs.d_ztval.ptr(), cs.d_azptr.ptr(), cs.d_azcol.ptr(), cs.d_az.ptr(), Er.ptr());
    hipLaunchKernelGGL(k_to_colmajor, dim3((unsigned)((nc * nc + 255) / 256)), dim3(256), 0, st, nc, Er.ptr(), E.ptr());
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
  }
  cs.d_piv.alloc(ctx, nc);
  if (d.precision == HZ_PREC_MIXED) {
    DevArray<c64> E32;
    E32.alloc(ctx, nc * nc);
    hipLaunchKernelGGL(k_c128_to_c64, dim3((unsigned)((nc * nc + 255) / 256)), dim3(256), 0, st, nc * nc, E.ptr(),
                       E32.ptr());
    cs.d_E32.alloc(ctx, nc * nc);
    lu_and_inverse<float>(ctx, nc, E32.ptr(), cs.d_piv.ptr(), cs.d_E32.ptr());
    HIP_CHECK(hipStreamSynchronize(st));
  } else {
    cs.d_E.alloc(ctx, nc * nc);
    lu_and_inverse<double>(ctx, nc, E.ptr(), cs.d_piv.ptr(), cs.d_E.ptr());
    HIP_CHECK(hipStreamSynchronize(st));
  }
}

template <typename T>
static void coarse_apply_t(Ctx* ctx, Ddm& d, int s, const c128* v, cplx<T>* q, cplx<T>* t, const cplx<T>* Einv,
                           const cplx<T>* az) {
  CoarseSpace& cs = *d.coarse;
  hipStream_t st = ctx->stream;
  const int64_t nc = cs.nc, n = d.op->mesh->n;
  constexpr int KS = 32;
  const int64_t kchunk = (nc + KS - 1) / KS;
  const size_t need = (size_t)(nc * s) * sizeof(cplx<T>);
  if (cs.w_y.bytes < need) {  // kept for the life of the ddm: no allocation on the solve path after the first call
    cs.w_y.alloc(ctx, need);
    cs.w_y2.alloc(ctx, need);
    cs.w_part.alloc(ctx, need * KS);
  }
  cplx<T>* y = cs.w_y.as<cplx<T>>();
  cplx<T>* y2 = cs.w_y2.as<cplx<T>>();
  hipLaunchKernelGGL(k_restrict<T>, dim3((unsigned)nc), dim3(1024), 0, st, nc, s, cs.d_ztptr.ptr(), cs.d_ztcol.ptr(),
                     cs.d_ztval.ptr(), v, y);
  hipLaunchKernelGGL(k_dense_apply<T>, dim3((unsigned)((nc + 63) / 64), KS), dim3(256), 0, st, nc, s, kchunk, Einv, y,
                     cs.w_part.as<cplx<T>>());
  hipLaunchKernelGGL(k_dense_reduce<T>, dim3((unsigned)((nc * s + 255) / 256)), dim3(256), 0, st, KS, nc * s,
                     cs.w_part.as<cplx<T>>(), y2);
  hipLaunchKernelGGL(k_prolong<T>, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, st, n, s, cs.d_zptr.ptr(),
                     cs.d_zcol.ptr(), cs.d_zval.ptr(), cs.d_azptr.ptr(), cs.d_azcol.ptr(), az, y2, v, q, t);
  HIP_CHECK(hipGetLastError());
}

void coarse_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c64* q, c64* t) {
  HZ_REQUIRE(d.precision == HZ_PREC_MIXED, HZ_ERR_STATE, "coarse correction: complex64 blocks need mixed precision");
  coarse_apply_t<float>(ctx, d, s, v, q, t, d.coarse->d_E32.ptr(), d.coarse->d_az32.ptr());
}

void coarse_apply(Ctx* ctx, Ddm& d, int s, const c128* v, c128* q, c128* t) {
  HZ_REQUIRE(d.precision != HZ_PREC_MIXED, HZ_ERR_STATE, "coarse correction: complex128 blocks need FP64");
  coarse_apply_t<double>(ctx, d, s, v, q, t, d.coarse->d_E.ptr(), d.coarse->d_az.ptr());
}

}  // namespace hz
