// Internal declarations of libhz (host + device).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hz.h"

namespace hz {

// ---------------------------------------------------------------- errors

struct Error : std::runtime_error {
  hz_status code;
  Error(hz_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(hz_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIP_CHECK(x) ::hz::hip_check((x), #x, __FILE__, __LINE__)
#define HZ_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) ::hz::fail(code, msg); \
  } while (0)

// ---------------------------------------------------------------- complex

template <typename T>
struct cplx {
  T re, im;
};
using c128 = cplx<double>;
using c64 = cplx<float>;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmk(T r, T i) {
  cplx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return cmk(a.re, -a.im); }
// c ? a : b per component (in device code a select on the struct itself can be lowered
// through scratch memory, which serialises the loads feeding it)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csel(bool c, cplx<T> a, cplx<T> b) {
  return cmk(c ? a.re : b.re, c ? a.im : b.im);
}
// a += b * c
template <typename T>
__host__ __device__ __forceinline__ void cfma(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// a -= b * c
template <typename T>
__host__ __device__ __forceinline__ void cfms(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fma(-b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(-b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename T>
__host__ __device__ __forceinline__ void cfma_conj(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    T r = b.im / b.re, d = b.re + b.im * r;
    return cmk((a.re + a.im * r) / d, (a.im - a.re * r) / d);
  } else {
    T r = b.re / b.im, d = b.re * r + b.im;
    return cmk((a.re * r + a.im) / d, (a.im * r - a.re) / d);
  }
}

// ---------------------------------------------------------------- device memory

struct Ctx;

// Page-locked host array (hipHostMalloc) for small results copied to the host every step:
// the copies are direct DMA transfers instead of staged ones.
template <typename T>
struct HostPinned {
  T* p = nullptr;
  HostPinned() = default;
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
  ~HostPinned() {
    if (p) (void)hipHostFree(p);
  }
  void alloc(size_t count) {
    HIP_CHECK(hipHostMalloc((void**)&p, std::max<size_t>(1, count) * sizeof(T), hipHostMallocDefault));
    for (size_t i = 0; i < count; ++i) p[i] = T{};
  }
  T& operator[](size_t i) { return p[i]; }
  const T& operator[](size_t i) const { return p[i]; }
};

// Owning device allocation (the context's allocator, else hipMalloc / hipFree); the bytes
// are charged to the context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Ctx* ctx = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept;
  ~DevBuf() { release(); }
  void alloc(Ctx* c, size_t nbytes);
  void release();
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

template <typename T>
struct DevArray {
  DevBuf buf;
  size_t n = 0;
  void alloc(Ctx* c, size_t count) {
    buf.alloc(c, count * sizeof(T));
    n = count;
  }
  void upload(Ctx* c, const T* host, size_t count);
  void upload(Ctx* c, const std::vector<T>& v) { upload(c, v.data(), v.size()); }
  void zero(Ctx* c);
  T* ptr() const { return buf.as<T>(); }
  size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------- objects

constexpr int kElemVol = 210;               // packed lower triangle of a 20x20 element matrix
constexpr int kFaceEnt = 55;                // packed lower triangle of a 10x10 face matrix
constexpr int kElemStride = kElemVol + 4 * kFaceEnt;  // 430 complex entries per tet

struct Mesh {
  int64_t T = 0, V = 0, n = 0;
  std::vector<int32_t> tets;       // T*4
  std::vector<double> coords;      // V*3
  std::vector<int32_t> tet_dofs;   // T*20
  std::vector<int64_t> nbr;        // T*4 neighbour tet or -1
  std::vector<int8_t> tag;         // T*4: HZ_BC_NONE interior, else boundary tag
  std::vector<uint8_t> dirichlet;  // n
  std::vector<double> dof_xyz;     // n*3
  // global CSR pattern
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  // device copies
  DevArray<int32_t> d_tets;
  DevArray<double> d_coords;
  DevArray<int32_t> d_tet_dofs;
  DevArray<uint8_t> d_dirichlet;
  // global pattern and the per-row element incidences that assemble it (impedance faces
  // flagged per tet)
  DevArray<int64_t> d_rowptr, d_inc_ptr;
  DevArray<int32_t> d_col, d_inc;
  DevArray<uint8_t> d_robin;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// element incidences of the rows of an assembled operator: row r's are idx[ptr[r] ..
// ptr[r + 1]), each 20 q + l (selected tet q, element node l), in ascending q
struct RowIncidence {
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
};

struct Operator {
  std::shared_ptr<Mesh> mesh;
  double freq = 0;
  bool has_q = false;
  std::vector<double> velocity, Q;  // host copies (per tet)
  DevArray<c128> d_k;          // per tet wavenumber k_e
  DevArray<c128> d_elem;       // T * kElemStride
  DevArray<c128> d_val;        // CSR values on the mesh's pattern
  DevArray<c64> d_val32;
  int64_t nnz() const { return (int64_t)mesh->col.size(); }
};

struct Ddm;  // defined in ddm.h

// A context: one GPU, one stream.
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  bool poisoned = false;
  // caller-supplied device allocator (hz_init_opts), null = hipMalloc / hipFree
  void* (*alloc_fn)(size_t, void*, void*) = nullptr;
  void (*free_fn)(void*, void*, void*) = nullptr;
  void* alloc_user = nullptr;
  size_t hbm_budget = 0;
  std::atomic<int64_t> bytes_in_use{0};
  std::mutex mu;  // protects handle tables
  uint64_t next_handle = 1;
  std::map<uint64_t, std::shared_ptr<Mesh>> meshes;
  std::map<uint64_t, std::shared_ptr<Operator>> ops;
  std::map<uint64_t, std::shared_ptr<Ddm>> ddms;
  // reference element tables live in __constant__ memory (per device, set at init)
  struct Serve* serve = nullptr;
  std::atomic<bool> serving{false};  // a scheduler thread owns the stream: only hz_serve_* calls
  struct Prof* prof = nullptr;  // live kernel accounting (hz_profile_*)
  bool trace = false;           // HZ_TRACE=1 at hz_init: per-step solver lines on stderr
  DevBuf krylov_ws;             // Krylov workspace kept between hz_solve calls
  DevBuf krylov_io;             // hz_solve's node-major right-hand-side and solution blocks
  bool krylov_busy = false;     // a job is using krylov_ws
  // while serving: one preconditioner solve workspace shared by every ddm (the scheduler
  // applies them one after another on the context stream); null otherwise
  struct PrecondWork* shared_pw = nullptr;
};

// reference element tables (host), see p3ref.cpp
struct P3Tables {
  double S[10][kElemVol];  // combined stiffness per (a<=b) pair, packed lower triangle
  double M[kElemVol];
  double F[4][kFaceEnt];   // face mass per face, packed over the face's nodes
  int face_nodes[4][10];   // element-local node ids of each face, ascending
};
const P3Tables& p3_tables();
void p3_upload_tables(Ctx* ctx);
// basis values at barycentric point (for point sources), host reference
void p3_eval_basis(const double lam[4], double phi[20]);

inline int packed(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// mesh.cpp
std::shared_ptr<Mesh> build_mesh(Ctx* ctx, int64_t T, const int32_t* tets, int64_t V, const double* coords,
                                 const int8_t* face_bc);
// the CSR pattern of the operator assembled from a set of tets (global ids `tets_sel`,
// ascending) with local dof numbering `loc` (global dof -> local id or -1), and its rows'
// element incidences (which the device fill sums over)
void build_pattern_and_incidence(const Mesh& m, const std::vector<int64_t>& tets_sel, const std::vector<int32_t>& loc,
                                 int64_t n_local, std::vector<int64_t>& rowptr, std::vector<int32_t>& col,
                                 RowIncidence& inc);

// assemble.hip
void launch_element_matrices(Ctx* ctx, const Mesh& m, Operator& op, const double* d_vel, const double* d_q);
void launch_point_sources(Ctx* ctx, const Mesh& m, int64_t ns, const double* d_xyz, const double* d_amp,
                          unsigned long long* d_best, c128* d_rhs);
// values of an operator assembled from its rows' element incidences: entry (r, c) sums, over
// the incidences of row r in ascending tet order, the element entry (node of r, node of c)
// and then the face entries of the tet's Robin faces (bitmask robin[q]; null: none) that hold
// both nodes.  Local ids map to global dofs through gdofs (null: the identity); tsel maps a
// selected tet to its global id (null: the identity).  Rows and columns flagged in dir (per
// local dof, nullable) become identity rows and columns.
void launch_incidence_fill(hipStream_t st, int64_t n_rows, const int64_t* d_rowptr, const int32_t* d_col,
                           const int32_t* d_gdofs, const int64_t* d_inc_ptr, const int32_t* d_inc,
                           const int32_t* d_tsel, const uint8_t* d_robin, const int32_t* d_tet_dofs,
                           const c128* d_elem, const uint8_t* d_dir, c128* d_val, c64* d_val32);

// spmm.hip: y = alpha A x + beta yin (yin may be null), A complex128 CSR, x complex<TX>
// (complex64 x is widened exactly), y complex128; node-major [n][s] blocks
template <typename TX>
void launch_spmm(hipStream_t st, int64_t n, int s, const int64_t* rowptr, const int32_t* col, const c128* val,
                 const cplx<TX>* x, c128* y, c128 alpha, c128 beta, const c128* yin);

// utilities
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body);
double wall_time();

}  // namespace hz
