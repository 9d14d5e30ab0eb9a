// C ABI of libhz (include/hz.h): argument checks, handle tables, host/device marshalling.
#include <algorithm>
#include <cmath>
#include <new>

#include "krylov.h"
#include "noalloc.h"
#include "prof.h"
#include "serve.h"

struct hz_ctx : hz::Ctx {};

namespace hz {

[[noreturn]] void fail(hz_status code, const std::string& msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    const char* base = std::strrchr(file, '/');
    throw Error(HZ_ERR_HIP, std::string(hipGetErrorString(e)) + " in " + what + " (" + (base ? base + 1 : file) + ":" +
                                std::to_string(line) + ")");
  }
}

DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
  if (this != &o) {
    release();
    p = o.p;
    bytes = o.bytes;
    ctx = o.ctx;
    o.p = nullptr;
    o.bytes = 0;
    o.ctx = nullptr;
  }
  return *this;
}

void DevBuf::alloc(Ctx* c, size_t nbytes) {
  release();
  if (nbytes == 0) nbytes = 16;
  void* q = nullptr;
  if (c->alloc_fn) {
    q = c->alloc_fn(nbytes, (void*)c->stream, c->alloc_user);
    if (!q) fail(HZ_ERR_OOM, "device allocation of " + std::to_string(nbytes) + " bytes failed (caller allocator)");
  } else {
    const hipError_t e = hipMalloc(&q, nbytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      size_t fr = 0, tot = 0;
      (void)hipMemGetInfo(&fr, &tot);
      fail(HZ_ERR_OOM, "device allocation of " + std::to_string(nbytes) + " bytes failed (device: " +
                           std::to_string(fr >> 20) + " of " + std::to_string(tot >> 20) + " MiB free; the library holds " +
                           std::to_string((int64_t)c->bytes_in_use >> 20) + " MiB)");
    }
  }
  p = q;
  bytes = nbytes;
  ctx = c;
  c->bytes_in_use += (int64_t)nbytes;
}

void DevBuf::release() {
  if (p) {
    if (ctx && ctx->free_fn)
      ctx->free_fn(p, (void*)ctx->stream, ctx->alloc_user);  // stream-ordered release
    else
      (void)hipFree(p);
    if (ctx) ctx->bytes_in_use -= (int64_t)bytes;
  }
  p = nullptr;
  bytes = 0;
  ctx = nullptr;
}

template <typename T>
void DevArray<T>::upload(Ctx* c, const T* host, size_t count) {
  alloc(c, count);
  if (count) {
    HIP_CHECK(hipMemcpyAsync(ptr(), host, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
  }
}
template <typename T>
void DevArray<T>::zero(Ctx* c) {
  if (n) HIP_CHECK(hipMemsetAsync(ptr(), 0, n * sizeof(T), c->stream));
}
template struct DevArray<int32_t>;
template struct DevArray<int64_t>;
template struct DevArray<uint32_t>;
template struct DevArray<uint8_t>;
template struct DevArray<double>;
template struct DevArray<c128>;
template struct DevArray<c64>;
template struct DevArray<FrontDesc>;
template struct DevArray<unsigned long long>;

}  // namespace hz

using namespace hz;

namespace {

template <typename F>
hz_status guard(hz_ctx* c, F&& f) {
  if (!c) return HZ_ERR_ARG;
  if (c->poisoned) {
    c->last_error = "context poisoned by an earlier HIP error";
    return HZ_ERR_HIP;
  }
  if (c->serving) {
    c->last_error = "the context is serving: only hz_serve_* calls until hz_serve_stop";
    return HZ_ERR_STATE;
  }
  try {
    HIP_CHECK(hipSetDevice(c->device));
    f();
    return HZ_OK;
  } catch (const Error& e) {
    c->last_error = e.what();
    if (e.code == HZ_ERR_HIP) c->poisoned = true;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return HZ_ERR_OOM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return HZ_ERR_STATE;
  }
}

template <typename M>
auto lookup(hz_ctx* c, M& table, hz_handle h, const char* what) -> decltype(table.begin()->second) {
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = table.find(h);
  if (it == table.end()) fail(HZ_ERR_ARG, std::string("unknown ") + what + " handle");
  return it->second;
}

hz_handle new_handle(hz_ctx* c) {
  std::lock_guard<std::mutex> lk(c->mu);
  return c->next_handle++;
}

// stage a [s][n] complex128 block on the device (copy if host)
struct Staged {
  DevArray<c128> buf;
  const c128* ptr = nullptr;
};

void stage_in(hz_ctx* c, const void* p, int mem, int64_t count, Staged& st) {
  HZ_REQUIRE(p, HZ_ERR_ARG, "null block pointer");
  HZ_REQUIRE(mem == HZ_MEM_HOST || mem == HZ_MEM_DEVICE, HZ_ERR_ARG, "bad memory kind");
  if (mem == HZ_MEM_DEVICE) {
    st.ptr = static_cast<const c128*>(p);
  } else {
    const double* h = static_cast<const double*>(p);
    for (int64_t i = 0; i < 2 * count; ++i) HZ_REQUIRE(std::isfinite(h[i]), HZ_ERR_ARG, "non-finite input value");
    st.buf.upload(c, static_cast<const c128*>(p), count);
    st.ptr = st.buf.ptr();
  }
}

void copy_out(hz_ctx* c, const c128* dev, void* dst, int mem, int64_t count) {
  HZ_REQUIRE(mem == HZ_MEM_HOST || mem == HZ_MEM_DEVICE, HZ_ERR_ARG, "bad memory kind");
  HIP_CHECK(hipMemcpyAsync(dst, dev, count * sizeof(c128),
                           mem == HZ_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
}

}  // namespace

extern "C" {

hz_status hz_init(hz_ctx** out, const hz_init_opts* opts) {
  if (!out) return HZ_ERR_ARG;
  *out = nullptr;
  if (opts && opts->struct_size != sizeof(hz_init_opts)) return HZ_ERR_ABI;
  hz_ctx* c = new (std::nothrow) hz_ctx();
  if (!c) return HZ_ERR_OOM;
  c->device = opts ? opts->device : 0;
  c->stream = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
  if (opts && ((opts->alloc == nullptr) != (opts->free == nullptr))) {
    delete c;
    return HZ_ERR_ARG;  // an allocator needs both calls
  }
  if (opts) {
    c->alloc_fn = opts->alloc;
    c->free_fn = opts->free;
    c->alloc_user = opts->alloc_user;
  }
  hz_status st = guard(c, [&] {
    int ndev = 0;
    HIP_CHECK(hipGetDeviceCount(&ndev));
    HZ_REQUIRE(c->device >= 0 && c->device < ndev, HZ_ERR_ARG, "hz_init: no such device");
    HIP_CHECK(hipSetDevice(c->device));
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    c->hbm_budget = (opts && opts->hbm_budget) ? opts->hbm_budget : (size_t)(0.9 * (double)fr);
    const char* tr = std::getenv("HZ_TRACE");
    c->trace = tr && tr[0] && tr[0] != '0';
    p3_upload_tables(c);
    noalloc_init(c->device);
  });
  if (st != HZ_OK) {
    delete c;
    return st;
  }
  *out = c;
  return HZ_OK;
}

void hz_finalize(hz_ctx* c) {
  if (!c) return;
  if (c->serve) {
    hz_serve_stop(c);
  }
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& kv : c->ddms) precond_release_workspace(*kv.second);
    c->krylov_ws.release();
    c->krylov_io.release();
    c->ddms.clear();
    c->ops.clear();
    c->meshes.clear();
  }
  delete c->prof;
  c->prof = nullptr;
  delete c;
}

const char* hz_last_error(const hz_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

hz_status hz_release(hz_ctx* c, hz_handle h) {
  return guard(c, [&] {
    HIP_CHECK(hipStreamSynchronize(c->stream));
    krylov_cache_release(c);  // releasing objects gives back the solves' cached workspace too
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->meshes.erase(h)) return;
    if (c->ops.erase(h)) return;
    auto it = c->ddms.find(h);
    if (it != c->ddms.end()) {
      precond_release_workspace(*it->second);
      c->ddms.erase(it);
      return;
    }
    fail(HZ_ERR_ARG, "hz_release: unknown handle");
  });
}

hz_status hz_mesh(hz_ctx* c, int64_t n_tets, const int32_t* tets, int64_t n_verts, const double* coords,
                  const int8_t* face_bc, hz_handle* mesh, int64_t* n_dofs) {
  return guard(c, [&] {
    HZ_REQUIRE(mesh && n_dofs, HZ_ERR_ARG, "hz_mesh: null output");
    auto m = build_mesh(c, n_tets, tets, n_verts, coords, face_bc);
    // global pattern and its rows' element incidences (impedance faces of the physical boundary)
    std::vector<int64_t> all(m->T);
    for (int64_t t = 0; t < m->T; ++t) all[t] = t;
    std::vector<int32_t> loc(m->n);
    for (int64_t g = 0; g < m->n; ++g) loc[g] = (int32_t)g;
    std::vector<uint8_t> robin(m->T, 0);
    for (int64_t t = 0; t < m->T; ++t)
      for (int f = 0; f < 4; ++f)
        if (m->tag[4 * t + f] == HZ_BC_IMPEDANCE) robin[t] |= (uint8_t)(1u << f);
    RowIncidence inc;
    build_pattern_and_incidence(*m, all, loc, m->n, m->rowptr, m->col, inc);
    m->d_rowptr.upload(c, m->rowptr);
    m->d_col.upload(c, m->col);
    m->d_inc_ptr.upload(c, inc.ptr);
    m->d_inc.upload(c, inc.idx);
    m->d_robin.upload(c, robin);
    const hz_handle h = new_handle(c);
    std::lock_guard<std::mutex> lk(c->mu);
    c->meshes[h] = m;
    *mesh = h;
    *n_dofs = m->n;
  });
}

hz_status hz_assemble(hz_ctx* c, hz_handle mesh, const double* velocity, const double* Q, double freq_hz,
                      hz_handle* op) {
  return guard(c, [&] {
    HZ_REQUIRE(velocity && op, HZ_ERR_ARG, "hz_assemble: null pointer");
    HZ_REQUIRE(std::isfinite(freq_hz) && freq_hz > 0, HZ_ERR_ARG, "hz_assemble: frequency must be > 0");
    auto m = lookup(c, c->meshes, mesh, "mesh");
    for (int64_t t = 0; t < m->T; ++t) {
      HZ_REQUIRE(std::isfinite(velocity[t]) && velocity[t] > 0, HZ_ERR_ARG, "hz_assemble: velocity must be finite and > 0");
      if (Q) HZ_REQUIRE(std::isfinite(Q[t]) && Q[t] > 0, HZ_ERR_ARG, "hz_assemble: Q must be finite and > 0");
    }
    auto o = std::make_shared<Operator>();
    o->mesh = m;
    o->freq = freq_hz;
    o->has_q = Q != nullptr;
    o->velocity.assign(velocity, velocity + m->T);
    if (Q) o->Q.assign(Q, Q + m->T);
    DevArray<double> dv, dq;
    dv.upload(c, o->velocity);
    if (Q) dq.upload(c, o->Q);
    o->d_k.alloc(c, m->T);
    o->d_elem.alloc(c, m->T * kElemStride);
    launch_element_matrices(c, *m, *o, dv.ptr(), Q ? dq.ptr() : nullptr);
    o->d_val.alloc(c, m->nnz());
    o->d_val32.alloc(c, m->nnz());
    launch_incidence_fill(c->stream, m->n, m->d_rowptr.ptr(), m->d_col.ptr(), nullptr, m->d_inc_ptr.ptr(),
                          m->d_inc.ptr(), nullptr, m->d_robin.ptr(), m->d_tet_dofs.ptr(), o->d_elem.ptr(),
                          m->d_dirichlet.ptr(), o->d_val.ptr(), o->d_val32.ptr());
    HIP_CHECK(hipStreamSynchronize(c->stream));
    // the element matrices are recomputed when a decomposition needs its local operators
    o->d_elem = DevArray<c128>();
    const hz_handle h = new_handle(c);
    std::lock_guard<std::mutex> lk(c->mu);
    c->ops[h] = o;
    *op = h;
  });
}

hz_status hz_setup_ddm_ex(hz_ctx* c, hz_handle op, const int32_t* partition, int32_t n_sub, int32_t overlap,
                          const hz_coarse_mesh* coarse, const hz_ddm_opts* opts, hz_handle* ddm) {
  return guard(c, [&] {
    HZ_REQUIRE(ddm, HZ_ERR_ARG, "hz_setup_ddm: null output");
    HZ_REQUIRE(opts && opts->struct_size == sizeof(hz_ddm_opts), HZ_ERR_ABI, "hz_setup_ddm_ex: bad options struct");
    auto o = lookup(c, c->ops, op, "operator");
    krylov_cache_release(c);  // set-up sizes its arena by the free memory
    auto d = build_ddm(c, o, partition, n_sub, overlap, coarse, opts->precision, opts->pou, opts->local_solver);
    const hz_handle h = new_handle(c);
    std::lock_guard<std::mutex> lk(c->mu);
    c->ddms[h] = d;
    *ddm = h;
  });
}

hz_status hz_setup_ddm(hz_ctx* c, hz_handle op, const int32_t* partition, int32_t n_sub, int32_t overlap,
                       const hz_coarse_mesh* coarse, int precision, hz_handle* ddm) {
  hz_ddm_opts o{};
  o.struct_size = sizeof(o);
  o.precision = precision;
  o.pou = HZ_POU_BOOLEAN;
  o.local_solver = HZ_LOCAL_EXACT;
  return hz_setup_ddm_ex(c, op, partition, n_sub, overlap, coarse, &o, ddm);
}

hz_status hz_get_pou(hz_ctx* c, hz_handle ddm, int32_t i, double* weights) {
  return guard(c, [&] {
    auto d = lookup(c, c->ddms, ddm, "ddm");
    HZ_REQUIRE(i >= 0 && i < d->n_sub && weights, HZ_ERR_ARG, "hz_get_pou: bad arguments");
    const Subdomain& S = d->subs[i];
    if (d->pou == HZ_POU_SMOOTH)
      std::copy(S.pouw.begin(), S.pouw.end(), weights);
    else
      for (int64_t l = 0; l < S.n; ++l) weights[l] = S.owned[l] ? 1.0 : 0.0;
  });
}

hz_status hz_solve_ex(hz_ctx* c, hz_handle ddm, int64_t n_rhs, const void* rhs, int rhs_mem, const hz_solve_opts* opts,
                      void* x, int x_mem, hz_col_info* info) {
  return guard(c, [&] {
    HZ_REQUIRE(opts && opts->struct_size == sizeof(hz_solve_opts), HZ_ERR_ABI, "hz_solve_ex: bad options struct");
    HZ_REQUIRE(n_rhs >= 1 && x && info, HZ_ERR_ARG, "hz_solve: bad arguments");
    HZ_REQUIRE(opts->tol >= 0 && std::isfinite(opts->tol), HZ_ERR_ARG, "hz_solve: bad tolerance");
    HZ_REQUIRE(opts->max_iter >= 1 || opts->fixed_iters > 0, HZ_ERR_ARG, "hz_solve: max_iter must be >= 1");
    auto d = lookup(c, c->ddms, ddm, "ddm");
    const int64_t n = d->op->mesh->n;
    Staged B;
    stage_in(c, rhs, rhs_mem, n_rhs * n, B);
    HZ_REQUIRE(count_nonfinite(c, B.ptr, n_rhs * n) == 0, HZ_ERR_ARG, "hz_solve: non-finite right-hand side");
    // device x: the blocks' solutions go straight to it; host x: through one device copy
    DevArray<c128> Xd;
    HZ_REQUIRE(x_mem == HZ_MEM_HOST || x_mem == HZ_MEM_DEVICE, HZ_ERR_ARG, "hz_solve: bad memory kind");
    if (x_mem == HZ_MEM_HOST) Xd.alloc(c, n_rhs * n);
    c128* Xout = x_mem == HZ_MEM_HOST ? Xd.ptr() : static_cast<c128*>(x);
    SolveOptions so;
    so.tol = opts->tol;
    so.max_iter = opts->max_iter > 0 ? opts->max_iter : 500;
    so.restart = opts->restart > 0 ? opts->restart : 40;
    so.fixed_iters = opts->fixed_iters;
    const bool z32 = d->precision == HZ_PREC_MIXED;
    // block width and restart length: a short memory supply narrows the block (automatic width)
    // before it shortens the restart, which changes the iteration
    const int want = so.fixed_iters > 0 ? std::max(so.restart, so.fixed_iters) : so.restart;
    int blk = (int)std::min<int64_t>(n_rhs, opts->block > 0 ? std::min(opts->block, 32) : 32);
    // the block's node-major right-hand side and solution (2 n b complex128) come on top
    int m = 0;
    if (opts->block <= 0) {
      for (int b = blk; b >= 1; b = b > 1 ? b / 2 : 0) {
        const int mb = FgmresJob::restart_fit(c, n, b, want, so.fixed_iters, z32, 2 * n * b * (int64_t)sizeof(c128));
        if (mb == want || b == 1) {
          blk = b;
          m = mb;
          break;
        }
      }
    } else {
      m = FgmresJob::restart_fit(c, n, blk, want, so.fixed_iters, z32, 2 * n * blk * (int64_t)sizeof(c128));
    }
    HZ_REQUIRE(m > 0, HZ_ERR_OOM,
               so.fixed_iters > 0 ? "hz_solve: the Krylov basis for fixed_iters steps does not fit in device memory"
                                  : "hz_solve: not even a restart length of 8 fits in device memory");
    bool all_ok = true;
    // the blocks' node-major right-hand side and solution, kept with the context between solves
    if ((int64_t)c->krylov_io.bytes < 2 * n * blk * (int64_t)sizeof(c128)) {
      c->krylov_io.release();
      c->krylov_io.alloc(c, 2 * n * blk * sizeof(c128));
    }
    c128* Bn = c->krylov_io.as<c128>();
    c128* Xn = Bn + n * blk;
    for (int64_t c0 = 0; c0 < n_rhs; c0 += blk) {
      const int s = (int)std::min<int64_t>(blk, n_rhs - c0);
      KrylovKernels K(c, n, s);
      K.to_node(B.ptr + c0 * n, Bn);
      std::vector<ColInfo> ci;
      fgmres(c, d, s, Bn, Xn, so, m, ci);
      K.from_node(Xn, Xout + c0 * n);
      for (int k = 0; k < s; ++k) {
        info[c0 + k].iters = ci[k].iters;
        info[c0 + k].restarts = ci[k].restarts;
        info[c0 + k].rel_residual = ci[k].rel_residual;
        info[c0 + k].status = ci[k].status;
        info[c0 + k].restart_len = ci[k].m;
        info[c0 + k].block = ci[k].block;
        all_ok = all_ok && ci[k].status == HZ_OK;
      }
    }
    if (x_mem == HZ_MEM_HOST) copy_out(c, Xd.ptr(), x, x_mem, n_rhs * n);
    HIP_CHECK(hipStreamSynchronize(c->stream));
    if (!all_ok) fail(HZ_ERR_NOT_CONVERGED, "hz_solve: max_iter reached before the tolerance");
  });
}

hz_status hz_solve(hz_ctx* c, hz_handle ddm, int64_t n_rhs, const void* rhs, int rhs_mem, double tol, int32_t max_iter,
                   void* x, int x_mem, hz_col_info* info) {
  hz_solve_opts o{};
  o.struct_size = sizeof(o);
  o.tol = tol;
  o.max_iter = max_iter;
  return hz_solve_ex(c, ddm, n_rhs, rhs, rhs_mem, &o, x, x_mem, info);
}

hz_status hz_point_sources(hz_ctx* c, hz_handle mesh, int64_t n_src, const double* xyz, const double* amp, void* rhs,
                           int rhs_mem) {
  return guard(c, [&] {
    HZ_REQUIRE(n_src >= 1 && xyz && rhs, HZ_ERR_ARG, "hz_point_sources: bad arguments");
    for (int64_t k = 0; k < 3 * n_src; ++k) HZ_REQUIRE(std::isfinite(xyz[k]), HZ_ERR_ARG, "hz_point_sources: non-finite position");
    auto m = lookup(c, c->meshes, mesh, "mesh");
    DevArray<double> dx, da;
    dx.upload(c, xyz, 3 * n_src);
    if (amp) da.upload(c, amp, 2 * n_src);
    DevArray<unsigned long long> best;
    best.alloc(c, n_src);
    DevArray<c128> out;
    out.alloc(c, n_src * m->n);
    launch_point_sources(c, *m, n_src, dx.ptr(), amp ? da.ptr() : nullptr, best.ptr(), out.ptr());
    copy_out(c, out.ptr(), rhs, rhs_mem, n_src * m->n);
  });
}

hz_status hz_spmm_noalloc(hz_ctx* c, hz_handle op, int64_t n_rhs, const void* x, void* y) {
  return guard(c, [&] {
    HZ_REQUIRE(n_rhs >= 1 && x && y, HZ_ERR_ARG, "hz_spmm_noalloc: bad arguments");
    auto o = lookup(c, c->ops, op, "operator");
    spmm_noalloc(c, *o, n_rhs, static_cast<const c128*>(x), static_cast<c128*>(y));
    HIP_CHECK(hipStreamSynchronize(c->stream));
  });
}

hz_status hz_spmm(hz_ctx* c, hz_handle op, int64_t n_rhs, const void* x, int x_mem, void* y, int y_mem) {
  return guard(c, [&] {
    HZ_REQUIRE(n_rhs >= 1 && y, HZ_ERR_ARG, "hz_spmm: bad arguments");
    auto o = lookup(c, c->ops, op, "operator");
    const int64_t n = o->mesh->n;
    Staged X;
    stage_in(c, x, x_mem, n_rhs * n, X);
    DevArray<c128> Yd, Xn, Yn;
    Yd.alloc(c, n_rhs * n);
    for (int64_t c0 = 0; c0 < n_rhs; c0 += 32) {
      const int s = (int)std::min<int64_t>(32, n_rhs - c0);
      Xn.alloc(c, n * s);
      Yn.alloc(c, n * s);
      KrylovKernels K(c, n, s);
      K.to_node(X.ptr + c0 * n, Xn.ptr());
      launch_spmm<double>(c->stream, n, s, o->mesh->d_rowptr.ptr(), o->mesh->d_col.ptr(), o->d_val.ptr(), Xn.ptr(),
                          Yn.ptr(), cmk(1.0, 0.0), cmk(0.0, 0.0), nullptr);
      K.from_node(Yn.ptr(), Yd.ptr() + c0 * n);
    }
    copy_out(c, Yd.ptr(), y, y_mem, n_rhs * n);
  });
}

hz_status hz_spmm_c64x(hz_ctx* c, hz_handle op, int64_t n_rhs, const void* x, int x_mem, void* y, int y_mem) {
  return guard(c, [&] {
    HZ_REQUIRE(n_rhs >= 1 && x && y, HZ_ERR_ARG, "hz_spmm_c64x: bad arguments");
    HZ_REQUIRE(x_mem == HZ_MEM_HOST || x_mem == HZ_MEM_DEVICE, HZ_ERR_ARG, "bad memory kind");
    auto o = lookup(c, c->ops, op, "operator");
    const int64_t n = o->mesh->n;
    DevArray<c64> Xh;
    const c64* X = static_cast<const c64*>(x);
    if (x_mem == HZ_MEM_HOST) {
      const float* h = static_cast<const float*>(x);
      for (int64_t i = 0; i < 2 * n_rhs * n; ++i) HZ_REQUIRE(std::isfinite(h[i]), HZ_ERR_ARG, "non-finite input value");
      Xh.upload(c, X, n_rhs * n);
      X = Xh.ptr();
    }
    DevArray<c128> Yd, Yn;
    DevArray<c64> Xn;
    Yd.alloc(c, n_rhs * n);
    for (int64_t c0 = 0; c0 < n_rhs; c0 += 32) {
      const int s = (int)std::min<int64_t>(32, n_rhs - c0);
      Xn.alloc(c, n * s);
      Yn.alloc(c, n * s);
      KrylovKernels K(c, n, s);
      K.to_node(X + c0 * n, Xn.ptr());
      launch_spmm<float>(c->stream, n, s, o->mesh->d_rowptr.ptr(), o->mesh->d_col.ptr(), o->d_val.ptr(), Xn.ptr(),
                         Yn.ptr(), cmk(1.0, 0.0), cmk(0.0, 0.0), nullptr);
      K.from_node(Yn.ptr(), Yd.ptr() + c0 * n);
    }
    copy_out(c, Yd.ptr(), y, y_mem, n_rhs * n);
  });
}

hz_status hz_precond(hz_ctx* c, hz_handle ddm, int64_t n_rhs, const void* v, int v_mem, void* z, int z_mem) {
  return guard(c, [&] {
    HZ_REQUIRE(n_rhs >= 1 && z, HZ_ERR_ARG, "hz_precond: bad arguments");
    auto d = lookup(c, c->ddms, ddm, "ddm");
    const int64_t n = d->op->mesh->n;
    Staged V;
    stage_in(c, v, v_mem, n_rhs * n, V);
    DevArray<c128> Zd, Vn, Zn;
    Zd.alloc(c, n_rhs * n);
    for (int64_t c0 = 0; c0 < n_rhs; c0 += 32) {
      const int s = (int)std::min<int64_t>(32, n_rhs - c0);
      Vn.alloc(c, n * s);
      Zn.alloc(c, n * s);
      KrylovKernels K(c, n, s);
      K.to_node(V.ptr + c0 * n, Vn.ptr());
      precond_apply(c, *d, s, Vn.ptr(), Zn.ptr());
      K.from_node(Zn.ptr(), Zd.ptr() + c0 * n);
    }
    copy_out(c, Zd.ptr(), z, z_mem, n_rhs * n);
  });
}

hz_status hz_ddm_stats_get(hz_ctx* c, hz_handle ddm, hz_ddm_stats* out) {
  return guard(c, [&] {
    HZ_REQUIRE(out, HZ_ERR_ARG, "null output");
    auto d = lookup(c, c->ddms, ddm, "ddm");
    out->n_dofs = d->op->mesh->n;
    out->nnz = d->op->mesh->nnz();
    out->n_sub = d->n_sub;
    out->local_dofs_total = d->n_local_total;
    out->factor_entries = d->factor_entries;
    out->n_fronts = (int64_t)d->fronts.size();
    out->n_levels = (int64_t)d->levels.size();
    out->max_front = d->max_front;
    out->n_coarse = d->coarse ? d->coarse->nc : 0;
    out->static_pivots = d->static_pivots;
    out->update_entries = d->update_entries;
    out->factor_useful = d->factor_useful;
    out->device_bytes = d->device_bytes();
    out->setup_seconds = d->setup_seconds;
    out->factor_seconds = d->factor_seconds;
    out->factor_flops = d->factor_flops;
    out->local_solver = d->local_solver;
    out->icc_entries = d->icc ? d->icc->nnz + d->n_local_total : 0;
    out->icc_levels = d->icc ? d->icc->n_fwd : 0;
  });
}

hz_status hz_ddm_levels(hz_ctx* c, hz_handle ddm, hz_ddm_level* out, int32_t max_levels, int32_t* n_levels) {
  return guard(c, [&] {
    HZ_REQUIRE(n_levels, HZ_ERR_ARG, "null level count");
    HZ_REQUIRE(out || max_levels <= 0, HZ_ERR_ARG, "null output");
    auto d = lookup(c, c->ddms, ddm, "ddm");
    const int32_t L = (int32_t)d->levels.size();
    for (int32_t i = 0; i < std::min(L, max_levels); ++i) {
      const Level& lv = d->levels[i];
      out[i].n_fronts = (int64_t)lv.fronts.size();
      out[i].max_pivots = lv.max_p;
      out[i].max_front = lv.max_f;
      out[i].sum_pivots = lv.sum_p;
      out[i].sum_front = lv.sum_f;
      out[i].factor_useful = lv.useful;
      const bool tuned = d->tile_fwd[0].size() == (size_t)L;
      out[i].fwd_tile_rows = tuned ? kFwdRowsMfma[d->tile_fwd[0][i]] : 0;
      out[i].bwd_tile_cols = tuned ? kBwdColsMfma[d->tile_bwd[0][i]] : 0;
    }
    *n_levels = L;
  });
}

hz_status hz_get_dofmap(hz_ctx* c, hz_handle mesh, int32_t* tet_dofs) {
  return guard(c, [&] {
    HZ_REQUIRE(tet_dofs, HZ_ERR_ARG, "null output");
    auto m = lookup(c, c->meshes, mesh, "mesh");
    std::copy(m->tet_dofs.begin(), m->tet_dofs.end(), tet_dofs);
  });
}

hz_status hz_get_csr_size(hz_ctx* c, hz_handle op, int64_t* n, int64_t* nnz) {
  return guard(c, [&] {
    auto o = lookup(c, c->ops, op, "operator");
    *n = o->mesh->n;
    *nnz = o->mesh->nnz();
  });
}

hz_status hz_get_csr(hz_ctx* c, hz_handle op, int64_t* rowptr, int32_t* col, double* val) {
  return guard(c, [&] {
    auto o = lookup(c, c->ops, op, "operator");
    if (rowptr) std::copy(o->mesh->rowptr.begin(), o->mesh->rowptr.end(), rowptr);
    if (col) std::copy(o->mesh->col.begin(), o->mesh->col.end(), col);
    if (val) copy_out(c, o->d_val.ptr(), val, HZ_MEM_HOST, o->nnz());
  });
}

hz_status hz_get_subdomain_size(hz_ctx* c, hz_handle ddm, int32_t i, int64_t* n_i, int64_t* nnz_i) {
  return guard(c, [&] {
    auto d = lookup(c, c->ddms, ddm, "ddm");
    HZ_REQUIRE(i >= 0 && i < d->n_sub, HZ_ERR_ARG, "subdomain index out of range");
    *n_i = d->subs[i].n;
    *nnz_i = (int64_t)d->subs[i].col.size();
  });
}

hz_status hz_get_subdomain(hz_ctx* c, hz_handle ddm, int32_t i, int32_t* gdofs, uint8_t* owned, int64_t* rowptr,
                           int32_t* col, double* val) {
  return guard(c, [&] {
    auto d = lookup(c, c->ddms, ddm, "ddm");
    HZ_REQUIRE(i >= 0 && i < d->n_sub, HZ_ERR_ARG, "subdomain index out of range");
    const Subdomain& S = d->subs[i];
    if (gdofs) std::copy(S.gdofs.begin(), S.gdofs.end(), gdofs);
    if (owned) std::copy(S.owned.begin(), S.owned.end(), owned);
    if (rowptr) std::copy(S.rowptr.begin(), S.rowptr.end(), rowptr);
    if (col) std::copy(S.col.begin(), S.col.end(), col);
    if (val) {
      HZ_REQUIRE(d->d_lval.ptr() != nullptr, HZ_ERR_STATE,
                 "hz_get_subdomain: the local operator values were released after the factorisation (over 2 GiB)");
      copy_out(c, d->d_lval.ptr() + S.csr_off, val, HZ_MEM_HOST, (int64_t)S.col.size());
    }
  });
}

hz_status hz_get_coarse_size(hz_ctx* c, hz_handle ddm, int64_t* n_c, int64_t* nnz) {
  return guard(c, [&] {
    auto d = lookup(c, c->ddms, ddm, "ddm");
    HZ_REQUIRE(d->coarse != nullptr, HZ_ERR_STATE, "ddm has no coarse space");
    *n_c = d->coarse->nc;
    *nnz = (int64_t)d->coarse->zcol.size();
  });
}

hz_status hz_get_coarse(hz_ctx* c, hz_handle ddm, int64_t* rowptr, int32_t* col, double* val) {
  return guard(c, [&] {
    auto d = lookup(c, c->ddms, ddm, "ddm");
    HZ_REQUIRE(d->coarse != nullptr, HZ_ERR_STATE, "ddm has no coarse space");
    const CoarseSpace& cs = *d->coarse;
    if (rowptr) std::copy(cs.zptr.begin(), cs.zptr.end(), rowptr);
    if (col) std::copy(cs.zcol.begin(), cs.zcol.end(), col);
    if (val) std::copy(cs.zval.begin(), cs.zval.end(), val);
  });
}

}  // extern "C"
