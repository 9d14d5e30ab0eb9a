// Serving: continuous batching of solve requests (hz_serve_*).
//
// A scheduler thread owns the context's stream while serving.  A request is split into
// parts (block-FGMRES jobs of at most 32 sources).  Requests wait in a FIFO queue; the parts
// of the queue head are admitted one at a time when a slot is free and the part's Krylov
// memory fits in the HBM budget next to the resident operators, factors and running parts.
// While the head waits for memory, parts of later requests that fit may start in its place
// (backfill), for at most kBackfillWindow seconds of the head's wait; after that admission is
// strictly FIFO until the head has started, so no request waits behind others forever.
// Each request's part width and restart length are chosen at submission: the widest part
// (32 columns and its halvings) whose restart length reaches 20 next to the resident objects,
// else the width that allows the longest restart (requests that fit at no restart length of at
// least 8 are refused).  Each
// scheduler tick advances every active job by one Arnoldi step: the blocks M^{-1} v of all
// jobs on the same operator are packed column-wise (first-fit decreasing, at most 32 columns
// a launch) into shared launches of the preconditioner and of the SpMM (so the factors and the
// matrix are read once for all of them), then each job does its own orthogonalisation and
// least-squares step.  A finished job writes its columns of the solution to the caller's
// block and frees its memory at once; a request completes when all its parts have.
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>

#include "serve.h"

namespace hz {

namespace {

__global__ void k_pack_cols(int64_t n, int s, int S, int off, const c128* __restrict__ src, c128* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t i = k / s;
  const int c = (int)(k - i * s);
  dst[i * S + off + c] = src[k];
}
template <typename T>
__global__ void k_unpack_cols(int64_t n, int s, int S, int off, const cplx<T>* __restrict__ src,
                              cplx<T>* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * s) return;
  const int64_t i = k / s;
  const int c = (int)(k - i * s);
  dst[k] = src[i * S + off + c];
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct Ticket {
  uint64_t id = 0;
  hz_request req{};
  std::shared_ptr<Ddm> ddm;
  double t_submit = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  double t_blocked = 0;  // when this request, at the queue head, first waited for memory (0: not waiting)
  int32_t status = HZ_OK;
  int m = 0;             // restart length (chosen at submission)
  int w = 32;            // part width: sources per part (chosen at submission)
  int nparts = 0;        // parts of at most w sources
  int admitted = 0;      // parts admitted by the scheduler
  int finished = 0;      // parts done
  int64_t held = 0;      // memory reserved for the admitted parts
  bool oom = false;      // a part could not start: no memory even alone, or a dependent block
  struct Part {
    int c0 = 0, s = 0;
    DevArray<c128> Bn, Xn;
    std::unique_ptr<FgmresJob> job;
    std::vector<ColInfo> info;  // kept when the job (and its Krylov memory) is released
    bool done = false;
  };
  std::vector<std::unique_ptr<Part>> parts;  // the admitted parts, in column order
};

struct Serve {
  Ctx* ctx = nullptr;
  int max_slots = 8;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false, failed = false;
  std::string error;
  std::deque<std::shared_ptr<Ticket>> queue;
  std::map<uint64_t, std::shared_ptr<Ticket>> tickets;
  std::vector<std::shared_ptr<Ticket>> running;
  uint64_t next_id = 1;
  int active_parts = 0;
  int64_t held = 0;  // memory reserved by all admitted requests
  int64_t base = 0;  // device memory of the resident objects and the packing buffers (fixed while serving)
  // stats
  std::vector<double> lat;
  int64_t completed = 0, rejected = 0, sources = 0, parts_done = 0, steps = 0;
  double t_first = -1, t_last = 0;
  DevArray<c128> packV, packZ, packW;
  DevArray<c64> packZ32;  // packed preconditioned columns of mixed-precision jobs
  // page-locked staging of a host request's columns (one part at a time): the caller's pageable
  // block is copied through it by host threads, so the device copies run at pinned-memory speed
  HostPinned<c128> stage;
  // the preconditioner solve workspace every resident ddm shares while serving
  PrecondWork pw;
};

static constexpr int kServeRestart = 40;
static constexpr int kGoodRestart = 20;
static constexpr int kMinRestart = 8;
static constexpr double kBackfillWindow = 30.0;

static int part_cols(const Ticket& t, int k) { return (int)std::min<int64_t>(t.w, t.req.n_rhs - t.w * (int64_t)k); }

// device memory of part k: its Krylov workspace and its node-major right-hand side and
// solution (which also stage its columns of a host request in and out)
static int64_t part_bytes(const Ticket& t, int k, int m) {
  const int64_t n = t.ddm->op->mesh->n;
  const int s = part_cols(t, k);
  return FgmresJob::bytes_needed(n, s, m, t.ddm->precision == HZ_PREC_MIXED) + 2 * n * s * (int64_t)sizeof(c128);
}

// start of part k of a request (scheduler thread, no lock held)
static void start_part(Serve& S, Ticket& t, int k) {
  Ctx* ctx = S.ctx;
  const int64_t n = t.ddm->op->mesh->n;
  SolveOptions o;
  o.tol = t.req.tol;
  o.max_iter = t.req.max_iter > 0 ? t.req.max_iter : 500;
  o.restart = t.m;
  auto p = std::make_unique<Ticket::Part>();
  p->c0 = t.w * k;
  p->s = part_cols(t, k);
  p->Bn.alloc(ctx, n * p->s);
  p->Xn.alloc(ctx, n * p->s);
  KrylovKernels K(ctx, n, p->s);
  // the part's columns are contiguous in the caller's [n_rhs][n] block; a host block is staged
  // through Xn (the solve zeroes it before use)
  const c128* cols = static_cast<const c128*>(t.req.rhs) + (int64_t)p->c0 * n;
  if (t.req.mem == HZ_MEM_HOST) {
    const int64_t cnt = n * p->s;
    parallel_for(cnt, [&](int64_t a, int64_t b) { std::memcpy(S.stage.p + a, cols + a, (b - a) * sizeof(c128)); });
    HIP_CHECK(hipMemcpyAsync(p->Xn.ptr(), S.stage.p, cnt * sizeof(c128), hipMemcpyHostToDevice, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));  // the staging buffer is reused at once
    K.to_node(p->Xn.ptr(), p->Bn.ptr());
  } else {
    K.to_node(cols, p->Bn.ptr());
  }
  p->job = std::make_unique<FgmresJob>(ctx, t.ddm, p->s, p->Bn.ptr(), p->Xn.ptr(), o, t.m);
  p->job->start();
  t.parts.push_back(std::move(p));
}

// a finished part's solution to the caller's block (through Bn, free now, for a host block);
// its device memory goes back at once
static void part_out(Serve& S, Ticket& t, Ticket::Part& p) {
  Ctx* ctx = S.ctx;
  const int64_t n = t.ddm->op->mesh->n;
  KrylovKernels K(ctx, n, p.s);
  c128* cols = static_cast<c128*>(t.req.x) + (int64_t)p.c0 * n;
  if (t.req.mem == HZ_MEM_HOST) {
    const int64_t cnt = n * p.s;
    K.from_node(p.Xn.ptr(), p.Bn.ptr());
    HIP_CHECK(hipMemcpyAsync(S.stage.p, p.Bn.ptr(), cnt * sizeof(c128), hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    parallel_for(cnt, [&](int64_t a, int64_t b) { std::memcpy(cols + a, S.stage.p + a, (b - a) * sizeof(c128)); });
  } else {
    K.from_node(p.Xn.ptr(), cols);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  }
  p.Bn = DevArray<c128>();
  p.Xn = DevArray<c128>();
}

static void finish_ticket(Serve& S, Ticket& t) {
  (void)S;
  int32_t st = HZ_OK;
  for (auto& p : t.parts) {
    for (int k = 0; k < p->s; ++k) {
      const ColInfo& ci = p->info[k];
      if (t.req.info) {
        hz_col_info& hi = t.req.info[p->c0 + k];
        hi.iters = ci.iters;
        hi.restarts = ci.restarts;
        hi.rel_residual = ci.rel_residual;
        hi.status = ci.status;
        hi.restart_len = ci.m;
        hi.block = ci.block;
      }
      if (ci.status != HZ_OK) st = HZ_ERR_NOT_CONVERGED;
    }
  }
  t.parts.clear();
  t.status = st;
}

// Shared launches for the jobs of one operator: first-fit decreasing into launches of at most
// 32 columns (the widest job first, each into the first launch with room), so that as few
// passes over the factors as possible serve them all.  Ties keep admission order.
static std::vector<std::vector<FgmresJob*>> pack_launches(const std::vector<FgmresJob*>& jobs) {
  std::vector<FgmresJob*> order(jobs);
  std::stable_sort(order.begin(), order.end(), [](const FgmresJob* x, const FgmresJob* y) { return x->s > y->s; });
  std::vector<std::vector<FgmresJob*>> bins;
  std::vector<int> width;
  for (FgmresJob* j : order) {
    size_t b = 0;
    while (b < bins.size() && width[b] + j->s > 32) ++b;
    if (b == bins.size()) {
      bins.emplace_back();
      width.push_back(0);
    }
    bins[b].push_back(j);
    width[b] += j->s;
  }
  return bins;
}

static void tick(Serve& S) {
  Ctx* ctx = S.ctx;
  hipStream_t st = ctx->stream;
  // group the active jobs by operator, pack up to 32 columns per shared launch
  std::map<Ddm*, std::vector<FgmresJob*>> groups;
  for (auto& t : S.running)
    for (auto& p : t->parts)
      if (!p->done) groups[t->ddm.get()].push_back(p->job.get());
  for (auto& [dp, jobs] : groups) {
    for (const std::vector<FgmresJob*>& bin : pack_launches(jobs)) {
      int cols = 0;
      for (FgmresJob* j : bin) cols += j->s;
      const int64_t n = dp->op->mesh->n;
      if (bin.size() == 1) {  // a single job needs no packing
        bin[0]->matvec();
      } else {
        const bool z32 = dp->precision == HZ_PREC_MIXED;
        const int64_t need = n * 32;
        if ((int64_t)S.packV.n < need) {
          S.packV.alloc(ctx, need);
          S.packW.alloc(ctx, need);
        }
        if (z32 && (int64_t)S.packZ32.n < need) S.packZ32.alloc(ctx, need);
        if (!z32 && (int64_t)S.packZ.n < need) S.packZ.alloc(ctx, need);
        int off = 0;
        for (FgmresJob* j : bin) {
          hipLaunchKernelGGL(k_pack_cols, dim3((unsigned)((n * j->s + 255) / 256)), dim3(256), 0, st, n, j->s, cols, off,
                             j->v_cur(), S.packV.ptr());
          off += j->s;
        }
        // one preconditioner apply and one SpMM for all packed columns (the operator is shared)
        const int64_t* rp = dp->op->mesh->d_rowptr.ptr();
        const int32_t* ci = dp->op->mesh->d_col.ptr();
        if (z32) {
          precond_apply(ctx, *dp, cols, S.packV.ptr(), S.packZ32.ptr());
          launch_spmm<float>(st, n, cols, rp, ci, dp->op->d_val.ptr(), S.packZ32.ptr(), S.packW.ptr(), cmk(1.0, 0.0),
                             cmk(0.0, 0.0), nullptr);
        } else {
          precond_apply(ctx, *dp, cols, S.packV.ptr(), S.packZ.ptr());
          launch_spmm<double>(st, n, cols, rp, ci, dp->op->d_val.ptr(), S.packZ.ptr(), S.packW.ptr(), cmk(1.0, 0.0),
                              cmk(0.0, 0.0), nullptr);
        }
        off = 0;
        for (FgmresJob* j : bin) {
          const dim3 grid((unsigned)((n * j->s + 255) / 256));
          if (z32)
            hipLaunchKernelGGL(k_unpack_cols<float>, grid, dim3(256), 0, st, n, j->s, cols, off, S.packZ32.ptr(),
                               j->z32_cur());
          else
            hipLaunchKernelGGL(k_unpack_cols<double>, grid, dim3(256), 0, st, n, j->s, cols, off, S.packZ.ptr(),
                               j->z_cur());
          hipLaunchKernelGGL(k_unpack_cols<double>, grid, dim3(256), 0, st, n, j->s, cols, off, S.packW.ptr(),
                             j->w_cur());
          off += j->s;
        }
        HIP_CHECK(hipGetLastError());
      }
    }
    for (FgmresJob* j : jobs) j->after_matvec();
    std::lock_guard<std::mutex> lk(S.mu);
    S.steps += (int64_t)jobs.size();
  }
  HIP_CHECK(hipStreamSynchronize(st));
  for (auto& t : S.running)
    for (auto& p : t->parts)
      if (!p->done && p->job->cycle_done() && p->job->end_cycle()) {
        p->done = true;
        p->info = p->job->info;
        p->job.reset();  // the Krylov workspace goes back at once
        part_out(S, *t, *p);
        std::lock_guard<std::mutex> lk(S.mu);
        ++t->finished;
        --S.active_parts;
        ++S.parts_done;
      }
}

static void scheduler(Serve* S) {
  Ctx* ctx = S->ctx;
  try {
    HIP_CHECK(hipSetDevice(ctx->device));
    for (;;) {
      std::vector<std::pair<std::shared_ptr<Ticket>, int>> admit;  // (request, part)
      {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->running.empty(); });
        if (S->stop && S->running.empty() && S->queue.empty()) break;  // stop drains every request
        // FIFO admission of parts by slots and memory; while the head waits for memory, later
        // requests whose parts fit may go first (backfill) for kBackfillWindow seconds of that
        // wait; the first part of an idle server is always admitted
        int64_t pending = 0;
        const double tnow = now_s();
        for (auto it = S->queue.begin(); it != S->queue.end();) {
          auto t = *it;
          const bool head = it == S->queue.begin();
          const int64_t pb = part_bytes(*t, t->admitted, t->m);
          const bool idle = S->active_parts == 0;
          const bool slots_ok = idle || S->active_parts + 1 <= S->max_slots;
          const bool mem_ok = idle || ctx->bytes_in_use + pending + pb <= (int64_t)ctx->hbm_budget;
          if (!slots_ok) break;
          if (!mem_ok) {
            if (!head) {
              ++it;  // a later request may still fit
              continue;
            }
            if (t->t_blocked == 0) t->t_blocked = tnow;
            if (tnow - t->t_blocked > kBackfillWindow) break;  // strict FIFO from now on
            ++it;
            continue;
          }
          if (head) t->t_blocked = 0;
          ++S->active_parts;
          pending += pb;
          t->held += pb;
          S->held += pb;
          if (t->state == 0) {  // first admission (a rolled-back request stays in running)
            t->state = 1;
            S->running.push_back(t);
          }
          admit.emplace_back(t, t->admitted++);
          if (t->admitted == t->nparts) it = S->queue.erase(it);  // else: its next part, same request
        }
      }
      // start the admitted parts; a part whose memory the allocator cannot give now goes
      // back to the head of the queue (it is retried when running parts have freed theirs),
      // or fails its request when nothing else is running
      for (size_t a = 0; a < admit.size(); ++a) {
        auto& [t, k] = admit[a];
        try {
          start_part(*S, *t, k);
        } catch (const Error& e) {
          if (e.code != HZ_ERR_OOM && e.code != HZ_ERR_ARG) throw;
          std::lock_guard<std::mutex> lk(S->mu);
          // undo this and every later admission of this round, latest first (FIFO order)
          for (size_t b = admit.size(); b-- > a;) {
            auto& [tb, kb] = admit[b];
            const int64_t pb = part_bytes(*tb, kb, tb->m);
            tb->held -= pb;
            S->held -= pb;
            --S->active_parts;
            --tb->admitted;
            if (std::find(S->queue.begin(), S->queue.end(), tb) == S->queue.end()) {  // back in FIFO place
              auto pos = std::find_if(S->queue.begin(), S->queue.end(),
                                      [&](const std::shared_ptr<Ticket>& q) { return q->id > tb->id; });
              S->queue.insert(pos, tb);
            }
          }
          if (e.code == HZ_ERR_ARG || S->active_parts == 0) {  // bad block, or it cannot fit even alone:
            t->status = e.code;                                  // the request fails
            t->oom = true;
            std::fprintf(stderr, "hz: serve: request %llu failed at part %d: %s\n", (unsigned long long)t->id, k, e.what());
          }
          break;
        }
      }
      // requests that failed to fit even alone: retire them (their started parts are dropped)
      {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = S->queue.begin(); it != S->queue.end();) {
          if ((*it)->oom) {
            auto t = *it;
            it = S->queue.erase(it);
            S->running.erase(std::remove(S->running.begin(), S->running.end(), t), S->running.end());
            for (auto& p : t->parts)
              if (!p->done) --S->active_parts;
            t->parts.clear();
            S->held -= t->held;
            t->held = 0;
            t->t_done = now_s();
            t->state = 2;
            S->rejected += 1;
            S->done_cv.notify_all();
          } else {
            ++it;
          }
        }
      }
      if (!S->running.empty()) tick(*S);
      // complete finished requests
      std::vector<std::shared_ptr<Ticket>> fin;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = S->running.begin(); it != S->running.end();) {
          if ((*it)->finished == (*it)->nparts) {
            fin.push_back(*it);
            it = S->running.erase(it);
          } else {
            ++it;
          }
        }
      }
      for (auto& t : fin) {
        finish_ticket(*S, *t);
        std::lock_guard<std::mutex> lk(S->mu);
        t->t_done = now_s();
        t->state = 2;
        S->held -= t->held;
        t->held = 0;
        S->lat.push_back(t->t_done - t->t_submit);
        S->completed += 1;
        S->sources += t->req.n_rhs;
        S->t_last = t->t_done;
        S->done_cv.notify_all();
      }
    }
  } catch (const std::exception& e) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->failed = true;
    S->error = e.what();
    for (auto& t : S->running) {
      t->state = 2;
      t->status = HZ_ERR_HIP;
    }
    for (auto& t : S->queue) {
      t->state = 2;
      t->status = HZ_ERR_STATE;
    }
    S->running.clear();
    S->queue.clear();
    S->done_cv.notify_all();
  }
}

}  // namespace hz

using namespace hz;

extern "C" {

hz_status hz_serve_start(hz_ctx* c, int32_t max_slots) {
  Ctx* x = reinterpret_cast<Ctx*>(c);
  if (!x || max_slots < 1) return HZ_ERR_ARG;
  if (x->poisoned) return HZ_ERR_HIP;
  if (x->serve) return HZ_ERR_STATE;
  krylov_cache_release(x);  // admission counts what the context holds
  auto* S = new Serve();
  S->ctx = x;
  S->max_slots = max_slots;
  // the shared launches' packing buffers, sized for the largest resident operator, so that a
  // tick allocates nothing; with them the resident memory is fixed until hz_serve_stop (the
  // context refuses other calls meanwhile)
  try {
    int64_t nmax = 0;
    bool mixed = false, full = false;
    {
      std::lock_guard<std::mutex> lk(x->mu);
      for (auto& kv : x->ddms) {
        nmax = std::max<int64_t>(nmax, kv.second->op->mesh->n);
        (kv.second->precision == HZ_PREC_MIXED ? mixed : full) = true;
      }
    }
    if (nmax > 0) {
      S->packV.alloc(x, nmax * 32);
      S->packW.alloc(x, nmax * 32);
      if (mixed) S->packZ32.alloc(x, nmax * 32);
      if (full) S->packZ.alloc(x, nmax * 32);
      S->stage.alloc(nmax * 32);
      // one solve workspace for all ddms, grown here to what a 32-column apply of each needs
      // (which also tunes their sweep tiles for 32 columns), so that serving's memory is fixed
      std::vector<std::shared_ptr<Ddm>> ds;
      {
        std::lock_guard<std::mutex> lk(x->mu);
        for (auto& kv : x->ddms) ds.push_back(kv.second);
      }
      for (auto& d : ds) precond_release_workspace(*d);
      x->shared_pw = &S->pw;
      HIP_CHECK(hipMemsetAsync(S->packV.ptr(), 0, (size_t)nmax * 32 * sizeof(c128), x->stream));
      for (auto& d : ds) {
        if (d->precision == HZ_PREC_MIXED)
          precond_apply(x, *d, 32, S->packV.ptr(), S->packZ32.ptr());
        else
          precond_apply(x, *d, 32, S->packV.ptr(), S->packZ.ptr());
      }
      HIP_CHECK(hipStreamSynchronize(x->stream));
    }
  } catch (const Error& e) {
    x->shared_pw = nullptr;
    x->last_error = e.what();
    delete S;
    return e.code;
  }
  S->base = x->bytes_in_use;
  x->serving = true;
  x->serve = S;
  S->th = std::thread(scheduler, S);
  return HZ_OK;
}

hz_status hz_serve_submit(hz_ctx* c, const hz_request* req, uint64_t* ticket) {
  Ctx* x = reinterpret_cast<Ctx*>(c);
  if (!x || !req || !ticket) return HZ_ERR_ARG;
  if (req->struct_size != sizeof(hz_request)) return HZ_ERR_ABI;
  Serve* S = x->serve;
  if (!S) return HZ_ERR_STATE;
  if (req->n_rhs < 1 || !req->rhs || !req->x || !(req->tol >= 0) || (req->mem != HZ_MEM_HOST && req->mem != HZ_MEM_DEVICE))
    return HZ_ERR_ARG;
  std::shared_ptr<Ddm> d;
  {
    std::lock_guard<std::mutex> lk(x->mu);
    auto it = x->ddms.find(req->ddm);
    if (it == x->ddms.end()) return HZ_ERR_ARG;
    d = it->second;
  }
  auto t = std::make_shared<Ticket>();
  t->req = *req;
  t->ddm = d;
  t->t_submit = now_s();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->failed) return HZ_ERR_STATE;
  // part width and restart length: for each width (32 and its halvings, never past n_rhs) the
  // longest restart (up to 40) with which the first part fits in the budget left after the
  // resident objects; the widest width reaching kGoodRestart, else the longest restart (the
  // wider width on a tie); never admissible below kMinRestart
  const int64_t avail = (int64_t)x->hbm_budget - S->base;  // what a part running alone may use
  t->m = 0;
  int best_w = 0, best_m = 0;
  for (int w = (int)std::min<int64_t>(32, req->n_rhs); w >= 1; w = w > 1 ? w / 2 : 0) {
    t->w = w;
    int mw = 0;
    for (int m = kServeRestart; m >= kMinRestart; --m)
      if (part_bytes(*t, 0, m) <= avail) {
        mw = m;
        break;
      }
    if (mw >= kGoodRestart) {
      best_w = w;
      best_m = mw;
      break;
    }
    if (mw > best_m) {
      best_w = w;
      best_m = mw;
    }
  }
  t->w = best_w > 0 ? best_w : 32;
  t->m = best_m;
  t->nparts = (int)((req->n_rhs + t->w - 1) / t->w);
  if (t->m == 0) {
    S->rejected += 1;
    return HZ_ERR_BUSY;
  }
  t->id = S->next_id++;
  if (S->t_first < 0) S->t_first = t->t_submit;
  S->tickets[t->id] = t;
  S->queue.push_back(t);
  *ticket = t->id;
  S->cv.notify_all();
  return HZ_OK;
}

hz_status hz_serve_poll(hz_ctx* c, uint64_t ticket, int* done) {
  Ctx* x = reinterpret_cast<Ctx*>(c);
  if (!x || !done) return HZ_ERR_ARG;
  Serve* S = x->serve;
  if (!S) return HZ_ERR_STATE;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return HZ_ERR_ARG;
  *done = it->second->state == 2;
  return HZ_OK;
}

hz_status hz_serve_wait(hz_ctx* c, uint64_t ticket, int32_t* status) {
  Ctx* x = reinterpret_cast<Ctx*>(c);
  if (!x) return HZ_ERR_ARG;
  Serve* S = x->serve;
  if (!S) return HZ_ERR_STATE;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return HZ_ERR_ARG;
  auto t = it->second;
  S->done_cv.wait(lk, [&] { return t->state == 2; });
  if (status) *status = t->status;
  S->tickets.erase(ticket);
  if (S->failed) {
    x->last_error = "serving stopped: " + S->error;
    return HZ_ERR_HIP;
  }
  return HZ_OK;
}

hz_status hz_serve_stats_get(hz_ctx* c, hz_serve_stats* out) {
  Ctx* x = reinterpret_cast<Ctx*>(c);
  if (!x || !out) return HZ_ERR_ARG;
  Serve* S = x->serve;
  if (!S) return HZ_ERR_STATE;
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> l = S->lat;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    const double pos = q * (double)(l.size() - 1);
    const size_t i = (size_t)std::floor(pos);
    const double f = pos - (double)i;
    return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
  };
  out->p50_s = pct(0.50);
  out->p99_s = pct(0.99);
  out->sources_per_s = (S->completed > 0 && S->t_last > S->t_first) ? S->sources / (S->t_last - S->t_first) : 0.0;
  out->completed = S->completed;
  out->rejected = S->rejected;
  out->parts_done = S->parts_done;
  out->steps = S->steps;
  out->active_parts = S->active_parts;
  return HZ_OK;
}

hz_status hz_serve_stop(hz_ctx* c) {
  Ctx* x = reinterpret_cast<Ctx*>(c);
  if (!x) return HZ_ERR_ARG;
  Serve* S = x->serve;
  if (!S) return HZ_ERR_STATE;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  if (S->th.joinable()) S->th.join();  // running requests finish first
  const bool failed = S->failed;
  if (failed) x->last_error = "serving stopped: " + S->error;
  x->serve = nullptr;
  x->serving = false;
  x->shared_pw = nullptr;  // the ddms grow their own workspaces again
  delete S;
  if (failed) x->poisoned = true;
  return failed ? HZ_ERR_HIP : HZ_OK;
}

}  // extern "C"
