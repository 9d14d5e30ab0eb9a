// Live kernel accounting (hz_profile_enable / hz_profile_get).
#include "prof.h"

namespace hz {

Prof::~Prof() {
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

static hipEvent_t take_event(Prof& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}

int prof_begin(Ctx* ctx, int kid, double bytes, double flops) {
  if (!ctx->prof || !ctx->prof->on) return -1;
  Prof& p = *ctx->prof;
  ProfRec r{kid, take_event(p), take_event(p), bytes, flops};
  HIP_CHECK(hipEventRecord(r.a, ctx->stream));
  p.recs.push_back(r);
  return (int)p.recs.size() - 1;
}

void prof_end(Ctx* ctx, int idx) {
  if (idx < 0 || !ctx->prof) return;
  (void)hipEventRecord(ctx->prof->recs[idx].b, ctx->stream);
}

}  // namespace hz

using namespace hz;

extern "C" {

hz_status hz_profile_enable(hz_ctx* c, int on) {
  if (!c) return HZ_ERR_ARG;
  Ctx* x = reinterpret_cast<Ctx*>(c);
  try {
    HIP_CHECK(hipStreamSynchronize(x->stream));
    if (!x->prof) x->prof = new Prof();
    if (on) {
      for (auto& r : x->prof->recs) {
        x->prof->pool.push_back(r.a);
        x->prof->pool.push_back(r.b);
      }
      x->prof->recs.clear();
    }
    x->prof->on = on != 0;
    return HZ_OK;
  } catch (const Error& e) {
    x->last_error = e.what();
    return e.code;
  }
}

hz_status hz_profile_get(hz_ctx* c, int kid, hz_kernel_stat* out) {
  if (!c || !out || kid < 0 || kid >= HZ_K_COUNT) return HZ_ERR_ARG;
  Ctx* x = reinterpret_cast<Ctx*>(c);
  try {
    HIP_CHECK(hipStreamSynchronize(x->stream));
    *out = hz_kernel_stat{0, 0.0, 0.0, 0.0};
    if (!x->prof) return HZ_OK;
    for (auto& r : x->prof->recs) {
      if (r.kid != kid) continue;
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
      out->launches += 1;
      out->seconds += 1e-3 * ms;
      out->bytes += r.bytes;
      out->flops += r.flops;
    }
    return HZ_OK;
  } catch (const Error& e) {
    x->last_error = e.what();
    return e.code;
  }
}

}  // extern "C"
