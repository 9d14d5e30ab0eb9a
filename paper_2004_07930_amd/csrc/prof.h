// Live kernel accounting (hz_profile_*): HIP events around launches of selected kernel
// classes, with the algorithmic bytes / flops of each launch.
#pragma once

#include "hz_internal.h"

namespace hz {

struct ProfRec {
  int kid;
  hipEvent_t a, b;
  double bytes, flops;
};

struct Prof {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  ~Prof();
};

// returns a record index (or -1 when recording is off); call prof_end with it after the launch
int prof_begin(Ctx* ctx, int kid, double bytes, double flops);
void prof_end(Ctx* ctx, int idx);

struct ProfScope {
  Ctx* ctx;
  int idx;
  ProfScope(Ctx* c, int kid, double bytes, double flops) : ctx(c), idx(prof_begin(c, kid, bytes, flops)) {}
  ~ProfScope() { prof_end(ctx, idx); }
};

}  // namespace hz
