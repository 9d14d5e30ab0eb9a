// Entry points that allocate no device memory (noalloc.hip).
#pragma once

#include "hz_internal.h"

namespace hz {

// complex128 entries of the per-device scratch array (128 MiB)
constexpr int64_t kNoallocScratchEntries = int64_t(1) << 23;

// looks up the scratch array's address on `device` (current) once; called by hz_init
void noalloc_init(int device);
// y = A x for device blocks [n_rhs][n] through the scratch array, on the context's stream
void spmm_noalloc(Ctx* c, const Operator& op, int64_t n_rhs, const c128* x, c128* y);

}  // namespace hz
