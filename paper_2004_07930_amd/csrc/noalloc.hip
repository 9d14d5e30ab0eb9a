// Scratch memory of hz_spmm_noalloc: the operator product of hz_spmm for callers that cannot
// allocate device memory.  Its node-major staging copies of x and y live in one file-scope
// device array instead of allocations.  The array is a per-device object of the code object:
// each GPU the library runs on holds its own copy, at its own address, until the process ends.
// Host code never passes the array's name to a kernel (on the host it names a stand-in, not
// device memory): its device address is looked up once per device with hipGetSymbolAddress
// while that device is current (hz_init) and only that address is used.
#include <cstdio>

#include "krylov.h"
#include "noalloc.h"

namespace hz {

namespace {

__device__ __align__(256) c128 scratch[kNoallocScratchEntries];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
c128* g_scratch[kMaxDevices] = {};

}  // namespace

void noalloc_init(int device) {
  HZ_REQUIRE(device >= 0 && device < kMaxDevices, HZ_ERR_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return;
  void* p = nullptr;
  HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  HZ_REQUIRE(p != nullptr, HZ_ERR_HIP, "no device address for the scratch array");
  g_scratch[device] = static_cast<c128*>(p);
}

void spmm_noalloc(Ctx* c, const Operator& op, int64_t n_rhs, const c128* x, c128* y) {
  c128* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = c->device >= 0 && c->device < kMaxDevices ? g_scratch[c->device] : nullptr;
  }
  HZ_REQUIRE(base, HZ_ERR_STATE, "hz_spmm_noalloc: scratch memory of this device was not set up by hz_init");
  const int64_t n = op.mesh->n;
  // one column needs its node-major x and y copies: 2 n entries
  HZ_REQUIRE(2 * n <= kNoallocScratchEntries, HZ_ERR_ARG,
             "hz_spmm_noalloc: operator too large for the scratch memory (at most " +
                 std::to_string(kNoallocScratchEntries / 2) + " dofs)");
  const int64_t cols = std::min<int64_t>(32, kNoallocScratchEntries / (2 * n));
  for (int64_t c0 = 0; c0 < n_rhs; c0 += cols) {
    const int s = (int)std::min<int64_t>(cols, n_rhs - c0);
    c128* xn = base;
    c128* yn = base + n * s;
    KrylovKernels K(c, n, s);
    K.to_node(x + c0 * n, xn);
    launch_spmm<double>(c->stream, n, s, op.mesh->d_rowptr.ptr(), op.mesh->d_col.ptr(), op.d_val.ptr(), xn, yn,
                        cmk(1.0, 0.0), cmk(0.0, 0.0), nullptr);
    K.from_node(yn, y + c0 * n);
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace hz
