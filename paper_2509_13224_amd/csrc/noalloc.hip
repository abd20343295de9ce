// Allocation-free TT inner product for callers that cannot allocate device memory (work under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The temporaries of the contraction chain (the interface matrices, the partially contracted
// core and the partial tiles of split GEMMs) live in one file-scope device array of fixed size
// instead of the context's workspace.  Each device holds its own copy of the array for the
// life of the process; its device address is looked up once per device (at context creation)
// and used from then on, since the array's name in host code is only a host-side stand-in.
// Every call on a device shares that device's array, so calls that overlap on one device
// (two streams, or two threads) race; nothing in it needs to start at zero (the chain writes
// every element before it reads it).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "runtime.hpp"

namespace ttiga {

// 64 MiB: enough for ranks up to 128 at mode sizes up to 256, or ranks 64 at 1024
constexpr size_t kNoAllocScratchDoubles = size_t(8) << 20;

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
std::mutex g_mu;
std::map<int, double*> g_addr;  // device -> address of that device's scratch
}  // namespace

size_t noalloc_scratch_bytes() { return sizeof(double) * kNoAllocScratchDoubles; }

// The device address of `scratch` on the current device; looked up once per device.
double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_addr.find(device);
  if (it != g_addr.end()) return it->second;
  int cur = -1;
  TTIGA_HIP(hipGetDevice(&cur));
  TTIGA_CHECK(cur == device, TTIGA_E_STATE, "scratch lookup with another device current");
  void* ptr = nullptr;
  const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  TTIGA_CHECK(rc == hipSuccess && ptr != nullptr, TTIGA_E_HIP,
              std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc));
  g_addr[device] = static_cast<double*>(ptr);
  return static_cast<double*>(ptr);
}

void tt_dot_noalloc(Context& ctx, const ttiga_tt_view& x, const ttiga_tt_view& y, double* out_dev) {
  TTIGA_CHECK(out_dev != nullptr, TTIGA_E_ARG, "null output");
  TTIGA_CHECK(!ctx.prof.on, TTIGA_E_STATE, "profiling records events: switch it off for the allocation-free dot");
  int n[3], rx[4], ry[4];
  const double* xc[3];
  const double* yc[3];
  for (int k = 0; k < 4; ++k) {
    rx[k] = x.r[k];
    ry[k] = y.r[k];
  }
  TTIGA_CHECK(rx[0] == 1 && rx[3] == 1 && ry[0] == 1 && ry[3] == 1, TTIGA_E_ARG, "TT view needs r0 = r3 = 1");
  for (int k = 0; k < 3; ++k) {
    TTIGA_CHECK(x.n[k] == y.n[k], TTIGA_E_ARG, "dot: mode sizes differ");
    TTIGA_CHECK(x.n[k] > 0 && rx[k + 1] > 0 && ry[k + 1] > 0 && x.core[k] && y.core[k], TTIGA_E_ARG,
                "bad TT view");
    n[k] = x.n[k];
    xc[k] = x.core[k];
    yc[k] = y.core[k];
  }
  const size_t need = tt_dot_scratch_doubles(n, rx, ry);
  TTIGA_CHECK(need <= kNoAllocScratchDoubles, TTIGA_E_ARG,
              "dot needs " + std::to_string(need * sizeof(double)) + " bytes of scratch; the allocation-free " +
                  "entry point has " + std::to_string(noalloc_scratch_bytes()));
  tt_dot_cores(ctx, n, rx, xc, ry, yc, out_dev, noalloc_scratch(ctx.device));
}

}  // namespace ttiga
