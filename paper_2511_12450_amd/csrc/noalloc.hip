// lm_matvec_noalloc: the layered FMM matvec with its per-launch workspace in
// a static device array instead of library allocations, for callers that
// cannot allocate device memory (code under stream capture, serving loops
// that forbid hipMalloc).
//
// `scratch` is one file-scope __device__ array; every GPU the library runs on
// holds its own copy until the process ends.  In host code its name is only
// a stand-in for the symbol, so the device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and only that
// address is handed to kernels.  Every call on a device shares the array and
// leaves its contents behind: the matvec clears what it needs cleared
// (local expansions) itself, and calls that overlap on one device race.
#include <mutex>

#include "lm_internal.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[LM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch (resolved on the first call on it).
lm_status scratch_ptr(void** out) {
  int dev = 0;
  LM_TRY_HIP(hipGetDevice(&dev));
  LM_CHECK(dev >= 0 && dev < kMaxDevices, LM_EINTERNAL, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    LM_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    LM_CHECK(p, LM_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return LM_OK;
}

}  // namespace

extern "C" lm_status lm_matvec_noalloc(lm_geom g, int precision, int n_rhs, const void* x, void* y,
                                       void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_CHECK(precision == LM_FP64 || precision == LM_MIXED, LM_EINVAL, "precision must be LM_FP64 or LM_MIXED");
  LM_CHECK(n_rhs >= 1, LM_EINVAL, "n_rhs must be >= 1");
  LM_CHECK(x && y && x != y, LM_EINVAL, "x and y must be distinct device pointers");
  hipStream_t s = (hipStream_t)hip_stream;
  // the dense operator needs no workspace
  if (g->method == LM_DENSE) return dense_matvec(g, precision, n_rhs, x, y, s);
  void* base = nullptr;
  LM_TRY(scratch_ptr(&base));
  return fmm_matvec_in(g, precision, n_rhs, x, y, base, (size_t)LM_NOALLOC_SCRATCH_BYTES, s);
}
