// Static device scratch of the allocation-free render entry point
// (nsl_render_noalloc): room for the prepared MFMA operands of the larger
// field shape and one request record.  Each GPU the library runs on holds
// its own copy of the array until the process ends; its address on the
// current device is looked up once per device and kept.
#include <mutex>

#include "kernels.h"
#include "net.h"

namespace nsl {

namespace {

constexpr size_t round256(size_t n) { return (n + 255) / 256 * 256; }
constexpr size_t prep_floats_full = (size_t)NetFull::FWD_FLOATS + NetFull::BWD_FLOATS;
constexpr size_t prep_floats_tiny = (size_t)NetTiny::FWD_FLOATS + NetTiny::BWD_FLOATS;
constexpr size_t kPrepBytes =
    round256(sizeof(float) * (prep_floats_full > prep_floats_tiny ? prep_floats_full : prep_floats_tiny));
constexpr size_t kScratchBytes = kPrepBytes + round256(sizeof(nsl_render_request));
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

hipError_t noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return hipSuccess;
}

}  // namespace nsl
