// nncp_norm_sq_noalloc: ||X||^2 (FP64) without any device allocation, for
// callers that cannot allocate (code under HIP graph capture, serving loops
// that admit jobs without touching the allocator).
//
// The two-stage reduction of nncp_norm_sq needs scratch: one FP64 partial per
// work-group and the arrival counter of the last-group reduction. Here that
// scratch is a file-scope device array, one copy per GPU for the life of the
// process. Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): each device's address is looked up once
// with hipGetSymbolAddress, with that device current, and kept per device.
#include <mutex>

#include "nncp_internal.hpp"

using namespace nncpk;

namespace {

// kNormSqMaxBlocks FP64 partials, then the arrival counter (in the last slot's
// 8 bytes; the rest of that 256-byte line is unused). 8.2 KB per device.
constexpr int kScratchDoubles = kNormSqMaxBlocks + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
int scratch_for_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NNCP_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return NNCP_EDEVICE;
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return NNCP_OK;
}

}  // namespace

extern "C" int nncp_norm_sq_noalloc(const void* X, int dtype, int64_t n, double* out_dev, void* stream) {
  if (!X || !out_dev || n < 1 || dtype < NNCP_F32 || dtype > NNCP_F16) return NNCP_EINVAL;
  const int nb = norm_sq_blocks(n);
  if (nb > kNormSqMaxBlocks) return NNCP_EINVAL;  // more partials than the scratch holds
  double* sp = nullptr;
  int st = scratch_for_current_device(&sp);
  if (st != NNCP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  unsigned* counter = (unsigned*)(sp + kNormSqMaxBlocks);
  // the counter must start at zero: cleared by a kernel (no memset node under capture)
  if (fill_u32_launch(counter, 1, 0u, s) != hipSuccess) return NNCP_EDEVICE;
  if (norm_sq_launch(X, dtype, n, out_dev, sp, counter, nb, s) != hipSuccess) return NNCP_EDEVICE;
  return NNCP_OK;
}
