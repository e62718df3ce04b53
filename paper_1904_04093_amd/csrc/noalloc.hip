// Allocation-free residual entry point (gabp_residual_noalloc).
//
// gabp_residual reduces its norms through per-block partial sums held in context-owned
// device memory and reads them back to the host. This variant keeps the partials and the
// reduced scalars in one file-scope device array instead and writes the norms to device
// memory, so a call allocates nothing, never waits for the stream and can be recorded into
// a HIP graph. The array exists once per GPU for the life of the process; host code reaches
// it only through the device address looked up here (its name on the host side is a
// stand-in, not a device pointer).
#include <mutex>

#include "gabp_internal.h"

namespace gabp {

constexpr int64_t kScratchDoubles = 262144;   // 2 MiB: 3 partials per residual block + 4

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `dev` (the current device), looked up once per device;
// gabp_setup calls this for its device, so the lookup happens before any capture.
int scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GABP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  if (out) *out = g_scratch_ptr[dev];
  return GABP_OK;
}

namespace {

// red[0] = ||r||_2^2, red[1] = ||r||_inf, red[2] = ||b||_2^2 -> the three norms
__global__ void k_norms_out(const double* __restrict__ red, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = sqrt(red[0]);
    out[1] = red[1];
    out[2] = sqrt(red[2]);
  }
}

}  // namespace
}  // namespace gabp

using namespace gabp;

extern "C" int gabp_residual_noalloc(gabp_ctx* c, const double* b, const double* x, double* r,
                                     int32_t transposed, double* norms, hipStream_t s) {
  if (!c || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  const int64_t need = 3 * static_cast<int64_t>(c->nred) + 4;
  if (need > kScratchDoubles)
    return fail(GABP_EINVAL, "context too large for the static scratch array: at most " +
                                 std::to_string((kScratchDoubles - 4) / 3 * kRedBlock) +
                                 " rows");
  GABP_HIP(hipSetDevice(c->device));
  double* base = nullptr;
  const int st = scratch_on(c->device, &base);
  if (st != GABP_OK) return st;
  double* partials = base;
  double* red = base + 3 * static_cast<int64_t>(c->nred);
  const double* coef = transposed ? c->L.aT : c->L.val;
  GABP_HIP(launch_residual(&c->L, coef, b, x, nullptr, nullptr, r, partials, c->nred, red, s,
                           norms != nullptr));
  if (norms) {
    k_norms_out<<<1, 64, 0, s>>>(red, norms);
    GABP_HIP(hipGetLastError());
  }
  return GABP_OK;
}
