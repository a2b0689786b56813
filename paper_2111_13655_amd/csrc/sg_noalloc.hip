// sg_propagate_noalloc: the propagators of sg_propagate with their work
// vectors, projection partials and coefficient slots in a fixed, file-scope
// device array instead of buffers allocated for the call.  For callers that
// cannot allocate device memory (tight serving loops, harnesses that forbid
// it).  The array is per device (each GPU the library runs on holds its own
// copy until the process ends); every call on one device shares it, so calls
// that overlap on one device race.
#include <mutex>

#include "sg_internal.h"

namespace {

constexpr int64_t kScratchBytes = int64_t(64) << 20;
constexpr int kMaxDevices = 64;

// The scratch region.  Host code never passes this name to a kernel or a
// copy: on the host it is a stand-in, not a device address; the device
// address comes from hipGetSymbolAddress, once per device.
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device must be
// current).  Looked up once per device.
sg_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return sg::fail(SG_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return sg::hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return SG_OK;
}

}  // namespace

using namespace sg;

extern "C" {

int64_t sg_noalloc_scratch_bytes(void) { return kScratchBytes; }

sg_status sg_propagate_noalloc(sg_problem *p, void *psi, double dt, int32_t nsteps,
                               int32_t method, int32_t order, double tol, sg_precision prec,
                               int32_t check_every, sg_prop_stats *stats, double *norm_trace,
                               double *energy_trace, void *stream) {
  int m = 0, nvec = 0;
  sg_status st = propagate_check(p, psi, dt, nsteps, method, order, prec, check_every, &m, &nvec);
  if (st != SG_OK) return st;
  int64_t off[5];
  const int64_t need = propagate_layout(p->h.ncs, method, order, m, nvec, off);
  if (need > kScratchBytes)
    return fail(SG_EINVAL, "work buffers of " + std::to_string(need) +
                               " bytes exceed the fixed scratch of " +
                               std::to_string(kScratchBytes) +
                               " bytes; use sg_propagate or a smaller order");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device) return fail(SG_EINVAL, "the problem lives on another device");
  void *base = nullptr;
  if ((st = scratch_address(dev, &base)) != SG_OK) return st;
  char *b = (char *)base;
  PropBuffers B;
  B.owned = false;
  B.v = (double2 *)(b + off[0]);
  if (method == SG_PROP_SIL) {
    B.partials = (double *)(b + off[1]);
    B.coef = (double *)(b + off[2]);
    B.lz = (double *)(b + off[3]);
    B.npart = (double *)(b + off[4]);
  } else if (method == SG_PROP_BS || method == SG_PROP_RK) {
    B.coef = (double *)(b + off[2]);
  }
  return propagate_run(p, psi, dt, nsteps, method, order, m, nvec, tol, prec, check_every, stats,
                       norm_trace, energy_trace, stream, B, true);
}

}  // extern "C"
