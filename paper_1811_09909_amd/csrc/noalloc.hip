// hdg_rhs_noalloc: the right-hand side g of the trace system (eq.
// trace_linear_system) from a volume source, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops).
// hdg_rhs stages the per-element loads in memory the handle allocated at
// setup; this variant stages them in a fixed device array of this file, so
// a call makes no allocation of any kind.  The array is one per GPU the
// library runs on (each holds its own copy until the process ends); its
// device address is taken once per device, with that device current, at the
// first hdg_setup on it.
#include <mutex>

#include "hdg_internal.hpp"

namespace hdg {

// largest staging the allocation-free call supports: N_T * ((k+1)^d +
// 2 d (k+1)^(d-1)) doubles (64 MiB: e.g. 256 x 256 elements up to k = 6,
// 512 x 512 up to k = 2)
constexpr long RHS_SCRATCH_DOUBLES = 8L << 20;

static __device__ __align__(256) double scratch[RHS_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[MAX_DEVICES] = {};
}  // namespace

// this device's copy of `scratch`, looked up once per device with the
// device current (the array's host-side name is not a device address)
double* scratch_ptr() {
  int dev = 0;
  HDG_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw HipError{hipErrorInvalidDevice, "scratch: device index"};
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    HDG_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    scratch_dev[dev] = static_cast<double*>(p);
  }
  return scratch_dev[dev];
}

long scratch_capacity() { return RHS_SCRATCH_DOUBLES; }

}  // namespace hdg

extern "C" hdg_status hdg_rhs_noalloc(hdg_handle h, const double* rhs, int rhs_kind, const double* g_dirichlet,
                                      double* g) {
  if (!h || !rhs || !g) return HDG_ERR_INVALID_ARG;
  if (rhs_kind != HDG_RHS_F_NODAL && rhs_kind != HDG_RHS_F_LOAD) return HDG_ERR_INVALID_ARG;
  try {
    if (!hdg::rhs_supported(h, rhs_kind, g_dirichlet)) return HDG_ERR_UNSUPPORTED;
    const long need = hdg::rhs_staging_doubles(h);
    if (need > hdg::RHS_SCRATCH_DOUBLES) return HDG_ERR_UNSUPPORTED;
    hdg::rhs_with_staging(h, rhs, rhs_kind, g_dirichlet, g, hdg::scratch_ptr());
    return HDG_OK;
  } catch (const hdg::HipError&) {
    return HDG_ERR_DEVICE;
  }
}
