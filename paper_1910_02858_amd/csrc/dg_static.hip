// Entry points that allocate no device memory, for callers that cannot call hipMalloc (code
// under HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// Their scratch lives in one file-scope device array per GPU, `scratch`, sized
// DG_NOALLOC_SCRATCH_DOUBLES.  In host code the array's name is only a host-side stand-in, so
// the device address of each GPU's copy is looked up once, with hipGetSymbolAddress while that
// GPU is current (dg_init calls dg_static_scratch_setup), kept per device, and passed to the
// kernels as an ordinary pointer.  Every call on one GPU shares that GPU's copy, and each GPU
// holds it until the process ends: calls that overlap in time on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dg_internal.h"

static __device__ __align__(256) double scratch[DG_NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each GPU, nullptr until looked up

}  // namespace

namespace dg {

int static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return DG_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return DG_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return DG_ERR_HIP;
  }
  g_ptr[device] = static_cast<double *>(p);
  return DG_OK;
}

}  // namespace dg

extern "C" int dg_integrals_noalloc(dg_handle *h, const double *U, double *out_dev) {
  if (!h) return DG_ERR_ARG;
  if (!U || !out_dev || (reinterpret_cast<uintptr_t>(U) & 7u) || (reinterpret_cast<uintptr_t>(out_dev) & 7u)) {
    h->err = "U and out_dev must be non-NULL, 8-byte aligned device pointers";
    return DG_ERR_ARG;
  }
  const size_t need = (size_t)h->K * 8;
  if (need > (size_t)DG_NOALLOC_SCRATCH_DOUBLES) {
    h->err = "dg_integrals_noalloc: the mesh has more elements than the static scratch holds (8 doubles per "
             "element, at most " + std::to_string(DG_NOALLOC_SCRATCH_DOUBLES / 8) + " elements)";
    return DG_ERR_UNSUPPORTED;
  }
  double *partial = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (h->device >= 0 && h->device < kMaxDevices) partial = g_ptr[h->device];
  }
  if (!partial) {
    h->err = "dg_integrals_noalloc: no scratch address for the handle's device";
    return DG_ERR_HIP;
  }
  const dg::Geo g = h->geo();
  int rc;
  switch (h->N) {
#define DG_CASE(NN) \
  case NN: rc = dg::launch_reduce<NN>(g, h->ph, dg::RED_INTEGRALS, U, 0.0, partial, h->stream); break;
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: rc = DG_ERR_UNSUPPORTED;
  }
  if (!rc) rc = dg::launch_final_reduce(dg::RED_INTEGRALS, partial, h->K, out_dev, h->stream);
  if (rc) h->err = "launch of the integral reduction failed";
  return rc;
}
