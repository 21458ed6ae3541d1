// Allocation-free Schur-complement apply.
//
// edd_apply_S needs one interior-length work vector, t = K_II^{-1} (K [0; v])_I,
// which normally lives in the handle's own buffer.  edd_apply_S_noalloc takes
// it from `scratch`, a static device array of fixed size, so the call makes
// no device allocation of any kind.  Each GPU holds its own copy of the array
// at its own address; the address is looked up once per device, at handle
// set-up, with that device current, and kept here.
#include <map>
#include <mutex>

#include "internal.h"

namespace edd {

namespace {

__device__ __align__(256) double scratch[EDD_NOALLOC_MAX_INTERIOR_DOFS];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device -> address of its `scratch`

}  // namespace

// Resolve the device address of `scratch` for p->device (current during
// set-up) once per device and record it on the handle.
int scratch_init(edd_problem *p) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(p->device);
  if (it != g_scratch_ptr.end()) {
    p->scratch_d = it->second;
    return EDD_OK;
  }
  int cur = -1;
  int rc = check_hip(p, hipGetDevice(&cur));
  if (rc) return rc;
  if (cur != p->device) return EDD_ESTATE;
  double *ptr = nullptr;
  rc = check_hip(p, hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
  if (rc) return rc;
  if (!ptr) return EDD_EHIP;
  g_scratch_ptr[p->device] = ptr;
  p->scratch_d = ptr;
  return EDD_OK;
}

}  // namespace edd

extern "C" int edd_apply_S_noalloc(edd_problem *p, const double *v_dev, double *y_dev,
                                   int precision) {
  using namespace edd;
  if (!p || !v_dev || !y_dev) return EDD_EINVAL;
  if (precision != EDD_F64 && precision != EDD_F32) return EDD_EINVAL;
  if (p->n_idofs > (int64_t)EDD_NOALLOC_MAX_INTERIOR_DOFS) return EDD_EINVAL;
  if (!p->scratch_d) return EDD_ESTATE;
  if (!p->have_moduli) return EDD_ESTATE;
  if (!(p->factor_precision & precision)) return EDD_ESTATE;
  // per-launch timing creates HIP events on demand: suspend it for the call
  const bool kt = p->kt_enabled;
  p->kt_enabled = false;
  apply_S_with(p, v_dev, y_dev, precision, p->scratch_d);
  p->kt_enabled = kt;
  return check_hip(p, hipGetLastError());
}
