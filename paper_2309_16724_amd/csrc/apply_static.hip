// dmrg_apply_H_static: H.psi without any device allocation.  The stripe
// workspace, partial tiles and stripe slices that dmrg_apply_H takes from
// the plan's own buffers live here in one file-scope device array instead,
// for callers that cannot allocate (code under graph capture of their own,
// tight serving loops, harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>
#include <mutex>
#include <string>
#include "plan.hpp"

namespace {

constexpr int64_t SCRATCH_BYTES = DMRG_STATIC_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;

// Every GPU the library runs on holds its own copy until the process ends.
// In host code the name is a host-side stand-in: only the address returned by
// hipGetSymbolAddress (per device) may be passed to kernels.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};

// device address of `scratch` on the current device (looked up once per device)
int scratch_ptr(char **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    dmrg::set_error(std::string("dmrg_apply_H_static: no usable current device: ") + hipGetErrorString(e));
    return DMRG_EHIP;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      dmrg::set_error(std::string("dmrg_apply_H_static: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return DMRG_EHIP;
    }
    g_scratch[dev] = p;
  }
  *out = (char *)g_scratch[dev];
  return DMRG_OK;
}

}  // namespace

extern "C" int dmrg_apply_H_static(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream) {
  if (!p || !psi || !hpsi) { dmrg::set_error("null argument"); return DMRG_EINVAL; }
  if (psi == hpsi) { dmrg::set_error("psi and hpsi must not alias"); return DMRG_EINVAL; }
  int64_t off[dmrg::SCRATCH_REGIONS];
  const int64_t need = dmrg::plan_scratch_layout(p, off);
  if (need > SCRATCH_BYTES) {
    dmrg::set_error("dmrg_apply_H_static: the plan needs " + std::to_string(need) +
                    " bytes of scratch memory, more than the static " + std::to_string(SCRATCH_BYTES) +
                    "; build the plan with a smaller workspace_bytes (its stripe workspace is cut into more "
                    "launches)");
    return DMRG_EINVAL;
  }
  char *base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  return dmrg::enqueue_scratch(p, psi, hpsi, stream, base);
}
