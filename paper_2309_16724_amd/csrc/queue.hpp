// Device side of the per-XCD work queues (see XcdQueues in plan.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include "plan.hpp"

namespace dmrg {

// the XCD the calling wavefront runs on (HW_REG_XCC_ID)
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & (NXCD - 1); }

// Next tile for a caller on XCD x: the next entry of range x, then of the
// other ranges in turn; -1 once every range is exhausted.  qi holds the
// number of ranges found exhausted so far (the caller's state, starting at 0).
// One lane calls it; each returned index is handed out exactly once.
__device__ __forceinline__ int queue_next(const XcdQueues &q, int32_t *counters, int x, int &qi) {
  for (; qi < NXCD; qi++) {
    const int qq = (x + qi) & (NXCD - 1);
    const int len = q.start[qq + 1] - q.start[qq];
    if (len <= 0) continue;
    const int k = atomicAdd(counters + qq, 1);
    if (k < len) return q.start[qq] + k;
  }
  return -1;
}

}  // namespace dmrg
