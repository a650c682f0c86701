// Kernel launchers (device code in kern_*.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace triot {

hipError_t launch_coiter(int co_op, const CoLaunch &L, hipStream_t st);
hipError_t launch_batched(int co_op, const CoPlan *plans, const uint32_t *ustart, uint32_t nitems,
                          uint32_t total, int blocks, hipStream_t st);
hipError_t launch_moments(const SegLaunch &L, hipStream_t st);
hipError_t launch_moments_adj(const SegLaunch &L, hipStream_t st);
int segment_blocks_per_cu(bool adj, bool cov, int dm, bool vec4);

}  // namespace triot
