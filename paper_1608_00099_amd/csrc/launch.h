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
hipError_t launch_dot(const SegLaunch &L, hipStream_t st);
hipError_t launch_bbox(const SegLaunch &L, hipStream_t st);
hipError_t launch_conv(const ConvLaunch &L, hipStream_t st);
uint32_t conv_lds_words();
hipError_t launch_marginal(const MargLaunch &L, hipStream_t st);

}  // namespace triot
