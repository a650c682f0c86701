// Kernel launchers (device code in kern_*.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace triot {

hipError_t launch_coiter(int co_op, const CoLaunch &L, hipStream_t st);
// One persistent launch over a device table of item plans.
struct BatchLaunch {
    const CoPlan *plans;      // device: the item plans
    const uint32_t *ustart;   // device: each item's first work unit, then the total
    const uint32_t *uitem;    // device: the item of every work unit, or null (then
                              // the kernel searches ustart)
    uint32_t nitems;
    uint32_t total;           // work units over all items
    uint32_t rows_max;        // largest rows per box among items with RB > 1 (0: none)
    int blocks;               // requested grid (clamped to what fits at once)
    int cus;
    int cache;                // cache policy
    uint32_t rr;              // 0: contiguous unit ranges per workgroup, 1: round-robin
    int launched;             // out: the grid launched
};
hipError_t launch_batched(int co_op, BatchLaunch &B, hipStream_t st);
hipError_t launch_moments(const SegLaunch &L, hipStream_t st);
hipError_t launch_moments_adj(const SegLaunch &L, hipStream_t st);
int segment_blocks_per_cu(bool adj, bool cov, int dm, bool vec4, int stage);
hipError_t launch_dot(const SegLaunch &L, hipStream_t st);
hipError_t launch_bbox(const SegLaunch &L, hipStream_t st);
hipError_t launch_conv(const ConvLaunch &L, hipStream_t st);
uint32_t conv_lds_words();
hipError_t launch_marginal(const MargLaunch &L, hipStream_t st);

}  // namespace triot
