// Host planner: validation (once per call over shapes, Section 4) and the
// launch plan of one co-iteration.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "common.h"

namespace triot {

// Launch schedule knobs (defaults, or the autotuner's choice).
struct Sched {
    int vec_max = 4;        // widest vector (words) allowed: 1, 2 or 4
    int cache = 1;          // cache policy: 0 normal, 1 non-temporal loads and
                            // stores, 2 non-temporal loads only
    int blocks_per_cu = 4;  // persistent workgroups per CU
    int order = 0;          // unit order: 0 blocked ranges, 1 round-robin
    bool small_units = true;  // shrink units of small problems (not for batch items)
    bool no_vec2 = false;     // lanes of 4 or 1 words only (the batched kernel)
    int rb_max = RB_MAX;    // rows per box (LDS table) upper bound
    int pe_target = 8192;   // elements per work unit
};

// One validated, normalized request.
struct Request {
    triot_op op;
    int n;                           // operands
    int d;
    int64_t shape[MAXT][MAXD];
    int64_t counter[MAXD];
    int64_t base[MAXT];
    void *ptr[MAXT];
    int elem_bytes;                  // element size of COPY / EMBED_FILL (4 or 8), else 4
    int64_t npoints;                 // counter points
    const void *params;
    // Byte range [span_lo, span_hi) each operand touches over the counter
    // (empty when equal), and which operands are written; set by validate
    // for the element-wise ops that check aliasing.
    uint64_t span_lo[MAXT], span_hi[MAXT];
    bool written[MAXT];
};

struct CoLaunch {
    CoPlan plan;
    int dims;                 // the merged counter (before any split)
    int64_t extents[MAXD];    // its extents, inner axis in elements
    int blocks;               // requested grid (the launch keeps it within what fits at once)
    int cus;                  // compute units of the device planned for
    int unroll;               // elements per thread per step (fixed: 4)
    int cache;                // cache policy (Sched::cache)
    bool rows1;     // RB == 1
    bool unit;      // every inner stride is 1
};

struct SegLaunch {
    SegPlan plan;
    int blocks;
    int dm;         // accumulator positions of the moments pass: the kept axes
                    // with the covariance, else 8 or 32
    int dmax;       // register tier of the adjoint (8 or 32)
};

struct ConvLaunch {
    ConvPlan plan;
};

struct MargLaunch {
    MargPlan plan;
};

// Number of compute units of the current device (cached per device).
int device_cus();

triot_status validate(triot_op op, int n, int d, const int64_t *shapes, const int64_t *counter,
                      void *const *tensors, const int64_t *bases, const void *params, Request *r);

bool is_segment_op(triot_op op);

triot_status plan_coiter(const Request &r, const Sched &s, int cus, CoLaunch *out);
triot_status plan_segment(const Request &r, int cus, SegLaunch *out);

size_t segment_workspace_bytes(const SegLaunch &l);

triot_status plan_conv(const Request &r, ConvLaunch *out);
triot_status plan_marginal(const Request &r, int cus, MargLaunch *out);
size_t marginal_workspace_bytes(int cus);

// Key of the schedule cache: everything the plan shape depends on.
std::string sched_key(const Request &r);

}  // namespace triot
