// Internal plan layouts shared by the host planner and the gfx950 kernels.
//
// A plan is everything a kernel needs to co-iterate, passed by value as the
// kernel argument (the kernel-argument segment is constant memory read
// through the scalar cache), or, for batches, stored in device memory.
#pragma once

#include <stdint.h>

#include "triot.h"

namespace triot {

constexpr int MAXD = TRIOT_MAX_D;
constexpr int MAXT = TRIOT_MAX_TENSORS;
constexpr uint32_t NOBOUND = 0xFFFFFFFFu;
constexpr int NT = 256;           // threads per workgroup (4 wave64)
constexpr int RB_MAX = 1024;      // LDS row-table capacity (rows per box)
constexpr int SEG_MAX = 32;       // per-thread segment length of the row kernels
constexpr int DOT_QUADS = 4;      // word quads per lane and tile of the inner product's quad walk
constexpr int MOM_TERMS_MAX = 1 + MAXD + 8 * 9 / 2;  // covariance limited to 8 axes

// Internal op ids of the element-wise family (kernel template argument).
enum CoOp : int {
    CO_COPY = 0,
    CO_FILL = 1,
    CO_MUL_ACC = 2,
    CO_MUL = 3,
    CO_MUL_ADJ = 4,
    CO_INDEX = 5,
    CO_XPYX_MZ = 6,
};

// Division of a 32-bit n by an invariant divisor c >= 2 (Granlund &
// Montgomery, PLDI 1994, round-up multiplier with add-back):
//   h = mulhi(n, m);  q = (h + ((n - h) >> 1)) >> s
// with l = ceil(log2 c), m = floor(2^32 (2^l - c) / c) + 1, s = l - 1.
struct AxisDiv {
    uint32_t c, m, s, pad;
};

// ---------------------------------------------------------------------
// Element-wise co-iteration plan (one lane per counter element).
//
// The planned counter has D axes (extent-1 axes dropped, adjacent axes
// merged where every operand is contiguous across them): D-1 outer axes
// and one inner axis of extent L in units of `vec` 4-byte words (outer
// strides and bases in words).
// The outer axes split into `nhigh` high axes and `nlow` low axes.  A
// *box* is one value of the high axes: RB = prod(low extents) rows of L
// elements.  Every workgroup tabulates, once, the offset of each box row
// relative to the box start (low axes only, so the table is the same for
// every box); a work unit is one box part of at most PE elements, whose
// high tuple is decoded once, uniformly, by magic division.
struct CoPlan {
    uint32_t D, n, nhigh, nlow;
    uint32_t L;          // inner extent
    uint32_t Lm;         // ceil(2^32 / L): e / L == mulhi(e, Lm) for e < 2^32 / L (RB > 1)
    uint32_t RB;         // rows per box
    uint32_t BE;         // elements per box (RB * L)
    uint32_t parts;      // units per box
    uint32_t PE;         // elements per unit
    AxisDiv partdiv;     // unit -> (box, part); c == 1 means parts == 1
    uint32_t nunits;     // boxes * parts
    uint32_t predmask;   // bit k: operand k only where t lies inside its window
    uint32_t esz;        // bytes per vector element (4 * vec)
    uint32_t vec;
    // Ragged rows: when the inner extent is not a multiple of vec, each row
    // ends in a vector moved back by tshift bytes so that it ends at the row
    // end; of its vec words only the last vec - tskip are new (tskip = 0:
    // rows are whole vectors).
    uint32_t tshift;
    uint32_t tskip;
    // EMBED_FILL with vectors: the source's inner window extent in elements
    // (NOBOUND = none).  A vector wholly inside it is loaded whole, one
    // straddling it word by word, and the rest of the vector is zero.
    uint32_t ibel;
    uint32_t unit;       // 1 when every inner stride is 1
    uint32_t interleave; // unit order: 0 a contiguous range of units per
                         // workgroup, 1 units dealt round-robin
    // Split axis: the outermost low axis may be the lower part (m digits)
    // of a counter axis of extent `sc` whose upper part (ceil(sc/m) blocks)
    // is the innermost high axis.  The last block covers sc - hi*m < m
    // digits, a prefix of the box; window bounds on that axis become a
    // per-box limit on the low digit (stored in the row mask word).
    uint32_t split;      // 0 or 1
    uint32_t sm;         // digits per block (m)
    uint32_t sc;         // true extent of the split axis
    uint32_t rows_below; // box rows per low digit of the split axis
    uint32_t sbound[MAXT];            // window extent on the split axis (NOBOUND = none)
    AxisDiv ax[MAXD];                 // outer axes, outermost first
    int64_t stride[MAXT][MAXD];       // outer strides per operand (4-byte words)
    uint32_t bound[MAXT][MAXD];       // window extent per outer axis (NOBOUND = unchecked)
    uint32_t ibound[MAXT];            // window extent on the inner axis
    uint32_t istride[MAXT];           // inner stride (vector units)
    int64_t base[MAXT];               // 4-byte words
    uint64_t ptr[MAXT];               // device byte addresses
    uint64_t npoints;                 // counter points (INDEX output leading dimension)
    uint64_t cstride[MAXD];           // counter flat stride of each high axis (INDEX)
};

// ---------------------------------------------------------------------
// Row-segment plan (moments and their adjoint: one thread per segment).
//
// Logical axes only (extent-1 axes dropped, no merging, the tuple is read):
// D axes, D-1 outer and the inner one of extent L.  Each row splits into G
// segments of at most S elements; a thread folds one segment at a time.
// The moments pass loads a segment with 16-byte accesses when `vec4`; the
// adjoint stages NT consecutive segments through LDS when `full`.
struct SegPlan {
    uint32_t D, n;
    uint32_t d_orig;
    uint32_t L, S, G;
    AxisDiv gdiv;             // segment -> (row, part of row); c == 1 means G == 1
    uint32_t rows;            // counter rows (< 2^32)
    uint32_t full;            // every operand contiguous over the counter
    uint32_t vec4;            // every operand contiguous along the row and L % 4 == 0
    uint32_t stage;           // 1, 2 tiles through LDS (rows of 4-16 words, 32-word segments); 3 short rows batched;
                              // 4 row blocks: segments of rb whole rows (16 words) through LDS;
                              // 5 rows of exactly 16 words, per-lane loads;
                              // 6 rows of 16 words end to end, quads of 16 rows per load, row sums (moments)
                              //   or row masks (bounding box) formed across lanes
    uint32_t rb;              // stage 4: rows per segment (16 / L)
    uint32_t quads;           // DOT: one word quad per lane (vec4, quads < 2^31, not staged)
    AxisDiv qdiv;             // quads: quad -> (row, quad in row), divisor L / 4
    uint64_t nquads;          // quads: rows * L / 4
    uint32_t flags;           // TRIOT_MOMENTS_* bits
    uint32_t nblocks;         // grid size (moments: number of partials)
    uint32_t nterms;          // accumulated terms: 1 + D (+ D(D+1)/2)
    uint64_t nseg;            // rows * G
    uint64_t ntiles;          // ceil(nseg / NT)
    AxisDiv ax[MAXD];         // outer axes 0..D-2
    double center[MAXD];      // shift (c-1)/2 per kept axis
    uint32_t orig[MAXD];      // original axis of kept axis i
    int64_t stride[4][MAXD];  // element strides per operand (inner at D-1)
    int64_t base[4];
    uint64_t ptr[4];
    uint64_t out32;           // MOMENTS: float results
    uint64_t out64;           // MOMENTS: optional double results; ADJ: moments in
    uint64_t gmom;            // ADJ: float partials
    uint64_t ws;              // MOMENTS: partials + ticket
};

// ---------------------------------------------------------------------
// Naive convolution plan (one thread per output element).
struct ConvPlan {
    uint32_t d;
    uint32_t lds;             // 1: both inputs staged in LDS
    uint64_t nout;            // output elements (< 2^32)
    uint32_t nl, nr;          // input elements (LDS staging sizes)
    AxisDiv ax[MAXD];         // output extents (axes 1..d-1 divided)
    uint32_t ls[MAXD], rs[MAXD];
    int64_t lstride[MAXD], rstride[MAXD];
    uint64_t out, lhs, rhs;   // device addresses (float64)
};

// ---------------------------------------------------------------------
// Marginalization plan: thread (o, p) sums part p of the reduced sub-box
// of kept tuple o; a second pass adds the parts in order when parts > 1.
struct MargPlan {
    uint32_t n, dk, dr;       // operands, kept axes, reduced axes
    uint32_t parts;
    // Walk of a part: mode 0 one element at a time; mode 1 four at a time
    // (the innermost reduced axis is every operand's last axis, extent a
    // multiple of 4, part boundaries multiples of 4); mode 2 interleaved
    // (one reduced axis, contiguous in every operand: lane l of a wave
    // takes elements chunk * clen + l + 64 s, so a wave's loads are
    // coalesced); mode 4 columns (one kept axis, innermost and unit-stride,
    // one reduced axis: thread (q, p) adds outputs 4q .. 4q + 3 over rows
    // p, p + parts, .., so a wave's loads cover consecutive rows); mode 5
    // short runs (one reduced axis, innermost and unit-stride, of 4 .. 64
    // elements, a power of 2: nred / 4 lanes per output, a word quad each).
    uint32_t mode;
    uint32_t clen;            // mode 2: elements per chunk (64 lanes)
    uint64_t nout;            // kept tuples (< 2^32)
    uint64_t nred;            // reduced tuples
    AxisDiv kax[MAXD];        // kept extents, outermost first
    AxisDiv rax[MAXD];        // reduced extents, outermost first
    int64_t kstride[4][MAXD]; // element strides of the kept axes per operand
    int64_t rstride[4][MAXD]; // element strides of the reduced axes per operand
    int64_t base[4];
    uint64_t ptr[4];
    uint64_t out32, out64, ws;
};

// Host-side helpers (plan.cpp).
bool magic_for(uint32_t c, AxisDiv *out);

}  // namespace triot
