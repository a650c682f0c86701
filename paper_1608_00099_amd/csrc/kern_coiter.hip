// Element-wise co-iteration kernels for gfx950 (CDNA4, wave64).
//
// One lane per counter element, elements in row-major counter order, so
// that consecutive lanes touch consecutive addresses along the innermost
// (collapsed) axis of every operand.  The flat -> tuple decode of the paper
// (Section 1, reindexing by remainder and quotient) is split in three:
//   - the high axes of a work unit are decoded once, uniformly (scalar
//     registers), by magic-number division, giving every operand's 64-bit
//     box base;
//   - the low axes are decoded once per workgroup into an LDS table of
//     32-bit row offsets, identical for every box;
//   - per element only row = e / L (one mulhi) and the table lookup remain.
// Offsets are the row-major (Horner) sums of Section 1.  Windows (slices
// with a bias, Section 4) enter through the operand bases, partial reads
// (zero-filled embedding, adjoints) through per-axis window bounds.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"

namespace triot {

__device__ __forceinline__ uint32_t div_u32(uint32_t n, const AxisDiv &a)
{
    uint32_t h = __umulhi(n, a.m);
    return (h + ((n - h) >> 1)) >> a.s;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); consecutive logical blocks should share an XCD so that neighbouring
// work units (and the partially written cache lines between them) meet in
// one L2.
__device__ __forceinline__ uint32_t logical_block()
{
    uint32_t g = gridDim.x, b = blockIdx.x;
    if ((g & 7u) == 0)
        return (b & 7u) * (g >> 3) + (b >> 3);
    return b;
}

// Global-address-space pointers: loads and stores then address memory as a
// uniform 64-bit base (scalar registers) plus a 32-bit per-lane offset.
#define GLOBAL __attribute__((address_space(1)))
typedef GLOBAL char gchar;

// Cache policy of a launch (a schedule knob): CP_NONTEMP_LS marks loads and
// stores non-temporal (streamed past the caches, the right hint for data
// touched once), CP_NONTEMP_L the loads only (windowed stores that leave
// partial cache lines can merge better in L2 when cached normally).
enum { CP_NORMAL = 0, CP_NONTEMP_LS = 1, CP_NONTEMP_L = 2 };

template <class T, int CP> __device__ __forceinline__ T gload(const gchar *p, uint32_t off)
{
    const GLOBAL T *a = (const GLOBAL T *)(p + off);
    if constexpr (CP == CP_NORMAL)
        return *a;
    else
        return __builtin_nontemporal_load(a);
}

template <class T, int CP> __device__ __forceinline__ void gstore(gchar *p, uint32_t off, T v)
{
    GLOBAL T *a = (GLOBAL T *)(p + off);
    if constexpr (CP == CP_NONTEMP_LS)
        __builtin_nontemporal_store(v, a);
    else
        *a = v;
}

// Store of a ragged row's last vector: only its words from `skip` on are
// new (the others belong to the vector before it, stored by another lane).
// 1 <= skip < V.
//
// whole_tail: the read-modify-write ops (x += y*z, out = a*b in place,
// benchmark 3's update) store the last vector whole when the vector before
// it belongs to the previous lane of the same wavefront: both then sit in
// the same load and store instructions of one step, a wavefront issues all
// of a step's loads before its stores, so the shared words were loaded
// unchanged by both lanes and both store the same bits there.  The first
// lane of a wavefront (its predecessor belongs to another wavefront, which
// may already have stored) keeps the word-wise store.  A whole store is
// part of the same store instruction as its predecessor's and the two fill
// their cache lines together, where word stores issued after it reach
// memory as separate partial writes.
template <class T, int CP>
__device__ __forceinline__ void gstore_tail(gchar *p, uint32_t off, T v, uint32_t skip)
{
    if constexpr (sizeof(T) > 4) {
        constexpr int V = sizeof(T) / 4;
        typedef __typeof__(v[0] + 0) W;
#pragma unroll
        for (int c = 1; c < V; ++c) {
            W w = v[c];
            if ((uint32_t)c >= skip)
                gstore<W, CP>(p, off + 4u * c, w);
        }
    }
}

template <int V> struct Vec;
template <> struct Vec<1> {
    typedef uint32_t U;
    typedef float F;
};
// Vectors are only 4-byte aligned in memory (rows may start at any word).
template <> struct Vec<2> {
    typedef uint32_t U __attribute__((ext_vector_type(2), aligned(4)));
    typedef float F __attribute__((ext_vector_type(2), aligned(4)));
};
template <> struct Vec<4> {
    typedef uint32_t U __attribute__((ext_vector_type(4), aligned(4)));
    typedef float F __attribute__((ext_vector_type(4), aligned(4)));
};

// The box-row table in LDS, sized per launch (dynamic shared memory) so that
// small boxes leave room for more resident workgroups: per operand, `rs`
// pre-adjusted byte offsets of the box rows (operand-major), then, for the
// predicated ops, `rs` row masks (bits 0-7: the row lies inside operand k's
// window; bits 8-31: the row's digit on the split axis).
extern __shared__ uint32_t lds_rows[];

struct RowTable {
    uint32_t *t;
    uint32_t rs;               // row stride: the plan's rows per box
    __device__ __forceinline__ uint32_t off(int k, uint32_t r) const { return t[(uint32_t)k * rs + r]; }
    __device__ __forceinline__ uint32_t mask(uint32_t n, uint32_t r) const { return t[n * rs + r]; }
};

// Tabulate the box rows: decode each row over the low axes and store, per
// operand, row offset * 4 - row * L * istride * esz (bytes; row offsets are
// in 4-byte words, the inner axis in vectors of esz bytes) so that element
// e of the box sits at table[row] + e * istride * esz bytes from the box
// base.  Row masks are stored when PRED.
template <bool PRED>
__device__ void fill_table(const CoPlan &P, const RowTable &T)
{
    const uint32_t n = P.n, nhigh = P.nhigh, nlow = P.nlow;
    for (uint32_t r = threadIdx.x; r < P.RB; r += NT) {
        uint32_t rel[MAXT];
#pragma unroll
        for (int k = 0; k < MAXT; ++k)
            rel[k] = 0;
        uint32_t mask = 0xFFu;
        uint32_t q = r;
        uint32_t t = 0;
        for (int j = (int)(nhigh + nlow) - 1; j >= (int)nhigh; --j) {
            const AxisDiv a = P.ax[j];
            if (j == (int)nhigh) {
                t = q;                       // outermost low axis: the rest
            } else {
                uint32_t qq = div_u32(q, a);
                t = q - qq * a.c;
                q = qq;
            }
#pragma unroll
            for (int k = 0; k < MAXT; ++k) {
                if (k < (int)n) {
                    rel[k] += t * (uint32_t)P.stride[k][j];
                    if (t >= P.bound[k][j])
                        mask &= ~(1u << k);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < MAXT; ++k)
            if (k < (int)n)
                T.t[(uint32_t)k * T.rs + r] = rel[k] * 4u - r * P.L * P.istride[k] * P.esz;
        // t now holds the outermost low digit (the split axis' digit if split)
        if (PRED)
            T.t[n * T.rs + r] = mask | (t << 8);
    }
}

template <int OP> struct OpInfo;
template <> struct OpInfo<CO_COPY> { static constexpr int N = 2; static constexpr bool PRED = false; };
template <> struct OpInfo<CO_FILL> { static constexpr int N = 2; static constexpr bool PRED = true; };
template <> struct OpInfo<CO_MUL_ACC> { static constexpr int N = 3; static constexpr bool PRED = false; };
template <> struct OpInfo<CO_MUL> { static constexpr int N = 3; static constexpr bool PRED = false; };
template <> struct OpInfo<CO_MUL_ADJ> { static constexpr int N = 5; static constexpr bool PRED = true; };
template <> struct OpInfo<CO_INDEX> { static constexpr int N = MAXT; static constexpr bool PRED = false; };
template <> struct OpInfo<CO_XPYX_MZ> { static constexpr int N = 3; static constexpr bool PRED = false; };

// Process one work unit (a part of one box).  BATCH: called from the batched
// kernel (which keeps EMBED_FILL's lower-register body, see below).
template <int OP, int V, int U, bool ROWS1, bool UNIT, int CP, bool RAG, bool BATCH = false>
__device__ __forceinline__ void run_unit(const CoPlan &P, uint32_t unit, const RowTable &T)
{
    typedef typename Vec<V>::U VU;
    typedef typename Vec<V>::F VF;
    constexpr int N = OpInfo<OP>::N;
    const uint32_t n = (OP == CO_INDEX) ? P.n : (uint32_t)N;

    // ---- uniform: unit -> (box, part) -> high tuple -> box bases ----
    uint32_t box, part;
    if (P.partdiv.c == 1) {
        box = unit;
        part = 0;
    } else {
        box = div_u32(unit, P.partdiv);
        part = unit - box * P.parts;
    }
    int64_t bb[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
        bb[k] = (k < (int)n) ? P.base[k] : 0;
    uint32_t himask = 0xFFFFFFFFu;
    uint32_t blk = 0;          // block digit of the split axis
    uint64_t fbase = 0;        // counter flat index of the box start (INDEX)
    {
        uint32_t q = box;
        for (int i = (int)P.nhigh - 1; i >= 0; --i) {
            uint32_t t;
            if (i == 0) {
                t = q;
            } else {
                const AxisDiv a = P.ax[i];
                uint32_t qq = div_u32(q, a);
                t = q - qq * a.c;
                q = qq;
            }
            if (i == (int)P.nhigh - 1)
                blk = t;
            if (OP == CO_INDEX)
                fbase += (uint64_t)t * P.cstride[i];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k < (int)n) {
                    bb[k] += (int64_t)t * P.stride[k][i];
                    if (OpInfo<OP>::PRED && t >= P.bound[k][i])
                        himask &= ~(1u << k);
                }
            }
        }
    }
    uint32_t bev = P.BE;       // elements of this box (a prefix when split)
    uint32_t lolim[N];         // per operand: limit on the split digit
#pragma unroll
    for (int k = 0; k < N; ++k)
        lolim[k] = 0xFFFFFFFFu;
    if (P.split) {
        const uint32_t first = blk * P.sm;
        const uint32_t rows = min(P.sm, P.sc - first);
        bev = rows * P.rows_below * P.L;
        if (OpInfo<OP>::PRED) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const uint32_t b = P.sbound[k < (int)n ? k : 0];
                lolim[k] = (b == NOBOUND) ? 0xFFFFFFFFu : (b > first ? b - first : 0u);
            }
        }
    }
    const uint32_t e0 = part * P.PE;
    const uint32_t e1 = min(e0 + P.PE, bev);
    if (e0 >= e1)
        return;
    // Single-row boxes: the base moves to the vector before the unit's
    // first (the row start for the first unit), so that the per-lane
    // offsets stay non-negative for a ragged row's last vector, moved back
    // by up to V - 1 words, when it is the first vector of a unit.
    const uint32_t eb = (ROWS1 && e0 >= 1u) ? e0 - 1u : 0u;
    if (ROWS1) {
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k < (int)n)
                bb[k] += (int64_t)eb * P.istride[k] * V;
    }
    constexpr uint32_t esz = 4u * V;   // == P.esz: the launcher picks V = P.vec
    gchar *bp[N];
    uint32_t isb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        bp[k] = (gchar *)(uintptr_t)(P.ptr[k < (int)n ? k : 0]) + bb[k] * (int64_t)4;
        isb[k] = UNIT ? esz : P.istride[k < (int)n ? k : 0] * esz;
    }

    // ---- per element ----
    const uint32_t lastj = P.L - 1;
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += NT * U) {
        uint32_t ev[U];
        bool valid[U];
        bool tl[U];              // a ragged row's last vector
        uint32_t off[N][U];
        uint32_t pm[U];
        uint32_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t x = e + (uint32_t)u * NT;
            valid[u] = x < e1;
            x = valid[u] ? x : e0;
            ev[u] = x;
            uint32_t row, j;
            if (ROWS1) {
                row = 0;
                j = x;
            } else {
                row = __umulhi(x, P.Lm);
                j = x - row * P.L;
            }
            jj[u] = j;
            tl[u] = RAG && j == lastj;
            pm[u] = 0xFFFFFFFFu;
            if (OpInfo<OP>::PRED) {
                const uint32_t rm = ROWS1 ? 0xFFu : T.mask(n, row);
                const uint32_t dig = rm >> 8;
                uint32_t m = himask & rm & 0xFFu;
#pragma unroll
                for (int k = 0; k < N; ++k)
                    if (j >= P.ibound[k] || dig >= lolim[k])
                        m &= ~(1u << k);
                pm[u] = m;
            }
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k < (int)n) {
                    uint32_t rel = ROWS1 ? 0u : T.off(k, row);
                    uint32_t xe = ROWS1 ? (x - eb) : x;
                    off[k][u] = rel + xe * isb[k] - (tl[u] ? P.tshift : 0u);
                }
            }
        }

        if constexpr (OP == CO_COPY) {
            // A ragged row's last vector is stored whole: the words it shares
            // with the vector before it get the same source words again (the
            // destination is either disjoint from the source or the source).
            VU v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u])
                    v[u] = gload<VU, CP>(bp[1], off[1][u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u])
                    gstore<VU, CP>(bp[0], off[0][u], v[u]);
        } else if constexpr (OP == CO_FILL && !BATCH) {
            // Vectors: the source's inner bound is checked per word (ibel);
            // the destination vector, a ragged row's last included, is
            // stored whole (shared words get the same value twice).  The
            // registers of a vector are written by loads only (a vector
            // straddling the bound loads its words, the ones past the bound
            // from the last word before it) and words outside the source
            // are zeroed after the step's loads: no register is written by
            // an ALU instruction while a load to it may be in flight in
            // another lane, so the step waits for its loads once, before
            // its stores (one counter covers loads and stores: a wait
            // between them would also wait for the stores already issued).
            VU v[U];
            bool keep[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                asm volatile("" : "=v"(v[u]));   // defined without an instruction
                const bool rd = valid[u] && (pm[u] & 2u);
                if constexpr (V == 1) {
                    keep[u][0] = rd;
                    if (rd)
                        v[u] = gload<VU, CP>(bp[1], off[1][u]);
                } else {
                    const uint32_t jel = jj[u] * V - (tl[u] ? P.tskip : 0u);
                    // word addresses formed before any load of the step, in
                    // registers no load of it writes
                    uint32_t wa[V];
                    const uint32_t last = P.ibel - 1u - jel;   // < V - 1 where used
#pragma unroll
                    for (int c = 0; c < V; ++c) {
                        keep[u][c] = rd && jel + (uint32_t)c < P.ibel;
                        wa[c] = off[1][u] + 4u * min((uint32_t)c, last);
                        asm volatile("" : "+v"(wa[c]));
                    }
                    if (rd && jel + V <= P.ibel) {
                        v[u] = gload<VU, CP>(bp[1], off[1][u]);
                    } else if (rd && jel < P.ibel) {
#pragma unroll
                        for (int c = 0; c < V; ++c)
                            v[u][c] = gload<uint32_t, CP>(bp[1], wa[c]);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (V == 1) {
                    v[u] = keep[u][0] ? v[u] : (VU)0u;
                } else {
#pragma unroll
                    for (int c = 0; c < V; ++c)
                        v[u][c] = keep[u][c] ? v[u][c] : 0u;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u])
                    gstore<VU, CP>(bp[0], off[0][u], v[u]);
        } else if constexpr (OP == CO_FILL) {
            // The batched kernel's body: the same values with fewer
            // registers (its instance holds every lane-width variant, and
            // the body above would cost it two of eight workgroups per CU,
            // more than the waits it saves).  A straddling vector loads its
            // words in place, which waits for loads in flight.
            VU v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                v[u] = (VU)0u;
                if (valid[u] && (pm[u] & 2u)) {
                    if constexpr (V == 1) {
                        v[u] = gload<VU, CP>(bp[1], off[1][u]);
                    } else {
                        const uint32_t jel = jj[u] * V - (tl[u] ? P.tskip : 0u);
                        if (jel + V <= P.ibel) {
                            v[u] = gload<VU, CP>(bp[1], off[1][u]);
                        } else {
#pragma unroll
                            for (int c = 0; c < V; ++c)
                                if (jel + (uint32_t)c < P.ibel)
                                    v[u][c] = gload<uint32_t, CP>(bp[1], off[1][u] + 4u * c);
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u])
                    gstore<VU, CP>(bp[0], off[0][u], v[u]);
        } else if constexpr (OP == CO_MUL_ACC) {
            VF x[U], y[U], z[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) {
                    x[u] = gload<VF, CP>(bp[0], off[0][u]);
                    y[u] = gload<VF, CP>(bp[1], off[1][u]);
                    z[u] = gload<VF, CP>(bp[2], off[2][u]);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) {
                    VF prod = y[u] * z[u];       // rounded once (no contraction)
                    if (tl[u] && (threadIdx.x & 63u) != 0)
                        gstore<VF, CP>(bp[0], off[0][u], x[u] + prod);   // see whole_tail
                    else if (tl[u])
                        gstore_tail<VF, CP>(bp[0], off[0][u], x[u] + prod, P.tskip);
                    else
                        gstore<VF, CP>(bp[0], off[0][u], x[u] + prod);
                }
        } else if constexpr (OP == CO_XPYX_MZ) {
            VF x[U], y[U], z[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) {
                    x[u] = gload<VF, CP>(bp[0], off[0][u]);
                    y[u] = gload<VF, CP>(bp[1], off[1][u]);
                    z[u] = gload<VF, CP>(bp[2], off[2][u]);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) {
                    // (x + y*x) - z, each operation rounded once
                    VF prod = y[u] * x[u];
                    VF sum = x[u] + prod;
                    if (tl[u] && (threadIdx.x & 63u) != 0)
                        gstore<VF, CP>(bp[0], off[0][u], sum - z[u]);     // see whole_tail
                    else if (tl[u])
                        gstore_tail<VF, CP>(bp[0], off[0][u], sum - z[u], P.tskip);
                    else
                        gstore<VF, CP>(bp[0], off[0][u], sum - z[u]);
                }
        } else if constexpr (OP == CO_MUL) {
            VF a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) {
                    a[u] = gload<VF, CP>(bp[1], off[1][u]);
                    b[u] = gload<VF, CP>(bp[2], off[2][u]);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) {
                    // x may be y or z (in place)
                    if (tl[u] && (threadIdx.x & 63u) != 0)
                        gstore<VF, CP>(bp[0], off[0][u], a[u] * b[u]);    // see whole_tail
                    else if (tl[u])
                        gstore_tail<VF, CP>(bp[0], off[0][u], a[u] * b[u], P.tskip);
                    else
                        gstore<VF, CP>(bp[0], off[0][u], a[u] * b[u]);
                }
        } else if constexpr (OP == CO_MUL_ADJ) {
            // operands: 0 ga, 1 gb, 2 gout, 3 a, 4 b
            VF g[U], a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                g[u] = (VF)0.0f;
                a[u] = (VF)0.0f;
                b[u] = (VF)0.0f;
                const bool inI = valid[u] && (pm[u] & 4u);
                if (inI) {
                    g[u] = gload<VF, CP>(bp[2], off[2][u]);
                    if (pm[u] & 2u)
                        a[u] = gload<VF, CP>(bp[3], off[3][u]);
                    if (pm[u] & 1u)
                        b[u] = gload<VF, CP>(bp[4], off[4][u]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!valid[u])
                    continue;
                const bool inI = (pm[u] & 4u) != 0;
                if (pm[u] & 1u)
                    gstore<VF, CP>(bp[0], off[0][u], inI ? g[u] * b[u] : (VF)0.0f);
                if (pm[u] & 2u)
                    gstore<VF, CP>(bp[1], off[1][u], inI ? g[u] * a[u] : (VF)0.0f);
            }
        } else if constexpr (OP == CO_INDEX) {
            // Element offsets (base included) of every operand, row-major
            // counter index f = box * BE + e.
            int64_t *out = (int64_t *)(uintptr_t)P.ptr[0];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!valid[u])
                    continue;
                uint64_t f = fbase + ev[u];
#pragma unroll
                for (int k = 0; k < N; ++k)
                    if (k < (int)n)
                        out[(uint64_t)k * P.npoints + f] = bb[k] + (int64_t)(off[k][u] >> 2);  // esz == 4
            }
        }
        (void)jj;
    }
}

template <int OP, int V, int U, bool ROWS1, bool UNIT, int CP, bool RAG>
__global__ __launch_bounds__(NT) void coiter_kernel(const CoPlan P)
{
    const RowTable T{lds_rows, P.RB};
    if (!ROWS1) {
        fill_table<OpInfo<OP>::PRED>(P, T);
        __syncthreads();
    }
    const uint32_t lb = logical_block();
    const uint32_t g = gridDim.x;
    if (P.interleave) {
        // round-robin: at any moment the grid sweeps one window of memory
        for (uint64_t u = lb; u < P.nunits; u += g)
            run_unit<OP, V, U, ROWS1, UNIT, CP, RAG>(P, (uint32_t)u, T);
    } else {
        const uint32_t u0 = (uint32_t)(((uint64_t)lb * P.nunits) / g);
        const uint32_t u1 = (uint32_t)(((uint64_t)(lb + 1) * P.nunits) / g);
        for (uint32_t u = u0; u < u1; ++u)
            run_unit<OP, V, U, ROWS1, UNIT, CP, RAG>(P, u, T);
    }
}

// ---------------------------------------------------------------------
// Batched persistent kernel: one launch over a device table of item plans.
// Work units of all items are numbered consecutively (ustart holds each
// item's first unit).  Every workgroup walks either a contiguous range of
// units (rr == 0) or every g-th unit from its own (rr == 1: at any moment
// the grid sweeps one window of memory), and re-tabulates its box rows
// whenever it enters a new item.  Each item runs with its own lane width:
// 4 words (unit-stride rows, ragged or not) or 1.
// ---------------------------------------------------------------------
template <int OP, int U, int CP>
__global__ __launch_bounds__(NT) void batched_kernel(const CoPlan *__restrict__ plans,
                                                     const uint32_t *__restrict__ ustart,
                                                     const uint32_t *__restrict__ uitem,
                                                     uint32_t nitems, uint32_t total, uint32_t rr)
{
    const uint32_t lb = logical_block();
    const uint32_t g = gridDim.x;
    uint32_t u, uend, step;
    if (rr) {
        u = lb;
        uend = total;
        step = g;
    } else {
        u = (uint32_t)(((uint64_t)lb * total) / g);
        uend = (uint32_t)(((uint64_t)(lb + 1) * total) / g);
        step = 1;
    }
    // The current item's plan lives in LDS (one coalesced copy per item), so
    // the per-unit decode never waits on global memory.
    __shared__ CoPlan Ps;
    uint32_t item = 0, first = 0, next = 0;    // next == 0: nothing loaded yet
    for (; u < uend; u += step) {
        if (u >= next) {
            // the item holding u: one load from the unit table, else the
            // last item whose first unit is <= u (binary search; empty items
            // share their first unit with the next item)
            if (uitem) {
                item = uitem[u];
            } else {
                uint32_t lo = item, hi = nitems;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (ustart[mid] <= u)
                        lo = mid;
                    else
                        hi = mid;
                }
                item = lo;
            }
            first = ustart[item];
            next = ustart[item + 1];
            __syncthreads();
            const uint32_t *src = (const uint32_t *)(plans + item);
            uint32_t *dst = (uint32_t *)&Ps;
            for (uint32_t i = threadIdx.x; i < sizeof(CoPlan) / 4; i += NT)
                dst[i] = src[i];
            __syncthreads();
            if (Ps.RB > 1)
                fill_table<OpInfo<OP>::PRED>(Ps, RowTable{lds_rows, Ps.RB});
            __syncthreads();
        }
        const CoPlan &P = Ps;
        const RowTable T{lds_rows, P.RB};
        const bool rows1 = P.RB == 1;
        const uint32_t lu = u - first;
        if (P.vec == 4) {
            // 4-word lanes: unit-stride rows, possibly ragged
            if (P.tskip) {
                if (rows1)
                    run_unit<OP, 4, U, true, true, CP, true, true>(P, lu, T);
                else
                    run_unit<OP, 4, U, false, true, CP, true, true>(P, lu, T);
            } else {
                if (rows1)
                    run_unit<OP, 4, U, true, true, CP, false, true>(P, lu, T);
                else
                    run_unit<OP, 4, U, false, true, CP, false, true>(P, lu, T);
            }
        } else if (rows1) {
            if (P.unit)
                run_unit<OP, 1, U, true, true, CP, false, true>(P, lu, T);
            else
                run_unit<OP, 1, U, true, false, CP, false, true>(P, lu, T);
        } else {
            if (P.unit)
                run_unit<OP, 1, U, false, true, CP, false, true>(P, lu, T);
            else
                run_unit<OP, 1, U, false, false, CP, false, true>(P, lu, T);
        }
    }
}

// ---------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------

// Workgroups of `kern` that fit on one CU at once with `lds` bytes of
// dynamic LDS (0 if the runtime cannot tell).  `cache` is the calling
// kernel's own memo, by LDS size in KiB (the query asks for the rounded-up
// size).
static int resident_per_cu(const void *kern, size_t lds, int (&cache)[64])
{
    const size_t kib = (lds + 1023) / 1024;
    if (kib < 64 && cache[kib] > 0)
        return cache[kib];
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, kib * 1024) != hipSuccess)
        return 0;
    if (kib < 64 && nb > 0)
        cache[kib] = nb;
    return nb;
}

// A persistent grid (each workgroup owns a fixed share of the work) larger
// than what fits at once would run its last workgroups after the others:
// keep it within the resident capacity (a multiple of 8 for whole XCDs).
static int clamp_resident(int blocks, int per_cu, int cus)
{
    if (per_cu <= 0 || cus <= 0)
        return blocks;
    const int cap = per_cu * cus;
    return blocks > cap ? cap : blocks;
}

template <int OP, int V, int U, bool ROWS1, bool UNIT, int CP, bool RAG = false>
static hipError_t go(const CoLaunch &L, hipStream_t st)
{
    static int occ[64];
    const auto kern = coiter_kernel<OP, V, U, ROWS1, UNIT, CP, RAG>;
    const size_t lds =
        ROWS1 ? 0 : (size_t)L.plan.RB * (L.plan.n + (OpInfo<OP>::PRED ? 1 : 0)) * 4u;
    const int blocks =
        clamp_resident(L.blocks, resident_per_cu(reinterpret_cast<const void *>(kern), lds, occ),
                       L.cus);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, L.plan);
    return hipGetLastError();
}

template <int OP, int V, int U, int CP>
static hipError_t pick_rows(const CoLaunch &L, hipStream_t st)
{
    if (L.plan.tskip) {
        // ragged rows: planned only for vectors of unit-stride rows, for
        // ops without window predicates and EMBED_FILL
        if constexpr (V > 1 && (!OpInfo<OP>::PRED || OP == CO_FILL) && OP != CO_INDEX) {
            if (!L.unit)
                return hipErrorInvalidValue;
            return L.rows1 ? go<OP, V, U, true, true, CP, true>(L, st)
                           : go<OP, V, U, false, true, CP, true>(L, st);
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (L.rows1)
        return L.unit ? go<OP, V, U, true, true, CP>(L, st) : go<OP, V, U, true, false, CP>(L, st);
    return L.unit ? go<OP, V, U, false, true, CP>(L, st) : go<OP, V, U, false, false, CP>(L, st);
}

template <int OP, int CP>
static hipError_t pick_vec(const CoLaunch &L, hipStream_t st)
{
    constexpr int U = 4;
    if constexpr (OP == CO_INDEX) {
        return pick_rows<OP, 1, U, CP>(L, st);
    } else {
        switch (L.plan.vec) {
        case 4: return pick_rows<OP, 4, U, CP>(L, st);
        case 2: return pick_rows<OP, 2, U, CP>(L, st);
        default: return pick_rows<OP, 1, U, CP>(L, st);
        }
    }
}

template <int OP>
static hipError_t pick_cache(const CoLaunch &L, hipStream_t st)
{
    switch (L.cache) {
    case CP_NONTEMP_LS: return pick_vec<OP, CP_NONTEMP_LS>(L, st);
    case CP_NONTEMP_L: return pick_vec<OP, CP_NONTEMP_L>(L, st);
    default: return pick_vec<OP, CP_NORMAL>(L, st);
    }
}

hipError_t launch_coiter(int co_op, const CoLaunch &L, hipStream_t st)
{
    switch (co_op) {
    case CO_COPY: return pick_cache<CO_COPY>(L, st);
    case CO_FILL: return pick_cache<CO_FILL>(L, st);
    case CO_MUL_ACC: return pick_cache<CO_MUL_ACC>(L, st);
    case CO_MUL: return pick_cache<CO_MUL>(L, st);
    case CO_MUL_ADJ: return pick_cache<CO_MUL_ADJ>(L, st);
    case CO_XPYX_MZ: return pick_cache<CO_XPYX_MZ>(L, st);
    case CO_INDEX: return pick_vec<CO_INDEX, CP_NORMAL>(L, st);
    default: return hipErrorInvalidValue;
    }
}

template <int OP, int CP>
static void go_batched(BatchLaunch &B, hipStream_t st)
{
    static int occ[64];
    const auto kern = batched_kernel<OP, 4, CP>;
    const size_t lds = (size_t)B.rows_max * (OpInfo<OP>::N + (OpInfo<OP>::PRED ? 1 : 0)) * 4u;
    B.launched = clamp_resident(
        B.blocks, resident_per_cu(reinterpret_cast<const void *>(kern), lds, occ), B.cus);
    hipLaunchKernelGGL(kern, dim3(B.launched), dim3(NT), lds, st, B.plans, B.ustart, B.uitem,
                       B.nitems, B.total, B.rr);
}

template <int OP>
static void pick_batched(BatchLaunch &B, hipStream_t st)
{
    switch (B.cache) {
    case CP_NONTEMP_LS: go_batched<OP, CP_NONTEMP_LS>(B, st); break;
    case CP_NONTEMP_L: go_batched<OP, CP_NONTEMP_L>(B, st); break;
    default: go_batched<OP, CP_NORMAL>(B, st); break;
    }
}

hipError_t launch_batched(int co_op, BatchLaunch &B, hipStream_t st)
{
    switch (co_op) {
    case CO_COPY: pick_batched<CO_COPY>(B, st); break;
    case CO_FILL: pick_batched<CO_FILL>(B, st); break;
    case CO_MUL_ACC: pick_batched<CO_MUL_ACC>(B, st); break;
    case CO_MUL: pick_batched<CO_MUL>(B, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace triot
