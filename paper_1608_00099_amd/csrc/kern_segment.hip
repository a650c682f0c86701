// Tuple-reading row kernels for gfx950: index-weighted moments (Algorithm 11
// of the paper, read as E[t_i] of a PMF, plus the covariance of t) and their
// adjoint (the index-weighted scatter of the gradient), the inner product
// (benchmark 2 of Section 3) and the nonzero bounding box (Section 2).
//
// One thread per row segment (at most SEG_MAX consecutive elements of one
// counter row).  Inside a segment only the inner coordinate j varies, so the
// per-element work is three float64 sums, taken as running sums that never
// form j (three additions per element), and the outer coordinates enter
// once per segment ("row factoring").  The coordinates are shifted by the
// centre (c_i - 1)/2 of every axis, which keeps the covariance free of
// cancellation (the shifted-data variance algorithm of Chan, Golub &
// LeVeque).  A thread loads its own segment: consecutive threads hold
// consecutive segments, so a wave's loads cover one contiguous range.
//
// Partial sums are float64 per thread (on CDNA the float64 FMA issues at the
// same rate as an unpacked float32 FMA), reduced across the wave by DPP,
// across the workgroup through LDS, and across workgroups by a second
// kernel (one wave per result) that adds the per-workgroup partials in a
// fixed order.  No float atomics: the result is deterministic.  Ordering
// that combine behind the first kernel by the stream, rather than by a
// device-scope fence in every workgroup (which on CDNA writes back the whole
// L2 of the XCD), costs one short launch.
//
// Accumulator positions: p = 0 is the inner axis (D-1), p >= 1 the outer
// axis D-1-p, so that register arrays are indexed by compile-time positions.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"

namespace triot {

__device__ __forceinline__ uint32_t sdiv_u32(uint32_t n, const AxisDiv &a)
{
    uint32_t h = __umulhi(n, a.m);
    return (h + ((n - h) >> 1)) >> a.s;
}

__device__ __forceinline__ uint32_t seg_logical_block()
{
    uint32_t g = gridDim.x, b = blockIdx.x;
    if ((g & 7u) == 0)
        return (b & 7u) * (g >> 3) + (b >> 3);
    return b;
}

// The 32-axis instances of the row kernels read their plan in place, from
// the kernel-argument segment (explicit arguments start at its offset 0):
// a by-value aggregate parameter indexed at run time (the axis tables) is
// otherwise copied to per-lane scratch memory first, which the compiler
// does for those larger instances.
#define SEG_PLAN_FOR(DM) \
    const SegPlan &P = (DM) > 8 ? *(const SegPlan *)__builtin_amdgcn_kernarg_segment_ptr() : plan

#define GLOBAL __attribute__((address_space(1)))
#define SHARED __attribute__((address_space(3)))

// LDS staging: one padding word every 32 words keeps the per-thread segment
// reads (stride L words across lanes) spread over the banks.
constexpr int STAGE_WORDS = NT * SEG_MAX + (NT * SEG_MAX) / 32 + 32;
__device__ __forceinline__ uint32_t sidx(uint32_t e) { return e + (e >> 5); }

template <int DMAX, bool COV> struct Terms {
    static constexpr int K = 1;                       // first moment sums start here
    static constexpr int C = 1 + DMAX;                // second moment sums start here
    static constexpr int T = 1 + DMAX + (COV ? DMAX * (DMAX + 1) / 2 : 0);
    __host__ __device__ static constexpr int c(int p, int q)   // p <= q
    {
        return C + p * DMAX - p * (p - 1) / 2 + (q - p);
    }
};

// Segment s -> (row, first j, length) and its first element in row-major
// counter order.
struct Seg {
    uint32_t row, j0, len;
};

__device__ __forceinline__ Seg seg_of(const SegPlan &P, uint64_t s)
{
    Seg g;
    uint32_t s32 = (uint32_t)s;  // rows * G < 2^32 * G; G == 1 keeps s < 2^32
    if (P.gdiv.c == 1) {
        g.row = s32;
        g.j0 = 0;
    } else if (P.nseg <= 0xFFFFFFFFull) {
        // fewer than 2^32 segments (uniform): 32-bit magic division by G
        const uint32_t row = sdiv_u32(s32, P.gdiv);
        g.row = row;
        g.j0 = (s32 - row * P.G) * P.S;
    } else {
        // s < rows * G may exceed 32 bits only when G > 1; split it.
        uint64_t row = s / P.G;
        g.row = (uint32_t)row;
        g.j0 = (uint32_t)(s - row * P.G) * P.S;
    }
    g.len = min(P.S, P.L - g.j0);
    return g;
}

__device__ __forceinline__ uint64_t seg_start(const SegPlan &P, const Seg &g)
{
    return (uint64_t)g.row * P.L + g.j0;
}

// Outer coordinates of a row, shifted by the axis centres, at positions
// 1..D-1 (position p is axis D-1-p).
template <int DMAX>
__device__ __forceinline__ void row_coords(const SegPlan &P, uint32_t row, double u[DMAX],
                                           uint32_t t[DMAX])
{
    uint32_t q = row;
    const int D = (int)P.D;
#pragma unroll
    for (int p = 1; p < DMAX; ++p) {
        if (p < D) {
            const int i = D - 1 - p;
            uint32_t digit;
            if (i == 0) {
                digit = q;
            } else {
                const AxisDiv a = P.ax[i];
                uint32_t qq = sdiv_u32(q, a);
                digit = q - qq * a.c;
                q = qq;
            }
            t[p] = digit;
            u[p] = (double)digit - P.center[i];
        } else {
            t[p] = 0;
            u[p] = 0.0;
        }
    }
}

template <int DMAX>
__device__ __forceinline__ int64_t row_offset(const SegPlan &P, int k, const uint32_t t[DMAX])
{
    int64_t off = P.base[k];
    const int D = (int)P.D;
#pragma unroll
    for (int p = 1; p < DMAX; ++p)
        if (p < D)
            off += (int64_t)t[p] * P.stride[k][D - 1 - p];
    return off;
}

// Cross-lane sums by DPP (data-parallel primitives: an operand read from
// another lane of the same row of 16 inside the ALU instruction, no LDS
// traffic).  A float64 moves as its two 32-bit halves through the same lane
// pattern; lanes of rows outside ROWS receive +0.0.
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xF, false);
    const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xF, false);
    return __hiloint2double(h2, l2);
}

enum : int {
    DPP_QUAD_XOR1 = 0xB1,      // quad_perm [1,0,3,2]
    DPP_QUAD_XOR2 = 0x4E,      // quad_perm [2,3,0,1]
    DPP_ROW_MIRROR = 0x140,    // lane i of a row of 16 reads lane 15 - i
    DPP_HALF_MIRROR = 0x141,   // lane i of a half row of 8 reads lane 7 - i
    DPP_ROW_BCAST15 = 0x142,   // lane 15 of each row to every lane of the next row
    DPP_ROW_BCAST31 = 0x143,   // lane 31 to every lane of rows 2 and 3
};

// Every lane of each row of 16 gets the sum of its row's 16 values.
__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_f64<DPP_QUAD_XOR1, 0xF>(v);
    v += dpp_f64<DPP_QUAD_XOR2, 0xF>(v);
    v += dpp_f64<DPP_HALF_MIRROR, 0xF>(v);
    v += dpp_f64<DPP_ROW_MIRROR, 0xF>(v);
    return v;
}

// Over the four lanes of a quad, lane q receives the sum of v[q] (a
// reduce-scatter in two exchanges: with the lane two apart, each lane keeps
// the pair of values whose index shares its bit 1 and hands over the other
// pair; with the neighbour, it keeps the value whose index is its own lane
// number).  Fixed order: deterministic.
__device__ __forceinline__ double quad_scatter(const double v[4])
{
    const uint32_t q = threadIdx.x & 3u;
    const bool b1 = (q & 2u) != 0u, b0 = (q & 1u) != 0u;
    double k0 = b1 ? v[2] : v[0], k1 = b1 ? v[3] : v[1];
    const double h0 = b1 ? v[0] : v[2], h1 = b1 ? v[1] : v[3];
    k0 += dpp_f64<DPP_QUAD_XOR2, 0xF>(h0);
    k1 += dpp_f64<DPP_QUAD_XOR2, 0xF>(h1);
    const double k = b0 ? k1 : k0, h = b0 ? k0 : k1;
    return k + dpp_f64<DPP_QUAD_XOR1, 0xF>(h);
}

// quad_scatter's exchange pattern for 32-bit masks combined by OR: lane q
// receives the OR of v[q] over its quad.
__device__ __forceinline__ uint32_t quad_scatter_or(const uint32_t v[4])
{
    const uint32_t q = threadIdx.x & 3u;
    const bool b1 = (q & 2u) != 0u, b0 = (q & 1u) != 0u;
    uint32_t k0 = b1 ? v[2] : v[0], k1 = b1 ? v[3] : v[1];
    const uint32_t h0 = b1 ? v[0] : v[2], h1 = b1 ? v[1] : v[3];
    k0 |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h0, DPP_QUAD_XOR2, 0xF, 0xF, false);
    k1 |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h1, DPP_QUAD_XOR2, 0xF, 0xF, false);
    const uint32_t k = b0 ? k1 : k0, h = b0 ? k0 : k1;
    return k | (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h, DPP_QUAD_XOR1, 0xF, 0xF, false);
}

// Sum over the 32 lanes of each half wave; the sum is valid in the half
// wave's LAST lane (31 or 63).  Fixed order: deterministic.
__device__ __forceinline__ double half_wave_sum(double v)
{
    v = row16_sum(v);
    return v + dpp_f64<DPP_ROW_BCAST15, 0xA>(v);    // rows 1 and 3 add rows 0 and 2
}

// Sum over the 64 lanes of a wave, valid in lane 63.
__device__ __forceinline__ double wave_sum(double v)
{
    v = half_wave_sum(v);
    return v + dpp_f64<DPP_ROW_BCAST31, 0xC>(v);    // rows 2 and 3 add lane 31
}

// Minimum (MAX: maximum) over the 64 lanes of a wave by DPP, in the lane
// pattern of wave_sum, valid in lane 63.  Lanes of rows that a step leaves
// out receive the identity (all ones for the minimum, 0 for the maximum).
template <bool MAX> __device__ __forceinline__ uint32_t wave_minmax(uint32_t v)
{
    constexpr int ID = MAX ? 0 : -1;
    auto f = [](uint32_t a, int b) { return MAX ? max(a, (uint32_t)b) : min(a, (uint32_t)b); };
    v = f(v, __builtin_amdgcn_update_dpp(ID, (int)v, DPP_QUAD_XOR1, 0xF, 0xF, false));
    v = f(v, __builtin_amdgcn_update_dpp(ID, (int)v, DPP_QUAD_XOR2, 0xF, 0xF, false));
    v = f(v, __builtin_amdgcn_update_dpp(ID, (int)v, DPP_HALF_MIRROR, 0xF, 0xF, false));
    v = f(v, __builtin_amdgcn_update_dpp(ID, (int)v, DPP_ROW_MIRROR, 0xF, 0xF, false));
    v = f(v, __builtin_amdgcn_update_dpp(ID, (int)v, DPP_ROW_BCAST15, 0xA, 0xF, false));
    return f(v, __builtin_amdgcn_update_dpp(ID, (int)v, DPP_ROW_BCAST31, 0xC, 0xF, false));
}

// Workgroup sum of the per-thread terms acc[0..T) into dst[0..T), in a
// fixed order.  Eight terms at a time pass through LDS transposed: thread t
// stores its eight values at x[q][t]; then the 32 threads of half wave q sum
// term q, each over eight stored values, and the half wave folds its 32
// sums by DPP.  A butterfly over all 64 lanes per term instead would
// cost each wave 12 cross-lane reads per term, and those all queue on the
// CU's one LDS unit.
template <int T>
__device__ __forceinline__ void block_sums(const double *acc, double (*x)[NT], double *dst)
{
    static_assert(NT == 256, "eight half waves per workgroup");
    const int tid = threadIdx.x;
    const int q = tid >> 5, part = tid & 31;
#pragma unroll
    for (int i0 = 0; i0 < T; i0 += 8) {
        __syncthreads();   // the previous chunk's reads are done
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i0 + k < T)
                x[k][tid] = acc[i0 + k];
        __syncthreads();
        double v = 0.0;
        if (i0 + q < T) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                v += x[q][k * 32 + part];
        }
        v = half_wave_sum(v);
        if (part == 31 && i0 + q < T)
            dst[i0 + q] = v;
    }
    __syncthreads();
}

// Sums of one segment of len <= SEG_MAX consecutive elements: with the
// running sums A += w_j, B += A, C += B taken for j = 0 .. len-1,
//   A = sum w,   B = sum w (r + 1),   C = sum w (r + 1)(r + 2) / 2,
// where r = len - 1 - j counts from the segment's end, so that
//   sum w r = B - A  and  sum w r^2 = 2C - 3B + A,
// and, with e = len - 1, the sums over the local coordinate j = e - r are
//   sum w j = e A - sum w r,   sum w j^2 = e^2 A - 2 e sum w r + sum w r^2.
// No coordinate is ever formed per element (three float64 additions each).
// The segment is loaded and folded in halves of HALF words (fewer live
// registers; a row of at most HALF words never touches the second half).
constexpr int HALF = SEG_MAX / 2;

typedef float f4v __attribute__((ext_vector_type(4), aligned(4)));

// Load through the global address space, non-temporal when NTL (streamed
// data: no reuse, and no allocation that would first have to evict lines
// another kernel left dirty).
template <bool NTL> __device__ __forceinline__ f4v ldg(const GLOBAL f4v *p)
{
    if constexpr (NTL)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NTL> __device__ __forceinline__ float ldg(const GLOBAL float *p)
{
    if constexpr (NTL)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Weights of a half segment: float words for one operand; with several
// operands (MULTI) their product, formed in float64 in operand order (the
// definition's w = prod_k v_k; a float32 product would round).
template <bool MULTI> struct HalfW {
    float w[HALF];
    __device__ __forceinline__ double at(int j) const { return (double)w[j]; }
    __device__ __forceinline__ double at_or_zero(int j, bool keep) const
    {
        return (double)(keep ? w[j] : 0.0f);
    }
};
template <> struct HalfW<true> {
    double w[HALF];
    __device__ __forceinline__ double at(int j) const { return w[j]; }
    __device__ __forceinline__ double at_or_zero(int j, bool keep) const
    {
        return keep ? w[j] : 0.0;
    }
};

// Loads words [h0, h0 + HALF) of a segment of every operand.  VEC: 16-byte
// loads (every operand contiguous along the row, len a multiple of 4);
// else one word per element and operand.  Loads are issued
// unconditionally (indices clamped into the segment) so that they are all
// in flight together; the elements past len are never summed.
template <bool VEC, bool NTL>
__device__ __forceinline__ void load_words(const SegPlan &P, int k, const int64_t off[4],
                                           uint32_t len, uint32_t h0, float v[HALF])
{
    if constexpr (VEC) {
        const uint32_t qmax = (len >> 2) - 1;   // last quad of the segment
        const GLOBAL f4v *pk =
            (const GLOBAL f4v *)((const GLOBAL float *)(uintptr_t)P.ptr[k] + off[k]);
#pragma unroll
        for (int q = 0; q < HALF / 4; ++q) {
            const f4v x = ldg<NTL>(pk + min((h0 >> 2) + (uint32_t)q, qmax));
            v[4 * q + 0] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
        const int D = (int)P.D;
        const GLOBAL float *pk = (const GLOBAL float *)(uintptr_t)P.ptr[k] + off[k];
        const int64_t ik = P.stride[k][D - 1];
#pragma unroll
        for (int j = 0; j < HALF; ++j)
            v[j] = ldg<NTL>(pk + (int64_t)min(h0 + (uint32_t)j, len - 1) * ik);
    }
}

template <bool VEC, bool NTL, bool MULTI>
__device__ __forceinline__ void seg_load_half(const SegPlan &P, const int64_t off[4], uint32_t len,
                                              uint32_t h0, HalfW<MULTI> &W)
{
    if constexpr (!MULTI) {
        load_words<VEC, NTL>(P, 0, off, len, h0, W.w);
    } else {
        // the first two operands' loads go out together
        float v[HALF], x[HALF];
        load_words<VEC, NTL>(P, 0, off, len, h0, v);
        load_words<VEC, NTL>(P, 1, off, len, h0, x);
#pragma unroll
        for (int j = 0; j < HALF; ++j)
            W.w[j] = (double)v[j] * (double)x[j];
#pragma unroll
        for (int k = 2; k < 4; ++k) {
            if (k < (int)P.n) {
                load_words<VEC, NTL>(P, k, off, len, h0, v);
#pragma unroll
                for (int j = 0; j < HALF; ++j)
                    W.w[j] *= (double)v[j];
            }
        }
    }
}

// Folds one segment whose first half w0 is already loaded.  The second
// half, when len > HALF, is loaded here before the first half is summed, so
// both halves' loads are in flight together.
// ORDER: 0 the mass only, 1 with the first sum, 2 with the second too.
template <bool VEC, bool NTL, bool MULTI, int ORDER>
__device__ __forceinline__ void seg_moments(const SegPlan &P, const int64_t off[4], uint32_t len,
                                            const HalfW<MULTI> &w0, double &s0, double &s1,
                                            double &s2)
{
    constexpr bool SECOND = ORDER >= 2;
    double A = 0.0, B = 0.0, C = 0.0;
    HalfW<MULTI> w1;
    if (len > (uint32_t)HALF)
        seg_load_half<VEC, NTL, MULTI>(P, off, len, HALF, w1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t h0 = (uint32_t)(h * HALF);
        if (h == 0 || len > h0) {
#pragma unroll
            for (int j = 0; j < HALF; ++j) {
                if (h0 + (uint32_t)j < len) {
                    A += (h == 0) ? w0.at(j) : w1.at(j);
                    if (ORDER >= 1)
                        B += A;
                    if (SECOND)
                        C += B;
                }
            }
        }
    }
    const double e = (double)len - 1.0;
    const double r1 = B - A;
    s0 = A;
    s1 = fma(e, A, -r1);
    if (SECOND) {
        const double r2 = fma(2.0, C, fma(-3.0, B, A));
        s2 = fma(e, fma(e, A, -2.0 * r1), r2);
    } else {
        s2 = 0.0;
    }
}

// The same three sums for the moments pass, formed directly: the
// multipliers j and j^2 are compile-time constants of the unrolled loop, so
// each element costs one float64 addition and two fused multiply-adds, in
// two independent partial sums per moment (no running-sum chain).
// Elements past len (the loads are clamped into the segment) enter as
// zero, a select on the loaded word; when every segment is HALF words long
// (S == HALF, G == 1: uniform over the launch) no select is needed.  Fewer
// registers than the running sums (the covariance instance of 6 axes: 126
// VGPRs against 138), which lets the staged pass run 3 workgroups per CU.
template <bool MULTI>
__device__ __forceinline__ void seg_sums_both(const SegPlan &P, uint32_t len, const HalfW<MULTI> &w0,
                                              const HalfW<MULTI> &w1, double &s0, double &s1,
                                              double &s2)
{
    double a[2] = {0.0, 0.0}, b[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
    // every segment S words long (uniform): a half wholly inside needs no select
    const bool whole = P.L % P.S == 0u;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t h0 = (uint32_t)(h * HALF);
        if (h == 0 || len > h0) {
            const HalfW<MULTI> &W = (h == 0) ? w0 : w1;
            const bool plain = whole && P.S >= h0 + (uint32_t)HALF;
#pragma unroll
            for (int j = 0; j < HALF; ++j) {
                const double w = plain ? W.at(j) : W.at_or_zero(j, h0 + (uint32_t)j < len);
                const int jj = h * HALF + j;
                a[j & 1] += w;
                b[j & 1] = fma((double)jj, w, b[j & 1]);
                c[j & 1] = fma((double)(jj * jj), w, c[j & 1]);
            }
        }
    }
    s0 = a[0] + a[1];
    s1 = b[0] + b[1];
    s2 = c[0] + c[1];
}

// WHOLE: every segment is exactly HALF words (S == HALF, G == 1), known at
// compile time: the instance carries no second-half path.
template <bool VEC, bool NTL, bool MULTI, bool WHOLE = false>
__device__ __forceinline__ void seg_sums_fma(const SegPlan &P, const int64_t off[4], uint32_t len,
                                             const HalfW<MULTI> &w0, double &s0, double &s1,
                                             double &s2)
{
    if (WHOLE || (P.S == (uint32_t)HALF && P.G == 1u)) {
        // every segment is exactly HALF words (uniform): no second half and
        // no select
        double a[2] = {0.0, 0.0}, b[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const double w = w0.at(j);
            a[j & 1] += w;
            b[j & 1] = fma((double)j, w, b[j & 1]);
            c[j & 1] = fma((double)(j * j), w, c[j & 1]);
        }
        s0 = a[0] + a[1];
        s1 = b[0] + b[1];
        s2 = c[0] + c[1];
        return;
    }
    if constexpr (!WHOLE) {
        HalfW<MULTI> w1;
        if (len > (uint32_t)HALF)
            seg_load_half<VEC, NTL, MULTI>(P, off, len, HALF, w1);
        seg_sums_both<MULTI>(P, len, w0, w1, s0, s1, s2);
    }
}

// Staged tile loads (plan flag `stage`: every operand contiguous over the
// counter, rows of L = 4, 8 or 16 words, so G == 1 and a wave's 64
// segments are one range of 64 L consecutive words).  Per-lane segment
// loads put 64 lanes on 64 different 64-byte pieces in every instruction:
// the L1 sends each piece to L2 as a request of its own, and on MI355X the
// address unit then stalls on the L1 for about half of the moments pass.
// Here lane i of load k takes word quad 64 k + i of the wave's range (each
// instruction covers 1 KiB of consecutive memory, whole lines), writes it
// to the wave's LDS rows, and reads its own segment back (the inner product,
// which needs only the total, adds the fetched quads directly).  LDS rows
// are padded to an odd number of quads (4, 12 or 20 words), which spreads
// the per-lane 16-byte reads of eight lanes over all banks.
typedef float f4l __attribute__((ext_vector_type(4)));   // 16-byte aligned (LDS)
constexpr int STG_ROW = 20;                              // LDS words per row at L = 16

__device__ __forceinline__ uint32_t stg_row(uint32_t S)
{
    return S == 4 ? 4u : (S == 8 ? 12u : (S == 16 ? 20u : 36u));
}
constexpr int STG_ROW32 = 36;                            // LDS words per row at S = 32

// Orders this wave's LDS accesses on both sides (no instruction: a wave's
// LDS operations complete in order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Segments of this wave in tile `tile` (0 past the end); uniform per wave.
__device__ __forceinline__ uint32_t stage_count(const SegPlan &P, uint64_t tile)
{
    const uint64_t s0 = tile * NT + (threadIdx.x & ~63u);
    if (tile >= P.ntiles || s0 >= P.nseg)
        return 0u;
    const uint64_t left = P.nseg - s0;
    return left < 64u ? (uint32_t)left : 64u;
}

__device__ __forceinline__ uint32_t stage_shift(uint32_t S)   // log2(quads per segment)
{
    return S == 4 ? 0u : (S == 8 ? 1u : (S == 16 ? 2u : 3u));
}

// The global loads of a staged tile of operand k: lane i takes quads
// i, 64 + i, .. of the wave's range into x (indices clamped into the
// range; the LDS pass drops the copies).
template <bool NTL, int QN = HALF / 4>
__device__ __forceinline__ void stage_fetch(const SegPlan &P, int k, uint64_t tile, float x[4 * QN])
{
    const uint32_t cnt = stage_count(P, tile);
    if (cnt == 0u)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t sh = stage_shift(P.S);
    const uint32_t nq = cnt << sh;
    const uint64_t s0 = tile * NT + (threadIdx.x & ~63u);
    const GLOBAL f4v *src =
        (const GLOBAL f4v *)((const GLOBAL float *)(uintptr_t)P.ptr[k] + P.base[k] +
                             (int64_t)(s0 * P.S));
#pragma unroll
    for (int i = 0; i < QN; ++i) {
        if ((uint32_t)i < (1u << sh)) {
            const f4v y = ldg<NTL>(src + min((uint32_t)i * 64u + lane, nq - 1u));
            x[4 * i + 0] = y.x;
            x[4 * i + 1] = y.y;
            x[4 * i + 2] = y.z;
            x[4 * i + 3] = y.w;
        }
    }
}

// Writes the fetched quads to the wave's LDS rows.  Every lane of the
// wave takes part.
template <int QN = HALF / 4>
__device__ __forceinline__ void stage_put(const SegPlan &P, uint64_t tile, const float x[4 * QN],
                                          SHARED float *lds)
{
    const uint32_t cnt = stage_count(P, tile);
    if (cnt == 0u)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t row = stg_row(P.S), sh = stage_shift(P.S);
    const uint32_t nq = cnt << sh;
    wave_lds_sync();   // this wave's reads of the previous tile are done
#pragma unroll
    for (int i = 0; i < QN; ++i) {
        const uint32_t q = (uint32_t)i * 64u + lane;
        if ((uint32_t)i < (1u << sh) && q < nq) {
            const uint32_t r = q >> sh, c = q & ((1u << sh) - 1u);
            *(SHARED f4l *)(lds + r * row + 4u * c) = f4l{x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]};
        }
    }
    wave_lds_sync();
}

// Reads quads Q0 .. Q0 + QN - 1 of this lane's segment back from the
// wave's LDS rows into v (lanes past the last segment read nothing).
template <int QN = HALF / 4, int Q0 = 0>
__device__ __forceinline__ void stage_get(const SegPlan &P, uint64_t tile, const SHARED float *lds,
                                          float v[4 * QN])
{
    const uint32_t cnt = stage_count(P, tile);
    const uint32_t lane = threadIdx.x & 63u;
    if (lane >= cnt)
        return;
    const uint32_t row = stg_row(P.S), sh = stage_shift(P.S);
#pragma unroll
    for (int i = 0; i < QN; ++i) {
        if ((uint32_t)(Q0 + i) < (1u << sh)) {
            const f4l y = *(const SHARED f4l *)(lds + lane * row + 4u * (uint32_t)(Q0 + i));
            v[4 * i + 0] = y.x;
            v[4 * i + 1] = y.y;
            v[4 * i + 2] = y.z;
            v[4 * i + 3] = y.w;
        }
    }
}

// Writes the fetched quads to the wave's LDS rows and reads this lane's
// segment back into v (stage_put and stage_get in one pass).  Every lane of
// the wave takes part.
template <int QN = HALF / 4>
__device__ __forceinline__ void stage_scatter(const SegPlan &P, uint64_t tile, const float x[4 * QN],
                                              SHARED float *lds, float v[4 * QN])
{
    const uint32_t cnt = stage_count(P, tile);
    if (cnt == 0u)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t row = stg_row(P.S), sh = stage_shift(P.S);
    const uint32_t nq = cnt << sh;
    wave_lds_sync();   // this wave's reads of the previous tile are done
#pragma unroll
    for (int i = 0; i < QN; ++i) {
        const uint32_t q = (uint32_t)i * 64u + lane;
        if ((uint32_t)i < (1u << sh) && q < nq) {
            const uint32_t r = q >> sh, c = q & ((1u << sh) - 1u);
            *(SHARED f4l *)(lds + r * row + 4u * c) = f4l{x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]};
        }
    }
    wave_lds_sync();
    if (lane < cnt) {
#pragma unroll
        for (int i = 0; i < QN; ++i) {
            if ((uint32_t)i < (1u << sh)) {
                const f4l y = *(const SHARED f4l *)(lds + lane * row + 4u * (uint32_t)i);
                v[4 * i + 0] = y.x;
                v[4 * i + 1] = y.y;
                v[4 * i + 2] = y.z;
                v[4 * i + 3] = y.w;
            }
        }
    }
}

template <bool NTL>
__device__ __forceinline__ void stage_words(const SegPlan &P, int k, uint64_t tile, SHARED float *lds,
                                            float v[HALF])
{
    float x[HALF];
    stage_fetch<NTL>(P, k, tile, x);
    stage_scatter(P, tile, x, lds, v);
}

// The weights of this lane's segment through stage_words: the float words
// of one operand, or the float64 product over several (operand order).
template <bool NTL, bool MULTI>
__device__ __forceinline__ void stage_half(const SegPlan &P, uint64_t tile, SHARED float *lds,
                                           HalfW<MULTI> &W)
{
    if constexpr (!MULTI) {
        stage_words<NTL>(P, 0, tile, lds, W.w);
    } else {
        float v[HALF];
        stage_words<NTL>(P, 0, tile, lds, v);
#pragma unroll
        for (int j = 0; j < HALF; ++j)
            W.w[j] = (double)v[j];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            if (k < (int)P.n) {
                stage_words<NTL>(P, k, tile, lds, v);
#pragma unroll
                for (int j = 0; j < HALF; ++j)
                    W.w[j] *= (double)v[j];
            }
        }
    }
}

// Segments of 32 words (S == 32, L a multiple of 32, every operand
// contiguous over the counter): both halves of this lane's segment through
// one staged pass (eight quads per lane; LDS rows of 36 words, an odd
// number of quads).
template <bool NTL, bool MULTI>
__device__ __forceinline__ void stage_seg32(const SegPlan &P, uint64_t tile, SHARED float *lds,
                                            HalfW<MULTI> &W0, HalfW<MULTI> &W1)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k == 0 || (MULTI && k < (int)P.n)) {
            float x[SEG_MAX], v[SEG_MAX];
            stage_fetch<NTL, SEG_MAX / 4>(P, k, tile, x);
            stage_scatter<SEG_MAX / 4>(P, tile, x, lds, v);
#pragma unroll
            for (int j = 0; j < HALF; ++j) {
                if constexpr (!MULTI) {
                    W0.w[j] = v[j];
                    W1.w[j] = v[HALF + j];
                } else if (k == 0) {
                    W0.w[j] = (double)v[j];
                    W1.w[j] = (double)v[HALF + j];
                } else {
                    W0.w[j] *= (double)v[j];
                    W1.w[j] *= (double)v[HALF + j];
                }
            }
        }
    }
}

// Element offsets of a segment's first element in every operand.
template <int DM>
__device__ __forceinline__ void seg_offsets(const SegPlan &P, const Seg &sg, int64_t off[4])
{
    if (P.full) {
        const int64_t f = (int64_t)sg.row * P.L + sg.j0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            off[k] = P.base[k] + f;
    } else {
        const int D = (int)P.D;
        double u[DM];
        uint32_t tt[DM];
        row_coords<DM>(P, sg.row, u, tt);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            off[k] = (k < (int)P.n) ? row_offset<DM>(P, k, tt) + (int64_t)sg.j0 * P.stride[k][D - 1]
                                    : 0;
    }
}

// Main pass: every workgroup folds tiles of NT consecutive segments, dealt
// round-robin (the grid sweeps memory in one window), into per-thread
// float64 accumulators [M, K_p, C_pq] over centred coordinates, then
// reduces them across the workgroup (wave shuffles, then LDS, fixed
// order) into one partial per term, written term-major to the workspace.
// DM: accumulator positions (the exact number of kept axes for the
// covariance tier; 8 or 32 for first moments only).
// Resident workgroups per CU the register allocation aims at: 2, the
// number the pass runs (room for both halves of a segment in flight beside
// the accumulators).
template <int DM, bool COV, bool MULTI> constexpr int moments_min_blocks()
{
    return 2;
}

// Folds one segment's sums (s0, s1, s2 along the inner axis) into the
// accumulators: the outer coordinates enter once per segment.
template <int DM, bool COV>
__device__ __forceinline__ void seg_fold(const SegPlan &P, const Seg &sg, double s0, double s1,
                                         double s2, double cin, double *acc)
{
    typedef Terms<DM, COV> TT;
    double u[DM];
    uint32_t tt[DM];
    row_coords<DM>(P, sg.row, u, tt);
    // inner axis: u_in = a + j with a = j0 - centre
    const double a = (double)sg.j0 - cin;
    const double A1 = fma(a, s0, s1);                       // sum w u_in
    acc[0] += s0;
    acc[TT::K + 0] += A1;
#pragma unroll
    for (int p = 1; p < DM; ++p)
        acc[TT::K + p] = fma(u[p], s0, acc[TT::K + p]);
    if constexpr (COV) {
        const double A2 = fma(a, fma(a, s0, 2.0 * s1), s2);  // sum w u_in^2
        acc[TT::c(0, 0)] += A2;
#pragma unroll
        for (int p = 1; p < DM; ++p)
            acc[TT::c(0, p)] = fma(u[p], A1, acc[TT::c(0, p)]);
#pragma unroll
        for (int q = 1; q < DM; ++q) {
            const double uq = u[q] * s0;
#pragma unroll
            for (int p = 1; p <= q; ++p)
                acc[TT::c(p, q)] = fma(u[p], uq, acc[TT::c(p, q)]);
        }
    }
}

// Row blocks (rows of LL = 2, 4 or 8 words laid end to end): a segment of
// 16 words holds 16 / LL whole rows, which differ only in the next axis
// (position 1; the plan makes its extent a multiple of 16 / LL).  With
// ja = j % LL and jb = j / LL the segment gives S0 = sum w, Sa = sum ja w,
// Saa = sum ja^2 w, Sb = sum jb w, Sbb = sum jb^2 w and Sab = sum ja jb w
// (compile-time multipliers; the second moments only with COV).
template <int LL, bool COV>
__device__ __forceinline__ void rowblock_sums(const float v[16], double S[6])
{
    double acc[6][2] = {};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int ja = j % LL, jb = j / LL;
        const double w = (double)v[j];
        acc[0][j & 1] += w;
        acc[1][j & 1] = fma((double)ja, w, acc[1][j & 1]);
        acc[3][j & 1] = fma((double)jb, w, acc[3][j & 1]);
        if constexpr (COV) {
            acc[2][j & 1] = fma((double)(ja * ja), w, acc[2][j & 1]);
            acc[4][j & 1] = fma((double)(jb * jb), w, acc[4][j & 1]);
            acc[5][j & 1] = fma((double)(ja * jb), w, acc[5][j & 1]);
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
        S[i] = acc[i][0] + acc[i][1];
}

// Folds a row block: positions 0 (inner) and 1 (the next axis, from the
// block's first row) from the block sums, the outer positions once.
template <int DM, bool COV>
__device__ __forceinline__ void rowblock_fold(const SegPlan &P, uint32_t row, const double S[6],
                                              double cin, double *acc)
{
    typedef Terms<DM, COV> TT;
    double u[DM];
    uint32_t tt[DM];
    row_coords<DM>(P, row, u, tt);
    const double a = -cin, b = u[1];
    const double A1 = fma(a, S[0], S[1]);   // sum w u_0
    const double B1 = fma(b, S[0], S[3]);   // sum w u_1
    acc[0] += S[0];
    acc[TT::K + 0] += A1;
    acc[TT::K + 1] += B1;
#pragma unroll
    for (int p = 2; p < DM; ++p)
        acc[TT::K + p] = fma(u[p], S[0], acc[TT::K + p]);
    if constexpr (COV) {
        acc[TT::c(0, 0)] += fma(a, fma(a, S[0], 2.0 * S[1]), S[2]);   // sum w u_0^2
        acc[TT::c(1, 1)] += fma(b, fma(b, S[0], 2.0 * S[3]), S[4]);   // sum w u_1^2
        acc[TT::c(0, 1)] += fma(a, B1, fma(b, S[1], S[5]));          // sum w u_0 u_1
#pragma unroll
        for (int p = 2; p < DM; ++p) {
            acc[TT::c(0, p)] = fma(u[p], A1, acc[TT::c(0, p)]);
            acc[TT::c(1, p)] = fma(u[p], B1, acc[TT::c(1, p)]);
        }
#pragma unroll
        for (int q = 2; q < DM; ++q) {
            const double uq = u[q] * S[0];
#pragma unroll
            for (int p = 2; p <= q; ++p)
                acc[TT::c(p, q)] = fma(u[p], uq, acc[TT::c(p, q)]);
        }
    }
}

// Short segments (rows of at most 8 words, one operand): a segment per lane
// is a single small load, so a loop of one tile at a time waits out a full
// memory round trip per handful of words.  Here every lane loads its
// segments of SHORT_TILES consecutive tiles first (half as many in the
// 32-axis tier; at most two 16-byte loads, or eight words, each), then
// folds them in tile order.
constexpr int SHORT_TILES = 8;
constexpr int SHORT_W = 8;

template <bool VEC, bool NTL>
__device__ __forceinline__ void short_load(const SegPlan &P, const int64_t off[4], uint32_t len,
                                           float v[SHORT_W])
{
    const GLOBAL float *p0 = (const GLOBAL float *)(uintptr_t)P.ptr[0] + off[0];
    if constexpr (VEC) {
        const uint32_t qmax = (len >> 2) - 1;
#pragma unroll
        for (int q = 0; q < SHORT_W / 4; ++q) {
            const f4v x = ldg<NTL>((const GLOBAL f4v *)p0 + min((uint32_t)q, qmax));
            v[4 * q + 0] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
        const int64_t ik = P.stride[0][P.D - 1];
#pragma unroll
        for (int j = 0; j < SHORT_W; ++j)
            v[j] = ldg<NTL>(p0 + (int64_t)min((uint32_t)j, len - 1) * ik);
    }
}

// Sums of a short segment over its local coordinate j: w, j w, j^2 w
// (words past len enter as zero).
__device__ __forceinline__ void short_sums(uint32_t len, const float v[SHORT_W], double &s0,
                                           double &s1, double &s2)
{
    double a[2] = {0.0, 0.0}, b[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < SHORT_W; ++j) {
        const double w = (double)((uint32_t)j < len ? v[j] : 0.0f);
        a[j & 1] += w;
        b[j & 1] = fma((double)j, w, b[j & 1]);
        c[j & 1] = fma((double)(j * j), w, c[j & 1]);
    }
    s0 = a[0] + a[1];
    s1 = b[0] + b[1];
    s2 = c[0] + c[1];
}

// STG: 0 per-lane segment loads; 1 staged tile loads of rows of 4, 8 or 16
// words; 2 staged loads of 32-word segments (both halves); 3 short segments
// (at most 8 words, one operand), SHORT_TILES tiles per pass; 4 row blocks
// (16-word segments of whole short rows, staged); 5 per-lane loads of
// segments of exactly 16 words (rows of 16 words); 6 rows of 16 words laid
// end to end, one operand, loaded as quads of 16 rows, row sums across lanes.
template <int DM, bool COV, bool VEC, bool MULTI, bool NTL = true, int STG = 0>
__global__ __launch_bounds__(NT, (moments_min_blocks<DM, COV, MULTI>())) void moments_kernel(const SegPlan plan)
{
    SEG_PLAN_FOR(DM);
    typedef Terms<DM, COV> TT;
    constexpr int T = TT::T;
    __shared__ double xch[8][NT];
    __shared__ double tot[T];
    __shared__ __align__(16) float
        stg[(STG == 1 || STG == 2 || STG == 4) ? NT / 64 : 1]
           [STG == 2 ? 64 * STG_ROW32 : ((STG == 1 || STG == 4) ? 64 * STG_ROW : 4)];

    double acc[T];
#pragma unroll
    for (int i = 0; i < T; ++i)
        acc[i] = 0.0;

    const int D = COV ? DM : (int)P.D;
    const double cin = P.center[D - 1];
    const uint32_t lb = seg_logical_block();
    const uint64_t g = gridDim.x;

    if constexpr (STG == 4) {
        SHARED float *lds = (SHARED float *)stg[threadIdx.x >> 6];
        for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
            const uint64_t s = tile * NT + threadIdx.x;
            float v[16];
            stage_words<NTL>(P, 0, tile, lds, v);
            if (s < P.nseg) {
                double S[6];
                if (P.L == 2)
                    rowblock_sums<2, COV>(v, S);
                else if (P.L == 4)
                    rowblock_sums<4, COV>(v, S);
                else
                    rowblock_sums<8, COV>(v, S);
                rowblock_fold<DM, COV>(P, (uint32_t)s * P.rb, S, cin, acc);
            }
        }
    } else if constexpr (STG == 6) {
        // Rows of 16 words laid end to end, one operand: the wave's 64 rows
        // of a tile are 4 KiB of consecutive memory.  Load k gives lane l
        // quad l & 3 of row 16 k + l / 4 (each instruction covers 1 KiB,
        // whole lines); the lane sums its four words for each k, and the
        // quad's reduce-scatter leaves lane l the sums of row 16 (l & 3) +
        // l / 4, which it folds.
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t q = lane & 3u;
        const GLOBAL f4v *src =
            (const GLOBAL f4v *)((const GLOBAL float *)(uintptr_t)P.ptr[0] + P.base[0]);
        const double jq = (double)(4u * q);      // the lane's first column
        for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
            const uint64_t r0 = tile * NT + (threadIdx.x & ~63u) + (lane >> 2);
            const uint64_t last = P.nseg - 1u;
            f4v x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)         // rows past the end: the last row (never folded)
                x[k] = ldg<NTL>(src + 4u * min(r0 + 16u * (uint32_t)k, last) + q);
            double a[4], b[4], c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double w0 = (double)x[k].x, w1 = (double)x[k].y;
                const double w2 = (double)x[k].z, w3 = (double)x[k].w;
                // column j = 4q + e: sums of w, e w, e^2 w, then shifted by 4q
                const double s0 = (w0 + w1) + (w2 + w3);
                const double s1 = fma(3.0, w3, fma(2.0, w2, w1));
                const double s2 = fma(9.0, w3, fma(4.0, w2, w1));
                a[k] = s0;
                b[k] = fma(jq, s0, s1);
                c[k] = fma(jq, fma(jq, s0, 2.0 * s1), s2);
            }
            const double s0 = quad_scatter(a), s1 = quad_scatter(b), s2 = quad_scatter(c);
            const uint64_t row = r0 + 16u * q;
            if (row < P.nseg)
                seg_fold<DM, COV>(P, Seg{(uint32_t)row, 0u, 16u}, s0, s1, s2, cin, acc);
        }
    } else if constexpr (STG == 3) {
        // block lb takes tiles lb*K .. lb*K + K-1, then (lb + g)*K .. (K
        // halved for the 32-axis tier: its accumulators leave fewer registers)
        constexpr int K = DM > 8 ? SHORT_TILES / 2 : SHORT_TILES;
        for (uint64_t t0 = (uint64_t)lb * K; t0 < P.ntiles; t0 += g * K) {
            float v[K][SHORT_W];
            Seg sg[K];
            bool ok[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t s = (t0 + (uint64_t)k) * NT + threadIdx.x;
                ok[k] = t0 + (uint64_t)k < P.ntiles && s < P.nseg;
                sg[k] = Seg{0, 0, 0};
                if (ok[k]) {
                    int64_t off[4];
                    sg[k] = seg_of(P, s);
                    seg_offsets<DM>(P, sg[k], off);
                    short_load<VEC, NTL>(P, off, sg[k].len, v[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (ok[k]) {
                    double s0, s1, s2;
                    short_sums(sg[k].len, v[k], s0, s1, s2);
                    seg_fold<DM, COV>(P, sg[k], s0, s1, s2, cin, acc);
                }
            }
        }
    } else {
    for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
        const uint64_t s = tile * NT + threadIdx.x;
        const bool valid = s < P.nseg;
        Seg sg{0, 0, 0};
        int64_t off[4];
        HalfW<MULTI> w0, w1;
        if constexpr (STG == 2) {
            stage_seg32<NTL, MULTI>(P, tile, (SHARED float *)stg[threadIdx.x >> 6], w0, w1);
            if (valid)
                sg = seg_of(P, s);
        } else if constexpr (STG == 1) {
            stage_half<NTL, MULTI>(P, tile, (SHARED float *)stg[threadIdx.x >> 6], w0);
            if (valid) {
                sg = seg_of(P, s);
                seg_offsets<DM>(P, sg, off);
            }
        } else if (valid) {
            sg = seg_of(P, s);
            seg_offsets<DM>(P, sg, off);
            seg_load_half<VEC, NTL, MULTI>(P, off, sg.len, 0, w0);
        }
        if (valid) {
            double s0, s1, s2;
            if constexpr (STG == 2)
                seg_sums_both<MULTI>(P, sg.len, w0, w1, s0, s1, s2);
            else
                seg_sums_fma<VEC, NTL, MULTI, STG == 5>(P, off, sg.len, w0, s0, s1, s2);
            seg_fold<DM, COV>(P, sg, s0, s1, s2, cin, acc);
        }
    }
    }

    // ---- workgroup reduction (fixed order) ----
    block_sums<T>(acc, xch, tot);
    // Partials are term-major (term i of block b at i * nblocks + b) so the
    // combining workgroup reads them with coalesced loads.
    double *partials = (double *)((char *)(uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    for (int i = threadIdx.x; i < T; i += NT)
        partials[(size_t)i * nb + blockIdx.x] = tot[i];
}

// Combines the per-workgroup partials of moments_kernel into the caller's
// layout [M, E, C]: one wavefront per output value, launched right after
// the main pass on the same stream (the kernel boundary makes every partial
// visible; no device-wide fence per workgroup).  Output o needs at most
// four terms (M; K_p for E_i; K_p, K_q and C_pq for C_ij): lane l adds the
// partials of blocks l, l + 64, .. of each, all loads of a pass in flight
// together, then the wave folds its 64 sums by DPP.  Fixed order
// throughout: deterministic.
constexpr int ONT = 64;
// Threads of the one-workgroup combines (inner product, bounding box).
constexpr int FNT = 1024;

template <int DM, bool COV>
__global__ __launch_bounds__(ONT) void moments_out_kernel(const SegPlan P)
{
    typedef Terms<DM, COV> TT;
    const int D = (int)P.D;
    const int d = (int)P.d_orig;
    const int o = blockIdx.x;
    const int lane = threadIdx.x;
    // position (accumulator index) of original axis i, -1 when dropped
    auto pos_of = [&](int i) -> int {
        for (int p = 0; p < D; ++p)
            if ((int)P.orig[D - 1 - p] == i)
                return p;
        return -1;
    };
    int term[4] = {0, 0, 0, 0};
    int nt = 1;                // terms this output reads (term[0] is M)
    int p = -1, q = -1;
    bool dropped = false;      // a dropped axis: the plain definition's 0/M
    if (o >= 1 && o <= d) {
        p = pos_of(o - 1);
        if (p < 0) {
            dropped = true;
        } else {
            term[1] = TT::K + p;
            nt = 2;
        }
    } else if (o > d) {
        // o -> (i, j), i <= j, in the row-major upper triangle
        int r = o - 1 - d, i = 0;
        while (r >= d - i) {
            r -= d - i;
            ++i;
        }
        const int j = i + r;
        p = pos_of(i);
        q = pos_of(j);
        if (p < 0 || q < 0 || !COV) {
            dropped = true;
        } else {
            term[1] = TT::K + p;
            term[2] = TT::K + q;
            term[3] = TT::c(p < q ? p : q, p < q ? q : p);
            nt = 4;
        }
    }
    const GLOBAL double *partials = (const GLOBAL double *)((uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    constexpr int BATCH = 8;             // loads in flight per term and thread
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b0 = 0; b0 < nb; b0 += ONT * BATCH) {
        double x[4][BATCH];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const GLOBAL double *row = partials + (size_t)term[k] * nb;
#pragma unroll
            for (int c = 0; c < BATCH; ++c) {
                const uint32_t b = b0 + (uint32_t)(c * ONT + lane);
                x[k][c] = (k < nt) ? row[b < nb ? b : 0u] : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < BATCH; ++c)
                s[k] += (b0 + (uint32_t)(c * ONT + lane) < nb) ? x[k][c] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        s[k] = wave_sum(s[k]);
    if (lane != ONT - 1)
        return;
    const double M = s[0];
    double v;
    if (o == 0) {
        v = M;
    } else if (dropped) {
        v = 0.0 / M;
    } else if (o <= d) {
        v = P.center[D - 1 - p] + s[1] / M;
    } else {
        const double ei = s[1] / M, ej = s[2] / M;
        v = s[3] / M - ei * ej;
    }
    ((float *)(uintptr_t)P.out32)[o] = (float)v;
    if (P.out64)
        ((double *)(uintptr_t)P.out64)[o] = v;
}

// ---------------------------------------------------------------------
// Adjoint: g[t] = gM + (1/M) [ sum_i gE_i (t_i - E_i)
//                              + sum_{i<=j} gC_ij ((t_i - E_i)(t_j - E_j) - C_ij) ]
// Along a segment only the inner coordinate moves, so with v = j - E_in
//     g = A + v (B + Gam v)
// where A and B depend on the row's outer coordinates only.
// ---------------------------------------------------------------------
template <int DMAX, bool COV>
__global__ __launch_bounds__(NT) void moments_adj_kernel(const SegPlan P)
{
    __shared__ float stage[STAGE_WORDS];
    // Effective coefficients over the kept axes at compile-time positions
    // (extent-1 axes have t = 0 and fold into constants).
    __shared__ double sE[DMAX], sgE[DMAX], sgC[DMAX][DMAX];
    __shared__ double sconst, sMinv, sgM;

    const int D = (int)P.D;
    const int d = (int)P.d_orig;
    const bool cov = COV && (P.flags & TRIOT_MOMENTS_COV);
    const double *mom = (const double *)(uintptr_t)P.out64;
    const float *gmom = (const float *)(uintptr_t)P.gmom;
    if (threadIdx.x == 0) {
        // original axis -> position (or -1 for an extent-1 axis)
        int pos[MAXD];
        for (int i = 0; i < MAXD; ++i)
            pos[i] = -1;
        for (int p = 0; p < D; ++p) {
            uint32_t o = P.orig[D - 1 - p];
            if (o != 0xFFFFFFFFu)
                pos[o] = p;
        }
        for (int p = 0; p < DMAX; ++p) {
            sE[p] = 0.0;
            sgE[p] = 0.0;
            for (int q = 0; q < DMAX; ++q)
                sgC[p][q] = 0.0;
        }
        double c0 = 0.0;
        for (int i = 0; i < d; ++i) {
            const double Ei = mom[1 + i];
            const double gEi = (double)gmom[1 + i];
            if (pos[i] >= 0) {
                sE[pos[i]] = Ei;
                sgE[pos[i]] += gEi;
            } else {
                c0 += gEi * (0.0 - Ei);
            }
        }
        if (cov) {
            int idx = 1 + d;
            for (int i = 0; i < d; ++i)
                for (int j = i; j < d; ++j, ++idx) {
                    const double gc = (double)gmom[idx];
                    const double Cij = mom[idx];
                    c0 -= gc * Cij;
                    const int pi = pos[i], pj = pos[j];
                    const double ki = 0.0 - mom[1 + i], kj = 0.0 - mom[1 + j];
                    if (pi >= 0 && pj >= 0) {
                        const int lo = pi < pj ? pi : pj, hi = pi < pj ? pj : pi;
                        sgC[lo][hi] += gc;
                    } else if (pi >= 0) {
                        sgE[pi] += gc * kj;        // (t_i - E_i) * kappa_j
                    } else if (pj >= 0) {
                        sgE[pj] += gc * ki;
                    } else {
                        c0 += gc * ki * kj;
                    }
                }
        }
        sconst = c0;
        sMinv = 1.0 / mom[0];
        sgM = (double)gmom[0];
    }
    __syncthreads();

    const uint32_t lb = seg_logical_block();
    const uint64_t g = gridDim.x;
    const uint64_t t0 = (lb * P.ntiles) / g;
    const uint64_t t1 = ((lb + 1) * P.ntiles) / g;
    float *gout = (float *)(uintptr_t)P.ptr[0];
    const double Minv = sMinv, gM = sgM;

    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint64_t s0 = tile * NT;
        const uint32_t nsg = (uint32_t)min((uint64_t)NT, P.nseg - s0);
        const Seg first = seg_of(P, s0);
        const Seg last = seg_of(P, s0 + nsg - 1);
        const uint64_t f0 = seg_start(P, first);
        const uint32_t nel = (uint32_t)(seg_start(P, last) + last.len - f0);
        if (threadIdx.x < nsg) {
            const Seg sg = seg_of(P, s0 + threadIdx.x);
            double u[DMAX];
            uint32_t tt[DMAX];
            row_coords<DMAX>(P, sg.row, u, tt);
            // delta_p = t - E over the outer positions
            double dl[DMAX];
#pragma unroll
            for (int p = 1; p < DMAX; ++p)
                dl[p] = (p < D) ? (double)tt[p] - sE[p] : 0.0;
            double A = sconst, B = sgE[0];
#pragma unroll
            for (int p = 1; p < DMAX; ++p)
                A = fma(sgE[p], dl[p], A);
            if (cov) {
#pragma unroll
                for (int p = 1; p < DMAX; ++p) {
                    B = fma(sgC[0][p], dl[p], B);
                    double s = 0.0;
#pragma unroll
                    for (int q = p; q < DMAX; ++q)
                        s = fma(sgC[p][q], dl[q], s);
                    A = fma(dl[p], s, A);
                }
            }
            A = fma(A, Minv, gM);
            B *= Minv;
            const double Gm = cov ? sgC[0][0] * Minv : 0.0;
            const double v0 = (double)sg.j0 - sE[0];
            if (P.full) {
                const uint32_t loc = (uint32_t)(seg_start(P, sg) - f0);
                for (uint32_t jl = 0; jl < sg.len; ++jl) {
                    const double v = v0 + (double)jl;
                    stage[sidx(loc + jl)] = (float)fma(v, fma(Gm, v, B), A);
                }
            } else {
                const int64_t ro = row_offset<DMAX>(P, 0, tt);
                for (uint32_t jl = 0; jl < sg.len; ++jl) {
                    const double v = v0 + (double)jl;
                    gout[ro + (int64_t)(sg.j0 + jl) * P.stride[0][D - 1]] =
                        (float)fma(v, fma(Gm, v, B), A);
                }
            }
        }
        if (P.full) {
            __syncthreads();
            GLOBAL float *dst = (GLOBAL float *)(uintptr_t)P.ptr[0] + P.base[0] + (int64_t)f0;
            for (uint32_t e = threadIdx.x; e < nel; e += NT)
                dst[e] = stage[sidx(e)];
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------
// Inner product (benchmark 2 of Section 3): the mass of the weights alone,
// through the same segments, loads and fixed-order reductions.
// ---------------------------------------------------------------------
template <int DM, bool VEC, bool MULTI, bool NTL = true>
__global__ __launch_bounds__(NT, 4) void dot_kernel(const SegPlan plan)
{
    SEG_PLAN_FOR(DM);
    __shared__ double xch[8][NT];
    __shared__ double tot[1];
    double acc[1] = {0.0};
    const uint32_t lb = seg_logical_block();
    const uint64_t g = gridDim.x;
    if (VEC && P.quads) {
        // One word quad per lane: tile t holds quads t * NT * DOT_QUADS + u * NT
        // + i (u < DOT_QUADS), so each load instruction of the workgroup
        // covers NT consecutive quads (whole rows of the counter).
        const int D = (int)P.D;
        const uint32_t qpr = P.qdiv.c;
        for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
            const uint32_t q0 = (uint32_t)(tile * NT * DOT_QUADS) + threadIdx.x;
            f4v x[DOT_QUADS][4];
            bool ok[DOT_QUADS];
#pragma unroll
            for (int u = 0; u < DOT_QUADS; ++u) {
                const uint32_t q = q0 + (uint32_t)(u * NT);
                ok[u] = q < P.nquads;
                const uint32_t qq = ok[u] ? q : 0u;
                const uint32_t row = qpr == 1u ? qq : sdiv_u32(qq, P.qdiv);
                const uint32_t col = qq - row * qpr;
                double uu[DM];
                uint32_t tt[DM];
                row_coords<DM>(P, row, uu, tt);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (k < (int)P.n) {
                        const int64_t off = row_offset<DM>(P, k, tt) + (int64_t)col * 4 * P.stride[k][D - 1];
                        x[u][k] = ldg<NTL>((const GLOBAL f4v *)((const GLOBAL float *)(uintptr_t)P.ptr[k] + off));
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < DOT_QUADS; ++u) {
                if (ok[u]) {
                    double w[4] = {(double)x[u][0].x, (double)x[u][0].y, (double)x[u][0].z,
                                   (double)x[u][0].w};
#pragma unroll
                    for (int k = 1; k < 4; ++k) {
                        if (k < (int)P.n) {
                            w[0] *= (double)x[u][k].x;
                            w[1] *= (double)x[u][k].y;
                            w[2] *= (double)x[u][k].z;
                            w[3] *= (double)x[u][k].w;
                        }
                    }
                    acc[0] += w[0];
                    acc[0] += w[1];
                    acc[0] += w[2];
                    acc[0] += w[3];
                }
            }
        }
    } else {
        for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
            const uint64_t s = tile * NT + threadIdx.x;
            if (VEC && P.stage) {
                // every operand contiguous over the counter: only the total
                // is needed, so each lane adds the products of the quads it
                // fetched (no pass through LDS; the clamped copies past the
                // wave's range are skipped)
                const uint32_t cnt = stage_count(P, tile);
                if (cnt) {
                    const uint32_t lane = threadIdx.x & 63u;
                    const uint32_t sh = stage_shift(P.S);
                    const uint32_t nq = cnt << sh;
                    // products formed in float64 in operand order (rows of
                    // 4 or 8 words fetch fewer than HALF words: the rest stay
                    // zero and are never added)
                    float x[HALF] = {};
                    double w[HALF];
                    stage_fetch<NTL>(P, 0, tile, x);
#pragma unroll
                    for (int j = 0; j < HALF; ++j)
                        w[j] = (double)x[j];
#pragma unroll
                    for (int k = 1; k < 4; ++k) {
                        if (MULTI && k < (int)P.n) {
                            stage_fetch<NTL>(P, k, tile, x);
#pragma unroll
                            for (int j = 0; j < HALF; ++j)
                                w[j] *= (double)x[j];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < HALF / 4; ++i) {
                        if ((uint32_t)i < (1u << sh) && (uint32_t)i * 64u + lane < nq) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                acc[0] += w[4 * i + e];
                        }
                    }
                }
            } else if (s < P.nseg) {
                const Seg sg = seg_of(P, s);
                int64_t off[4];
                HalfW<MULTI> w0;
                seg_offsets<DM>(P, sg, off);
                seg_load_half<VEC, NTL, MULTI>(P, off, sg.len, 0, w0);
                double s0, s1, s2;
                seg_moments<VEC, NTL, MULTI, 0>(P, off, sg.len, w0, s0, s1, s2);
                acc[0] += s0;
            }
        }
    }
    block_sums<1>(acc, xch, tot);
    if (threadIdx.x == 0)
        ((double *)((char *)(uintptr_t)P.ws + 256))[blockIdx.x] = tot[0];
}

// Sum of the per-workgroup partials, written as float32 to out32[0] and,
// when requested, float64 to out64[0].  One workgroup of FNT threads:
// thread t loads partials t, t + FNT, .. (all loads of a pass in flight
// together), then the workgroup folds in a fixed tree (half-wave shuffles,
// then the half waves' sums in order).
__global__ __launch_bounds__(FNT) void dot_final_kernel(const SegPlan P)
{
    __shared__ double hw[FNT / 32];
    const GLOBAL double *partials = (const GLOBAL double *)((uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    double v = 0.0;
    for (uint32_t b = threadIdx.x; b < nb; b += FNT)
        v += partials[b];
    v = half_wave_sum(v);
    if ((threadIdx.x & 31) == 31)
        hw[threadIdx.x >> 5] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < FNT / 32; ++i)
            t += hw[i];
        ((float *)(uintptr_t)P.out32)[0] = (float)t;
        if (P.out64)
            ((double *)(uintptr_t)P.out64)[0] = t;
    }
}

// ---------------------------------------------------------------------
// Nonzero bounding box (Section 2): per counter position, the least and
// greatest digit at which every operand is nonzero.  Each operand is
// compared with zero separately (a float32 product of nonzero values may
// underflow to zero; the reals' product is nonzero exactly when every
// factor is).  Per segment a bit mask of the qualifying elements gives the
// inner extent; the outer digits enter once per segment.  Minima and
// maxima do not depend on the order of combination: LDS atomics fold the
// workgroup, a second kernel the workgroups.  hi is kept as digit + 1 so
// that 0 means "none".
// ---------------------------------------------------------------------
template <bool VEC, bool NTL>
__device__ __forceinline__ uint32_t seg_nonzero_half(const SegPlan &P, const int64_t off[4],
                                                     uint32_t len, uint32_t h0)
{
    const int n = (int)P.n;
    uint32_t m = 0xFFFFu;
    if constexpr (VEC) {
        const uint32_t qmax = (len >> 2) - 1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < n) {
                const GLOBAL f4v *pk =
                    (const GLOBAL f4v *)((const GLOBAL float *)(uintptr_t)P.ptr[k] + off[k]);
                f4v v[HALF / 4];
#pragma unroll
                for (int q = 0; q < HALF / 4; ++q)
                    v[q] = ldg<NTL>(pk + min((h0 >> 2) + (uint32_t)q, qmax));
                uint32_t mk = 0;
#pragma unroll
                for (int q = 0; q < HALF / 4; ++q) {
                    mk |= (v[q].x != 0.0f ? 1u : 0u) << (4 * q + 0);
                    mk |= (v[q].y != 0.0f ? 1u : 0u) << (4 * q + 1);
                    mk |= (v[q].z != 0.0f ? 1u : 0u) << (4 * q + 2);
                    mk |= (v[q].w != 0.0f ? 1u : 0u) << (4 * q + 3);
                }
                m &= mk;
            }
        }
    } else {
        const int D = (int)P.D;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < n) {
                const GLOBAL float *pk = (const GLOBAL float *)(uintptr_t)P.ptr[k] + off[k];
                const int64_t ik = P.stride[k][D - 1];
                float v[HALF];
#pragma unroll
                for (int j = 0; j < HALF; ++j)
                    v[j] = ldg<NTL>(pk + (int64_t)min(h0 + (uint32_t)j, len - 1) * ik);
                uint32_t mk = 0;
#pragma unroll
                for (int j = 0; j < HALF; ++j)
                    mk |= (v[j] != 0.0f ? 1u : 0u) << j;
                m &= mk;
            }
        }
    }
    // keep only the elements of the segment
    const uint32_t rem = len > h0 ? len - h0 : 0u;
    if (rem < (uint32_t)HALF)
        m &= (1u << rem) - 1u;
    return m;
}

// W32: the instance for staged 32-word segments (its LDS rows and
// registers: 2 workgroups per CU, the number the plan runs).
template <int DM, bool VEC, bool NTL = true, bool W32 = false>
__global__ __launch_bounds__(NT, (W32 || DM > 8) ? 2 : 4) void bbox_kernel(const SegPlan plan)
{
    SEG_PLAN_FOR(DM);
    __shared__ uint32_t slo[DM], shi[DM];
    __shared__ __align__(16) float
        stg[VEC ? NT / 64 : 1][W32 ? 64 * STG_ROW32 : (VEC ? 64 * STG_ROW : 4)];
    const int D = (int)P.D;
    uint32_t lo[DM], hi[DM];
#pragma unroll
    for (int p = 0; p < DM; ++p) {
        lo[p] = 0xFFFFFFFFu;
        hi[p] = 0u;
    }
    for (int p = threadIdx.x; p < DM; p += NT) {
        slo[p] = 0xFFFFFFFFu;
        shi[p] = 0u;
    }
    const uint32_t lb = seg_logical_block();
    const uint64_t g = gridDim.x;
    if (VEC && !W32 && P.stage == 6) {
        // Rows of 16 words laid end to end: load r gives lane l quad l & 3 of
        // row 16 r + l / 4 of the wave's 64 rows (1 KiB per instruction); the
        // lane's 4-bit masks of its words, shifted to their columns, are
        // combined across the quad so that lane l holds the 16-bit mask of
        // row 16 (l & 3) + l / 4.
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t q = lane & 3u;
        for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
            const uint64_t r0 = tile * NT + (threadIdx.x & ~63u) + (lane >> 2);
            const uint64_t last = P.nseg - 1u;
            uint32_t mk[4] = {0xFu, 0xFu, 0xFu, 0xFu};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < (int)P.n) {
                    const GLOBAL f4v *src =
                        (const GLOBAL f4v *)((const GLOBAL float *)(uintptr_t)P.ptr[k] + P.base[k]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {   // rows past the end: the last row (never folded)
                        const f4v y = ldg<NTL>(src + 4u * min(r0 + 16u * (uint32_t)r, last) + q);
                        mk[r] &= (y.x != 0.0f ? 1u : 0u) | (y.y != 0.0f ? 2u : 0u) |
                                 (y.z != 0.0f ? 4u : 0u) | (y.w != 0.0f ? 8u : 0u);
                    }
                }
            }
            uint32_t v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[r] = mk[r] << (4u * q);
            const uint32_t m = quad_scatter_or(v);
            const uint64_t row = r0 + 16u * q;
            if (row < P.nseg && m) {
                double u[DM];
                uint32_t tt[DM];
                row_coords<DM>(P, (uint32_t)row, u, tt);
                lo[0] = min(lo[0], (uint32_t)(__ffs(m) - 1));
                hi[0] = max(hi[0], (uint32_t)(32 - __clz(m)));
#pragma unroll
                for (int p = 1; p < DM; ++p) {
                    if (p < D) {
                        lo[p] = min(lo[p], tt[p]);
                        hi[p] = max(hi[p], tt[p] + 1u);
                    }
                }
            }
        }
    } else
    for (uint64_t tile = lb; tile < P.ntiles; tile += g) {
        const uint64_t s = tile * NT + threadIdx.x;
        uint32_t staged = 0xFFFFFFFFu;   // staged tiles: the nonzero mask of the segment
        if (VEC && !W32 && P.stage == 1) {
            SHARED float *lds = (SHARED float *)stg[threadIdx.x >> 6];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < (int)P.n) {
                    float v[HALF];
                    stage_words<NTL>(P, k, tile, lds, v);
                    uint32_t mk = 0;
#pragma unroll
                    for (int j = 0; j < HALF; ++j)
                        mk |= (v[j] != 0.0f ? 1u : 0u) << j;
                    staged &= mk;
                }
            }
        } else if constexpr (W32) {
            // segments of 32 words laid end to end: both halves at once
            SHARED float *lds = (SHARED float *)stg[threadIdx.x >> 6];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < (int)P.n) {
                    float x[SEG_MAX];
                    stage_fetch<NTL, SEG_MAX / 4>(P, k, tile, x);
                    stage_put<SEG_MAX / 4>(P, tile, x, lds);
                    float v[HALF];
                    uint32_t mk = 0;
                    stage_get<HALF / 4, 0>(P, tile, lds, v);
#pragma unroll
                    for (int j = 0; j < HALF; ++j)
                        mk |= (v[j] != 0.0f ? 1u : 0u) << j;
                    stage_get<HALF / 4, HALF / 4>(P, tile, lds, v);
#pragma unroll
                    for (int j = 0; j < HALF; ++j)
                        mk |= (v[j] != 0.0f ? 1u : 0u) << (HALF + j);
                    staged &= mk;
                }
            }
        }
        if (s < P.nseg) {
            const Seg sg = seg_of(P, s);
            int64_t off[4];
            seg_offsets<DM>(P, sg, off);
            uint32_t m;
            if (VEC && P.stage) {
                m = sg.len >= 32u ? staged : staged & ((1u << sg.len) - 1u);
            } else {
                m = seg_nonzero_half<VEC, NTL>(P, off, sg.len, 0);
                if (sg.len > (uint32_t)HALF)
                    m |= seg_nonzero_half<VEC, NTL>(P, off, sg.len, HALF) << HALF;
            }
            if (m) {
                double u[DM];
                uint32_t tt[DM];
                row_coords<DM>(P, sg.row, u, tt);
                const uint32_t jmin = sg.j0 + (uint32_t)(__ffs(m) - 1);
                const uint32_t jmax = sg.j0 + (uint32_t)(31 - __clz(m));
                lo[0] = min(lo[0], jmin);
                hi[0] = max(hi[0], jmax + 1u);
#pragma unroll
                for (int p = 1; p < DM; ++p) {
                    if (p < D) {
                        lo[p] = min(lo[p], tt[p]);
                        hi[p] = max(hi[p], tt[p] + 1u);
                    }
                }
            }
        }
    }
    // fold the wave first (DPP, into lane 63), then one LDS atomic per wave
    // and position: 256 same-address atomics per position would serialize
#pragma unroll
    for (int p = 0; p < DM; ++p) {
        if (p < D) {
            lo[p] = wave_minmax<false>(lo[p]);
            hi[p] = wave_minmax<true>(hi[p]);
        }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 63) {
#pragma unroll
        for (int p = 0; p < DM; ++p) {
            if (p < D && hi[p]) {
                atomicMin(&slo[p], lo[p]);
                atomicMax(&shi[p], hi[p]);
            }
        }
    }
    __syncthreads();
    // partials: 2*DM words per block, position-major (coalesced combine)
    uint32_t *partials = (uint32_t *)((char *)(uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    for (int p = threadIdx.x; p < DM; p += NT) {
        partials[(size_t)(2 * p) * nb + blockIdx.x] = slo[p];
        partials[(size_t)(2 * p + 1) * nb + blockIdx.x] = shi[p];
    }
}

// Combines the bbox partials and writes [lo_i, hi_i] per original axis
// (int64; -1 everywhere when nothing qualifies; 0 on extent-1 axes).  One
// workgroup of FNT threads: thread t loads block t's 2 * D words at once
// (one round trip), then folds them into LDS with min / max atomics, which
// do not depend on order.
template <int DM>
__global__ __launch_bounds__(FNT) void bbox_final_kernel(const SegPlan P)
{
    __shared__ uint32_t flo[DM], fhi[DM];
    __shared__ int pos_of[MAXD];
    const int D = (int)P.D;
    const GLOBAL uint32_t *partials = (const GLOBAL uint32_t *)((uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    for (int p = threadIdx.x; p < DM; p += FNT) {
        flo[p] = 0xFFFFFFFFu;
        fhi[p] = 0u;
    }
    if (threadIdx.x < MAXD)
        pos_of[threadIdx.x] = -1;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += FNT) {
        const uint32_t b = b0 + threadIdx.x;
        uint32_t l[DM], h[DM];
#pragma unroll
        for (int p = 0; p < DM; ++p) {
            l[p] = 0xFFFFFFFFu;
            h[p] = 0u;
            if (p < D && b < nb) {
                l[p] = partials[(size_t)(2 * p) * nb + b];
                h[p] = partials[(size_t)(2 * p + 1) * nb + b];
            }
        }
        // wave folds by DPP (into lane 63), then one LDS atomic per wave and
        // position
#pragma unroll
        for (int p = 0; p < DM; ++p) {
            if (p < D) {
                l[p] = wave_minmax<false>(l[p]);
                h[p] = wave_minmax<true>(h[p]);
            }
        }
        if ((threadIdx.x & 63) == 63) {
#pragma unroll
            for (int p = 0; p < DM; ++p) {
                if (p < D && h[p]) {
                    atomicMin(&flo[p], l[p]);
                    atomicMax(&fhi[p], h[p]);
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        for (int p = 0; p < D; ++p) {
            uint32_t o = P.orig[D - 1 - p];
            if (o != 0xFFFFFFFFu)
                pos_of[o] = p;
        }
    }
    __syncthreads();
    const bool found = fhi[0] != 0u;
    int64_t *out = (int64_t *)(uintptr_t)P.out32;
    const int d = (int)P.d_orig;
    for (int i = threadIdx.x; i < d; i += FNT) {
        const int p = pos_of[i];
        int64_t a = -1, b = -1;
        if (found) {
            a = (p < 0) ? 0 : (int64_t)flo[p];
            b = (p < 0) ? 0 : (int64_t)fhi[p] - 1;
        }
        out[2 * i] = a;
        out[2 * i + 1] = b;
    }
}

// ---------------------------------------------------------------------

template <int DM, bool COV>
static hipError_t go_moments(const SegLaunch &L, hipStream_t st)
{
    const bool multi = L.plan.n > 1;
    const bool cached = (L.plan.flags & TRIOT_MOMENTS_CACHED) != 0;
    const int k = (L.plan.vec4 ? 4 : 0) + (multi ? 2 : 0) + (cached ? 1 : 0);
    if (L.plan.stage == 1) {   // staged tile loads: instances of their own (their LDS rows)
        switch (k) {
        case 7: hipLaunchKernelGGL((moments_kernel<DM, COV, true, true, false, 1>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 6: hipLaunchKernelGGL((moments_kernel<DM, COV, true, true, true, 1>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 5: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false, 1>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 4: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true, 1>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        default: return hipErrorInvalidValue;   // the plan stages whole-quad rows only
        }
    } else if (L.plan.stage == 6) {   // rows of 16 words end to end, one operand (the plan's rule)
        switch (k) {
        case 5: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false, 6>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 4: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true, 6>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        default: return hipErrorInvalidValue;
        }
    } else if (L.plan.stage == 5) {   // rows of exactly 16 words, per-lane loads
        switch (k) {
        case 7: hipLaunchKernelGGL((moments_kernel<DM, COV, true, true, false, 5>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 6: hipLaunchKernelGGL((moments_kernel<DM, COV, true, true, true, 5>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 5: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false, 5>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 4: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true, 5>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        default: return hipErrorInvalidValue;   // the plan takes whole-quad rows only
        }
    } else if (L.plan.stage == 4) {   // row blocks, one operand, two axes or more (the plan's rule)
        if constexpr (DM >= 2) {
            if (cached)
                hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false, 4>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
            else
                hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true, 4>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (L.plan.stage == 3) {   // short segments, one operand (the plan's rule)
        switch (k) {
        case 5: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false, 3>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 4: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true, 3>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 1: hipLaunchKernelGGL((moments_kernel<DM, COV, false, false, false, 3>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 0: hipLaunchKernelGGL((moments_kernel<DM, COV, false, false, true, 3>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        default: return hipErrorInvalidValue;
        }
    } else if (L.plan.stage == 2) {   // one operand only (the plan's rule)
        switch (k) {
        case 5: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false, 2>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        case 4: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true, 2>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
        default: return hipErrorInvalidValue;
        }
    } else {
    switch (k) {
    case 7: hipLaunchKernelGGL((moments_kernel<DM, COV, true, true, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    case 6: hipLaunchKernelGGL((moments_kernel<DM, COV, true, true, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    case 5: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    case 4: hipLaunchKernelGGL((moments_kernel<DM, COV, true, false, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    case 3: hipLaunchKernelGGL((moments_kernel<DM, COV, false, true, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    case 2: hipLaunchKernelGGL((moments_kernel<DM, COV, false, true, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    case 1: hipLaunchKernelGGL((moments_kernel<DM, COV, false, false, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    default: hipLaunchKernelGGL((moments_kernel<DM, COV, false, false, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan); break;
    }
    }
    const int d = (int)L.plan.d_orig;
    const int nout = 1 + d + (COV ? d * (d + 1) / 2 : 0);
    hipLaunchKernelGGL((moments_out_kernel<DM, COV>), dim3(nout), dim3(ONT), 0, st, L.plan);
    return hipGetLastError();
}

hipError_t launch_moments(const SegLaunch &L, hipStream_t st)
{
    const bool cov = (L.plan.flags & TRIOT_MOMENTS_COV) != 0;
    if (cov) {
        switch (L.dm) {
        case 1: return go_moments<1, true>(L, st);
        case 2: return go_moments<2, true>(L, st);
        case 3: return go_moments<3, true>(L, st);
        case 4: return go_moments<4, true>(L, st);
        case 5: return go_moments<5, true>(L, st);
        case 6: return go_moments<6, true>(L, st);
        case 7: return go_moments<7, true>(L, st);
        case 8: return go_moments<8, true>(L, st);
        default: return hipErrorInvalidValue;
        }
    }
    return L.dm <= 8 ? go_moments<8, false>(L, st) : go_moments<32, false>(L, st);
}

template <int DM>
static void go_dot(const SegLaunch &L, hipStream_t st)
{
    const bool multi = L.plan.n > 1;
    if (L.plan.vec4) {
        if (multi)
            hipLaunchKernelGGL((dot_kernel<DM, true, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        else
            hipLaunchKernelGGL((dot_kernel<DM, true, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
    } else {
        if (multi)
            hipLaunchKernelGGL((dot_kernel<DM, false, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        else
            hipLaunchKernelGGL((dot_kernel<DM, false, false>), dim3(L.blocks), dim3(NT), 0, st,
                               L.plan);
    }
}

hipError_t launch_dot(const SegLaunch &L, hipStream_t st)
{
    // the word-quad walk over at most 3 axes: an instance whose axis loops
    // unroll to 3 (fewer run-time axis tests per quad; its other paths are
    // never launched, they would spill)
    if (L.plan.quads && L.plan.D <= 3)
        go_dot<3>(L, st);
    else if (L.dm <= 8)
        go_dot<8>(L, st);
    else
        go_dot<32>(L, st);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(FNT), 0, st, L.plan);
    return hipGetLastError();
}

hipError_t launch_bbox(const SegLaunch &L, hipStream_t st)
{
    const bool w32 = L.plan.stage == 2;   // staged 32-word segments (vec4 implied)
    if (L.dm <= 8) {
        if (w32)
            hipLaunchKernelGGL((bbox_kernel<8, true, true, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        else if (L.plan.vec4)
            hipLaunchKernelGGL((bbox_kernel<8, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        else
            hipLaunchKernelGGL((bbox_kernel<8, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        hipLaunchKernelGGL((bbox_final_kernel<8>), dim3(1), dim3(FNT), 0, st, L.plan);
    } else {
        if (w32)
            hipLaunchKernelGGL((bbox_kernel<32, true, true, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        else if (L.plan.vec4)
            hipLaunchKernelGGL((bbox_kernel<32, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        else
            hipLaunchKernelGGL((bbox_kernel<32, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        hipLaunchKernelGGL((bbox_final_kernel<32>), dim3(1), dim3(FNT), 0, st, L.plan);
    }
    return hipGetLastError();
}

hipError_t launch_moments_adj(const SegLaunch &L, hipStream_t st)
{
    const bool cov = (L.plan.flags & TRIOT_MOMENTS_COV) != 0;
    if (cov) {
        hipLaunchKernelGGL((moments_adj_kernel<8, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
    } else if (L.dmax <= 8) {
        hipLaunchKernelGGL((moments_adj_kernel<8, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
    } else {
        hipLaunchKernelGGL((moments_adj_kernel<32, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
    }
    return hipGetLastError();
}

}  // namespace triot

namespace triot {

// Resident workgroups per CU of the row kernels (their register needs
// differ by instance), asked of the runtime once per instance; 2 when no
// device answers.
template <class K> static int occupancy(K kernel)
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, NT, 0);
    return (e == hipSuccess && nb > 0) ? nb : 2;
}

template <int DM, bool COV> static int occ_moments(bool vec4, int stage)
{
    static int cache[2][7] = {{0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0}};
    int &c = cache[vec4 ? 1 : 0][stage < 7 ? stage : 0];
    if (!c) {
        switch (stage) {
        case 6: c = occupancy(moments_kernel<DM, COV, true, false, true, 6>); break;
        case 5: c = occupancy(moments_kernel<DM, COV, true, false, true, 5>); break;
        case 4:
            if constexpr (DM >= 2)
                c = occupancy(moments_kernel<DM, COV, true, false, true, 4>);
            else
                c = 2;
            break;
        case 1: c = occupancy(moments_kernel<DM, COV, true, false, true, 1>); break;
        case 2: c = occupancy(moments_kernel<DM, COV, true, false, true, 2>); break;
        case 3:
            c = vec4 ? occupancy(moments_kernel<DM, COV, true, false, true, 3>)
                     : occupancy(moments_kernel<DM, COV, false, false, true, 3>);
            break;
        default:
            c = vec4 ? occupancy(moments_kernel<DM, COV, true, false>)
                     : occupancy(moments_kernel<DM, COV, false, false>);
        }
    }
    return c;
}

int segment_blocks_per_cu(bool adj, bool cov, int dm, bool vec4, int stage)
{
    if (adj) {
        static int cache[3] = {0, 0, 0};
        const int i = cov ? 0 : (dm <= 8 ? 1 : 2);
        if (!cache[i])
            cache[i] = cov ? occupancy(moments_adj_kernel<8, true>)
                           : (dm <= 8 ? occupancy(moments_adj_kernel<8, false>)
                                      : occupancy(moments_adj_kernel<32, false>));
        return cache[i];
    }
    if (cov) {
        switch (dm) {
        case 1: return occ_moments<1, true>(vec4, stage);
        case 2: return occ_moments<2, true>(vec4, stage);
        case 3: return occ_moments<3, true>(vec4, stage);
        case 4: return occ_moments<4, true>(vec4, stage);
        case 5: return occ_moments<5, true>(vec4, stage);
        case 6: return occ_moments<6, true>(vec4, stage);
        case 7: return occ_moments<7, true>(vec4, stage);
        default: return occ_moments<8, true>(vec4, stage);
        }
    }
    return dm <= 8 ? occ_moments<8, false>(vec4, stage) : occ_moments<32, false>(vec4, stage);
}

}  // namespace triot
