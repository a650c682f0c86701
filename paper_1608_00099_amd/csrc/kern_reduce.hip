// Tuple-reading kernels with a different shape of work for gfx950: the
// naive multidimensional convolution (Algorithms 14 and 15 of the paper)
// and marginalization (sums over a subset of axes, Section 2).
//
// Convolution, as a gather: thread v computes one output element
//     out[v] = sum over t in lhs, 0 <= v - t < rs, of lhs[t] * rhs[v - t],
// visiting t in lexicographic order.  For a fixed v the paper's loops (lhs
// tuples outside, rhs tuples inside, result[t + u] += lhs[t] * rhs[u])
// add exactly these terms in exactly this order, so with the product and
// the sum rounded separately the result is the paper's bit for bit, with
// no atomics.  The valid t form a box [max(0, v - rs + 1), min(v, ls - 1)];
// along its innermost axis the lhs index rises by one and the rhs index
// falls by one.  Inputs small enough are staged in LDS once per workgroup.
//
// Marginalization: thread (o, p) decodes kept tuple o and the start of
// part p of the reduced sub-box, then walks that part in lexicographic
// order with an odometer (per-operand offsets advanced by stride, reset on
// carry).  Consecutive threads hold consecutive kept tuples, so when the
// innermost axis is kept, a wave's loads are contiguous.  With several
// parts a second kernel adds them in order.  Deterministic.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "launch.h"

namespace triot {

#define GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ uint32_t rdiv_u32(uint32_t n, const AxisDiv &a)
{
    uint32_t h = __umulhi(n, a.m);
    return (h + ((n - h) >> 1)) >> a.s;
}

constexpr int CONV_NT = 64;   // one wave per workgroup: outputs spread over more CUs
constexpr uint32_t CONV_LDS_WORDS = 8192;   // float64 words of LDS staging (64 KiB)

// Copies n float64 words from global memory to LDS with 16 loads in flight
// per thread (one round trip per 16 * CONV_NT words, not per CONV_NT).
__device__ __forceinline__ void stage_lds(double *dst, const GLOBAL double *src, uint32_t n)
{
    constexpr int K = 16;
    for (uint32_t b = threadIdx.x; b < n; b += K * CONV_NT) {
        double tmp[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const uint32_t i = b + (uint32_t)u * CONV_NT;
            tmp[u] = src[i < n ? i : 0u];
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const uint32_t i = b + (uint32_t)u * CONV_NT;
            if (i < n)
                dst[i] = tmp[u];
        }
    }
}

template <bool LDS>
__global__ __launch_bounds__(CONV_NT) void conv_kernel(const ConvPlan P)
{
    extern __shared__ double sm[];
    const GLOBAL double *gl = (const GLOBAL double *)(uintptr_t)P.lhs;
    const GLOBAL double *gr = (const GLOBAL double *)(uintptr_t)P.rhs;
    if (LDS) {
        stage_lds(sm, gl, P.nl);
        stage_lds(sm + P.nl, gr, P.nr);
        __syncthreads();
    }
    const double *L = LDS ? sm : (const double *)gl;
    const double *R = LDS ? sm + P.nl : (const double *)gr;
    const uint64_t f = (uint64_t)blockIdx.x * CONV_NT + threadIdx.x;
    if (f >= P.nout)
        return;
    const int d = (int)P.d;
    // output tuple v (row-major over ls + rs - 1)
    uint32_t v[MAXD];
    uint32_t q = (uint32_t)f;
    for (int i = d - 1; i >= 1; --i) {
        if (P.ax[i].c == 1) {
            v[i] = 0;
            continue;
        }
        const uint32_t qq = rdiv_u32(q, P.ax[i]);
        v[i] = q - qq * P.ax[i].c;
        q = qq;
    }
    if (d > 0)
        v[0] = q;
    // the box of valid lhs tuples and the offsets of its first tuple
    uint32_t lo[MAXD], hi[MAXD], t[MAXD];
    int64_t lrow = 0, rrow = 0;
    for (int i = 0; i < d; ++i) {
        lo[i] = v[i] + 1 > P.rs[i] ? v[i] + 1 - P.rs[i] : 0u;
        hi[i] = min(v[i], P.ls[i] - 1);
        t[i] = lo[i];
        lrow += (int64_t)lo[i] * P.lstride[i];
        rrow += (int64_t)(v[i] - lo[i]) * P.rstride[i];
    }
    double acc = 0.0;
    if (d == 0) {
        acc = acc + L[0] * R[0];
    } else {
        const int in = d - 1;
        const uint32_t nin = hi[in] - lo[in] + 1;
        while (true) {
            // innermost axis (unit stride in both inputs): lhs index up by
            // one, rhs index down by one; loads run ahead of the sequential
            // additions, which keep the paper's order
            const double *lp = L + lrow;
            const double *rp = R + rrow;
            uint32_t k = 0;
            for (; k + 4 <= nin; k += 4) {
                const double a0 = lp[k], a1 = lp[k + 1], a2 = lp[k + 2], a3 = lp[k + 3];
                const double b0 = rp[-(int64_t)k], b1 = rp[-(int64_t)k - 1];
                const double b2 = rp[-(int64_t)k - 2], b3 = rp[-(int64_t)k - 3];
                const double p0 = a0 * b0, p1 = a1 * b1, p2 = a2 * b2, p3 = a3 * b3;
                acc = acc + p0;
                acc = acc + p1;
                acc = acc + p2;
                acc = acc + p3;
            }
            for (; k < nin; ++k) {
                const double prod = lp[k] * rp[-(int64_t)k];
                acc = acc + prod;
            }
            // next tuple of the outer axes (carry), else done
            int i = in - 1;
            for (; i >= 0; --i) {
                if (t[i] < hi[i]) {
                    ++t[i];
                    lrow += P.lstride[i];
                    rrow -= P.rstride[i];
                    break;
                }
                lrow -= (int64_t)(t[i] - lo[i]) * P.lstride[i];
                rrow += (int64_t)(t[i] - lo[i]) * P.rstride[i];
                t[i] = lo[i];
            }
            if (i < 0)
                break;
        }
    }
    ((GLOBAL double *)(uintptr_t)P.out)[f] = acc;
}

// The same gather for a dimension D known at compile time (1..4): the
// per-axis state lives in registers, and the valid box is walked as one
// flattened loop in lexicographic order.  DEPTH steps of index arithmetic
// and their loads run ahead of the DEPTH additions, which stay in order
// (few waves share a CU here, so the loads' latency must overlap within
// the thread).  IDX: 32-bit indices when the inputs sit in LDS.
template <int D, bool LDS>
__global__ __launch_bounds__(CONV_NT) void conv_kernel_d(const ConvPlan P)
{
    typedef typename std::conditional<LDS, int32_t, int64_t>::type IDX;
    constexpr int DEPTH = 16;
    extern __shared__ double sm[];
    const GLOBAL double *gl = (const GLOBAL double *)(uintptr_t)P.lhs;
    const GLOBAL double *gr = (const GLOBAL double *)(uintptr_t)P.rhs;
    if (LDS) {
        stage_lds(sm, gl, P.nl);
        stage_lds(sm + P.nl, gr, P.nr);
        __syncthreads();
    }
    const double *L = LDS ? sm : (const double *)gl;
    const double *R = LDS ? sm + P.nl : (const double *)gr;
    const uint64_t f = (uint64_t)blockIdx.x * CONV_NT + threadIdx.x;
    if (f >= P.nout)
        return;
    uint32_t v[D];
    uint32_t q = (uint32_t)f;
#pragma unroll
    for (int i = D - 1; i >= 1; --i) {
        if (P.ax[i].c == 1) {
            v[i] = 0;
        } else {
            const uint32_t qq = rdiv_u32(q, P.ax[i]);
            v[i] = q - qq * P.ax[i].c;
            q = qq;
        }
    }
    v[0] = q;
    uint32_t nbox[D], c[D];
    IDX li = 0, ri = 0, lst[D], rst[D];
    uint32_t total = 1;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const uint32_t lo = v[i] + 1 > P.rs[i] ? v[i] + 1 - P.rs[i] : 0u;
        const uint32_t hi = min(v[i], P.ls[i] - 1);
        nbox[i] = hi - lo + 1;
        total *= nbox[i];
        c[i] = 0;
        lst[i] = (IDX)P.lstride[i];
        rst[i] = (IDX)P.rstride[i];
        li += (IDX)lo * lst[i];
        ri += (IDX)(v[i] - lo) * rst[i];
    }
    // advance (li, ri) to the next tuple of the box, lexicographically
    auto step = [&]() {
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            ++c[i];
            li += lst[i];
            ri -= rst[i];
            if (i == 0 || c[i] < nbox[i])
                break;
            li -= (IDX)nbox[i] * lst[i];
            ri += (IDX)nbox[i] * rst[i];
            c[i] = 0;
        }
    };
    double acc = 0.0;
    for (uint32_t s0 = 0; s0 < total; s0 += DEPTH) {
        double a[DEPTH], b[DEPTH];
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) {
            const bool ok = s0 + (uint32_t)u < total;
            a[u] = L[ok ? li : 0];
            b[u] = R[ok ? ri : 0];
            if (s0 + (uint32_t)u + 1 < total)
                step();
        }
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) {
            if (s0 + (uint32_t)u < total) {
                const double prod = a[u] * b[u];
                acc = acc + prod;
            }
        }
    }
    ((GLOBAL double *)(uintptr_t)P.out)[f] = acc;
}

// Dimensions 1 and 2 (benchmark 4 is 2-d): the box is walked as nested
// loops, rows of the lhs box outside, inside them chunks of 8 terms read at
// fixed offsets from one row pointer (no per-term index arithmetic or
// carry).  The inputs sit in LDS between 8 words of padding on each side,
// so the chunk's reads past a row's end stay inside the allocation; those
// terms are never added.  The additions keep the paper's order.
constexpr uint32_t CONV_PAD = 8;

template <int D>
__global__ __launch_bounds__(CONV_NT) void conv_kernel_rows(const ConvPlan P)
{
    extern __shared__ double sm[];
    double *Ls = sm + CONV_PAD;
    double *Rs = sm + CONV_PAD + P.nl + CONV_PAD;
    stage_lds(Ls, (const GLOBAL double *)(uintptr_t)P.lhs, P.nl);
    stage_lds(Rs, (const GLOBAL double *)(uintptr_t)P.rhs, P.nr);
    __syncthreads();
    const uint64_t f = (uint64_t)blockIdx.x * CONV_NT + threadIdx.x;
    if (f >= P.nout)
        return;
    // output tuple (v0, v1); for D == 1 the outer axis is a single row
    uint32_t v0 = 0, v1;
    if (D == 2) {
        if (P.ax[1].c == 1) {
            v1 = 0;
            v0 = (uint32_t)f;
        } else {
            v0 = rdiv_u32((uint32_t)f, P.ax[1]);
            v1 = (uint32_t)f - v0 * P.ax[1].c;
        }
    } else {
        v1 = (uint32_t)f;
    }
    const uint32_t ls0 = D == 2 ? P.ls[0] : 1u, rs0 = D == 2 ? P.rs[0] : 1u;
    const uint32_t ls1 = P.ls[D - 1], rs1 = P.rs[D - 1];
    const uint32_t lo0 = v0 + 1 > rs0 ? v0 + 1 - rs0 : 0u, hi0 = min(v0, ls0 - 1);
    const uint32_t lo1 = v1 + 1 > rs1 ? v1 + 1 - rs1 : 0u, hi1 = min(v1, ls1 - 1);
    const uint32_t n0 = hi0 - lo0 + 1, n1 = hi1 - lo1 + 1;
    int32_t lrow = (int32_t)(lo0 * ls1 + lo1);
    int32_t rrow = (int32_t)((v0 - lo0) * rs1 + (v1 - lo1));
    double acc = 0.0;
    if (ls1 <= 8) {
        // Rows of at most 8 terms: one chunk per row, and the next row's
        // words are read from LDS before this row's terms are added (two
        // buffers in turn), so LDS latency overlaps the add chain.
        double a0[8], b0[8], a1[8], b1[8];
        auto ld = [&](double (&a)[8], double (&b)[8], int32_t lr, int32_t rr) {
            const double *lp = Ls + lr;
            const double *rp = Rs + rr;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a[u] = lp[u];
                b[u] = rp[-u];
            }
        };
        auto add = [&](const double (&a)[8], const double (&b)[8]) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if ((uint32_t)u < n1) {
                    const double prod = a[u] * b[u];
                    acc = acc + prod;
                }
            }
        };
        ld(a0, b0, lrow, rrow);
        uint32_t j = 0;
        for (; j + 2 <= n0; j += 2) {
            ld(a1, b1, lrow + (int32_t)ls1, rrow - (int32_t)rs1);
            add(a0, b0);
            lrow += 2 * (int32_t)ls1;
            rrow -= 2 * (int32_t)rs1;
            if (j + 2 < n0)
                ld(a0, b0, lrow, rrow);
            add(a1, b1);
        }
        if (j < n0)
            add(a0, b0);
        ((GLOBAL double *)(uintptr_t)P.out)[f] = acc;
        return;
    }
    for (uint32_t j = 0; j < n0; ++j) {
        const double *lp = Ls + lrow;
        const double *rp = Rs + rrow;
        for (uint32_t k0 = 0; k0 < n1; k0 += 8) {
            double a[8], b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a[u] = lp[k0 + u];
                b[u] = rp[-(int32_t)k0 - u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (k0 + (uint32_t)u < n1) {
                    const double prod = a[u] * b[u];
                    acc = acc + prod;
                }
            }
        }
        lrow += (int32_t)ls1;
        rrow -= (int32_t)rs1;
    }
    ((GLOBAL double *)(uintptr_t)P.out)[f] = acc;
}

template <bool LDS>
static void go_conv(const ConvLaunch &L, uint32_t blocks, size_t bytes, hipStream_t st)
{
    switch (L.plan.d) {
    case 1: hipLaunchKernelGGL((conv_kernel_d<1, LDS>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan); break;
    case 2: hipLaunchKernelGGL((conv_kernel_d<2, LDS>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan); break;
    case 3: hipLaunchKernelGGL((conv_kernel_d<3, LDS>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan); break;
    case 4: hipLaunchKernelGGL((conv_kernel_d<4, LDS>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan); break;
    default: hipLaunchKernelGGL((conv_kernel<LDS>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan); break;
    }
}

hipError_t launch_conv(const ConvLaunch &L, hipStream_t st)
{
    const uint32_t blocks = (uint32_t)((L.plan.nout + CONV_NT - 1) / CONV_NT);
    if (L.plan.lds && (L.plan.d == 1 || L.plan.d == 2)) {
        const size_t bytes = (size_t)(L.plan.nl + L.plan.nr + 3 * CONV_PAD) * sizeof(double);
        if (L.plan.d == 1)
            hipLaunchKernelGGL((conv_kernel_rows<1>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan);
        else
            hipLaunchKernelGGL((conv_kernel_rows<2>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan);
        return hipGetLastError();
    }
    if (L.plan.lds)
        go_conv<true>(L, blocks, (size_t)(L.plan.nl + L.plan.nr) * sizeof(double), st);
    else
        go_conv<false>(L, blocks, 0, st);
    return hipGetLastError();
}

uint32_t conv_lds_words() { return CONV_LDS_WORDS - 3 * 8; }

// ---------------------------------------------------------------------
// Marginalization
// ---------------------------------------------------------------------
constexpr int MARG_NT = 256;

// Kept tuple o -> the element offsets of its reduced sub-box's origin.
__device__ __forceinline__ void marginal_kept(const MargPlan &P, uint32_t o, int64_t off[4])
{
    const int n = (int)P.n, dk = (int)P.dk;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        off[k] = P.base[k];
    uint32_t q = o;
    for (int i = dk - 1; i >= 0; --i) {
        uint32_t digit;
        if (i == 0) {
            digit = q;
        } else {
            const uint32_t qq = rdiv_u32(q, P.kax[i]);
            digit = q - qq * P.kax[i].c;
            q = qq;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < n)
                off[k] += (int64_t)digit * P.kstride[k][i];
    }
}

typedef float mf4 __attribute__((ext_vector_type(4), aligned(4)));

// The marginal walks read every operand word once: non-temporal loads.
// Loads that allocate in the caches must first evict what is there, and
// after a kernel that wrote a large buffer the memory-side cache holds its
// dirty lines, whose write-back then competes with these reads (measured on
// 16^6 after a 1 GiB write: 34.2 against 26.6 us with the cache clean).
__device__ __forceinline__ mf4 mload4(const GLOBAL float *p)
{
    return __builtin_nontemporal_load((const GLOBAL mf4 *)p);
}

__device__ __forceinline__ float mload1(const GLOBAL float *p)
{
    return __builtin_nontemporal_load(p);
}

// Thread (o, p) adds part p of kept tuple o's reduced sub-box in
// lexicographic order.  RD > 0: exactly RD reduced axes, known at compile
// time (the odometer in registers); RD == 0: any number.  W = 4: the
// innermost reduced axis is every operand's last axis with an extent that
// is a multiple of 4, and the walk loads four consecutive elements at a
// time (added in order, as one at a time would).
template <int RD, int W>
__global__ __launch_bounds__(MARG_NT) void marginal_kernel(const MargPlan P)
{
    const uint64_t gid = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    const uint64_t total = P.nout * P.parts;
    if (gid >= total)
        return;
    const uint32_t o = (uint32_t)(gid % P.nout);
    const uint32_t p = (uint32_t)(gid / P.nout);
    const int n = (int)P.n, dr = RD > 0 ? RD : (int)P.dr;
    constexpr int TN = RD > 0 ? RD : MAXD;
    int64_t off[4];
    marginal_kept(P, o, off);
    // part p of the reduced sub-box: flat range [r0, r1), in steps of W
    const uint64_t units = P.nred / W;
    const uint64_t r0 = (uint64_t)p * units / P.parts * W;
    const uint64_t r1 = (uint64_t)(p + 1) * units / P.parts * W;
    uint32_t t[TN];
    {
        uint64_t q = r0;
#pragma unroll
        for (int i = dr - 1; i >= 0; --i) {
            const uint64_t c = P.rax[i].c;
            const uint64_t digit = (i == 0) ? q : q % c;
            q = (i == 0) ? 0 : q / c;
            t[i] = (uint32_t)digit;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < n)
                    off[k] += (int64_t)digit * P.rstride[k][i];
        }
    }
    // Eight steps at a time: their offsets (odometer steps), then all
    // their loads, then their weights added in order.
    auto step = [&]() {
#pragma unroll
        for (int i = dr - 1; i >= 0; --i) {
            const uint32_t inc = (i == dr - 1) ? (uint32_t)W : 1u;
            t[i] += inc;
            if (t[i] < P.rax[i].c || i == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < n)
                        off[k] += (int64_t)inc * P.rstride[k][i];
                break;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < n)
                    off[k] -= (int64_t)(t[i] - inc) * P.rstride[k][i];
            t[i] = 0;
        }
    };
    constexpr int LA = 8;
    double acc = 0.0;
    for (uint64_t r = r0; r < r1; r += LA * W) {
        float v[LA][4][W];
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const bool ok = r + (uint64_t)u * W < r1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < n) {
                    const GLOBAL float *pk = (const GLOBAL float *)(uintptr_t)P.ptr[k];
                    if constexpr (W == 4) {
                        const mf4 x = mload4(pk + (ok ? off[k] : P.base[k]));
                        v[u][k][0] = x.x;
                        v[u][k][1] = x.y;
                        v[u][k][2] = x.z;
                        v[u][k][3] = x.w;
                    } else {
                        v[u][k][0] = mload1(pk + (ok ? off[k] : P.base[k]));
                    }
                }
            }
            if (r + (uint64_t)(u + 1) * W < r1)
                step();
        }
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            if (r + (uint64_t)u * W < r1) {
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    double w = 1.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (k < n)
                            w *= (double)v[u][k][e];
                    acc += w;
                }
            }
        }
    }
    if (P.parts == 1) {
        ((float *)(uintptr_t)P.out32)[o] = (float)acc;
        if (P.out64)
            ((double *)(uintptr_t)P.out64)[o] = acc;
    } else {
        ((double *)((char *)(uintptr_t)P.ws + 256))[(uint64_t)o * P.parts + p] = acc;
    }
}

// One contiguous reduced run per kept tuple (one reduced axis, stride 1 in
// every operand): part p = 64 c + l of output o is lane l of chunk c, the
// elements c * clen + l + 64 s of the run, so every load of a wave reads
// 64 consecutive elements.  Each lane adds its elements in order; the
// parts are then combined in order by the final kernels.
__global__ __launch_bounds__(MARG_NT) void marginal_inter_kernel(const MargPlan P)
{
    const uint64_t gid = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    const uint64_t total = P.nout * P.parts;
    if (gid >= total)
        return;
    const uint32_t o = (uint32_t)(gid / P.parts);     // a wave shares its output
    const uint32_t p = (uint32_t)(gid - (uint64_t)o * P.parts);
    const int n = (int)P.n;
    int64_t off[4];
    marginal_kept(P, o, off);
    const uint64_t c0 = (uint64_t)(p >> 6) * P.clen;
    const uint64_t end = min(c0 + P.clen, P.nred);
    constexpr int LA = 8;
    double acc = 0.0;
    for (uint64_t r = c0 + (p & 63u); r < end; r += 64 * LA) {
        float v[LA][4];
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const uint64_t e = r + (uint64_t)u * 64;
            const uint64_t ee = e < end ? e : c0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < n)
                    v[u][k] = mload1((const GLOBAL float *)(uintptr_t)P.ptr[k] + off[k] + (int64_t)ee);
        }
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            if (r + (uint64_t)u * 64 < end) {
                double w = 1.0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < n)
                        w *= (double)v[u][k];
                acc += w;
            }
        }
    }
    ((double *)((char *)(uintptr_t)P.ws + 256))[(uint64_t)o * P.parts + p] = acc;
}

// Columns: one kept axis, innermost and unit-stride in every operand, and
// one reduced axis.  Thread (q, p), q fastest, adds outputs 4q .. 4q + 3
// (one 16-byte load per operand and row) over rows p, p + parts, p +
// 2 parts, .. in order, so the lanes of a wave read consecutive rows: a
// contiguous range when the rows are adjacent.  The parts are combined in
// order by the final kernels.
__global__ __launch_bounds__(MARG_NT) void marginal_cols_kernel(const MargPlan P)
{
    const uint32_t quads = (uint32_t)(P.nout / 4);
    const uint64_t gid = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    if (gid >= (uint64_t)quads * P.parts)
        return;
    const uint32_t q = (uint32_t)(gid % quads);
    const uint64_t p = gid / quads;
    const int n = (int)P.n;
    constexpr int LA = 8;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint64_t r0 = p; r0 < P.nred; r0 += (uint64_t)LA * P.parts) {
        float v[LA][4][4];
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const uint64_t r = r0 + (uint64_t)u * P.parts;
            const uint64_t rr = r < P.nred ? r : p;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < n) {
                    const mf4 x = mload4((const GLOBAL float *)(uintptr_t)P.ptr[k] +
                                                       P.base[k] + 4 * (int64_t)q +
                                                       (int64_t)rr * P.rstride[k][0]);
                    v[u][k][0] = x.x;
                    v[u][k][1] = x.y;
                    v[u][k][2] = x.z;
                    v[u][k][3] = x.w;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            if (r0 + (uint64_t)u * P.parts < P.nred) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double w = 1.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (k < n)
                            w *= (double)v[u][k][e];
                    acc[e] += w;
                }
            }
        }
    }
    double *part = (double *)((char *)(uintptr_t)P.ws + 256);
#pragma unroll
    for (int e = 0; e < 4; ++e)
        part[(uint64_t)(4 * q + (uint32_t)e) * P.parts + p] = acc[e];
}

// Short runs: the one reduced axis is innermost and unit-stride, of R = 4
// .. 64 elements (a power of 2).  Lane group g = R / 4 per output: lane c of
// the group loads quad c of the run (so a wave's loads cover 64 consecutive
// quads when the runs are adjacent), adds its four weights in order, and
// the group folds its sums by butterflies (fixed order); lane 0 of the
// group writes the output.  Lanes past the last output load output 0's run
// and write nothing (every lane takes part in the butterflies).  (Four
// blocks of quads per workgroup, their loads in flight together, measured
// no faster.)
__global__ __launch_bounds__(MARG_NT) void marginal_runs_kernel(const MargPlan P)
{
    const uint32_t g = (uint32_t)(P.nred / 4);
    const uint64_t gid = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    const uint64_t o = gid / g;
    const uint32_t c = (uint32_t)(gid % g);
    const bool ok = o < P.nout;
    const int n = (int)P.n;
    int64_t off[4];
    marginal_kept(P, ok ? (uint32_t)o : 0u, off);
    float v[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < n) {
            const mf4 x = mload4((const GLOBAL float *)(uintptr_t)P.ptr[k] + off[k] +
                                               4 * (int64_t)c);
            v[k][0] = x.x;
            v[k][1] = x.y;
            v[k][2] = x.z;
            v[k][3] = x.w;
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double w = 1.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < n)
                w *= (double)v[k][e];
        acc += w;
    }
    for (uint32_t k = 1; k < g; k <<= 1)
        acc += __shfl_xor(acc, (int)k, 64);
    if (ok && c == 0) {
        ((float *)(uintptr_t)P.out32)[o] = (float)acc;
        if (P.out64)
            ((double *)(uintptr_t)P.out64)[o] = acc;
    }
}

// One workgroup of MARG_FNT threads per output: thread t adds parts t,
// t + MARG_FNT, .. (16 loads in flight per thread: up to 16384 parts in one
// round trip), then the workgroup folds in a fixed tree (wave butterflies,
// then the waves' sums in order).
constexpr int MARG_FNT = 1024;

__global__ __launch_bounds__(MARG_FNT) void marginal_final_kernel(const MargPlan P)
{
    __shared__ double ws[MARG_FNT / 64];
    const uint64_t o = blockIdx.x;
    const GLOBAL double *part = (const GLOBAL double *)((uintptr_t)P.ws + 256) + o * P.parts;
    constexpr int K = 16;
    double acc = 0.0;
    for (uint32_t b = threadIdx.x; b < P.parts; b += K * MARG_FNT) {
        double x[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const uint32_t p = b + (uint32_t)u * MARG_FNT;
            x[u] = part[p < P.parts ? p : 0u];
        }
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (b + (uint32_t)u * MARG_FNT < P.parts)
                acc += x[u];
    }
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1)
        acc += __shfl_xor(acc, k, 64);
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < MARG_FNT / 64; ++w)
            t += ws[w];
        ((float *)(uintptr_t)P.out32)[o] = (float)t;
        if (P.out64)
            ((double *)(uintptr_t)P.out64)[o] = t;
    }
}

// Few parts per output: one thread per output adds them in order, 16 loads
// in flight at a time.
__global__ __launch_bounds__(MARG_NT) void marginal_final_seq_kernel(const MargPlan P)
{
    const uint64_t o = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    if (o >= P.nout)
        return;
    const GLOBAL double *part = (const GLOBAL double *)((uintptr_t)P.ws + 256) + o * P.parts;
    constexpr int K = 16;
    double acc = 0.0;
    for (uint32_t b = 0; b < P.parts; b += K) {
        double x[K];
#pragma unroll
        for (int u = 0; u < K; ++u)
            x[u] = part[b + u < P.parts ? b + u : 0u];
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (b + (uint32_t)u < P.parts)
                acc += x[u];
    }
    ((float *)(uintptr_t)P.out32)[o] = (float)acc;
    if (P.out64)
        ((double *)(uintptr_t)P.out64)[o] = acc;
}

template <int W> static void go_marginal(const MargLaunch &L, uint32_t blocks, hipStream_t st)
{
    switch (L.plan.dr) {
    case 1: hipLaunchKernelGGL((marginal_kernel<1, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    case 2: hipLaunchKernelGGL((marginal_kernel<2, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    case 3: hipLaunchKernelGGL((marginal_kernel<3, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    case 4: hipLaunchKernelGGL((marginal_kernel<4, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    case 5: hipLaunchKernelGGL((marginal_kernel<5, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    case 6: hipLaunchKernelGGL((marginal_kernel<6, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    default: hipLaunchKernelGGL((marginal_kernel<0, W>), dim3(blocks), dim3(MARG_NT), 0, st, L.plan); break;
    }
}

hipError_t launch_marginal(const MargLaunch &L, hipStream_t st)
{
    const uint64_t total = L.plan.mode == 5   ? L.plan.nout * (L.plan.nred / 4)
                           : L.plan.mode == 4 ? L.plan.nout / 4 * L.plan.parts
                                              : L.plan.nout * L.plan.parts;
    const uint32_t blocks = (uint32_t)((total + MARG_NT - 1) / MARG_NT);
    if (L.plan.mode == 5)
        hipLaunchKernelGGL(marginal_runs_kernel, dim3(blocks), dim3(MARG_NT), 0, st, L.plan);
    else if (L.plan.mode == 4)
        hipLaunchKernelGGL(marginal_cols_kernel, dim3(blocks), dim3(MARG_NT), 0, st, L.plan);
    else if (L.plan.mode == 2)
        hipLaunchKernelGGL(marginal_inter_kernel, dim3(blocks), dim3(MARG_NT), 0, st, L.plan);
    else if (L.plan.mode == 1)
        go_marginal<4>(L, blocks, st);
    else
        go_marginal<1>(L, blocks, st);
    if (L.plan.parts >= 256) {
        hipLaunchKernelGGL(marginal_final_kernel, dim3((uint32_t)L.plan.nout), dim3(MARG_FNT), 0, st,
                           L.plan);
    } else if (L.plan.parts > 1) {
        const uint32_t fb = (uint32_t)((L.plan.nout + MARG_NT - 1) / MARG_NT);
        hipLaunchKernelGGL(marginal_final_seq_kernel, dim3(fb), dim3(MARG_NT), 0, st, L.plan);
    }
    return hipGetLastError();
}

}  // namespace triot
