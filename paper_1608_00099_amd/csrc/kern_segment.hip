// Tuple-reading row kernels for gfx950: index-weighted moments (Algorithm 11
// of the paper, read as E[t_i] of a PMF, plus the covariance of t) and their
// adjoint (the index-weighted scatter of the gradient).
//
// One thread per row segment (at most SEG_MAX consecutive elements of one
// counter row).  Inside a segment only the inner coordinate j varies, so the
// per-element work is three float64 sums,
//     r0 = sum w,  r1 = sum w*jl,  r2 = sum w*jl^2      (jl = j - j0),
// and the outer coordinates enter once per segment ("row factoring").  The
// coordinates are shifted by the centre (c_i - 1)/2 of every axis, which keeps
// the covariance free of cancellation (the shifted-data variance algorithm of
// Chan, Golub & LeVeque).  When the operands are contiguous over the counter,
// a workgroup stages its NT consecutive segments through LDS, so global
// memory sees only coalesced, lane-consecutive accesses.
//
// Partial sums are float64 per thread (on CDNA the float64 FMA issues at the
// same rate as an unpacked float32 FMA), reduced across the wave with
// shuffles, across the workgroup through LDS, and across workgroups by a
// second, one-workgroup kernel that adds the per-workgroup partials in fixed
// order with TwoSum compensation.  No float atomics: the result is
// deterministic.  Ordering that combine behind the first kernel by the
// stream, rather than by a device-scope fence in every workgroup (which on
// CDNA writes back the whole L2 of the XCD), costs one short launch.
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

#define GLOBAL __attribute__((address_space(1)))

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

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Error-free sum (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <int DMAX, bool COV>
__global__ __launch_bounds__(NT) void moments_kernel(const SegPlan P)
{
    typedef Terms<DMAX, COV> TT;
    constexpr int T = TT::T;
    __shared__ float stage[STAGE_WORDS];
    __shared__ double red[NT / 64][T];

    double acc[T];
#pragma unroll
    for (int i = 0; i < T; ++i)
        acc[i] = 0.0;

    const int D = (int)P.D;
    const double cin = P.center[D - 1];
    const uint32_t lb = seg_logical_block();
    const uint64_t g = gridDim.x;
    const uint64_t t0 = (lb * P.ntiles) / g;
    const uint64_t t1 = ((lb + 1) * P.ntiles) / g;

    // Tile geometry: NT consecutive segments, a contiguous range of nel
    // counter points starting at flat index f0.
    auto geom = [&](uint64_t tile, uint64_t &s0, uint32_t &nsg, uint64_t &f0, uint32_t &nel) {
        s0 = tile * NT;
        nsg = (uint32_t)min((uint64_t)NT, P.nseg - s0);
        const Seg first = seg_of(P, s0);
        const Seg last = seg_of(P, s0 + nsg - 1);
        f0 = seg_start(P, first);
        nel = (uint32_t)(seg_start(P, last) + last.len - f0);
    };
    // Software pipeline for contiguous operands: the weights of the next
    // tile are loaded into registers (groups of 8 independent loads, indices
    // clamped into the tile so that no load sits behind a branch) while the
    // current tile is folded from LDS.
    constexpr int PRE = SEG_MAX;  // words per thread per tile (nel <= NT * SEG_MAX)
    float pre[PRE];
    auto load_tile = [&](uint64_t f0, uint32_t nel) {
#pragma unroll
        for (int gq = 0; gq < PRE / 8; ++gq) {
            if ((uint32_t)(gq * 8 * NT) < nel) {
                uint32_t ec[8];
                const GLOBAL float *w0 = (const GLOBAL float *)(uintptr_t)P.ptr[0] + P.base[0] + f0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    ec[u] = min(threadIdx.x + (uint32_t)((gq * 8 + u) * NT), nel - 1);
                    pre[gq * 8 + u] = w0[ec[u]];
                }
                if (P.n > 1) {
#pragma unroll
                    for (int k = 1; k < 4; ++k) {
                        if (k < (int)P.n) {
                            const GLOBAL float *wk =
                                (const GLOBAL float *)(uintptr_t)P.ptr[k] + P.base[k] + f0;
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                pre[gq * 8 + u] *= wk[ec[u]];
                        }
                    }
                }
            }
        }
    };
    if (P.full && t0 < t1) {
        uint64_t s0, f0;
        uint32_t nsg, nel;
        geom(t0, s0, nsg, f0, nel);
        load_tile(f0, nel);
    }

    for (uint64_t tile = t0; tile < t1; ++tile) {
        uint64_t s0, f0;
        uint32_t nsg, nel;
        geom(tile, s0, nsg, f0, nel);
        if (P.full) {
            __syncthreads();               // the previous tile's reads are done
#pragma unroll
            for (int i = 0; i < PRE; ++i) {
                const uint32_t e = threadIdx.x + (uint32_t)(i * NT);
                if (e < nel)
                    stage[sidx(e)] = pre[i];
            }
            __syncthreads();
            if (tile + 1 < t1) {
                uint64_t s0n, f0n;
                uint32_t nsgn, neln;
                geom(tile + 1, s0n, nsgn, f0n, neln);
                load_tile(f0n, neln);      // in flight during the fold below
            }
        }
        if (threadIdx.x < nsg) {
            const Seg sg = seg_of(P, s0 + threadIdx.x);
            double u[DMAX];
            uint32_t tt[DMAX];
            row_coords<DMAX>(P, sg.row, u, tt);
            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
            if (P.full) {
                const uint32_t loc = (uint32_t)(seg_start(P, sg) - f0);
                for (uint32_t jl = 0; jl < sg.len; ++jl) {
                    const double w = (double)stage[sidx(loc + jl)];
                    const double x = (double)jl;
                    r0 += w;
                    r1 = fma(w, x, r1);
                    r2 = fma(w * x, x, r2);
                }
            } else {
                int64_t ro[4];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    ro[k] = (k < (int)P.n) ? row_offset<DMAX>(P, k, tt) : 0;
                for (uint32_t jl = 0; jl < sg.len; ++jl) {
                    const int64_t j = sg.j0 + jl;
                    float wf = 1.0f;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (k < (int)P.n)
                            wf *= ((const float *)(uintptr_t)P.ptr[k])[ro[k] + j * P.stride[k][D - 1]];
                    const double w = (double)wf;
                    const double x = (double)jl;
                    r0 += w;
                    r1 = fma(w, x, r1);
                    r2 = fma(w * x, x, r2);
                }
            }
            // inner axis: u_in = a + jl with a = j0 - centre
            const double a = (double)sg.j0 - cin;
            const double A1 = fma(a, r0, r1);                       // sum w u_in
            const double A2 = fma(a, fma(a, r0, 2.0 * r1), r2);     // sum w u_in^2
            acc[0] += r0;
            acc[TT::K + 0] += A1;
#pragma unroll
            for (int p = 1; p < DMAX; ++p)
                acc[TT::K + p] = fma(u[p], r0, acc[TT::K + p]);
            if constexpr (COV) {
                acc[TT::c(0, 0)] += A2;
#pragma unroll
                for (int p = 1; p < DMAX; ++p)
                    acc[TT::c(0, p)] = fma(u[p], A1, acc[TT::c(0, p)]);
#pragma unroll
                for (int q = 1; q < DMAX; ++q) {
                    const double uq = u[q] * r0;
#pragma unroll
                    for (int p = 1; p <= q; ++p)
                        acc[TT::c(p, q)] = fma(u[p], uq, acc[TT::c(p, q)]);
                }
            }
        }
    }

    // ---- workgroup reduction (fixed order) ----
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        double v = wave_sum(acc[i]);
        if (lane == 0)
            red[wave][i] = v;
    }
    __syncthreads();
    // Partials are term-major (term i of block b at i * nblocks + b) so the
    // combining workgroup reads them with coalesced loads.
    double *partials = (double *)((char *)(uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    for (int i = threadIdx.x; i < T; i += NT) {
        double v = red[0][i];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w)
            v += red[w][i];
        partials[(size_t)i * nb + blockIdx.x] = v;
    }
}

// Combines the per-workgroup partials of moments_kernel (one workgroup,
// launched right after it on the same stream: the kernel boundary makes
// every partial visible without a device-wide cache write-back per block)
// and writes [M, E, C] in the caller's layout.
template <int DMAX, bool COV>
__global__ __launch_bounds__(NT) void moments_final_kernel(const SegPlan P)
{
    typedef Terms<DMAX, COV> TT;
    constexpr int T = TT::T;
    __shared__ double red[NT / 64][T];
    __shared__ double rc[NT / 64][T];
    __shared__ double tot[T];
    __shared__ int pos_of[MAXD];
    const int D = (int)P.D;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double *partials = (const double *)((const char *)(uintptr_t)P.ws + 256);
    const uint32_t nb = P.nblocks;
    // Every thread folds blocks tid, tid + NT, ... of every term into a
    // compensated (sum, error) pair; the pairs then meet in a fixed tree:
    // lanes by xor-shuffles, waves in index order.  Deterministic.
    constexpr int CH = 8;  // terms reduced together (bounds the registers)
    constexpr int TP = (T + CH - 1) / CH * CH;  // workspace rows (padded)
#pragma unroll
    for (int i0 = 0; i0 < TP; i0 += CH) {
        double ls[CH], lc[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            ls[q] = 0.0;
            lc[q] = 0.0;
        }
        for (uint32_t b0 = 0; b0 < nb; b0 += NT) {
            // unconditional loads (clamped block index), then a select
            const uint32_t b = b0 + threadIdx.x;
            const bool ok = b < nb;
            const uint32_t bc = ok ? b : 0u;
            double v[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q)
                v[q] = partials[(size_t)(i0 + q) * nb + bc];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                double e;
                two_sum(ls[q], ok ? v[q] : 0.0, ls[q], e);
                lc[q] += e;
            }
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int i = i0 + q;
            if (i >= T)
                break;
            double s = ls[q], c = lc[q];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double so = __shfl_xor(s, o, 64);
                const double co = __shfl_xor(c, o, 64);
                double e;
                // (lower lane first) keeps both lanes of a pair bit-identical
                if (lane & o)
                    two_sum(so, s, s, e);
                else
                    two_sum(s, so, s, e);
                c = (lane & o) ? (co + c) + e : (c + co) + e;
            }
            if (lane == 0) {
                red[wave][i] = s;
                rc[wave][i] = c;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < T; i += NT) {
        double s = red[0][i], c = rc[0][i];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            double e;
            two_sum(s, red[w][i], s, e);
            c = (c + rc[w][i]) + e;
        }
        tot[i] = s + c;
    }
    if (threadIdx.x < MAXD)
        pos_of[threadIdx.x] = -1;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int p = 0; p < D; ++p) {
            uint32_t o = P.orig[D - 1 - p];
            if (o != 0xFFFFFFFFu)
                pos_of[o] = p;
        }
    }
    __syncthreads();
    const int d = (int)P.d_orig;
    const bool cov = (P.flags & TRIOT_MOMENTS_COV) != 0;
    const int nout = 1 + d + (cov ? d * (d + 1) / 2 : 0);
    const double M = tot[0];
    float *out32 = (float *)(uintptr_t)P.out32;
    double *out64 = (double *)(uintptr_t)P.out64;
    for (int o = threadIdx.x; o < nout; o += NT) {
        double v;
        if (o == 0) {
            v = M;
        } else if (o <= d) {
            const int i = o - 1;
            const int p = pos_of[i];
            v = (p < 0) ? 0.0 / M : P.center[D - 1 - p] + tot[TT::K + p] / M;
        } else {
            // o -> (i, j), i <= j, in the row-major upper triangle
            int r = o - 1 - d, i = 0;
            while (r >= d - i) {
                r -= d - i;
                ++i;
            }
            const int j = i + r;
            const int p = pos_of[i], q = pos_of[j];
            if (p < 0 || q < 0) {
                v = 0.0 / M;
            } else {
                const int lo = p < q ? p : q, hi = p < q ? q : p;
                const double ei = tot[TT::K + p] / M, ej = tot[TT::K + q] / M;
                v = COV ? tot[TT::c(lo, hi)] / M - ei * ej : 0.0;
            }
        }
        out32[o] = (float)v;
        if (out64)
            out64[o] = v;
    }
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

hipError_t launch_moments(const SegLaunch &L, hipStream_t st)
{
    const bool cov = (L.plan.flags & TRIOT_MOMENTS_COV) != 0;
    if (cov) {
        hipLaunchKernelGGL((moments_kernel<8, true>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        hipLaunchKernelGGL((moments_final_kernel<8, true>), dim3(1), dim3(NT), 0, st, L.plan);
    } else if (L.dmax <= 8) {
        hipLaunchKernelGGL((moments_kernel<8, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        hipLaunchKernelGGL((moments_final_kernel<8, false>), dim3(1), dim3(NT), 0, st, L.plan);
    } else {
        hipLaunchKernelGGL((moments_kernel<32, false>), dim3(L.blocks), dim3(NT), 0, st, L.plan);
        hipLaunchKernelGGL((moments_final_kernel<32, false>), dim3(1), dim3(NT), 0, st, L.plan);
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

// Resident workgroups per CU of the row kernels (their register and LDS
// needs differ by tier), asked of the runtime once; 2 when no device answers.
int segment_blocks_per_cu(bool adj, bool cov, int dmax)
{
    static int cache[2][2][2] = {};
    const int a = adj ? 1 : 0, c = cov ? 1 : 0, m = dmax > 8 ? 1 : 0;
    if (!cache[a][c][m]) {
        int nb = 0;
        hipError_t e;
        if (!adj) {
            if (cov)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, moments_kernel<8, true>, NT, 0);
            else if (dmax <= 8)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, moments_kernel<8, false>, NT, 0);
            else
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, moments_kernel<32, false>, NT, 0);
        } else {
            if (cov)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, moments_adj_kernel<8, true>, NT, 0);
            else if (dmax <= 8)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, moments_adj_kernel<8, false>, NT,
                                                                 0);
            else
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, moments_adj_kernel<32, false>,
                                                                 NT, 0);
        }
        cache[a][c][m] = (e == hipSuccess && nb > 0) ? nb : 2;
    }
    return cache[a][c][m];
}

}  // namespace triot
