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

#include "common.h"
#include "launch.h"

namespace triot {

#define GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ uint32_t rdiv_u32(uint32_t n, const AxisDiv &a)
{
    uint32_t h = __umulhi(n, a.m);
    return (h + ((n - h) >> 1)) >> a.s;
}

constexpr int CONV_NT = 256;
constexpr uint32_t CONV_LDS_WORDS = 8192;   // float64 words of LDS staging (64 KiB)

template <bool LDS>
__global__ __launch_bounds__(CONV_NT) void conv_kernel(const ConvPlan P)
{
    extern __shared__ double sm[];
    const GLOBAL double *gl = (const GLOBAL double *)(uintptr_t)P.lhs;
    const GLOBAL double *gr = (const GLOBAL double *)(uintptr_t)P.rhs;
    if (LDS) {
        for (uint32_t i = threadIdx.x; i < P.nl; i += CONV_NT)
            sm[i] = gl[i];
        for (uint32_t i = threadIdx.x; i < P.nr; i += CONV_NT)
            sm[P.nl + i] = gr[i];
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
        const int64_t ls_in = P.lstride[in], rs_in = P.rstride[in];
        const uint32_t nin = hi[in] - lo[in] + 1;
        while (true) {
            // innermost axis: lhs index up by one, rhs index down by one
            int64_t li = lrow, ri = rrow;
            for (uint32_t k = 0; k < nin; ++k) {
                const double prod = L[li] * R[ri];
                acc = acc + prod;
                li += ls_in;
                ri -= rs_in;
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

hipError_t launch_conv(const ConvLaunch &L, hipStream_t st)
{
    const uint32_t blocks = (uint32_t)((L.plan.nout + CONV_NT - 1) / CONV_NT);
    if (L.plan.lds) {
        const size_t bytes = (size_t)(L.plan.nl + L.plan.nr) * sizeof(double);
        hipLaunchKernelGGL((conv_kernel<true>), dim3(blocks), dim3(CONV_NT), bytes, st, L.plan);
    } else {
        hipLaunchKernelGGL((conv_kernel<false>), dim3(blocks), dim3(CONV_NT), 0, st, L.plan);
    }
    return hipGetLastError();
}

uint32_t conv_lds_words() { return CONV_LDS_WORDS; }

// ---------------------------------------------------------------------
// Marginalization
// ---------------------------------------------------------------------
constexpr int MARG_NT = 256;

__global__ __launch_bounds__(MARG_NT) void marginal_kernel(const MargPlan P)
{
    const uint64_t gid = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    const uint64_t total = P.nout * P.parts;
    if (gid >= total)
        return;
    const uint32_t o = (uint32_t)(gid % P.nout);
    const uint32_t p = (uint32_t)(gid / P.nout);
    const int n = (int)P.n, dk = (int)P.dk, dr = (int)P.dr;
    int64_t off[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        off[k] = P.base[k];
    // kept tuple o
    {
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
    // part p of the reduced sub-box: flat range [r0, r1)
    const uint64_t r0 = (uint64_t)p * P.nred / P.parts;
    const uint64_t r1 = (uint64_t)(p + 1) * P.nred / P.parts;
    uint32_t t[MAXD];
    {
        uint64_t q = r0;
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
    double acc = 0.0;
    for (uint64_t r = r0; r < r1; ++r) {
        double w = 1.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < n)
                w *= (double)((const GLOBAL float *)(uintptr_t)P.ptr[k])[off[k]];
        acc += w;
        // advance the odometer over the reduced axes
        for (int i = dr - 1; i >= 0; --i) {
            if (++t[i] < P.rax[i].c || i == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < n)
                        off[k] += P.rstride[k][i];
                break;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < n)
                    off[k] -= (int64_t)(t[i] - 1) * P.rstride[k][i];
            t[i] = 0;
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

__global__ __launch_bounds__(MARG_NT) void marginal_final_kernel(const MargPlan P)
{
    const uint64_t o = (uint64_t)blockIdx.x * MARG_NT + threadIdx.x;
    if (o >= P.nout)
        return;
    const double *part = (const double *)((const char *)(uintptr_t)P.ws + 256) + o * P.parts;
    double acc = 0.0;
    for (uint32_t p = 0; p < P.parts; ++p)
        acc += part[p];
    ((float *)(uintptr_t)P.out32)[o] = (float)acc;
    if (P.out64)
        ((double *)(uintptr_t)P.out64)[o] = acc;
}

hipError_t launch_marginal(const MargLaunch &L, hipStream_t st)
{
    const uint64_t total = L.plan.nout * L.plan.parts;
    const uint32_t blocks = (uint32_t)((total + MARG_NT - 1) / MARG_NT);
    hipLaunchKernelGGL(marginal_kernel, dim3(blocks), dim3(MARG_NT), 0, st, L.plan);
    if (L.plan.parts > 1) {
        const uint32_t fb = (uint32_t)((L.plan.nout + MARG_NT - 1) / MARG_NT);
        hipLaunchKernelGGL(marginal_final_kernel, dim3(fb), dim3(MARG_NT), 0, st, L.plan);
    }
    return hipGetLastError();
}

}  // namespace triot
