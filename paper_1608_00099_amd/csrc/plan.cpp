// Host planner: one validation pass over shapes per call (Section 4: the
// bounds are checked once for the whole shapes, never per index), then the
// launch plan -- dropped and merged axes, vector width, the box split and
// the magic-division tables of the kernels.
#include "plan.h"

#include <hip/hip_runtime.h>

#include "launch.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace triot {

bool magic_for(uint32_t c, AxisDiv *out)
{
    if (c < 2)
        return false;
    uint32_t l = 0;
    while ((uint64_t(1) << l) < c)
        ++l;                                   // l = ceil(log2 c), 1..32
    uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - c)) / c + 1;
    out->c = c;
    out->m = (uint32_t)m;
    out->s = l - 1;
    out->pad = 0;
    return true;
}

static AxisDiv trivial_div()
{
    AxisDiv a;
    a.c = 1;
    a.m = 0;
    a.s = 0;
    a.pad = 0;
    return a;
}

int device_cus()
{
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    std::lock_guard<std::mutex> g(mu);
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

bool is_segment_op(triot_op op)
{
    return op == TRIOT_OP_MOMENTS || op == TRIOT_OP_MOMENTS_ADJ || op == TRIOT_OP_DOT ||
           op == TRIOT_OP_BBOX;
}

// Checked arithmetic on non-negative int64 values.
static bool mul_ok(int64_t a, int64_t b, int64_t *r)
{
    if (a == 0 || b == 0) {
        *r = 0;
        return true;
    }
    if (a > INT64_MAX / b)
        return false;
    *r = a * b;
    return true;
}

static bool add_ok(int64_t a, int64_t b, int64_t *r)
{
    if (a > INT64_MAX - b)
        return false;
    *r = a + b;
    return true;
}

// Which operands are read or written only where the tuple lies inside a
// window (the rest must contain the whole counter), and which window.
// role[k] = -1: must contain the counter; role[k] = j: predicated by
// operand j's window extents.
static void roles(triot_op op, int n, int role[MAXT])
{
    for (int k = 0; k < MAXT; ++k)
        role[k] = -1;
    if (op == TRIOT_OP_EMBED_FILL) {
        role[1] = 1;
    } else if (op == TRIOT_OP_MUL_ADJ) {
        role[0] = 0;   // ga: its own window
        role[1] = 1;   // gb: its own window
        role[2] = 2;   // gout, a, b: the intersection (gout's window)
        role[3] = 2;
        role[4] = 2;
    }
    (void)n;
}

static bool is_output(triot_op op, int k)
{
    switch (op) {
    case TRIOT_OP_COPY:
    case TRIOT_OP_EMBED_FILL:
    case TRIOT_OP_MUL_ACC:
    case TRIOT_OP_MUL:
    case TRIOT_OP_MOMENTS_ADJ:
    case TRIOT_OP_XPYX_MZ:
    case TRIOT_OP_CONV:
        return k == 0;
    case TRIOT_OP_MUL_ADJ:
        return k == 0 || k == 1;
    default:
        return false;
    }
}

triot_status validate(triot_op op, int n, int d, const int64_t *shapes, const int64_t *counter,
                      void *const *tensors, const int64_t *bases, const void *params, Request *r)
{
    std::memset(r, 0, sizeof(*r));
    if ((int)op < 0 || (int)op > (int)TRIOT_OP_CONV)
        return TRIOT_E_INVALID;
    bool n_ok = false;
    switch (op) {
    case TRIOT_OP_COPY:
    case TRIOT_OP_EMBED_FILL: n_ok = (n == 2); break;
    case TRIOT_OP_MUL_ACC:
    case TRIOT_OP_MUL:
    case TRIOT_OP_XPYX_MZ:
    case TRIOT_OP_CONV: n_ok = (n == 3); break;
    case TRIOT_OP_MOMENTS:
    case TRIOT_OP_DOT:
    case TRIOT_OP_MARGINAL:
    case TRIOT_OP_BBOX: n_ok = (n >= 1 && n <= 4); break;
    case TRIOT_OP_MOMENTS_ADJ: n_ok = (n == 1); break;
    case TRIOT_OP_MUL_ADJ: n_ok = (n == 5); break;
    case TRIOT_OP_INDEX: n_ok = (n >= 1 && n <= MAXT); break;
    }
    if (!n_ok)
        return TRIOT_E_INVALID;
    if (d < 0 || d > MAXD)
        return TRIOT_E_DIM;
    if ((d > 0 && !shapes) || !tensors)
        return TRIOT_E_INVALID;
    r->op = op;
    r->n = n;
    r->d = d;
    r->params = params;
    r->elem_bytes = 4;
    if (op == TRIOT_OP_COPY || op == TRIOT_OP_EMBED_FILL) {
        if (params) {
            int eb = ((const triot_copy_params *)params)->elem_bytes;
            if (eb != 4 && eb != 8)
                return TRIOT_E_INVALID;
            r->elem_bytes = eb;
        }
    } else if (op == TRIOT_OP_INDEX) {
        r->elem_bytes = 8;  // int64 output; operands carry no data
    } else if (op == TRIOT_OP_MOMENTS) {
        if (params) {
            int f = ((const triot_moments_params *)params)->flags;
            if (f & ~(TRIOT_MOMENTS_FIRST | TRIOT_MOMENTS_COV | TRIOT_MOMENTS_CACHED))
                return TRIOT_E_INVALID;
        }
    } else if (op == TRIOT_OP_MOMENTS_ADJ) {
        if (!params)
            return TRIOT_E_INVALID;
        int f = ((const triot_moments_adj_params *)params)->flags;
        if (f & ~(TRIOT_MOMENTS_FIRST | TRIOT_MOMENTS_COV))
            return TRIOT_E_INVALID;
    } else if (op == TRIOT_OP_MARGINAL) {
        if (!params)
            return TRIOT_E_INVALID;
        uint32_t km = ((const triot_marginal_params *)params)->keep_mask;
        if (d < 32 && (km >> d) != 0)
            return TRIOT_E_INVALID;
    } else if (op == TRIOT_OP_CONV) {
        r->elem_bytes = 8;
        if (bases)
            for (int k = 0; k < n; ++k)
                if (bases[k] != 0)
                    return TRIOT_E_UNSUPPORTED;
        // out = lhs + rhs - 1 on every axis, inputs non-empty
        for (int i = 0; i < d; ++i) {
            const int64_t so = shapes[i], sl = shapes[d + i], sr = shapes[2 * (size_t)d + i];
            if (sl < 1 || sr < 1 || so != sl + sr - 1)
                return TRIOT_E_BOUNDS;
            if (counter && counter[i] != so)
                return TRIOT_E_INVALID;
        }
    }

    int64_t total[MAXT];
    for (int k = 0; k < n; ++k) {
        int64_t t = 1;
        for (int i = 0; i < d; ++i) {
            int64_t s = shapes[(size_t)k * d + i];
            if (s < 0)
                return TRIOT_E_INVALID;
            r->shape[k][i] = s;
            if (!mul_ok(t, s, &t))
                return TRIOT_E_OVERFLOW;
        }
        int64_t bytes;
        if (!mul_ok(t, (int64_t)r->elem_bytes, &bytes) || bytes > (INT64_MAX >> 2))
            return TRIOT_E_OVERFLOW;
        total[k] = t;
        int64_t b = bases ? bases[k] : 0;
        if (b < 0 || (t > 0 && b >= t) || (t == 0 && b != 0))
            return TRIOT_E_BOUNDS;
        r->base[k] = b;
        r->ptr[k] = tensors[k];
    }

    // Window start tuple and available extents of every operand.
    int64_t avail[MAXT][MAXD];
    for (int k = 0; k < n; ++k) {
        int64_t f = r->base[k];
        for (int i = d - 1; i >= 0; --i) {
            int64_t s = r->shape[k][i];
            int64_t digit = s ? f % s : 0;
            f = s ? f / s : 0;
            avail[k][i] = s - digit;
        }
    }

    // Counter: explicit, or the op's default.
    for (int i = 0; i < d; ++i) {
        int64_t c;
        if (counter) {
            c = counter[i];
            if (c < 0)
                return TRIOT_E_INVALID;
        } else if (op == TRIOT_OP_EMBED_FILL || op == TRIOT_OP_MOMENTS_ADJ ||
                   op == TRIOT_OP_CONV) {
            c = avail[0][i];
        } else if (op == TRIOT_OP_MUL_ADJ) {
            c = std::max(avail[0][i], avail[1][i]);
        } else {
            c = avail[0][i];
            for (int k = 1; k < n; ++k)
                c = std::min(c, avail[k][i]);
        }
        r->counter[i] = c;
    }
    int64_t np = 1;
    for (int i = 0; i < d; ++i)
        if (!mul_ok(np, r->counter[i], &np))
            return TRIOT_E_OVERFLOW;
    r->npoints = np;

    int role[MAXT];
    roles(op, n, role);
    if (op == TRIOT_OP_CONV) {
        // The counter is the output shape; the inputs are read whole.
        if (np == 0)
            return TRIOT_OK;
        for (int k = 0; k < n; ++k)
            if (!tensors[k])
                return TRIOT_E_INVALID;
        uint64_t lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = (uint64_t)(uintptr_t)tensors[k];
            hi[k] = lo[k] + (uint64_t)total[k] * 8;
        }
        for (int k = 1; k < 3; ++k)
            if (lo[0] < hi[k] && lo[k] < hi[0])
                return TRIOT_E_ALIAS;
        return TRIOT_OK;
    }
    for (int k = 0; k < n; ++k) {
        if (role[k] >= 0)
            continue;
        for (int i = 0; i < d; ++i)
            if (r->counter[i] > avail[k][i])
                return TRIOT_E_BOUNDS;
    }
    if (op == TRIOT_OP_MUL_ADJ) {
        // The intersection (gout's window) must lie inside a's and b's.
        for (int i = 0; i < d; ++i)
            if (avail[2][i] > avail[3][i] || avail[2][i] > avail[4][i])
                return TRIOT_E_BOUNDS;
    }
    if (np == 0)
        return TRIOT_OK;

    for (int k = 0; k < n; ++k) {
        if (op == TRIOT_OP_INDEX && k > 0)
            continue;
        if (!tensors[k])
            return TRIOT_E_INVALID;
    }
    if (op == TRIOT_OP_INDEX) {
        int64_t outb;
        if (!mul_ok(np, (int64_t)n * 8, &outb))
            return TRIOT_E_OVERFLOW;
    }
    if (op == TRIOT_OP_MOMENTS_ADJ) {
        const triot_moments_adj_params *p = (const triot_moments_adj_params *)params;
        if (!p->mom || !p->gmom)
            return TRIOT_E_INVALID;
    }

    // Aliasing: byte range touched by each operand over the counter.
    if (op != TRIOT_OP_INDEX && op != TRIOT_OP_MOMENTS && op != TRIOT_OP_DOT &&
        op != TRIOT_OP_MARGINAL && op != TRIOT_OP_BBOX) {
        uint64_t lo[MAXT], hi[MAXT];
        int64_t eb = (op == TRIOT_OP_COPY || op == TRIOT_OP_EMBED_FILL) ? r->elem_bytes : 4;
        for (int k = 0; k < n; ++k) {
            int64_t span = 0;
            bool empty = false;
            for (int i = 0; i < d; ++i) {
                int64_t ext = r->counter[i];
                if (role[k] >= 0)
                    ext = std::min(ext, avail[role[k]][i]);
                if (ext <= 0) {
                    empty = true;
                    break;
                }
                int64_t stride = 1;
                for (int j = i + 1; j < d; ++j)
                    stride *= r->shape[k][j];
                span += (ext - 1) * stride;
            }
            uint64_t p = (uint64_t)(uintptr_t)tensors[k];
            lo[k] = p + (uint64_t)r->base[k] * eb;
            hi[k] = empty ? lo[k] : lo[k] + (uint64_t)(span + 1) * eb;
            r->span_lo[k] = lo[k];
            r->span_hi[k] = hi[k];
            r->written[k] = is_output(op, k);
        }
        for (int o = 0; o < n; ++o) {
            if (!is_output(op, o))
                continue;
            for (int k = 0; k < n; ++k) {
                if (k == o || lo[o] == hi[o] || lo[k] == hi[k])
                    continue;
                bool overlap = lo[o] < hi[k] && lo[k] < hi[o];
                if (!overlap)
                    continue;
                bool same_view = tensors[o] == tensors[k] && r->base[o] == r->base[k] &&
                                 std::memcmp(r->shape[o], r->shape[k], sizeof(int64_t) * d) == 0;
                if (!same_view || is_output(op, k))
                    return TRIOT_E_ALIAS;
            }
        }
    }
    (void)total;
    return TRIOT_OK;
}

// ---------------------------------------------------------------------
// Element-wise plan
// ---------------------------------------------------------------------

struct Ax {
    int64_t c;
    int64_t S[MAXT];  // element (word) strides
    int64_t B[MAXT];  // predicate extent, -1 when it can never fail
};

triot_status plan_coiter(const Request &r, const Sched &s, int cus, CoLaunch *out)
{
    std::memset(out, 0, sizeof(*out));
    CoPlan &P = out->plan;
    const int n = r.n, d = r.d;
    int role[MAXT];
    roles(r.op, n, role);

    // Window extents again (predicate bounds).
    int64_t avail[MAXT][MAXD];
    for (int k = 0; k < n; ++k) {
        int64_t f = r.base[k];
        for (int i = d - 1; i >= 0; --i) {
            int64_t sz = r.shape[k][i];
            int64_t digit = sz ? f % sz : 0;
            f = sz ? f / sz : 0;
            avail[k][i] = sz - digit;
        }
    }

    // 1. Logical axes with their strides; drop extent-1 axes.
    Ax ax[MAXD + 1];
    int na = 0;
    for (int i = 0; i < d; ++i) {
        if (r.counter[i] == 1)
            continue;
        Ax a;
        a.c = r.counter[i];
        for (int k = 0; k < n; ++k) {
            int64_t st = 1;
            for (int j = i + 1; j < d; ++j)
                st *= r.shape[k][j];
            a.S[k] = st;
            int64_t b = -1;
            if (role[k] >= 0 && avail[role[k]][i] < a.c)
                b = avail[role[k]][i];
            a.B[k] = b;
        }
        ax[na++] = a;
    }
    int64_t base[MAXT];
    for (int k = 0; k < n; ++k)
        base[k] = r.base[k];

    // 2. 8-byte elements move as two 4-byte words: a trailing word axis.
    const bool words2 = (r.op == TRIOT_OP_COPY || r.op == TRIOT_OP_EMBED_FILL) && r.elem_bytes == 8;
    if (words2) {
        for (int i = 0; i < na; ++i)
            for (int k = 0; k < n; ++k)
                ax[i].S[k] *= 2;
        for (int k = 0; k < n; ++k)
            base[k] *= 2;
        Ax w;
        w.c = 2;
        for (int k = 0; k < n; ++k) {
            w.S[k] = 1;
            w.B[k] = -1;
        }
        ax[na++] = w;
    }
    if (na == 0) {  // a scalar: one point
        Ax a;
        a.c = 1;
        for (int k = 0; k < n; ++k) {
            a.S[k] = 1;
            a.B[k] = -1;
        }
        ax[na++] = a;
    }

    // 3. Merge adjacent axes where every operand is contiguous across them
    //    and the inner one carries no live predicate (INDEX and the
    //    element-wise ops only read addresses, never the tuple).
    Ax m[MAXD + 1];
    int nm = 0;
    m[MAXD] = ax[na - 1];
    int front = MAXD;
    for (int i = na - 2; i >= 0; --i) {
        Ax &b = m[front];
        const Ax &a = ax[i];
        bool ok = true;
        for (int k = 0; k < n && ok; ++k) {
            int64_t want;
            if (b.B[k] != -1 || !mul_ok(b.c, b.S[k], &want) || a.S[k] != want)
                ok = false;
        }
        int64_t merged_c;
        if (ok && mul_ok(a.c, b.c, &merged_c)) {
            Ax c;
            c.c = merged_c;
            for (int k = 0; k < n; ++k) {
                c.S[k] = b.S[k];
                c.B[k] = a.B[k] == -1 ? -1 : a.B[k] * b.c;
            }
            m[front] = c;
        } else {
            m[--front] = a;
        }
    }
    for (int i = front; i <= MAXD; ++i)
        m[nm++] = m[i];
    const int D = nm;

    // 4. Vector width: every operand contiguous on the inner axis, and the
    //    inner extent and every inner window bound a multiple of the width,
    //    so that a vector never straddles two rows.  Addresses need only be
    //    4-byte aligned: multi-dword global accesses take any dword address
    //    on CDNA.  Strides and bases stay in 4-byte words.
    //    Ragged rows (an inner extent of at least 2 widths that is not a
    //    multiple of the width) still take the width when the op reads and
    //    writes every operand on the whole counter (no window predicates):
    //    each row's last vector is moved back to end at the row end, reads
    //    words of the vector before it again and stores only its new words.
    //    EMBED_FILL also takes ragged rows (its destination is the counter,
    //    stored whole like COPY's) and a source inner bound at any element:
    //    the kernel loads a vector that straddles it word by word.
    const Ax &in = m[D - 1];
    const bool fill_el = r.op == TRIOT_OP_EMBED_FILL && in.c < (int64_t(1) << 31);
    const bool ragged_ok = r.op == TRIOT_OP_COPY || r.op == TRIOT_OP_MUL_ACC ||
                           r.op == TRIOT_OP_MUL || r.op == TRIOT_OP_XPYX_MZ || fill_el;
    int vec = 1;
    int64_t rtail = 0;   // words in a row's last vector (0: whole vectors)
    if (r.op != TRIOT_OP_INDEX) {
        for (int v = std::min(4, std::max(1, s.vec_max)); v > 1; v >>= 1) {
            if (v == 2 && s.no_vec2)
                continue;
            const bool whole = (in.c % v) == 0 && in.c / v >= 2;
            const bool rag = !whole && ragged_ok && in.c > v;
            bool ok = whole || rag;
            for (int k = 0; k < n && ok; ++k) {
                if (in.S[k] != 1 || ((uintptr_t)r.ptr[k] % 4) != 0)
                    ok = false;
                if (in.B[k] != -1 && !fill_el && (rag || in.B[k] % v != 0))
                    ok = false;
            }
            if (ok) {
                vec = v;
                rtail = whole ? 0 : in.c % v;
                break;
            }
        }
    }
    const int64_t L = (in.c + vec - 1) / vec;
    const uint32_t esz = 4u * vec;
    if (L >= (int64_t(1) << 32))
        return TRIOT_E_UNSUPPORTED;
    for (int i = 0; i < D - 1; ++i)
        if (m[i].c >= (int64_t(1) << 32))
            return TRIOT_E_UNSUPPORTED;

    int64_t is[MAXT];
    for (int k = 0; k < n; ++k)
        is[k] = (in.S[k] == 1 && vec > 1) ? 1 : in.S[k];  // in vector units
    bool unit = true;
    for (int k = 0; k < n; ++k)
        if (is[k] != 1)
            unit = false;
    if ((int64_t)is[0] >= (int64_t(1) << 31))
        return TRIOT_E_UNSUPPORTED;
    for (int k = 0; k < n; ++k)
        if (is[k] * (int64_t)esz >= (int64_t(1) << 31))
            return TRIOT_E_UNSUPPORTED;

    // 5. Box: the fewest low axes whose rows reach the unit size, within the
    //    LDS table, the exact range of the row magic and 31-bit offsets.
    //    If the box is still short of a unit, the next axis is split: its
    //    lower m digits join the box, its blocks of m digits become a high
    //    axis (the last block being a shorter prefix of the box).
    const int nouter = D - 1;
    const int rb_cap = std::max(1, std::min(s.rb_max, RB_MAX));
    // Work-unit size: the schedule's, but small problems get smaller units
    // so that there are at least about 4 per CU (never below one tile of
    // NT * 4 vectors).
    int64_t pe_target = s.pe_target;
    {
        int64_t nvec = L;
        for (int i = 0; i < nouter; ++i)
            nvec = (nvec > (int64_t(1) << 40) / m[i].c) ? (int64_t(1) << 40) : nvec * m[i].c;
        const int64_t want = nvec / ((int64_t)cus * 4);
        if (s.small_units && want < pe_target)
            pe_target = std::max<int64_t>(NT * 4, want / (NT * 4) * (NT * 4));
    }
    // Does a box of the full low axes [first, nouter) plus mm digits of
    // axis `split_axis` (or none) satisfy the magic and offset limits?
    auto fits = [&](int first, int split_axis, int64_t mm, int64_t rows) -> bool {
        if ((unsigned __int128)rows * L * L > ((unsigned __int128)1 << 32))
            return false;
        for (int k = 0; k < n; ++k) {
            // byte span of one box in operand k (inner rows in vectors,
            // outer strides in words)
            __int128 span = (__int128)(L - 1) * is[k] * esz;
            for (int j = first; j < nouter; ++j)
                span += (__int128)(m[j].c - 1) * m[j].S[k] * 4;
            if (split_axis >= 0)
                span += (__int128)(mm - 1) * m[split_axis].S[k] * 4;
            if (span + esz >= ((__int128)1 << 31))
                return false;
        }
        return true;
    };
    int nfull = 0;
    int64_t RB = 1;
    for (int i = nouter - 1; i >= 0; --i) {
        if (RB * L >= pe_target)
            break;
        int64_t rb2 = RB * m[i].c;
        if (rb2 > rb_cap || !fits(i, -1, 1, rb2))
            break;
        RB = rb2;
        nfull++;
    }
    const int a = nouter - 1 - nfull;  // next axis, candidate for the split
    int64_t mm = 1;
    if (a >= 0 && RB * L < pe_target) {
        int64_t want = (pe_target + RB * L - 1) / (RB * L);
        mm = std::min<int64_t>({m[a].c - 1, want, (int64_t)rb_cap / RB});
        while (mm >= 2 && !fits(a + 1, a, mm, RB * mm))
            mm /= 2;
    }
    const bool split = mm >= 2;
    const int64_t rows_below = RB;
    if (split)
        RB *= mm;

    // Outer axes of the kernel: [0, a) unchanged, then (split) the block
    // axis and the digit axis, then the full low axes.
    struct KAx {
        int64_t c;
        int64_t S[MAXT];
        int64_t B[MAXT];
    };
    KAx kx[MAXD + 1];
    int nk = 0;
    const int first_low = split ? a : a + 1;
    for (int i = 0; i < first_low; ++i) {
        kx[nk].c = m[i].c;
        for (int k = 0; k < n; ++k) {
            kx[nk].S[k] = m[i].S[k];
            kx[nk].B[k] = m[i].B[k];
        }
        nk++;
    }
    if (split) {
        KAx hi, lo;
        hi.c = (m[a].c + mm - 1) / mm;
        lo.c = mm;
        for (int k = 0; k < n; ++k) {
            hi.S[k] = m[a].S[k] * mm;
            lo.S[k] = m[a].S[k];
            hi.B[k] = -1;   // the split axis' window bound is applied per box
            lo.B[k] = -1;
        }
        kx[nk++] = hi;
        kx[nk++] = lo;
    }
    for (int i = a + 1; i < nouter; ++i) {
        kx[nk].c = m[i].c;
        for (int k = 0; k < n; ++k) {
            kx[nk].S[k] = m[i].S[k];
            kx[nk].B[k] = m[i].B[k];
        }
        nk++;
    }
    const int nlow = nfull + (split ? 1 : 0);
    const int nhigh = nk - nlow;
    int64_t nboxes = 1;
    for (int i = 0; i < nhigh; ++i)
        nboxes *= kx[i].c;
    if (nboxes >= (int64_t(1) << 32))
        return TRIOT_E_UNSUPPORTED;
    for (int i = 0; i < nk; ++i)
        if (kx[i].c >= (int64_t(1) << 32))
            return TRIOT_E_UNSUPPORTED;

    int64_t BE = RB * L;
    int64_t pe_cap = pe_target;
    if (RB == 1) {
        for (int k = 0; k < n; ++k)
            pe_cap = std::min<int64_t>(pe_cap, ((int64_t(1) << 31) / ((int64_t)esz * is[k])) - 2);
    }
    pe_cap = std::max<int64_t>(pe_cap, 1);
    int64_t parts = (BE + pe_cap - 1) / pe_cap;
    int64_t PE = (BE + parts - 1) / parts;
    int64_t nunits = nboxes * parts;
    if (nunits >= (int64_t(1) << 32) || BE >= (int64_t(1) << 32))
        return TRIOT_E_UNSUPPORTED;

    // 6. The kernel argument.
    P.D = (uint32_t)(nk + 1);
    P.n = (uint32_t)n;
    P.nhigh = (uint32_t)nhigh;
    P.nlow = (uint32_t)nlow;
    P.L = (uint32_t)L;
    P.Lm = (RB > 1) ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)L - 1) / (uint64_t)L) : 0;
    P.RB = (uint32_t)RB;
    P.BE = (uint32_t)BE;
    P.parts = (uint32_t)parts;
    P.PE = (uint32_t)PE;
    if (parts > 1)
        magic_for((uint32_t)parts, &P.partdiv);
    else
        P.partdiv = trivial_div();
    P.nunits = (uint32_t)nunits;
    P.esz = esz;
    P.vec = (uint32_t)vec;
    P.tskip = rtail ? (uint32_t)(vec - rtail) : 0u;
    P.tshift = P.tskip * 4u;
    P.unit = unit ? 1u : 0u;
    P.interleave = s.order ? 1u : 0u;
    P.split = split ? 1u : 0u;
    P.sm = split ? (uint32_t)mm : 1u;
    P.sc = split ? (uint32_t)m[a].c : 1u;
    P.rows_below = (uint32_t)rows_below;
    uint32_t predmask = 0;
    for (int k = 0; k < n; ++k) {
        P.sbound[k] = NOBOUND;
        if (split && m[a].B[k] >= 0) {
            P.sbound[k] = (uint32_t)m[a].B[k];
            predmask |= 1u << k;
        }
    }
    for (int i = 0; i < nk; ++i) {
        if (kx[i].c >= 2)
            magic_for((uint32_t)kx[i].c, &P.ax[i]);
        else
            P.ax[i] = trivial_div();
        for (int k = 0; k < n; ++k) {
            P.stride[k][i] = kx[i].S[k];
            if (kx[i].B[k] >= 0) {
                P.bound[k][i] = (uint32_t)kx[i].B[k];
                predmask |= 1u << k;
            } else {
                P.bound[k][i] = NOBOUND;
            }
        }
    }
    // Counter flat stride of each high axis (the INDEX output position).
    {
        int64_t below = BE;   // elements of one full box
        for (int i = nhigh - 1; i >= 0; --i) {
            P.cstride[i] = (uint64_t)below;
            if (split && i == nhigh - 1)
                below = (int64_t)m[a].c * rows_below * L;   // the true extent of the split axis
            else
                below *= kx[i].c;
        }
    }
    P.ibel = NOBOUND;
    for (int k = 0; k < n; ++k) {
        P.istride[k] = (uint32_t)is[k];
        if (in.B[k] >= 0 && fill_el && vec > 1) {
            // element-precise source bound (k == 1, the only bounded operand)
            P.ibound[k] = NOBOUND;
            P.ibel = (uint32_t)in.B[k];
            predmask |= 1u << k;
        } else if (in.B[k] >= 0) {
            P.ibound[k] = (uint32_t)(in.B[k] / vec);
            predmask |= 1u << k;
        } else {
            P.ibound[k] = NOBOUND;
        }
        P.base[k] = base[k];
        P.ptr[k] = (uint64_t)(uintptr_t)r.ptr[k];
    }
    P.predmask = predmask;
    P.npoints = (uint64_t)r.npoints;
    out->dims = D;
    for (int i = 0; i < D; ++i)
        out->extents[i] = m[i].c;

    int blocks = (int)std::min<int64_t>(nunits, (int64_t)cus * std::max(1, s.blocks_per_cu));
    if (blocks > 8)
        blocks = (blocks + 7) / 8 * 8;
    out->blocks = std::max(blocks, 1);
    out->unroll = 4;
    out->cus = cus;
    out->cache = s.cache;
    out->rows1 = (RB == 1);
    out->unit = unit;
    return TRIOT_OK;
}

// ---------------------------------------------------------------------
// Row-segment plan (moments, moments adjoint)
// ---------------------------------------------------------------------

triot_status plan_segment(const Request &r, int cus, SegLaunch *out)
{
    std::memset(out, 0, sizeof(*out));
    SegPlan &P = out->plan;
    const int n = r.n, d = r.d;
    int flags = TRIOT_MOMENTS_FIRST;
    if (r.op == TRIOT_OP_MOMENTS && r.params)
        flags |= ((const triot_moments_params *)r.params)->flags;
    if (r.op == TRIOT_OP_MOMENTS_ADJ)
        flags |= ((const triot_moments_adj_params *)r.params)->flags;

    int kept[MAXD];
    int D = 0;
    for (int i = 0; i < d; ++i)
        if (r.counter[i] != 1)
            kept[D++] = i;
    const bool scalar = (D == 0);
    if (scalar)
        D = 1;
    if (flags & TRIOT_MOMENTS_COV) {
        if (D > 8)
            return TRIOT_E_UNSUPPORTED;
    }
    int64_t c[MAXD];
    for (int i = 0; i < D; ++i)
        c[i] = scalar ? 1 : r.counter[kept[i]];
    int64_t rows = 1;
    for (int i = 0; i < D - 1; ++i)
        rows *= c[i];
    if (rows >= (int64_t(1) << 32))
        return TRIOT_E_UNSUPPORTED;
    for (int i = 0; i < D; ++i)
        if (c[i] >= (int64_t(1) << 32))
            return TRIOT_E_UNSUPPORTED;
    const int64_t L = c[D - 1];
    const int64_t S = std::min<int64_t>(L, SEG_MAX);
    const int64_t G = (L + S - 1) / S;

    P.D = (uint32_t)D;
    P.n = (uint32_t)n;
    P.d_orig = (uint32_t)d;
    P.L = (uint32_t)L;
    P.S = (uint32_t)S;
    P.G = (uint32_t)G;
    if (G > 1)
        magic_for((uint32_t)G, &P.gdiv);
    else
        P.gdiv = trivial_div();
    P.rows = (uint32_t)rows;
    P.flags = (uint32_t)flags;
    P.nseg = (uint64_t)rows * (uint64_t)G;
    P.ntiles = (P.nseg + NT - 1) / NT;
    for (int i = 0; i < D - 1; ++i)
        magic_for((uint32_t)c[i], &P.ax[i]);
    for (int i = 0; i < D; ++i) {
        P.center[i] = 0.5 * (double)(c[i] - 1);
        P.orig[i] = scalar ? 0xFFFFFFFFu : (uint32_t)kept[i];
    }
    bool full = true;
    for (int k = 0; k < n; ++k) {
        int64_t want = 1;
        for (int i = D - 1; i >= 0; --i) {
            int64_t st = 1;
            if (!scalar)
                for (int j = kept[i] + 1; j < d; ++j)
                    st *= r.shape[k][j];
            P.stride[k][i] = st;
            if (st != want)
                full = false;
            want *= c[i];
        }
        P.base[k] = r.base[k];
        P.ptr[k] = (uint64_t)(uintptr_t)r.ptr[k];
    }
    P.full = full ? 1u : 0u;
    // 16-byte segment loads: every operand contiguous along the row and whole
    // quads per row (then every segment, S = min(L, 32), is whole quads too).
    bool vec4 = (L % 4) == 0;
    for (int k = 0; k < n; ++k)
        if (P.stride[k][D - 1] != 1 || ((uintptr_t)r.ptr[k] % 4) != 0)
            vec4 = false;
    P.vec4 = vec4 ? 1u : 0u;
    // Rows of 4, 8 or 16 words laid end to end: a wave's 64 segments are one
    // contiguous range, loaded line by line (the inner product adds the
    // fetched quads directly; the bounding box and the moments pass over
    // several operands, the latter for rows of 16 words from 2^21 rows on,
    // measured faster there and slower below, pass them through LDS).
    const bool stage_rows = full && vec4 && (L == 4 || L == 8 || L == 16);
    const bool stage_moments =
        r.op == TRIOT_OP_MOMENTS && n > 1 && L == 16 && rows >= (int64_t(1) << 21);
    P.stage = (stage_rows && (r.op == TRIOT_OP_DOT || r.op == TRIOT_OP_BBOX || stage_moments))
                  ? 1u : 0u;
    // Segments of 32 words laid end to end (rows a multiple of 32 words):
    // the moments pass (one operand) and the bounding box stage both halves
    // of every segment.
    if (((r.op == TRIOT_OP_MOMENTS && n == 1) || r.op == TRIOT_OP_BBOX) && full && vec4 &&
        S == 32 && L % 32 == 0)
        P.stage = 2u;
    // Rows of at most 8 words, one operand, any layout: the moments pass
    // loads the segments of several tiles before folding them.
    if (r.op == TRIOT_OP_MOMENTS && n == 1 && L <= 8 && !P.stage)
        P.stage = 3u;
    // The bounding box over rows of 16 words laid end to end: quads of 16
    // consecutive rows per load instruction, the row masks combined across
    // lanes (no LDS pass).
    if (r.op == TRIOT_OP_BBOX && P.stage == 1 && L == 16)
        P.stage = 6u;
    // Rows of 16 words laid end to end, one operand: every load instruction
    // covers quads of 16 consecutive rows, and the row sums are formed across
    // lanes (faster than the per-lane loads and than the LDS pass at every
    // size measured, with 4 workgroups per CU).
    if (r.op == TRIOT_OP_MOMENTS && n == 1 && full && vec4 && L == 16 && !P.stage)
        P.stage = 6u;
    // Rows of exactly 16 words otherwise (per-lane loads): an instance
    // without the second-half path of longer segments.
    if (r.op == TRIOT_OP_MOMENTS && vec4 && L == 16 && !P.stage)
        P.stage = 5u;
    // Rows of 2, 4 or 8 words laid end to end, one operand, the next axis a
    // multiple of 16 / L: the moments pass takes segments of 16 / L whole
    // rows (16 words), so that the outer coordinates enter once per 16
    // words instead of once per row.
    if (r.op == TRIOT_OP_MOMENTS && n == 1 && full && D >= 2 && (L == 2 || L == 4 || L == 8) &&
        c[D - 2] % (16 / L) == 0) {
        P.stage = 4u;
        P.rb = (uint32_t)(16 / L);
        P.S = 16;
        P.nseg = (uint64_t)rows / P.rb;
        P.ntiles = (P.nseg + NT - 1) / NT;
    }
    // Inner product over other layouts of whole quads: one quad per lane, so
    // that the 8 lanes of a 32-word row load its 128 bytes together (with a
    // segment per lane, every load instruction touches 64 lines).
    const uint64_t nquads = (uint64_t)rows * (uint64_t)(L / 4);
    P.quads = (vec4 && !P.stage && r.op == TRIOT_OP_DOT && nquads < (uint64_t(1) << 31)) ? 1u : 0u;
    if (P.quads) {
        P.nquads = nquads;
        if (!magic_for((uint32_t)(L / 4), &P.qdiv))
            P.qdiv = trivial_div();            // one quad per row: row = quad
        P.ntiles = (nquads + (uint64_t)NT * DOT_QUADS - 1) / ((uint64_t)NT * DOT_QUADS);
    }
    const bool cov = (flags & TRIOT_MOMENTS_COV) != 0;
    // Accumulator positions of the moments pass: exactly the kept axes with
    // the covariance (D <= 8), else a tier of 8 or 32; the adjoint keeps the
    // tiers 8 and 32.
    const int dmax = (D <= 8) ? 8 : 32;
    const int dm = cov ? D : dmax;
    // Workspace rows per block: M, dm first sums and, with the covariance,
    // dm(dm+1)/2 second sums, padded to a multiple of 8 (the final
    // reduction reads them 8 at a time, unconditionally).
    P.nterms = (uint32_t)((1 + dm + (cov ? dm * (dm + 1) / 2 : 0) + 7) / 8 * 8);
    if (r.op == TRIOT_OP_DOT)
        P.nterms = 8;                       // the mass alone
    else if (r.op == TRIOT_OP_BBOX)
        P.nterms = (uint32_t)(2 * dm);      // lo and hi + 1 per position (32-bit words)

    // Persistent grid: as many workgroups as can be resident at once (for
    // the moments pass at most 2 per CU, 3 when staged through LDS and 4 for
    // the quads of 16-word rows: each workgroup ends in a reduction of every
    // term, and measured on MI355X, 2 per CU beat 3 and 4 on the per-lane
    // loads).
    const bool adj = r.op == TRIOT_OP_MOMENTS_ADJ;
    // The inner product and the bounding box: 2 per CU, 4 where each load
    // instruction covers consecutive memory (the inner product's word quads
    // and tile loads, the bounding box's tile loads, of 8-axis
    // instances): each workgroup walks few tiles, and more workgroups keep
    // more loads in flight (measured on MI355X: the inner product of a
    // (2^9, 2^9, 2^5) window 34.0 -> 24.7 us, of two 16^6 operands 32.4 ->
    // 28.8 us; the 16^6 bounding box 31.9 -> 27.9 us).
    int bpc = 2;
    if (D <= 8 && ((r.op == TRIOT_OP_DOT && (P.quads || P.stage == 1)) ||
                   (r.op == TRIOT_OP_BBOX && (P.stage == 1 || P.stage == 6))))
        bpc = 4;
    if (r.op == TRIOT_OP_MOMENTS || adj)
        bpc = segment_blocks_per_cu(adj, cov, adj ? dmax : dm, vec4, (int)P.stage);
    // (the staged moments pass: 3 per CU, measured faster on large inputs;
    // the quads of 16-word rows: 4, measured faster than 2 or 3 from 32 MiB
    // of input up and level below)
    if (r.op == TRIOT_OP_MOMENTS)
        bpc = std::min(bpc, P.stage == 6 ? 4 : ((P.stage == 1 || P.stage == 2 || P.stage == 4) ? 3 : 2));
    int64_t blocks = std::min<int64_t>((int64_t)P.ntiles, (int64_t)cus * bpc);
    if (blocks > 8)
        blocks = (blocks + 7) / 8 * 8;
    blocks = std::max<int64_t>(blocks, 1);
    P.nblocks = (uint32_t)blocks;
    out->blocks = (int)blocks;
    out->dm = dm;
    out->dmax = dmax;
    return TRIOT_OK;
}

size_t segment_workspace_bytes(const SegLaunch &l)
{
    // Per-workgroup partial sums (float64), after a 256-byte aligned header.
    return 256 + (size_t)l.plan.nblocks * l.plan.nterms * sizeof(double);
}

std::string sched_key(const Request &r)
{
    std::string k;
    char buf[64];
    std::snprintf(buf, sizeof buf, "op%d:n%d:e%d:d%d", (int)r.op, r.n, r.elem_bytes, r.d);
    k += buf;
    k += ":c";
    for (int i = 0; i < r.d; ++i) {
        std::snprintf(buf, sizeof buf, "%lld,", (long long)r.counter[i]);
        k += buf;
    }
    for (int t = 0; t < r.n; ++t) {
        k += ":s";
        for (int i = 0; i < r.d; ++i) {
            std::snprintf(buf, sizeof buf, "%lld,", (long long)r.shape[t][i]);
            k += buf;
        }
        std::snprintf(buf, sizeof buf, "b%lld,a%d", (long long)(r.base[t] % 4),
                      (int)((uintptr_t)r.ptr[t] % 16));
        k += buf;
    }
    return k;
}


// ---------------------------------------------------------------------
// Naive convolution plan
// ---------------------------------------------------------------------
triot_status plan_conv(const Request &r, ConvLaunch *out)
{
    std::memset(out, 0, sizeof(*out));
    ConvPlan &P = out->plan;
    const int d = r.d;
    P.d = (uint32_t)d;
    uint64_t nout = 1, nl = 1, nr = 1;
    for (int i = 0; i < d; ++i) {
        const int64_t so = r.shape[0][i], sl = r.shape[1][i], sr = r.shape[2][i];
        if (so >= (int64_t(1) << 32))
            return TRIOT_E_UNSUPPORTED;
        nout *= (uint64_t)so;
        nl *= (uint64_t)sl;
        nr *= (uint64_t)sr;
        if (i >= 1) {
            if (so >= 2)
                magic_for((uint32_t)so, &P.ax[i]);
            else
                P.ax[i] = trivial_div();
        }
        P.ls[i] = (uint32_t)sl;
        P.rs[i] = (uint32_t)sr;
    }
    if (nout >= (uint64_t(1) << 32))
        return TRIOT_E_UNSUPPORTED;
    for (int i = d - 1; i >= 0; --i) {
        P.lstride[i] = (i == d - 1) ? 1 : P.lstride[i + 1] * (int64_t)P.ls[i + 1];
        P.rstride[i] = (i == d - 1) ? 1 : P.rstride[i + 1] * (int64_t)P.rs[i + 1];
    }
    P.nout = nout;
    P.nl = (uint32_t)std::min<uint64_t>(nl, 0xFFFFFFFFu);
    P.nr = (uint32_t)std::min<uint64_t>(nr, 0xFFFFFFFFu);
    P.lds = (nl + nr <= conv_lds_words()) ? 1u : 0u;
    P.out = (uint64_t)(uintptr_t)r.ptr[0];
    P.lhs = (uint64_t)(uintptr_t)r.ptr[1];
    P.rhs = (uint64_t)(uintptr_t)r.ptr[2];
    return TRIOT_OK;
}

// ---------------------------------------------------------------------
// Marginalization plan
// ---------------------------------------------------------------------
// Threads aimed at per launch: the reduced sub-box of each kept tuple is
// split into parts until about this many threads run.
static int64_t marginal_thread_target(int cus) { return (int64_t)cus * 1024; }

size_t marginal_workspace_bytes(int cus)
{
    // parts > 1 only when nout < target, and then nout * parts < 2 * target
    return 256 + (size_t)(2 * marginal_thread_target(cus)) * sizeof(double);
}

// Every operand's kept axis (the only one) has unit stride.
static bool kept_unit(const MargPlan &P, int n)
{
    for (int k = 0; k < n; ++k)
        if (P.kstride[k][0] != 1)
            return false;
    return true;
}

triot_status plan_marginal(const Request &r, int cus, MargLaunch *out)
{
    std::memset(out, 0, sizeof(*out));
    MargPlan &P = out->plan;
    const int n = r.n, d = r.d;
    const uint32_t km = ((const triot_marginal_params *)r.params)->keep_mask;
    // Non-trivial axes in order, then adjacent axes of the same kind (both
    // kept or both reduced) merged where every operand is contiguous across
    // them: the kept tuple's flat index and the set of reduced tuples are
    // unchanged, and a merged reduced run is walked in one stride.
    struct MAx {
        int64_t c;
        int64_t st[MAXT];
        bool keep;
    };
    MAx ax[MAXD];
    int na = 0;
    for (int i = 0; i < d; ++i) {
        const int64_t c = r.counter[i];
        if (c == 1)
            continue;             // contributes nothing to any offset or index
        MAx a;
        a.c = c;
        a.keep = ((km >> i) & 1u) != 0;
        for (int k = 0; k < n; ++k) {
            int64_t v = 1;
            for (int j2 = i + 1; j2 < d; ++j2)
                v *= r.shape[k][j2];
            a.st[k] = v;
        }
        if (na > 0 && ax[na - 1].keep == a.keep) {
            MAx &b = ax[na - 1];
            bool ok = true;
            for (int k = 0; k < n && ok; ++k)
                ok = b.st[k] == a.c * a.st[k];
            int64_t mc;
            if (ok && mul_ok(b.c, a.c, &mc)) {
                b.c = mc;
                for (int k = 0; k < n; ++k)
                    b.st[k] = a.st[k];
                continue;
            }
        }
        ax[na++] = a;
    }
    int dk = 0, dr = 0;
    uint64_t nout = 1, nred = 1;
    for (int i = 0; i < na; ++i) {
        if (ax[i].c >= (int64_t(1) << 32))
            return TRIOT_E_UNSUPPORTED;
        if (ax[i].keep) {
            magic_for((uint32_t)ax[i].c, &P.kax[dk]);
            for (int k = 0; k < n; ++k)
                P.kstride[k][dk] = ax[i].st[k];
            nout *= (uint64_t)ax[i].c;
            ++dk;
        } else {
            magic_for((uint32_t)ax[i].c, &P.rax[dr]);
            for (int k = 0; k < n; ++k)
                P.rstride[k][dr] = ax[i].st[k];
            nred *= (uint64_t)ax[i].c;
            ++dr;
        }
    }
    if (nout >= (uint64_t(1) << 32))
        return TRIOT_E_UNSUPPORTED;
    // the innermost axis is reduced and every operand's last axis
    bool inner_unit = dr > 0 && na > 0 && !ax[na - 1].keep;
    for (int k = 0; k < n && inner_unit; ++k)
        inner_unit = P.rstride[k][dr - 1] == 1;
    const int64_t target = marginal_thread_target(cus);
    uint64_t parts = 1;
    uint32_t mode = 0, clen = 0;
    if (inner_unit && dr == 1 && (nred == 4 || nred == 8 || nred == 16 || nred == 32 ||
                                  nred == 64) && (int64_t)nout * 64 > target) {
        // short runs: nred / 4 lanes per output, one word quad each, summed
        // by butterflies inside the lane group
        mode = 5;
    } else if (inner_unit && dr == 1 && nred >= 1024 && (int64_t)nout * 64 <= target) {
        // interleaved: chunks of >= 1024 elements, 64 lanes each
        const uint64_t chunks = std::max<uint64_t>(
            1, std::min<uint64_t>((nred + 1023) / 1024, (uint64_t)(target / ((int64_t)nout * 64))));
        clen = (uint32_t)((nred + chunks - 1) / chunks);
        clen = (clen + 63) / 64 * 64;
        parts = 64 * ((nred + clen - 1) / clen);
        mode = 2;
    } else if (dk == 1 && dr == 1 && ax[na - 1].keep && nout % 4 == 0 && nout <= 1024 &&
               (int64_t)nout < target && nred >= 256 && kept_unit(P, n)) {
        // columns: the kept axis is innermost and unit-stride, one reduced
        // axis; a lane takes four consecutive outputs, rows p, p + parts, ..
        // (nout * parts partials: at most 2 * target, the workspace's size)
        parts = std::min<uint64_t>((uint64_t)(2 * target) / nout, nred / 64);
        parts = std::max<uint64_t>(parts, 1);
        mode = 4;
    } else {
        const bool vec = inner_unit && (P.rax[dr - 1].c % 4) == 0;
        const uint64_t units = vec ? nred / 4 : nred;   // parts split whole vectors
        if ((int64_t)nout < target) {
            parts = (uint64_t)((target + (int64_t)nout - 1) / (int64_t)nout);
            // at least 64 reduced tuples per part
            parts = std::min<uint64_t>(parts, std::max<uint64_t>(1, nred / 64));
            parts = std::min<uint64_t>(parts, std::max<uint64_t>(1, units));
        }
        mode = vec ? 1 : 0;
    }
    P.n = (uint32_t)n;
    P.dk = (uint32_t)dk;
    P.dr = (uint32_t)dr;
    P.parts = (uint32_t)parts;
    P.mode = mode;
    P.clen = clen;
    P.nout = nout;
    P.nred = nred;
    for (int k = 0; k < n; ++k) {
        P.base[k] = r.base[k];
        P.ptr[k] = (uint64_t)(uintptr_t)r.ptr[k];
    }
    return TRIOT_OK;
}

}  // namespace triot
