/*
 * triot_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference for co-iteration over
 * tensors whose dimension and shapes are known only at run time
 * (Heyl & Serang, "TRIOT: Faster tensor manipulation in C++11",
 * arXiv 1608.00099).  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load it; the product library never does.
 * It shares no source, header, table or helper with the GPU library.
 *
 * Conventions (all from Section 1 of the paper):
 *   - a tensor of dimension d and shape s = (s_0..s_{d-1}) is a flat
 *     row-major array; the element at tuple t lives at flat position
 *     sum_i t_i * prod_{j>i} s_j (the sum-of-products equation of
 *     Section 1, equal to its Horner form);
 *   - an operand may be a window into a parent tensor: it carries a base
 *     element offset ("bias", Section 4, slices) that is added to every
 *     flat index computed with the parent's shape;
 *   - a co-iteration visits every tuple of a "counter" shape once, in
 *     lexicographic order (Section 1), produced by incrementing the tuple
 *     with carry, and applies an operation to the operands' elements at
 *     that tuple (Algorithms 8-10: for_each / apply / enumerate).
 *
 * Floating-point arithmetic follows plain ISO C with contraction off
 * (built with -ffp-contract=off): a float32 x + y*z is two roundings.
 * Moments are accumulated in double precision in visiting order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_D 32

enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_EDIM = 2, ORACLE_EBOUNDS = 3 };

/* ------------------------------------------------------------------ */
/* Index arithmetic                                                     */
/* ------------------------------------------------------------------ */

/* Flat row-major index of tuple t in shape s: the sum-of-products
 * definition of Section 1, evaluated from the last axis with a running
 * product of the trailing extents. */
uint64_t oracle_flat_index(const uint64_t *t, const uint64_t *s, int d)
{
    uint64_t off = 0, trailing = 1;
    for (int i = d - 1; i >= 0; --i) {
        off += t[i] * trailing;
        trailing *= s[i];
    }
    return off;
}

/* Next tuple in lexicographic order with respect to shape c: the last
 * axis counts fastest, and an axis that reaches its extent wraps to 0
 * and carries into the axis before it (Section 1, tuple iteration).
 * Returns 0 once the carry leaves axis 0, i.e. the traversal is over. */
int oracle_next_tuple(uint64_t *t, const uint64_t *c, int d)
{
    for (int i = d - 1; i >= 0; --i) {
        t[i] += 1;
        if (t[i] < c[i])
            return 1;
        t[i] = 0;
    }
    return 0;
}

/* Tuple of flat index f in shape s by repeated remainder and quotient,
 * last axis first (the reindexing derivation of Section 1). */
void oracle_unflatten(uint64_t f, const uint64_t *s, int d, uint64_t *t)
{
    for (int i = d - 1; i >= 0; --i) {
        t[i] = f % s[i];
        f /= s[i];
    }
}

/* ------------------------------------------------------------------ */
/* Operand descriptions and a traversal helper                          */
/* ------------------------------------------------------------------ */

typedef struct {
    unsigned char *data;   /* parent buffer */
    uint64_t shape[ORACLE_MAX_D];
    uint64_t base;         /* element offset of the window start */
    size_t elem;           /* bytes per element */
} operand;

static void set_operand(operand *o, void *data, const int64_t *shape,
                        int64_t base, int d, size_t elem)
{
    o->data = (unsigned char *)data;
    for (int i = 0; i < d; ++i)
        o->shape[i] = (uint64_t)shape[i];
    o->base = (uint64_t)base;
    o->elem = elem;
}

static unsigned char *at(const operand *o, const uint64_t *t, int d)
{
    uint64_t off = o->base + oracle_flat_index(t, o->shape, d);
    return o->data + off * o->elem;
}

/* Window start tuple of an operand (its base decoded in its own shape). */
static void window_start(const operand *o, int d, uint64_t *start)
{
    uint64_t total = 1;
    for (int i = 0; i < d; ++i)
        total *= o->shape[i];
    oracle_unflatten(total ? o->base % total : 0, o->shape, d, start);
}

/* The counter must fit inside the operand's window on every axis
 * (Algorithm 8's bounds check, done once per call, Section 4). */
static int fits(const operand *o, const uint64_t *c, int d)
{
    uint64_t start[ORACLE_MAX_D];
    window_start(o, d, start);
    for (int i = 0; i < d; ++i)
        if (start[i] + c[i] > o->shape[i])
            return 0;
    return 1;
}

/* Is tuple t inside the operand's window (used where an operand is only
 * read on part of the counter: zero-filled embedding, adjoints)? */
static int inside(const operand *o, const uint64_t *t, int d)
{
    uint64_t start[ORACLE_MAX_D];
    window_start(o, d, start);
    for (int i = 0; i < d; ++i)
        if (start[i] + t[i] >= o->shape[i])
            return 0;
    return 1;
}

static int load_counter(int d, const int64_t *counter, uint64_t *c,
                        uint64_t *npoints)
{
    if (d < 0 || d > ORACLE_MAX_D)
        return ORACLE_EDIM;
    uint64_t n = 1;
    for (int i = 0; i < d; ++i) {
        if (counter[i] < 0)
            return ORACLE_EINVAL;
        c[i] = (uint64_t)counter[i];
        n *= c[i];
    }
    *npoints = n;
    return ORACLE_OK;
}

static double rd(const unsigned char *p, int f64)
{
    if (f64) {
        double v;
        memcpy(&v, p, 8);
        return v;
    }
    float v;
    memcpy(&v, p, 4);
    return (double)v;
}

/* ------------------------------------------------------------------ */
/* Operations                                                           */
/* ------------------------------------------------------------------ */

/* COPY: dst[t] = src[t] for every counter tuple t, as raw element bytes.
 * With the counter equal to the source shape this is the zero-pad
 * embedding of Section 1 (into a pre-zeroed destination); with the
 * counter equal to the destination shape it is benchmark 1's crop
 * (Section 3, Algorithm 13).  Other destination elements are untouched. */
int oracle_copy(int d, const int64_t *counter,
                void *dst, const int64_t *dst_shape, int64_t dst_base,
                const void *src, const int64_t *src_shape, int64_t src_base,
                int elem_bytes)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, n;
    int rc = load_counter(d, counter, c, &n);
    if (rc)
        return rc;
    operand D, S;
    set_operand(&D, dst, dst_shape, dst_base, d, (size_t)elem_bytes);
    set_operand(&S, (void *)src, src_shape, src_base, d, (size_t)elem_bytes);
    if (!fits(&D, c, d) || !fits(&S, c, d))
        return ORACLE_EBOUNDS;
    if (n == 0)
        return ORACLE_OK;
    do {
        memcpy(at(&D, t, d), at(&S, t, d), (size_t)elem_bytes);
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* EMBED_FILL: over the counter (the destination region), write the
 * source element where the tuple lies inside the source window and +0.0
 * (all-zero bytes) elsewhere: the zero-padded tensor that precedes an FFT
 * convolution, written in one pass (Sections 1 and 3). */
int oracle_embed_fill(int d, const int64_t *counter,
                      void *dst, const int64_t *dst_shape, int64_t dst_base,
                      const void *src, const int64_t *src_shape,
                      int64_t src_base, int elem_bytes)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, n;
    int rc = load_counter(d, counter, c, &n);
    if (rc)
        return rc;
    operand D, S;
    set_operand(&D, dst, dst_shape, dst_base, d, (size_t)elem_bytes);
    set_operand(&S, (void *)src, src_shape, src_base, d, (size_t)elem_bytes);
    if (!fits(&D, c, d))
        return ORACLE_EBOUNDS;
    if (n == 0)
        return ORACLE_OK;
    do {
        if (inside(&S, t, d))
            memcpy(at(&D, t, d), at(&S, t, d), (size_t)elem_bytes);
        else
            memset(at(&D, t, d), 0, (size_t)elem_bytes);
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* MUL_ACC: x[t] = x[t] + y[t]*z[t] over the counter (benchmark 3's
 * broadcast update, Section 3), product and sum each rounded once. */
int oracle_mul_acc(int d, const int64_t *counter,
                   void *x, const int64_t *xs, int64_t xb,
                   const void *y, const int64_t *ys, int64_t yb,
                   const void *z, const int64_t *zs, int64_t zb, int f64)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, n;
    int rc = load_counter(d, counter, c, &n);
    if (rc)
        return rc;
    size_t e = f64 ? 8 : 4;
    operand X, Y, Z;
    set_operand(&X, x, xs, xb, d, e);
    set_operand(&Y, (void *)y, ys, yb, d, e);
    set_operand(&Z, (void *)z, zs, zb, d, e);
    if (!fits(&X, c, d) || !fits(&Y, c, d) || !fits(&Z, c, d))
        return ORACLE_EBOUNDS;
    if (n == 0)
        return ORACLE_OK;
    do {
        if (f64) {
            double *px = (double *)at(&X, t, d);
            double py = *(const double *)at(&Y, t, d);
            double pz = *(const double *)at(&Z, t, d);
            double prod = py * pz;
            *px = *px + prod;
        } else {
            float *px = (float *)at(&X, t, d);
            float py = *(const float *)at(&Y, t, d);
            float pz = *(const float *)at(&Z, t, d);
            float prod = py * pz;
            *px = *px + prod;
        }
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* MUL: out[t] = a[t]*b[t] over the counter (one rounding). */
int oracle_mul(int d, const int64_t *counter,
               void *o, const int64_t *os, int64_t ob,
               const void *a, const int64_t *as, int64_t ab,
               const void *b, const int64_t *bs, int64_t bb, int f64)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, n;
    int rc = load_counter(d, counter, c, &n);
    if (rc)
        return rc;
    size_t e = f64 ? 8 : 4;
    operand O, A, B;
    set_operand(&O, o, os, ob, d, e);
    set_operand(&A, (void *)a, as, ab, d, e);
    set_operand(&B, (void *)b, bs, bb, d, e);
    if (!fits(&O, c, d) || !fits(&A, c, d) || !fits(&B, c, d))
        return ORACLE_EBOUNDS;
    if (n == 0)
        return ORACLE_OK;
    do {
        if (f64) {
            double va = *(const double *)at(&A, t, d);
            double vb = *(const double *)at(&B, t, d);
            *(double *)at(&O, t, d) = va * vb;
        } else {
            float va = *(const float *)at(&A, t, d);
            float vb = *(const float *)at(&B, t, d);
            *(float *)at(&O, t, d) = va * vb;
        }
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* INDEX: out[k*N + f] = flat offset (base included) of the f-th counter
 * tuple in operand k, for n operands; N = number of counter tuples. */
int oracle_index(int n, int d, const int64_t *counter, const int64_t *shapes,
                 const int64_t *bases, int64_t *out)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, npts;
    int rc = load_counter(d, counter, c, &npts);
    if (rc)
        return rc;
    if (n < 1)
        return ORACLE_EINVAL;
    for (int k = 0; k < n; ++k) {
        operand O;
        set_operand(&O, NULL, shapes + (size_t)k * d, bases ? bases[k] : 0, d, 1);
        if (!fits(&O, c, d))
            return ORACLE_EBOUNDS;
    }
    if (npts == 0)
        return ORACLE_OK;
    uint64_t f = 0;
    do {
        for (int k = 0; k < n; ++k) {
            uint64_t s[ORACLE_MAX_D];
            for (int i = 0; i < d; ++i)
                s[i] = (uint64_t)shapes[(size_t)k * d + i];
            uint64_t b = bases ? (uint64_t)bases[k] : 0;
            out[(size_t)k * npts + f] = (int64_t)(b + oracle_flat_index(t, s, d));
        }
        ++f;
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* MOMENTS: index-weighted sums over the counter (Algorithm 11, which
 * Section 2 describes as an expected value when the weights are a PMF):
 *   w(t) = prod_k v_k(t)              (widened to double)
 *   M    = sum_t w(t)
 *   E_i  = (sum_t t_i w(t)) / M
 *   C_ij = (sum_t w(t) (t_i - E_i)(t_j - E_j)) / M     (i <= j)
 * out = [M, E_0..E_{d-1}, C_00, C_01, .., C_0(d-1), C_11, .., C_(d-1)(d-1)].
 * flags bit 1 requests the covariance; E is always produced.  Two
 * sequential passes in lexicographic order, all in double. */
int oracle_moments(int n, int d, const int64_t *counter, void *const *tensors,
                   const int64_t *shapes, const int64_t *bases, int f64,
                   int flags, double *out)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, npts;
    int rc = load_counter(d, counter, c, &npts);
    if (rc)
        return rc;
    if (n < 1 || n > 8)
        return ORACLE_EINVAL;
    operand V[8];
    for (int k = 0; k < n; ++k) {
        set_operand(&V[k], tensors[k], shapes + (size_t)k * d,
                    bases ? bases[k] : 0, d, f64 ? 8 : 4);
        if (!fits(&V[k], c, d))
            return ORACLE_EBOUNDS;
    }
    double M = 0.0, S[ORACLE_MAX_D] = {0};
    if (npts > 0) {
        do {
            double w = 1.0;
            for (int k = 0; k < n; ++k)
                w *= rd(at(&V[k], t, d), f64);
            M += w;
            for (int i = 0; i < d; ++i)
                S[i] += (double)t[i] * w;
        } while (oracle_next_tuple(t, c, d));
    }
    double E[ORACLE_MAX_D];
    out[0] = M;
    for (int i = 0; i < d; ++i) {
        E[i] = S[i] / M;
        out[1 + i] = E[i];
    }
    if (!(flags & 2))
        return ORACLE_OK;
    int ncov = d * (d + 1) / 2;
    double *K = (double *)calloc((size_t)(ncov > 0 ? ncov : 1), sizeof(double));
    if (!K)
        return ORACLE_EINVAL;
    memset(t, 0, sizeof(t));
    if (npts > 0) {
        do {
            double w = 1.0;
            for (int k = 0; k < n; ++k)
                w *= rd(at(&V[k], t, d), f64);
            int p = 0;
            for (int i = 0; i < d; ++i)
                for (int j = i; j < d; ++j)
                    K[p++] += w * ((double)t[i] - E[i]) * ((double)t[j] - E[j]);
        } while (oracle_next_tuple(t, c, d));
    }
    for (int p = 0; p < ncov; ++p)
        out[1 + d + p] = K[p] / M;
    free(K);
    return ORACLE_OK;
}

/* MOMENTS_ADJ: the gradient of a scalar loss with respect to every weight
 * w(t) of the counter, given the moments (M, E, C) and the loss's partial
 * derivatives (gM, gE, gC) laid out like the MOMENTS output:
 *   dM/dw(t)    = 1
 *   dE_i/dw(t)  = (t_i - E_i) / M
 *   dC_ij/dw(t) = ((t_i - E_i)(t_j - E_j) - C_ij) / M
 * (the E-dependence of C drops out because sum_t w (t_j - E_j) = 0).
 * g[t] = gM + sum_i gE_i dE_i/dw + sum_{i<=j} gC_ij dC_ij/dw, written to
 * the single operand g (float32 or double); flags bit 1 = use gC. */
int oracle_moments_adj(int d, const int64_t *counter, void *g,
                       const int64_t *gs, int64_t gb, int f64,
                       const double *mom, const double *gmom, int flags)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, npts;
    int rc = load_counter(d, counter, c, &npts);
    if (rc)
        return rc;
    operand G;
    set_operand(&G, g, gs, gb, d, f64 ? 8 : 4);
    if (!fits(&G, c, d))
        return ORACLE_EBOUNDS;
    if (npts == 0)
        return ORACLE_OK;
    double M = mom[0];
    do {
        double acc = 0.0;
        for (int i = 0; i < d; ++i)
            acc += gmom[1 + i] * ((double)t[i] - mom[1 + i]);
        if (flags & 2) {
            int p = 0;
            for (int i = 0; i < d; ++i)
                for (int j = i; j < d; ++j) {
                    double dij = ((double)t[i] - mom[1 + i]) * ((double)t[j] - mom[1 + j]);
                    acc += gmom[1 + d + p] * (dij - mom[1 + d + p]);
                    ++p;
                }
        }
        double v = gmom[0] + acc / M;
        if (f64)
            *(double *)at(&G, t, d) = v;
        else
            *(float *)at(&G, t, d) = (float)v;
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* MUL_ADJ: adjoint of out = a*b over the intersection I (the shape of
 * gout): over the whole shape of ga, ga[t] = gout[t]*b[t] for t in I and
 * 0 elsewhere; over the whole shape of gb, gb[t] = gout[t]*a[t] for t in
 * I and 0 elsewhere.  Shapes: ga like a, gb like b, I inside both. */
int oracle_mul_adj(int d, void *ga, const int64_t *sa, void *gb,
                   const int64_t *sb, const void *gout, const int64_t *si,
                   const void *a, const void *b, int f64)
{
    uint64_t ca[ORACLE_MAX_D], cb[ORACLE_MAX_D], ci[ORACLE_MAX_D];
    uint64_t na, nb, ni, t[ORACLE_MAX_D];
    int rc = load_counter(d, sa, ca, &na);
    if (!rc)
        rc = load_counter(d, sb, cb, &nb);
    if (!rc)
        rc = load_counter(d, si, ci, &ni);
    if (rc)
        return rc;
    for (int i = 0; i < d; ++i)
        if (ci[i] > ca[i] || ci[i] > cb[i])
            return ORACLE_EBOUNDS;
    size_t e = f64 ? 8 : 4;
    operand GA, GB, GO, A, B;
    set_operand(&GA, ga, sa, 0, d, e);
    set_operand(&GB, gb, sb, 0, d, e);
    set_operand(&GO, (void *)gout, si, 0, d, e);
    set_operand(&A, (void *)a, sa, 0, d, e);
    set_operand(&B, (void *)b, sb, 0, d, e);
    /* ga over the shape of a */
    memset(t, 0, sizeof(t));
    if (na > 0) {
        do {
            unsigned char *dst = at(&GA, t, d);
            if (inside(&GO, t, d)) {
                if (f64)
                    *(double *)dst = *(const double *)at(&GO, t, d) *
                                     *(const double *)at(&B, t, d);
                else
                    *(float *)dst = *(const float *)at(&GO, t, d) *
                                    *(const float *)at(&B, t, d);
            } else {
                memset(dst, 0, e);
            }
        } while (oracle_next_tuple(t, ca, d));
    }
    /* gb over the shape of b */
    memset(t, 0, sizeof(t));
    if (nb > 0) {
        do {
            unsigned char *dst = at(&GB, t, d);
            if (inside(&GO, t, d)) {
                if (f64)
                    *(double *)dst = *(const double *)at(&GO, t, d) *
                                     *(const double *)at(&A, t, d);
                else
                    *(float *)dst = *(const float *)at(&GO, t, d) *
                                    *(const float *)at(&A, t, d);
            } else {
                memset(dst, 0, e);
            }
        } while (oracle_next_tuple(t, cb, d));
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Further tuple-visiting operations (Sections 2 and 3)                 */
/* ------------------------------------------------------------------ */

/* DOT: the inner product over the shared tuples (benchmark 2 of
 * Section 3; Algorithm 8's captured-sum example):
 *   out = sum_t prod_k v_k(t)    (each value widened to double),
 * summed in double in lexicographic order. */
int oracle_dot(int n, int d, const int64_t *counter, void *const *tensors,
               const int64_t *shapes, const int64_t *bases, int f64,
               double *out)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, npts;
    int rc = load_counter(d, counter, c, &npts);
    if (rc)
        return rc;
    if (n < 1 || n > 8)
        return ORACLE_EINVAL;
    operand V[8];
    for (int k = 0; k < n; ++k) {
        set_operand(&V[k], tensors[k], shapes + (size_t)k * d,
                    bases ? bases[k] : 0, d, f64 ? 8 : 4);
        if (!fits(&V[k], c, d))
            return ORACLE_EBOUNDS;
    }
    double s = 0.0;
    if (npts > 0) {
        do {
            double w = 1.0;
            for (int k = 0; k < n; ++k)
                w *= rd(at(&V[k], t, d), f64);
            s += w;
        } while (oracle_next_tuple(t, c, d));
    }
    *out = s;
    return ORACLE_OK;
}

/* XPYX_MZ: x[t] <- x[t] + y[t]*x[t] - z[t] over the counter (benchmark 3
 * of Section 3), evaluated as written in C: the product, then the sum,
 * then the difference, each rounded once. */
int oracle_xpyx_mz(int d, const int64_t *counter,
                   void *x, const int64_t *xs, int64_t xb,
                   const void *y, const int64_t *ys, int64_t yb,
                   const void *z, const int64_t *zs, int64_t zb, int f64)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, n;
    int rc = load_counter(d, counter, c, &n);
    if (rc)
        return rc;
    size_t e = f64 ? 8 : 4;
    operand X, Y, Z;
    set_operand(&X, x, xs, xb, d, e);
    set_operand(&Y, (void *)y, ys, yb, d, e);
    set_operand(&Z, (void *)z, zs, zb, d, e);
    if (!fits(&X, c, d) || !fits(&Y, c, d) || !fits(&Z, c, d))
        return ORACLE_EBOUNDS;
    if (n == 0)
        return ORACLE_OK;
    do {
        if (f64) {
            double *px = (double *)at(&X, t, d);
            double vx = *px;
            double vy = *(const double *)at(&Y, t, d);
            double vz = *(const double *)at(&Z, t, d);
            double prod = vy * vx;
            double sum = vx + prod;
            *px = sum - vz;
        } else {
            float *px = (float *)at(&X, t, d);
            float vx = *px;
            float vy = *(const float *)at(&Y, t, d);
            float vz = *(const float *)at(&Z, t, d);
            float prod = vy * vx;
            float sum = vx + prod;
            *px = sum - vz;
        }
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* MARGINAL: sum the weights w(t) = prod_k v_k(t) (double) over the axes
 * whose keep flag is 0 (Section 2: marginalization needs the tuple).  The
 * output is a double tensor over the kept axes (their counter extents, in
 * axis order; a scalar when none is kept), zeroed first; every counter
 * tuple adds its weight to the output at its kept coordinates, visiting
 * the counter in lexicographic order. */
int oracle_marginal(int n, int d, const int64_t *counter, const int *keep,
                    void *const *tensors, const int64_t *shapes,
                    const int64_t *bases, int f64, double *out)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, npts;
    int rc = load_counter(d, counter, c, &npts);
    if (rc)
        return rc;
    if (n < 1 || n > 8)
        return ORACLE_EINVAL;
    operand V[8];
    for (int k = 0; k < n; ++k) {
        set_operand(&V[k], tensors[k], shapes + (size_t)k * d,
                    bases ? bases[k] : 0, d, f64 ? 8 : 4);
        if (!fits(&V[k], c, d))
            return ORACLE_EBOUNDS;
    }
    uint64_t ks[ORACLE_MAX_D], kt[ORACLE_MAX_D];
    int dk = 0;
    uint64_t nout = 1;
    for (int i = 0; i < d; ++i)
        if (keep[i]) {
            ks[dk++] = c[i];
            nout *= c[i];
        }
    for (uint64_t f = 0; f < nout; ++f)
        out[f] = 0.0;
    if (npts == 0)
        return ORACLE_OK;
    do {
        double w = 1.0;
        for (int k = 0; k < n; ++k)
            w *= rd(at(&V[k], t, d), f64);
        int j = 0;
        for (int i = 0; i < d; ++i)
            if (keep[i])
                kt[j++] = t[i];
        out[oracle_flat_index(kt, ks, dk)] += w;
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* BBOX: the bounding box of the tuples at which every operand is nonzero
 * (Section 2: the nonzero bounding box of an element-wise product; the
 * product of reals is nonzero exactly when every factor is, so no
 * floating-point product decides it; a NaN counts as nonzero).
 * out[2i] = min t_i, out[2i+1] = max t_i over those tuples; every entry is
 * -1 when there is none. */
int oracle_bbox(int n, int d, const int64_t *counter, void *const *tensors,
                const int64_t *shapes, const int64_t *bases, int f64,
                int64_t *out)
{
    uint64_t c[ORACLE_MAX_D], t[ORACLE_MAX_D] = {0}, npts;
    int rc = load_counter(d, counter, c, &npts);
    if (rc)
        return rc;
    if (n < 1 || n > 8)
        return ORACLE_EINVAL;
    operand V[8];
    for (int k = 0; k < n; ++k) {
        set_operand(&V[k], tensors[k], shapes + (size_t)k * d,
                    bases ? bases[k] : 0, d, f64 ? 8 : 4);
        if (!fits(&V[k], c, d))
            return ORACLE_EBOUNDS;
    }
    int found = 0;
    for (int i = 0; i < d; ++i) {
        out[2 * i] = -1;
        out[2 * i + 1] = -1;
    }
    if (npts == 0)
        return ORACLE_OK;
    do {
        int nz = 1;
        for (int k = 0; k < n && nz; ++k)
            if (!(rd(at(&V[k], t, d), f64) != 0.0))
                nz = 0;
        if (!nz)
            continue;
        for (int i = 0; i < d; ++i) {
            int64_t v = (int64_t)t[i];
            if (!found || v < out[2 * i])
                out[2 * i] = v;
            if (!found || v > out[2 * i + 1])
                out[2 * i + 1] = v;
        }
        found = 1;
    } while (oracle_next_tuple(t, c, d));
    return ORACLE_OK;
}

/* CONV: the naive multidimensional convolution of Section 3 (Algorithms
 * 14 and 15): result shape ls + rs - 1 on every axis, zeroed first; for
 * every tuple t of lhs in lexicographic order and, inside, every tuple u
 * of rhs in lexicographic order, result[t + u] += lhs[t] * rhs[u]
 * (double, product and sum each rounded once). */
int oracle_conv(int d, const double *lhs, const int64_t *ls, const double *rhs,
                const int64_t *rs, double *out)
{
    uint64_t cl[ORACLE_MAX_D], cr[ORACLE_MAX_D], co[ORACLE_MAX_D];
    uint64_t nl, nr, no;
    uint64_t t[ORACLE_MAX_D] = {0}, u[ORACLE_MAX_D], v[ORACLE_MAX_D];
    int rc = load_counter(d, ls, cl, &nl);
    if (!rc)
        rc = load_counter(d, rs, cr, &nr);
    if (rc)
        return rc;
    for (int i = 0; i < d; ++i) {
        if (cl[i] == 0 || cr[i] == 0)
            return ORACLE_EINVAL;
        co[i] = cl[i] + cr[i] - 1;
    }
    no = 1;
    for (int i = 0; i < d; ++i)
        no *= co[i];
    for (uint64_t f = 0; f < no; ++f)
        out[f] = 0.0;
    do {
        const double a = lhs[oracle_flat_index(t, cl, d)];
        memset(u, 0, sizeof(u));
        do {
            for (int i = 0; i < d; ++i)
                v[i] = t[i] + u[i];
            double prod = a * rhs[oracle_flat_index(u, cr, d)];
            double *o = &out[oracle_flat_index(v, co, d)];
            *o = *o + prod;
        } while (oracle_next_tuple(u, cr, d));
    } while (oracle_next_tuple(t, cl, d));
    return ORACLE_OK;
}
