/*
 * triot.h -- C ABI of the MI355X co-iteration library.
 *
 * Co-iteration over several tensors whose dimension d and shapes are known
 * only at run time (Heyl & Serang, "TRIOT: Faster tensor manipulation in
 * C++11", arXiv 1608.00099).  Every point t of a counter shape is an index
 * tuple; in every operand it maps to the row-major flat offset
 *     off_k(t) = base_k + sum_i t_i * prod_{j>i} s^k_j          (Section 1)
 * where s^k is operand k's (parent) shape and base_k the element offset of
 * its window start (Section 4, slices with a bias).  An operation is then
 * applied at every counter point (Algorithms 8-10: read-only, dest-only,
 * and tuple-reading co-iteration).
 *
 * Conventions for every entry point:
 *   - Shapes, counters and bases are HOST arrays of int64 (element units).
 *     shapes is n_tensors*d values, operand k's shape at shapes[k*d].
 *   - Tensor pointers are DEVICE pointers to row-major parent buffers.
 *     The caller owns every device buffer; the library never frees one.
 *   - All work is enqueued on `stream` (any HIP stream, including the null
 *     stream).  No entry point synchronises the host on the hot path;
 *     device faults surface at the caller's next synchronisation.
 *   - Validation happens once per call over shapes, never per index
 *     (Section 4).  Errors are returned as triot_status, never aborted.
 *   - d = 0 is a scalar (one point, the empty tuple).  A counter with an
 *     extent 0 has no points: the call returns TRIOT_OK and does nothing.
 *     Extent-1 axes are dropped before planning (Section 4: an axis of
 *     extent 1 adds nothing to any offset, so leaving it out changes no
 *     result).
 *   - Window bounds: base_k decodes (in operand k's shape) to a start
 *     tuple sigma^k; every operand that is read or written on the whole
 *     counter needs sigma^k_i + counter_i <= s^k_i on every axis i.
 *   - Aliasing: an output may be passed again, with the same pointer, base
 *     and shape, as an input of an element-wise op (x[t] += y[t]*x[t],
 *     Section 4).  Any other overlap of an output with another operand is
 *     rejected with TRIOT_E_ALIAS.
 */
#ifndef TRIOT_H
#define TRIOT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest supported tensor dimension (the paper's MAX_TENSOR_DIMENSION,
 * Section 2, Algorithm 8). */
#define TRIOT_MAX_D 32
/* Largest number of operands of one call. */
#define TRIOT_MAX_TENSORS 5

typedef enum triot_status {
    TRIOT_OK = 0,
    TRIOT_E_INVALID = 1,     /* null pointer with work > 0, bad op, n or params */
    TRIOT_E_DIM = 2,         /* d < 0 or d > TRIOT_MAX_D */
    TRIOT_E_BOUNDS = 3,      /* counter exceeds an operand window (Algorithm 8's check) */
    TRIOT_E_ALIAS = 4,       /* an output partially overlaps another operand */
    TRIOT_E_OVERFLOW = 5,    /* a size or offset does not fit in int64 */
    TRIOT_E_WORKSPACE = 6,   /* workspace missing or smaller than triot_workspace_size() */
    TRIOT_E_DEVICE = 7,      /* a HIP call failed (launch, graph, memory) */
    TRIOT_E_UNSUPPORTED = 8  /* valid request outside this build's limits (stated per op) */
} triot_status;

typedef enum triot_op {
    /* dst[t] = src[t] over the counter, as raw element bytes (4 or 8).
     * tensors = {dst, src}.  counter = src shape: zero-pad embedding into a
     * pre-zeroed dst (Section 1); counter = dst shape: benchmark 1's crop
     * (Section 3).  dst elements outside the counter are untouched.
     * params: const triot_copy_params* (NULL = 4-byte elements). */
    TRIOT_OP_COPY = 0,
    /* Over the counter (the dst region): dst[t] = src[t] where t lies in
     * the src window, else +0.0 (all-zero bytes).  The zero-padded tensor
     * ahead of an FFT convolution (Sections 1 and 3) in one pass.
     * tensors = {dst, src}; src may be smaller than the counter.
     * params: const triot_copy_params* (NULL = 4-byte elements). */
    TRIOT_OP_EMBED_FILL = 1,
    /* x[t] = x[t] + y[t]*z[t] in float32, product and sum rounded
     * separately (no fused multiply-add), over the counter; NULL counter =
     * elementwise minimum of the shapes, i.e. the tuples shared by all
     * operands (Section 3, benchmarks 2 and 3).  tensors = {x, y, z}. */
    TRIOT_OP_MUL_ACC = 2,
    /* out[t] = a[t]*b[t] in float32 over the counter (NULL = intersection).
     * tensors = {out, a, b}. */
    TRIOT_OP_MUL = 3,
    /* Index-weighted moments of w(t) = prod_k v_k(t) over the counter
     * (Algorithm 11, an expected value when w is a PMF, Section 2):
     *   M = sum w,  E_i = sum t_i w / M,
     *   C_ij = sum w (t_i - E_i)(t_j - E_j) / M   (population covariance).
     * tensors = {v_0, .., v_{n-1}}, float32, 1 <= n <= 4.
     * out (device, float32): [M, E_0..E_{d-1}] followed, with
     * TRIOT_MOMENTS_COV, by the upper triangle C_00, C_01, .., C_0(d-1),
     * C_11, .., C_(d-1)(d-1): 1 + d (+ d(d+1)/2) values.
     * params: const triot_moments_params*.  Accumulation is float64 over
     * coordinates shifted to the axis centres, summed across threads and
     * workgroups in a fixed tree; the result is deterministic for a given
     * device and launch.  Needs a workspace.
     * Enqueues two kernels (partial sums, then their combination).
     * Limits: the covariance needs d' <= 8 axes after dropping extent-1
     * axes (first moments: d' <= 32), and fewer than 2^32 counter rows. */
    TRIOT_OP_MOMENTS = 4,
    /* Gradient of a scalar loss with respect to every weight w(t), given
     * the moments and the loss's partials (gM, gE, gC):
     *   g[t] = gM + sum_i gE_i (t_i - E_i)/M
     *             + sum_{i<=j} gC_ij ((t_i - E_i)(t_j - E_j) - C_ij)/M.
     * tensors = {g} (float32 output over the counter).
     * params: const triot_moments_adj_params*.  Same limits as MOMENTS. */
    TRIOT_OP_MOMENTS_ADJ = 5,
    /* Adjoint of out = a*b over the intersection I (broadcast-scatter):
     *   ga[t] = gout[t]*b[t] for t in I, 0 elsewhere in ga's shape;
     *   gb[t] = gout[t]*a[t] for t in I, 0 elsewhere in gb's shape.
     * tensors = {ga, gb, gout, a, b}, float32; shapes: ga like a, gb like
     * b, gout = I inside both.  counter = NULL (elementwise maximum of
     * the ga and gb shapes) or that shape.  One fused pass. */
    TRIOT_OP_MUL_ADJ = 6,
    /* out[k*N + f] = off_k(t_f) (int64, bases included) for every operand
     * k and the f-th counter tuple t_f in row-major order; N = number of
     * counter tuples.  tensors[0] is the int64 output of n_tensors*N
     * values; all n shapes (including operand 0's) define offsets; the
     * other pointers are ignored.  For checking the index arithmetic. */
    TRIOT_OP_INDEX = 7,
    /* Inner product over the shared tuples (benchmark 2 of Section 3; the
     * captured-sum example of Algorithm 8):  out = sum_t prod_k v_k(t).
     * tensors = {v_0, .., v_{n-1}}, float32, 1 <= n <= 4; counter NULL =
     * the intersection.  out (device): one float32; params: optional
     * const triot_reduce_params* (a float64 copy).  float64 accumulation,
     * deterministic; needs a workspace; enqueues two kernels. */
    TRIOT_OP_DOT = 8,
    /* x[t] = (x[t] + y[t]*x[t]) - z[t] in float32 (benchmark 3 of Section
     * 3), each operation rounded once (no fused multiply-add), over the
     * counter (NULL = intersection).  tensors = {x, y, z}. */
    TRIOT_OP_XPYX_MZ = 9,
    /* Marginalization (Section 2): the sums of w(t) = prod_k v_k(t) over
     * the counter axes NOT flagged in params->keep_mask (bit i = keep axis
     * i).  tensors = {v_0, .., v_{n-1}}, float32, 1 <= n <= 4; counter
     * NULL = intersection.  out (device, float32): a row-major tensor over
     * the kept axes with their counter extents (one value when no axis is
     * kept).  params: const triot_marginal_params* (required).  float64
     * accumulation; deterministic; needs a workspace; two kernels. */
    TRIOT_OP_MARGINAL = 10,
    /* Bounding box of the tuples at which every operand is nonzero (the
     * nonzero bounding box of an element-wise product, Section 2; a NaN
     * counts as nonzero, +0.0 and -0.0 as zero).  tensors = {v_0, ..},
     * float32, 1 <= n <= 4; counter NULL = intersection.  out (device,
     * int64): [lo_0, hi_0, .., lo_{d-1}, hi_{d-1}] (inclusive), every
     * entry -1 when no tuple qualifies.  Needs a workspace; two kernels.
     * Limits: d' <= 32 kept axes, fewer than 2^32 counter rows. */
    TRIOT_OP_BBOX = 11,
    /* Naive multidimensional convolution (Algorithms 14 and 15 of Section
     * 3): out[v] = sum over lhs tuples t (lexicographic order) with
     * 0 <= v - t < rs of lhs[t] * rhs[v - t], float64, each product and sum
     * rounded once; the result equals the paper's loop order bit for bit.
     * tensors = {out, lhs, rhs}, float64; shapes = {ls + rs - 1, ls, rs}
     * (every extent of ls and rs >= 1); counter NULL or the out shape;
     * bases NULL or zero.  out must not overlap lhs or rhs. */
    TRIOT_OP_CONV = 12
} triot_op;

typedef struct triot_copy_params {
    int elem_bytes;          /* 4 (float32) or 8 (float64) */
} triot_copy_params;

#define TRIOT_MOMENTS_FIRST 1  /* M and E (always produced) */
#define TRIOT_MOMENTS_COV 2    /* add the covariance upper triangle */
/* A load hint, no effect on results: the operands were just written (by
 * the previous kernel of a pipeline) and may still sit in the caches, so
 * load them through the caches rather than streaming past them (the
 * default, faster for data that is not cached). */
#define TRIOT_MOMENTS_CACHED 4

typedef struct triot_moments_params {
    int flags;               /* TRIOT_MOMENTS_FIRST [| TRIOT_MOMENTS_COV] [| TRIOT_MOMENTS_CACHED] */
    double *out64;           /* optional device buffer: the same layout in float64 */
} triot_moments_params;

typedef struct triot_reduce_params {
    double *out64;           /* optional device buffer: the result in float64 */
} triot_reduce_params;

typedef struct triot_marginal_params {
    uint32_t keep_mask;      /* bit i set: counter axis i is kept in the output */
    double *out64;           /* optional device buffer: the result in float64 */
} triot_marginal_params;

typedef struct triot_moments_adj_params {
    int flags;               /* TRIOT_MOMENTS_COV: gmom carries gC */
    const double *mom;       /* device, float64 moments [M, E.., C..] as MOMENTS writes to out64 */
    const float *gmom;       /* device, float32 partials [gM, gE.., gC..], same layout */
} triot_moments_adj_params;

/* Run one co-iteration.
 *   op             the operation (see triot_op).
 *   n_tensors      number of operands, 1..TRIOT_MAX_TENSORS, fixed per op.
 *   d              tensor dimension, 0..TRIOT_MAX_D (all operands share d).
 *   shapes         host, n_tensors*d extents (>= 0).
 *   counter_shape  host, d extents, or NULL for the op's default.
 *   tensors        host array of n_tensors device pointers.
 *   bases          host, n_tensors element offsets, or NULL for all 0.
 *   params         host pointer to the op's params struct (or NULL).
 *   out            device pointer for ops with a reduced result (MOMENTS).
 *   workspace      device scratch of at least triot_workspace_size() bytes
 *                  for ops that need one (MOMENTS: per-workgroup partial
 *                  sums); its contents need no initialisation.  Calls that
 *                  share a workspace must not overlap in time.
 *   stream         HIP stream to enqueue on.
 * Returns TRIOT_OK or an error; on error nothing is enqueued. */
triot_status triot_apply(triot_op op, int n_tensors, int d, const int64_t *shapes,
                         const int64_t *counter_shape, void *const *tensors,
                         const int64_t *bases, const void *params, void *out,
                         void *workspace, size_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as triot_apply, with the same arguments except the workspace,
 * and the same results bit for bit.  The ops that need a workspace
 * (MOMENTS, DOT, BBOX, MARGINAL) use instead a scratch array of
 * TRIOT_NOALLOC_SCRATCH_BYTES that the library holds on each device in
 * static device memory, from the first call on that device until the
 * process ends; a problem whose triot_workspace_size() exceeds it returns
 * TRIOT_E_WORKSPACE and enqueues nothing.  The entry point calls no
 * hipMalloc, hipFree or other allocating routine.  Nothing in the scratch
 * needs initialisation (every partial is written before it is read); calls
 * on one device share its scratch, so calls whose work overlaps in time on
 * one device (on different streams, or from different threads) race and
 * give undefined results.  TRIOT_E_DEVICE when the scratch's device
 * address cannot be obtained. */
#define TRIOT_NOALLOC_SCRATCH_BYTES (8u << 20)
triot_status triot_apply_noalloc(triot_op op, int n_tensors, int d, const int64_t *shapes,
                                 const int64_t *counter_shape, void *const *tensors,
                                 const int64_t *bases, const void *params, void *out,
                                 hipStream_t stream);

/* Workspace bytes triot_apply needs for this problem (0 if none). */
size_t triot_workspace_size(triot_op op, int n_tensors, int d, const int64_t *shapes,
                            const int64_t *counter_shape);

/* ---- batched form ---------------------------------------------------- */

/* One independent co-iteration of a batch; fields as in triot_apply. */
typedef struct triot_item {
    int d;
    int n_tensors;
    const int64_t *shapes;
    const int64_t *counter_shape;  /* NULL = the op's default */
    void *const *tensors;
    const int64_t *bases;          /* NULL = all 0 */
} triot_item;

/* Opaque batch handle: the planned work table in device memory and the
 * captured hipGraph that replays the whole batch as one persistent launch.
 * Owned by the library from create until destroy. */
typedef struct triot_batch triot_batch;

triot_status triot_batch_create(triot_batch **handle);
void triot_batch_destroy(triot_batch *handle);

/* Apply op to every item of a batch of thousands of tensors of uneven d and
 * shape (for instance the zero-padding ahead of FFT convolutions) in ONE
 * persistent kernel launch that walks a device work table of
 * (item, tile) units.  The first call with a given batch plans it, uploads
 * the table and captures the launch in a hipGraph; later calls with the
 * same shapes, pointers and op replay the graph on `stream`; a different
 * batch re-plans.  Supported ops: COPY, EMBED_FILL, MUL_ACC, MUL.
 * params as in triot_apply (shared by all items).  Items run concurrently:
 * TRIOT_E_ALIAS when the output range of one item overlaps any operand
 * range (read or written) of another item, besides the per-item aliasing
 * rule of triot_apply; nothing is enqueued then.  TRIOT_E_UNSUPPORTED
 * when the work units of all items reach 2^31. */
triot_status triot_apply_batched(triot_op op, int n_items, const triot_item *items,
                                 const void *params, triot_batch *handle, hipStream_t stream);

/* Replay the batch last planned by triot_apply_batched on `stream`, without
 * re-validating the items: for serving loops that call the same batch
 * (same shapes, pointers and op) again and again.  The caller guarantees
 * that the buffers are still allocated.  TRIOT_E_INVALID if nothing was
 * planned on this handle yet. */
triot_status triot_batch_launch(triot_batch *handle, hipStream_t stream);

/* Launch statistics of the last batched call: units (tiles) in the work
 * table, blocks of the persistent launch, and whether the call replayed
 * a captured graph (1) or planned and captured it (0). */
triot_status triot_batch_info(const triot_batch *handle, int64_t *n_units, int *n_blocks,
                              int *replayed);

/* ---- tuning ----------------------------------------------------------- */

/* Time the candidate launch schedules (vector width, cache policy, blocks
 * per CU, unit order, box rows, work-unit size) of this exact problem with HIP events on `stream`,
 * keep the fastest for every later call with the same plan signature, and
 * append it to the JSON cache at cache_path (NULL = in memory only).  The
 * operation RUNS several times on the given buffers: pass scratch copies
 * for in-place ops.  Each candidate is timed cold, after a write over a
 * 512 MiB device buffer (larger than the memory-side cache) that the first
 * tuning on a device allocates and triot_tune_reset frees; when it cannot be
 * allocated, candidates are timed without it.  The cache named by the environment variable
 * TRIOT_TUNE_CACHE, if set, is loaded on first use; unreadable or corrupt
 * entries are ignored.  Synchronises `stream`. */
triot_status triot_autotune(triot_op op, int n_tensors, int d, const int64_t *shapes,
                            const int64_t *counter_shape, void *const *tensors,
                            const int64_t *bases, const void *params, void *out,
                            void *workspace, size_t workspace_bytes, hipStream_t stream,
                            const char *cache_path);

/* Forget every tuned or pinned schedule held in memory (the defaults apply
 * again) and free the autotuner's flush buffers.  Not to be called while a
 * triot_autotune call is running. */
void triot_tune_reset(void);

/* A launch schedule of the element-wise co-iteration kernels. */
typedef struct triot_schedule {
    int vec_max;             /* widest lane access in 4-byte words: 1, 2 or 4 */
    int cache_policy;        /* 0 normal, 1 non-temporal loads and stores,
                                2 non-temporal loads only */
    int blocks_per_cu;       /* persistent workgroups per compute unit, 1..32 */
    int box_rows_max;        /* rows per box (LDS row table), 1..1024 */
    int unit_elems;          /* elements per work unit, 64..2^24 */
    int unit_order;          /* 0: each workgroup takes a contiguous range of
                                work units; 1: units dealt round-robin */
} triot_schedule;

/* Pin the schedule of one problem (same plan signature as triot_autotune):
 * every later call with that signature uses it, until triot_tune_reset or
 * another pin or tuning of the same signature.  No device work.  Returns
 * TRIOT_E_INVALID for a knob out of range and TRIOT_E_UNSUPPORTED for the
 * tuple-reading row kernels (moments and their adjoint), which have one
 * schedule.  Any value in range gives the same results as the defaults
 * (schedules change the speed only). */
triot_status triot_schedule_set(triot_op op, int n_tensors, int d, const int64_t *shapes,
                                const int64_t *counter_shape, void *const *tensors,
                                const int64_t *bases, const void *params,
                                const triot_schedule *schedule);

/* The schedule triot_apply uses for this problem: the one pinned or tuned
 * for its plan signature, else the defaults (4-word lanes where the rows
 * allow, non-temporal loads and stores, units of 8192 lanes, 1024 box
 * rows; 4 workgroups per CU and contiguous unit ranges, or for a COPY,
 * MUL_ACC, MUL or XPYX_MZ of at least 2^25 counter points 1 workgroup per
 * CU and round-robin units).  Same
 * arguments and errors as triot_schedule_set; no device work. */
triot_status triot_schedule_get(triot_op op, int n_tensors, int d, const int64_t *shapes,
                                const int64_t *counter_shape, void *const *tensors,
                                const int64_t *bases, const void *params,
                                triot_schedule *schedule);

/* Set the launch schedule of a batch (lane width, cache policy, blocks per
 * CU, box rows, unit size, unit order; a vec_max of 4 lets items take
 * 4-word lanes, 1 or 2 keeps 1-word lanes; unit_order 0 gives each
 * workgroup a contiguous range of the work units of all items, 1 deals
 * them round-robin).  Releases the planned table and graph: the next
 * triot_apply_batched plans and captures afresh.  The default is 4-word
 * lanes, non-temporal loads and stores, 8 blocks per CU, units of 4096
 * lanes, 1024 box rows, round-robin units.  TRIOT_E_INVALID for a knob out
 * of range. */
triot_status triot_batch_set_schedule(triot_batch *handle, const triot_schedule *schedule);

/* The schedule a batch handle plans with: the one set by
 * triot_batch_set_schedule or chosen by triot_batch_autotune, else the
 * default above (a schedule tuned earlier for the same batch layout on
 * another handle is used by triot_apply_batched but not reported here).
 * No device work.  TRIOT_E_INVALID for null arguments. */
triot_status triot_batch_get_schedule(const triot_batch *handle, triot_schedule *schedule);

/* Autotuner of the batched persistent launch (the schedules of its work
 * table: the zero padding of thousands of ragged items ahead of FFT
 * convolutions, Section 3, in one launch).  Validates the batch as
 * triot_apply_batched does (same errors), then times the one persistent
 * launch of this batch on `stream` under candidate schedules -- lane width
 * (4 or 1 words), cache policy, workgroups per CU, work-unit size and unit
 * order, by coordinate descent from the handle's current schedule, two
 * passes -- each cold, after a write over a 512 MiB device buffer as in
 * triot_autotune.  The fastest becomes the handle's schedule (as if set by
 * triot_batch_set_schedule: the next triot_apply_batched plans and
 * captures with it), is remembered in memory for every later batch with
 * the same layout (op, element size, and every item's shapes, counter,
 * bases and address alignment; not the addresses), and is appended to the
 * JSON cache at cache_path (NULL = in memory only; TRIOT_TUNE_CACHE loads
 * such entries too).  The operation RUNS several times on the given
 * buffers: pass scratch copies for in-place ops (MUL_ACC).  Allocates
 * device memory for the candidate tables and frees it before returning;
 * synchronises `stream`.  A batch with no points returns TRIOT_OK and
 * changes nothing. */
triot_status triot_batch_autotune(triot_batch *handle, triot_op op, int n_items,
                                  const triot_item *items, const void *params,
                                  hipStream_t stream, const char *cache_path);

/* ---- diagnostics -------------------------------------------------------- */

const char *triot_status_string(triot_status status);

/* Multiplier m and shift s with which the kernels divide a 32-bit n by
 * the invariant divisor c: with h = (n*m) >> 32,
 *     n / c == (h + ((n - h) >> 1)) >> s            for every n < 2^32
 * (Granlund & Montgomery, "Division by invariant integers using
 * multiplication", PLDI 1994, the round-up variant with an add-back).
 * c >= 2.  Returns TRIOT_E_INVALID for c < 2. */
triot_status triot_divmod_magic(uint32_t c, uint32_t *m, uint32_t *s);

/* The launch plan triot_apply would use, for inspection and tests. */
typedef struct triot_plan_info {
    int kernel;              /* 0 = element-wise co-iteration, 1 = per-row segments (moments) */
    int dims;                /* axes after dropping extent-1 axes and merging */
    int64_t extents[TRIOT_MAX_D]; /* the planned counter, outermost first */
    int vec;                 /* 4-byte words per lane access (1, 2, 4) */
    int high_axes;           /* axes decoded once per box (per work unit) */
    int low_axes;            /* outer axes tabulated per box row */
    int64_t box_rows;        /* rows per box */
    int64_t units;           /* work units of the launch */
    int blocks;              /* workgroups of the launch */
    int threads;             /* threads per workgroup */
    int unroll;              /* elements per thread per step */
    int inner_unit;          /* 1 when every operand is contiguous on the inner axis */
    int cache_policy;        /* 0 normal, 1 non-temporal loads and stores,
                                2 non-temporal loads only */
    int unit_order;          /* 0 contiguous ranges, 1 round-robin */
    int row_tail;            /* inner extent not a multiple of vec: the words in
                                each row's last vector, which is moved back to
                                end at the row end (0: rows are whole vectors) */
} triot_plan_info;

triot_status triot_plan_describe(triot_op op, int n_tensors, int d, const int64_t *shapes,
                                 const int64_t *counter_shape, void *const *tensors,
                                 const int64_t *bases, const void *params,
                                 triot_plan_info *info);

#ifdef __cplusplus
}
#endif

#endif /* TRIOT_H */
