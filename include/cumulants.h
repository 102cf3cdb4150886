/*
 * cumulants.h -- C ABI of the MI355X (gfx950) moment and cumulant tensor
 * library.
 *
 * Method: Domino, Gawron, Pawela, "Efficient computation of higher order
 * cumulant tensors".  The library computes
 *   - the column means and centred data (Def. of the centred variable,
 *     Section 1.3),
 *   - the d-th moment tensor m_i = (1/t) sum_l prod_k x_{l,i_k}
 *     (Def. of the d-th moment, Section 1.3) in the block storage of
 *     Section 2.1, only on sorted block tuples (Alg. 1 and Alg. 2, with the
 *     sample range split into chunks and reduced as in Alg. 3),
 *   - the cumulants c_2..c_dmax by the recursion of Section 3.2 (eq. cum_r;
 *     Alg. 4 and Alg. 5): c_2 = m_2, c_3 = m_3, and for d >= 4 the central
 *     moment minus the sum over partitions of the d positions into >= 2
 *     parts of size >= 2 of products of lower-order cumulants,
 *   - the same for many datasets in one graph-captured run (cum_batch_*) and
 *     for a sliding window of samples (cum_stream_*, with the general
 *     formula of Section 5.3 as a second finalisation).
 * Normalisation is 1/t throughout (plug-in estimator, so c_2 is the biased
 * covariance).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Data X is t x n, rows = samples, columns = variables (the data matrix of
 *   Section 1.3), row-major with leading dimension ldx >= n.
 * - Pointers are DEVICE pointers unless marked (host).  The caller owns every
 *   buffer; the library never frees caller memory.  Scratch memory is the
 *   caller's workspace, sized by cum_workspace_size().  The library keeps
 *   small index tables of its own in device memory, one set per
 *   configuration (n, b, orders, precision, launch shape; not per sample
 *   count), allocated on first use and freed at process exit.  Batch plans
 *   and streams own their device state until destroyed.
 * - stream is a hipStream_t passed as void* (NULL = the default stream).
 *   Work is enqueued asynchronously on it; outputs are valid once the stream
 *   has reached that point.  Calls that share a workspace must not overlap.
 * - Arguments are validated on the host before anything is enqueued; an
 *   invalid call returns a status and enqueues nothing.  No C++ exception
 *   crosses this boundary.  cum_last_error() gives a message for the last
 *   failing call of the calling thread.
 *
 * Block storage (Section 2.1)
 * ---------------------------
 * With nbar = ceil(n/b), an order-d tensor is stored as the blocks of all
 * sorted block tuples j_1 <= ... <= j_d over 0..nbar-1, in lexicographic
 * order of the tuple; there are C(nbar+d-1, d) of them (the paper prints the
 * binomial as C(nbar+d-1, nbar), which miscounts for nbar >= 3).  Each block
 * is a padded b^d cube, in-block index row-major (first position slowest):
 *   offset(j, r) = rank(j) * b^d + sum_k r_k * b^(d-1-k),
 * holding the entry at variable multi-index (j_k*b + r_k)_k.  Diagonal blocks
 * hold all b^d entries, redundant ones included (Alg. 1 loops over the whole
 * block).  Positions whose variable index reaches n (ragged last block,
 * b_l = n - b(nbar-1)) hold 0.
 */
#ifndef CUMULANTS_H
#define CUMULANTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CUM_OK = 0,
    CUM_EINVAL = -1,       /* invalid argument (nothing enqueued)              */
    CUM_ENOMEM = -2,       /* workspace too small, or a table allocation failed */
    CUM_EHIP = -3,         /* a HIP runtime call failed (see cum_last_error)   */
    CUM_EUNSUPPORTED = -4  /* valid but unsupported combination                 */
} cum_status;

/* Arithmetic of the moment contraction (the sum over samples of Alg. 1).
 * Centring, the cross-chunk reduction and the cumulant recursion are FP64 in
 * every mode.  Calls that centre their own data (cum_cumulants, batches,
 * streams) with d_max >= 7 stage and contract in FP64 whatever prec says:
 * rounding the centred samples to FP32 alone leaves cumulants of orders 7
 * and above on heavy-tailed data more than 1e-6 (relative) off. */
typedef enum {
    CUM_F64 = 0,    /* FP64 data, FP64 matrix-core products and sums            */
    CUM_F32 = 1,    /* FP32 data, FP32 matrix-core products, FP32 sums over at  */
                    /* most 64 samples, then FP64                               */
    CUM_BF16X2 = 2, /* FP32 data; each half-product split into two BF16 terms, */
                    /* all 4 cross products on BF16 matrix cores, FP32 sums    */
                    /* over at most 64 samples, then FP64                       */
    CUM_BF16X3 = 3, /* as BF16X2 with a three-term split and the 6 cross       */
                    /* products of combined weight >= 2^-16                     */
    CUM_F16X2 = 4,  /* FP32 data, each variable's centred values first divided */
                    /* by a power of two that brings them below 32; each half- */
                    /* product v split into FP16 hi and lo = (v - hi) * 2^11   */
                    /* rounded to FP16 (22 bits of v), the 3 cross products    */
                    /* hh, hl, lh on FP16 matrix cores, FP32 sums over at most */
                    /* 64 samples, then FP64, the powers of two undone exactly */
                    /* (orders 2..6; calls with d_max >= 7 that centre their   */
                    /* own data stage in FP64 as for every prec)               */
    /* Not precisions: these give the enum the range of int32_t, so that an
     * unknown value is a valid cum_prec object that the library rejects with
     * CUM_EUNSUPPORTED (without them, reading one is undefined in C++). */
    CUM_PREC_RANGE_LO_ = -2147483647 - 1,
    CUM_PREC_RANGE_HI_ = 2147483647
} cum_prec;

/* Block layout of one order (Section 2.1). */
typedef struct {
    int32_t n, d, b;
    int32_t nbar;         /* ceil(n/b)                                       */
    int32_t b_last;       /* n - b*(nbar-1), size of the ragged last block   */
    int64_t nblocks;      /* C(nbar+d-1, d) sorted block tuples              */
    int64_t block_elems;  /* b^d                                             */
    int64_t elems;        /* nblocks * b^d stored doubles                    */
} cum_layout;

/* Largest supported order. */
#define CUM_MAX_ORDER 10

/* Host only.  Layout of the order-d block storage for n variables and block
 * size b.  Requires n >= 1, 1 <= b <= n, 1 <= d <= CUM_MAX_ORDER. */
cum_status cum_layout_query(int n, int d, int b, cum_layout *out /* host */);

/* Host only.  Bytes of device workspace needed by cum_cumulants(t, n, d_max,
 * b, prec) (from d_max = 7 on, this includes the central moments of orders
 * 2..d_max-2 in block storage); it is also enough for cum_center(t, n, prec)
 * and for cum_moment_blocks(t, n, d, b, prec) with d <= d_max. */
cum_status cum_workspace_size(int64_t t, int n, int d_max, int b, cum_prec prec, size_t *bytes /* host */);

/* Column means and centred data (Def. of the centred variable, Section 1.3).
 *   X     t x n FP64, leading dimension ldx >= n (read only)
 *   mean  n FP64 out: mean[i] = (1/t) sum_l X[l][i] (compensated FP64 sums in a
 *         fixed order)
 *   Xc    t x n out, leading dimension n: X[l][i] - mean[i] computed in FP64,
 *         stored as FP64 for CUM_F64 and rounded to FP32 (nearest-even) for
 *         every other prec.  May be NULL (means only).
 * Requires t >= 1, n >= 1. */
cum_status cum_center(const double *X, int64_t t, int n, int64_t ldx, cum_prec prec, double *mean, void *Xc,
                      void *ws, size_t ws_bytes, void *stream);

/* Order-d moment tensor of the data AS GIVEN (no centring), in block storage
 * (Def. of the d-th moment; Alg. 1 and 2; sample chunks reduced in FP64 in a
 * fixed order as in Alg. 3, divided by t once).
 *   Xc  t x n, leading dimension n, FP64 for CUM_F64, FP32 otherwise
 *   M   cum_layout.elems FP64 out
 * Requires t >= 1, 1 <= b <= n, 2 <= d <= CUM_MAX_ORDER.  Results are
 * deterministic: the same call gives bitwise the same output.  With
 * CUM_F16X2 (d <= 6, else CUM_EUNSUPPORTED) each variable is first divided
 * by a power of two that brings its values, about zero, below 32. */
cum_status cum_moment_blocks(const void *Xc, cum_prec prec, int64_t t, int n, int d, int b, double *M, void *ws,
                             size_t ws_bytes, void *stream);

/* Cumulant tensors c_2..c_dmax of X (Alg. 5 for every order in turn; orders
 * 7 and above use the equivalent moment-cumulant relation split at the first
 * position, over the central moments of lower orders kept in the workspace).
 *   X      t x n FP64, leading dimension ldx >= n
 *   mean   n FP64 out (the first cumulant), or NULL
 *   kappa  (host) array of d_max-1 device pointers; kappa[d-2] receives c_d
 *          in block storage (cum_layout(n, d, b).elems FP64 each)
 * The data are centred in FP64; only the moment contraction runs in prec
 * (in FP64 when d_max >= 7, see cum_prec).
 * Requires t >= 1, 1 <= b <= n, 2 <= d_max <= CUM_MAX_ORDER.  The first call
 * of a configuration builds its tables (device allocations); later calls
 * allocate nothing and enqueue only kernels, so they may be captured in a
 * HIP graph. */
cum_status cum_cumulants(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec,
                         double *mean, double *const *kappa /* host array */, void *ws, size_t ws_bytes,
                         void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as cum_cumulants (bitwise, for the same
 * configuration), with the workspace taken from a fixed scratch array that
 * the library holds on each GPU until the process ends, so the call
 * allocates nothing and needs no ws argument.
 *   - The scratch holds CUM_NOALLOC_SCRATCH_BYTES; a call that would need
 *     more than cum_workspace_size(t, n, d_max, b, prec) of it returns
 *     CUM_ENOMEM and enqueues nothing.
 *   - The configuration's device tables must already exist: run
 *     cum_cumulants once with the same n, b, d_max, prec, tuning and a t of
 *     the same sample-chunk count first; otherwise CUM_EUNSUPPORTED and
 *     nothing is enqueued.
 *   - Every call on one GPU shares that GPU's scratch, which keeps the last
 *     call's contents (nothing in it needs to start at zero).  Calls that
 *     overlap on one GPU (other streams, other threads) race on it.
 * Arguments as for cum_cumulants. */
#define CUM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
cum_status cum_cumulants_noalloc(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec,
                                 double *mean, double *const *kappa /* host array */, void *stream);

/* Unfold an order-d block-stored tensor to the dense n^d array (first index
 * slowest).  Entry i is read from the canonical stored copy: the position
 * reached by sorting i_1..i_d ascending, so the output is exactly symmetric
 * even where redundant stored copies differ in their last bits (Def. of a
 * super-symmetric tensor, Section 1.3; block storage, Section 2.1). */
cum_status cum_unfold(const double *blocks, int n, int d, int b, double *dense, void *stream);

/* Host only.  Block-storage offset of the canonical stored copy of the
 * multi-index idx[0..d-1] (each 0 <= idx[k] < n): the indices are sorted
 * ascending first. */
cum_status cum_stored_offset(int n, int d, int b, const int32_t *idx /* host */, int64_t *offset /* host */);

/* ------------------------------------------------------------------------
 * Autotuning of the contraction (the paper picks its block size b by
 * timing, Section 5.2; here b is the caller's storage choice, and the tuned
 * knobs are the block size the contraction works in and the launch's):
 *   shape         one wave's task in one order's (rows x columns) product:
 *                 0 = 32 x 32, 2 = 32 x 64 entries (four tasks per
 *                 work-group, packed so that waves have equal work);
 *   target_items  about how many (tile, sample-chunk) work items to create;
 *                 it sets the sample chunk length, hence the split over
 *                 samples and the size of the FP64 partial-sum buffer;
 *   inner_b       1..b: block size of the layout the contraction fills.
 *                 With inner_b = b every stored entry is summed, redundant
 *                 copies in diagonal blocks included (as Alg. 1 does); with
 *                 a smaller inner_b fewer redundant copies are summed (with
 *                 1, each distinct sorted variable tuple once), and the
 *                 reduction reads each stored entry's sums at its sorted
 *                 variable tuple.  Default 1.
 * A tuned choice applies to later calls with the same (t, n, d_max, b, prec)
 * and changes their workspace size: query cum_workspace_size afterwards.
 * With the environment variable CUM_TUNE_FILE set, choices are also read
 * from and written to that file (one line per shape).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t shape;
    int32_t target_items;
    int32_t inner_b;
    float ms;  /* autotune: measured time of the chosen configuration */
} cum_tuning;

/* Time every candidate configuration of cum_cumulants(t, n, d_max, b, prec)
 * on the caller's data X (t x n FP64, ld ldx, device) -- contraction plus
 * reduction and recursion, best of three after a warm-up, HIP events on
 * stream -- and keep the fastest.  Allocates and frees its own device
 * workspace; synchronises stream.  best (host) may be NULL. */
cum_status cum_autotune(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec,
                        void *stream, cum_tuning *best /* host */);

/* Host only.  Set (tune != NULL) or forget (tune == NULL) the configuration
 * used for cum_cumulants(t, n, d_max, b, prec).  CUM_EINVAL for an unknown
 * shape, target_items < 1 or inner_b outside 1..b. */
cum_status cum_set_tuning(int64_t t, int n, int d_max, int b, cum_prec prec, const cum_tuning *tune /* host */);

/* Host only.  How cum_cumulants(t, n, d_max, b, prec) splits its work in
 * its current configuration (tuned, else the defaults). */
typedef struct {
    int64_t nchunks;          /* sample chunks (each a run of whole stages)       */
    int64_t work_items;       /* (tile, chunk) items of the contraction launch    */
    int64_t tiles;            /* work-group tiles over all orders                 */
    int64_t partial_entries;  /* sums per chunk (layout of the inner block size)  */
    int64_t stored_entries;   /* outputs of orders 2..d_max in block storage      */
} cum_plan_info;
cum_status cum_get_plan_info(int64_t t, int n, int d_max, int b, cum_prec prec, cum_plan_info *info /* host out */);

/* Host only.  The configuration cum_cumulants(t, n, d_max, b, prec) uses:
 * the tuned one if there is one, else the defaults (ms = 0). */
cum_status cum_get_tuning(int64_t t, int n, int d_max, int b, cum_prec prec, cum_tuning *tune /* host out */);

/* ------------------------------------------------------------------------
 * Batched cumulants: many datasets of the same width n and uneven sample
 * counts, captured once in a HIP graph and replayed: one batched centring
 * launch, then the datasets in groups of about equal work (one group per 128
 * datasets, at most 4).  Each group is one launch of the moment contraction over
 * its (dataset, tile, sample-chunk) work items, in group order; a group's
 * chunk sums and finalisation (reduction and recursion, one launch per pair
 * of orders; orders 7 and above by the first-position formula over each
 * dataset's lower central moments) run on a second stream as soon as its
 * contraction is done, beside the next group's contraction, so the first
 * groups' results are ready before the whole batch is.  The environment
 * variable CUM_BATCH_GROUPS, read when a plan is laid out, fixes the group
 * count (at most 8).  Results are deterministic (the same plan gives bitwise the same
 * output on every run, and the group count does not change the bits) and
 * carry the accuracy of cum_cumulants() for the same prec.
 * ------------------------------------------------------------------------ */
typedef struct cum_batch cum_batch;

/* Host only (allocates the plan's device memory).  t_i (host, n_sets
 * entries, each >= 1).  With CUM_F16X2 each dataset has its own scales. */
cum_status cum_batch_create(int n_sets, const int64_t *t_i /* host */, int n, int d_max, int b, cum_prec prec,
                            cum_batch **plan /* host out */);

/*   X_i    (host) n_sets device pointers, dataset s is t_i[s] x n FP64, ld n
 *   kappa  (host) n_sets*(d_max-1) device pointers: kappa[s*(d_max-1)+d-2]
 *          receives c_d of dataset s in block storage
 *   mean   (host) n_sets device pointers (n FP64 each) or NULL
 * The first call captures the graph on stream; later calls copy the pointer
 * tables and replay it. */
cum_status cum_batch_run(cum_batch *plan, const double *const *X_i, double *const *kappa, double *const *mean,
                         void *stream);

/* Host only.  After a cum_batch_run has completed: per-dataset device
 * timestamps (ticks of the 100 MHz constant clock), written when the
 * dataset's last order was finalised, and the start timestamp of the run.
 * ticks: n_sets entries.  Frequency in Hz goes to *hz. */
cum_status cum_batch_timestamps(cum_batch *plan, uint64_t *start /* host */, uint64_t *ticks /* host */,
                                double *hz /* host */);

/* Time the batch's candidate configurations (inner block size x tile shape x
 * work-item target) on the datasets X_i (host array of device pointers) and keep the
 * fastest for this plan (and for later plans of the same shape and count);
 * the graph is captured again on the next run.  Synchronises the device.
 * best (host) may be NULL. */
cum_status cum_batch_autotune(cum_batch *plan, const double *const *X_i, cum_tuning *best /* host */);

cum_status cum_batch_destroy(cum_batch *plan);

/* ------------------------------------------------------------------------
 * Streaming windows.  Sums over samples are additive over disjoint sample
 * ranges (the chunk decomposition of Alg. 3, eq. mapred), so the moment sums
 * of a window of samples are the sums of its batches', and a batch leaves
 * the window by subtracting its sums.  A stream keeps, in FP64, the sums of
 * products of the shifted data y = x - c for orders 1..d_max (each sorted
 * variable tuple once) about a fixed shift c.  Cumulants of the window are
 * computed on demand: delta = mean(y), central moments by expanding
 * prod_k (y_k - delta_k) over the subsets of positions (binomial
 * re-centring), then the recursion of Section 3.2.  The products of each
 * batch run in prec as in cum_cumulants; the re-centring is exact algebra
 * in FP64, well conditioned while c stays near the window's mean (the
 * default shift is the first batch's mean).
 * ------------------------------------------------------------------------ */
typedef struct cum_stream cum_stream;

/* Host only (allocates the stream's device memory).  shift (host, n values)
 * or NULL: the mean of the first batch added becomes the shift.  With
 * CUM_F16X2 each batch has its own scales, bounding it about the shift. */
cum_status cum_stream_create(int n, int d_max, int b, cum_prec prec, const double *shift /* host */,
                             cum_stream **stream_out /* host out */);

/* Add (sign = +1) or remove (sign = -1) the batch X (t x n FP64, ld ldx,
 * device).  A removed batch must hold samples that were added (the window's
 * sums are exact sums, so removing what was added restores them up to
 * rounding).  CUM_EINVAL if the window would hold fewer than 0 samples.
 * Asynchronous on stream; when a batch is larger than any before, the
 * stream's workspace grows, which synchronises stream first. */
cum_status cum_stream_update(cum_stream *s, const double *X, int64_t t, int64_t ldx, int sign, void *stream);

/* The window's mean (device, n doubles, or NULL) and cumulants c_2..c_dmax
 * in block storage (kappa: host array of d_max-1 device pointers,
 * kappa[d-2] of cum_layout_query(n, d, b).elems doubles).  CUM_EINVAL if the
 * window holds no samples.  Asynchronous on stream. */
cum_status cum_stream_cumulants(cum_stream *s, double *mean, double *const *kappa, void *stream);

/* The same outputs by the general formula (eq. cumfmom, Section 5.3): each
 * cumulant as the sum over all B(d) set partitions of its positions of
 * (k-1)! (-1)^(k-1) (k parts) times the product of the window's moments
 * about the shift at the parts, with no centring and no recursion.  With
 * shift 0 the moments are raw moments: the general algorithm the paper
 * compares against, which loses accuracy to cancellation as the mean grows
 * against the spread.  Cost per entry grows with B(d) (15 at d = 4, 203 at
 * 6, 115975 at 10).  Asynchronous on stream. */
cum_status cum_stream_cumulants_moebius(cum_stream *s, double *mean, double *const *kappa, void *stream);

/* Host only.  Samples in the window. */
cum_status cum_stream_count(cum_stream *s, int64_t *t /* host out */);

/* Empty the window (the shift is kept).  Asynchronous on stream. */
cum_status cum_stream_reset(cum_stream *s, void *stream);

/* Synchronises the device, then frees the stream. */
cum_status cum_stream_destroy(cum_stream *s);

/* Host only.  Check that the moment-contraction tiling of order d covers
 * every stored entry exactly once and multiplies the variables stored there,
 * and that the rank table the reduction uses to find a sorted tuple's
 * partial sums gives every tuple's position (no GPU needed).  Returns CUM_OK
 * or CUM_EINVAL with a message. */
cum_status cum_plan_check(int n, int d, int b);

/* Host only.  Measurement helpers.  While enabled on the calling thread,
 * every kernel launch made by the entry points on that thread is bracketed by
 * two HIP events recorded on the launch's own stream.  cum_timing_read waits
 * for those events, writes the summed milliseconds and the launch count per
 * kernel kind (CUM_KIND_* below; arrays of CUM_NKINDS entries, host) and
 * forgets them.  Disabled by default; enabling adds two event records per
 * launch. */
#define CUM_KIND_CENTER 0  /* column sums, means, centring                   */
#define CUM_KIND_MOMENT 1  /* block moment contraction                       */
#define CUM_KIND_REDUCE 2  /* chunk reduction + cumulant recursion           */
#define CUM_KIND_UNFOLD 3  /* unfold to dense                                */
#define CUM_KIND_BATCH 4   /* a whole batched run (graph launch)             */
#define CUM_NKINDS 5
cum_status cum_timing_enable(int on);
cum_status cum_timing_read(double *ms /* host */, int64_t *launches /* host */);

const char *cum_status_str(cum_status s);
const char *cum_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CUMULANTS_H */
