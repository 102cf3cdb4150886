/*
 * Dense FP64 CPU oracle for moment and cumulant tensors of multivariate data.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never links, loads or calls it, and the two share no code.
 *
 * What it computes (Domino, Gawron, Pawela, "Efficient computation of higher
 * order cumulant tensors"):
 *   - the column means and the centred data X~ = X - E(X)   (Def. of the
 *     centred variable, Section 1.3);
 *   - the d-th moment tensor of X~, every entry of the full n^d tensor, as
 *     m_i = (1/t) * sum_l prod_k x~_{l,i_k}                 (Def. of the d-th
 *     moment tensor, Section 1.3);
 *   - the cumulants by the partition recursion of Section 3.2 (the final
 *     formula, eq. cum_r): c_2 = m_2, c_3 = m_3 and for d >= 4
 *     c_i = m_i - sum over set partitions of the d positions into >= 2 parts,
 *     each part of size >= 2, of the product of lower cumulants restricted to
 *     the part's positions.
 * There is no block structure, no symmetry and no blocking here: every
 * multi-index is computed on its own.  Sums over samples are Neumaier-
 * compensated and run in sample order; products run left to right in
 * position order.  Build with -O2 -ffp-contract=off and no fast-math.
 *
 * Readings taken where the paper is loose:
 *   - normalisation is 1/t everywhere (plug-in estimator, the derivatives at
 *     0 of the empirical cumulant generating function of Section 1.3);
 *   - "non-crossing sub-tuples" in the partition definition is read as
 *     pairwise disjoint parts (all set partitions), which the Stirling count
 *     and the crossing term of the printed 4th-cumulant formula require.
 *
 * Indexing is 0-based.  Dense tensors are stored in odometer order with the
 * first index slowest: offset(i) = sum_k i_k * n^(d-1-k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 10

/* ------------------------------------------------------------------ */
/* Compensated (Neumaier) accumulation.                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    double s, c;
} orc_acc;

static inline void acc_add(orc_acc *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double acc_value(const orc_acc *a) { return a->s + a->c; }

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

static long ipow(long a, int e) {
    long r = 1;
    for (int k = 0; k < e; ++k) r *= a;
    return r;
}

/* ------------------------------------------------------------------ */
/* Centring: Def. of the centred variable (Section 1.3).               */
/* mean[i] = (sum_l X[l*ldx+i]) / t, Xc[l*n+i] = X[l*ldx+i] - mean[i]. */
/* ------------------------------------------------------------------ */
int orc_center(const double *X, long t, int n, long ldx, double *mean, double *Xc) {
    if (!X || !mean || t < 1 || n < 1 || ldx < n) return -1;
    for (int i = 0; i < n; ++i) {
        orc_acc a = {0.0, 0.0};
        for (long l = 0; l < t; ++l) acc_add(&a, X[l * ldx + i]);
        mean[i] = acc_value(&a) / (double)t;
    }
    if (Xc) {
        for (long l = 0; l < t; ++l)
            for (int i = 0; i < n; ++i) Xc[l * n + i] = X[l * ldx + i] - mean[i];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Moment tensor: Def. of the d-th moment (Section 1.3), every entry.   */
/* ------------------------------------------------------------------ */
static double moment_entry(const double *Xc, long t, int n, int d, const int *idx) {
    orc_acc a = {0.0, 0.0};
    for (long l = 0; l < t; ++l) {
        const double *row = Xc + l * n;
        double p = row[idx[0]];
        for (int k = 1; k < d; ++k) p = p * row[idx[k]];
        acc_add(&a, p);
    }
    return acc_value(&a) / (double)t;
}

static void decode(long e, int n, int d, int *idx) {
    for (int k = d - 1; k >= 0; --k) {
        idx[k] = (int)(e % n);
        e /= n;
    }
}

int orc_moment_dense(const double *Xc, long t, int n, int d, double *M) {
    if (!Xc || !M || t < 1 || n < 1 || d < 1 || d > ORC_MAXD) return -1;
    long total = ipow(n, d);
#pragma omp parallel for schedule(dynamic, 64)
    for (long e = 0; e < total; ++e) {
        int idx[ORC_MAXD];
        decode(e, n, d, idx);
        M[e] = moment_entry(Xc, t, n, d, idx);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Set partitions (Section 3.1, partition definitions).                */
/* A partition of positions 0..d-1 is stored as a label per position:   */
/* labels are numbered in order of first appearance, so parts come out  */
/* ordered by their smallest position and each part lists positions in */
/* increasing order.  Every set partition is produced exactly once, by  */
/* placing position k either in one of the parts opened so far or in a */
/* new part.                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int d;
    int min_part;   /* keep partitions whose parts all have >= min_part elements */
    int min_parts;  /* keep partitions with >= min_parts parts                   */
    int count, cap;
    int *labels;    /* cap * d                                                   */
} part_list;

static void part_rec(part_list *pl, int *lab, int k, int nparts) {
    if (k == pl->d) {
        if (nparts < pl->min_parts) return;
        int size[ORC_MAXD] = {0};
        for (int a = 0; a < pl->d; ++a) size[lab[a]]++;
        for (int r = 0; r < nparts; ++r)
            if (size[r] < pl->min_part) return;
        if (pl->labels && pl->count < pl->cap) memcpy(pl->labels + (long)pl->count * pl->d, lab, sizeof(int) * pl->d);
        pl->count++;
        return;
    }
    for (int r = 0; r <= nparts; ++r) {
        lab[k] = r;
        part_rec(pl, lab, k + 1, r == nparts ? nparts + 1 : nparts);
    }
}

/* Enumerate the set partitions of d positions whose parts all have at least
 * min_part elements and which have at least min_parts parts.  Writes up to
 * cap label vectors (d ints each) into labels (may be NULL to count only) and
 * returns the total count, or -1 on bad arguments. */
int orc_partitions(int d, int min_part, int min_parts, int *labels, int cap) {
    if (d < 1 || d > ORC_MAXD) return -1;
    part_list pl = {d, min_part, min_parts, 0, cap, labels};
    int lab[ORC_MAXD];
    part_rec(&pl, lab, 0, 0);
    return pl.count;
}

/* Partitions used by the recursion: parts of size >= 2, at least 2 parts. */
static int recursion_partitions(int d, int **out) {
    int cnt = orc_partitions(d, 2, 2, NULL, 0);
    *out = NULL;
    if (cnt <= 0) return cnt;
    *out = (int *)malloc(sizeof(int) * (size_t)cnt * (size_t)d);
    if (!*out) return -2;
    orc_partitions(d, 2, 2, *out, cnt);
    return cnt;
}

/* ------------------------------------------------------------------ */
/* Cumulants, dense: the recursion of Section 3.2 (eq. cum_r) over the  */
/* full n^d tensors.  K[d-2] receives the order-d cumulant for          */
/* d = 2..dmax, each an n^d array.                                      */
/* ------------------------------------------------------------------ */
int orc_cumulants_dense(const double *Xc, long t, int n, int dmax, double **K) {
    if (!Xc || !K || t < 1 || n < 1 || dmax < 2 || dmax > ORC_MAXD) return -1;
    for (int d = 2; d <= dmax; ++d) {
        if (!K[d - 2]) return -1;
        int rc = orc_moment_dense(Xc, t, n, d, K[d - 2]);
        if (rc) return rc;
        if (d < 4) continue; /* c_2 = m_2 and c_3 = m_3 */
        int *parts = NULL;
        int np = recursion_partitions(d, &parts);
        if (np < 0) return np;
        long total = ipow(n, d);
#pragma omp parallel for schedule(static)
        for (long e = 0; e < total; ++e) {
            int idx[ORC_MAXD];
            decode(e, n, d, idx);
            double sum = 0.0;
            for (int z = 0; z < np; ++z) {
                const int *lab = parts + (long)z * d;
                int nparts = 0;
                for (int a = 0; a < d; ++a)
                    if (lab[a] + 1 > nparts) nparts = lab[a] + 1;
                double prod = 1.0;
                for (int r = 0; r < nparts; ++r) {
                    /* offset of the sub-index (positions of part r, ascending) */
                    long off = 0;
                    int m = 0;
                    for (int a = 0; a < d; ++a)
                        if (lab[a] == r) {
                            off = off * n + idx[a];
                            ++m;
                        }
                    prod = prod * K[m - 2][off];
                }
                sum = sum + prod;
            }
            K[d - 2][e] = K[d - 2][e] - sum;
        }
        free(parts);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cumulants at chosen multi-indices (sampled mode).                    */
/* For each requested index i of order d, every sub-index i_S (S a set */
/* of positions, ascending) with |S| >= 2 gets its moment from one pass */
/* over the samples, and its cumulant from the same recursion as the    */
/* dense routine, applied to S.  Subsets are visited in increasing     */
/* bit-mask order, so every proper subset is ready before S needs it.   */
/* The arithmetic (product order, summation order, partition order) is */
/* the dense routine's, so both give identical values.                  */
/* ------------------------------------------------------------------ */
int orc_cumulant_at(const double *Xc, long t, int n, int d, const int *idx, long count, double *out) {
    if (!Xc || !idx || !out || t < 1 || n < 1 || d < 2 || d > ORC_MAXD || count < 0) return -1;
    for (long q = 0; q < count * d; ++q)
        if (idx[q] < 0 || idx[q] >= n) return -1;
    /* partition tables for every subset size 4..d */
    int *parts[ORC_MAXD + 1] = {0};
    int nparts_of[ORC_MAXD + 1] = {0};
    for (int m = 4; m <= d; ++m) {
        nparts_of[m] = recursion_partitions(m, &parts[m]);
        if (nparts_of[m] < 0) return nparts_of[m];
    }
    const int nmask = 1 << d;
    int rc = 0;
#pragma omp parallel
    {
        orc_acc *acc = (orc_acc *)malloc(sizeof(orc_acc) * (size_t)nmask);
        double *prod = (double *)malloc(sizeof(double) * (size_t)nmask);
        double *kap = (double *)malloc(sizeof(double) * (size_t)nmask);
        int ok = acc && prod && kap;
#pragma omp for schedule(dynamic, 1)
        for (long q = 0; q < count; ++q) {
            if (!ok) {
#pragma omp atomic write
                rc = -2;
                continue;
            }
            const int *ix = idx + q * d;
            for (int s = 0; s < nmask; ++s) acc[s].s = acc[s].c = 0.0;
            for (long l = 0; l < t; ++l) {
                const double *row = Xc + l * n;
                /* prod[S] = product over the positions of S in ascending order */
                for (int s = 1; s < nmask; ++s) {
                    int top = 31 - __builtin_clz((unsigned)s);
                    int rest = s & ~(1 << top);
                    prod[s] = rest ? prod[rest] * row[ix[top]] : row[ix[top]];
                    if (__builtin_popcount((unsigned)s) >= 2) acc_add(&acc[s], prod[s]);
                }
            }
            for (int s = 1; s < nmask; ++s) {
                int m = __builtin_popcount((unsigned)s);
                if (m < 2) continue;
                double mom = acc_value(&acc[s]) / (double)t;
                if (m < 4) {
                    kap[s] = mom;
                    continue;
                }
                int pos[ORC_MAXD], mm = 0;
                for (int a = 0; a < d; ++a)
                    if (s >> a & 1) pos[mm++] = a;
                double sum = 0.0;
                for (int z = 0; z < nparts_of[m]; ++z) {
                    const int *lab = parts[m] + (long)z * m;
                    int np = 0;
                    for (int a = 0; a < m; ++a)
                        if (lab[a] + 1 > np) np = lab[a] + 1;
                    double pr = 1.0;
                    for (int r = 0; r < np; ++r) {
                        int sub = 0;
                        for (int a = 0; a < m; ++a)
                            if (lab[a] == r) sub |= 1 << pos[a];
                        pr = pr * kap[sub];
                    }
                    sum = sum + pr;
                }
                kap[s] = mom - sum;
            }
            out[q] = kap[nmask - 1];
        }
        free(acc);
        free(prod);
        free(kap);
    }
    for (int m = 4; m <= d; ++m) free(parts[m]);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Block storage (Section 2.1), as read by the tests.                   */
/* Blocks are the sorted block tuples j_1 <= ... <= j_d over            */
/* nbar = ceil(n/b) block indices, in lexicographic order; each block is */
/* a b^d cube, in-block index row-major (first position slowest).       */
/* Entries whose variable index j_k*b + r_k falls beyond n are padding. */
/* The tuples are produced by a plain odometer over [0,nbar)^d that     */
/* keeps only the non-decreasing ones.                                  */
/* ------------------------------------------------------------------ */
static long sorted_tuples(int nbar, int d, int *out /* may be NULL */) {
    long total = ipow(nbar, d), cnt = 0;
    int j[ORC_MAXD];
    for (long e = 0; e < total; ++e) {
        decode(e, nbar, d, j);
        int ok = 1;
        for (int k = 1; k < d; ++k)
            if (j[k] < j[k - 1]) ok = 0;
        if (!ok) continue;
        if (out) memcpy(out + cnt * d, j, sizeof(int) * d);
        ++cnt;
    }
    return cnt;
}

/* Number of stored entries (blocks * b^d). */
long orc_block_elems(int n, int d, int b) {
    if (n < 1 || d < 1 || d > ORC_MAXD || b < 1 || b > n) return -1;
    int nbar = (n + b - 1) / b;
    return sorted_tuples(nbar, d, NULL) * ipow(b, d);
}

/* For each stored offset, the multi-index it holds (d ints), or all -1 for
 * a padding position. */
int orc_block_indices(int n, int d, int b, const long *offsets, long count, int *idx) {
    if (n < 1 || d < 1 || d > ORC_MAXD || b < 1 || b > n || count < 0) return -1;
    int nbar = (n + b - 1) / b;
    long nblk = sorted_tuples(nbar, d, NULL);
    int *tup = (int *)malloc(sizeof(int) * (size_t)(nblk * d));
    if (!tup) return -2;
    sorted_tuples(nbar, d, tup);
    long be = ipow(b, d);
    for (long q = 0; q < count; ++q) {
        long o = offsets[q];
        int *ix = idx + q * d;
        if (o < 0 || o >= nblk * be) {
            free(tup);
            return -1;
        }
        long blk = o / be, in = o % be;
        int r[ORC_MAXD];
        decode(in, b, d, r);
        int pad = 0;
        for (int k = 0; k < d; ++k) {
            ix[k] = tup[blk * d + k] * b + r[k];
            if (ix[k] >= n) pad = 1;
        }
        if (pad)
            for (int k = 0; k < d; ++k) ix[k] = -1;
    }
    free(tup);
    return 0;
}

/* Read the dense n^d tensor at every stored position (no averaging). */
int orc_fold(const double *dense, int n, int d, int b, double *blocks) {
    if (!dense || !blocks || n < 1 || d < 1 || d > ORC_MAXD || b < 1 || b > n) return -1;
    int nbar = (n + b - 1) / b;
    long nblk = sorted_tuples(nbar, d, NULL);
    int *tup = (int *)malloc(sizeof(int) * (size_t)(nblk * d));
    if (!tup) return -2;
    sorted_tuples(nbar, d, tup);
    long be = ipow(b, d);
    for (long blk = 0; blk < nblk; ++blk) {
        for (long in = 0; in < be; ++in) {
            int r[ORC_MAXD];
            decode(in, b, d, r);
            long off = 0;
            int pad = 0;
            for (int k = 0; k < d; ++k) {
                int v = tup[blk * d + k] * b + r[k];
                if (v >= n) pad = 1;
                off = off * n + v;
            }
            blocks[blk * be + in] = pad ? 0.0 : dense[off];
        }
    }
    free(tup);
    return 0;
}
