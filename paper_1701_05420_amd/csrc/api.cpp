// Host planner and C ABI (include/cumulants.h).
//
// For each (n, b, d) the planner builds, once, the row (prefix) and column
// (suffix) feature tables of the order's contraction, the (v, w) rank table,
// per-32-block validity bounds, the sorted block tuples and the partition
// masks used by the recursion, and uploads them.  For each call shape it
// builds the tile list and the work-item list (tiles x sample chunks, ordered
// so that all items of one chunk land on the same XCD).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cumulants.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace cum {

static thread_local std::string g_last_error;

static cum_status fail(cum_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(CUM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// ---------------------------------------------------------------------------
// optional per-launch timing with HIP events on the launch's stream
// ---------------------------------------------------------------------------
struct TimedLaunch {
    hipEvent_t a, b;
    int kind;
};
static thread_local bool g_timing = false;
static thread_local std::vector<TimedLaunch> g_timed;

template <typename F>
static hipError_t timed(int kind, hipStream_t s, F &&launch) {
    if (!g_timing) return launch();
    TimedLaunch tl{nullptr, nullptr, kind};
    hipError_t e;
    if ((e = hipEventCreate(&tl.a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&tl.b)) != hipSuccess) return e;
    if ((e = hipEventRecord(tl.a, s)) != hipSuccess) return e;
    e = launch();
    hipError_t e2 = hipEventRecord(tl.b, s);
    g_timed.push_back(tl);
    return e != hipSuccess ? e : e2;
}

// ---------------------------------------------------------------------------
// combinatorics (host)
// ---------------------------------------------------------------------------
static int64_t binom(int64_t a, int64_t r) {
    if (r < 0 || a < r) return 0;
    __int128 v = 1;
    for (int64_t i = 1; i <= r; ++i) {
        v = v * (a - r + i) / i;
        if (v > (__int128)INT64_MAX) return -1;
    }
    return (int64_t)v;
}

// b^e for b >= 1, saturating at INT64_MAX (so that size guards on user
// input see a too-large value rather than a wrapped one).
static int64_t ipow64(int64_t b, int e) {
    int64_t r = 1;
    for (int k = 0; k < e; ++k) {
        if (b > 1 && r > INT64_MAX / b) return INT64_MAX;
        r *= b;
    }
    return r;
}

// Term of the lexicographic rank contributed by tuple position k of an
// order-d tuple, moving from previous entry a to entry c.
static int64_t rank_term(int nbar, int d, int k, int a, int c) {
    return binom(nbar - a + d - k - 1, d - k) - binom(nbar - c + d - k - 1, d - k);
}

static int64_t rank_sorted_host(const int *u, int m, int nbar) {
    int64_t s = 0;
    int prev = 0;
    for (int k = 0; k < m; ++k) {
        s += rank_term(nbar, m, k, prev, u[k]);
        prev = u[k];
    }
    return s;
}

// All sorted (non-decreasing) m-tuples over 0..nbar-1 in lexicographic order.
static std::vector<std::vector<int>> sorted_tuples(int nbar, int m) {
    std::vector<std::vector<int>> out;
    std::vector<int> u(m, 0);
    if (m == 0) {
        out.push_back(u);
        return out;
    }
    while (true) {
        out.push_back(u);
        int k = m - 1;
        while (k >= 0 && u[k] == nbar - 1) --k;
        if (k < 0) break;
        int v = u[k] + 1;
        for (int q = k; q < m; ++q) u[q] = v;
    }
    return out;
}

// Set partitions of d positions with every part of size >= 2 and at least
// two parts, as position masks.  Restricted growth strings a_0..a_{d-1}
// (a_0 = 0, a_k <= 1 + max of the earlier entries) are visited in
// lexicographic order, advancing the rightmost entry that can still grow
// (Knuth's Algorithm 7.2.1.5H, the generator the paper cites), and filtered.
static std::vector<std::vector<uint16_t>> recursion_partitions(int d) {
    std::vector<std::vector<uint16_t>> out;
    if (d < 4) return out;
    std::vector<int> a(d, 0);
    while (true) {
        int nparts = 0;
        for (int k = 0; k < d; ++k) nparts = std::max(nparts, a[k] + 1);
        std::vector<uint16_t> masks(nparts, 0);
        for (int k = 0; k < d; ++k) masks[a[k]] |= (uint16_t)(1u << k);
        bool ok = nparts >= 2;
        for (uint16_t m : masks)
            if (__builtin_popcount(m) < 2) ok = false;
        if (ok) out.push_back(masks);
        int k = d - 1;
        while (k >= 1) {
            int lim = 0;
            for (int q = 0; q < k; ++q) lim = std::max(lim, a[q] + 1);
            if (a[k] < lim) break;
            --k;
        }
        if (k < 1) break;
        ++a[k];
        for (int q = k + 1; q < d; ++q) a[q] = 0;
    }
    return out;
}

// Every set partition of d positions (restricted growth strings, in their
// lexicographic order), each as its part masks in order of first position,
// with the weight (k-1)! (-1)^(k-1) of a partition into k parts (the
// moment-to-cumulant formula eq. cumfmom).
static void all_partitions(int d, std::vector<std::vector<uint16_t>> &parts, std::vector<double> &weight) {
    std::vector<int> a(d, 0);
    while (true) {
        int k = 0;
        for (int q = 0; q < d; ++q) k = std::max(k, a[q] + 1);
        std::vector<uint16_t> masks(k, 0);
        for (int q = 0; q < d; ++q) masks[a[q]] |= (uint16_t)(1u << q);
        double f = 1.0;
        for (int q = 2; q < k; ++q) f *= q;
        parts.push_back(masks);
        weight.push_back((k - 1) % 2 ? -f : f);
        int q = d - 1;
        while (q >= 1) {
            int lim = 0;
            for (int r = 0; r < q; ++r) lim = std::max(lim, a[r] + 1);
            if (a[q] < lim) break;
            --q;
        }
        if (q < 1) break;
        ++a[q];
        for (int r = q + 1; r < d; ++r) a[r] = 0;
    }
}

// ---------------------------------------------------------------------------
// device buffers owned by the library
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

template <typename T>
static cum_status upload(DevBuf &dst, const std::vector<T> &src) {
    size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
    if (dst.p) {
        (void)hipFree(dst.p);
        dst.p = nullptr;
    }
    HIP_TRY(hipMalloc(&dst.p, bytes));
    if (!src.empty()) HIP_TRY(hipMemcpy(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return CUM_OK;
}

// ---------------------------------------------------------------------------
// per-order plan
// ---------------------------------------------------------------------------
struct OrderPlan {
    int n = 0, b = 0, d = 0, p = 0, q = 0, nbar = 0, nr = 0, nc = 0;
    int64_t nblocks = 0, elems = 0;
    std::vector<Feat> rows, cols;
    std::vector<int32_t> rb_vmin, cb_wmax;  // per 32-row / 32-column block
    std::vector<int32_t> rv16, cw16;        // per 16-row / 16-column block
    std::vector<int64_t> H;
    std::vector<int64_t> prank;  // d x (nbar + 1): b^d * C(nbar - x + d - k - 1, d - k)
    std::vector<uint8_t> tuples;
    std::vector<int32_t> parts;   // npart x (d/2), packed mask | where << 10
    int npart = 0;
    std::vector<int32_t> terms;   // orders >= 7: nterm x 2 (set A with position 0, its complement)
    std::vector<int32_t> tpw;     // their multipliers b^|high positions| (see RedOrder::tpw)
    int nterm = 0;
    int qe = 0;                   // see RedOrder::qe, RedOrder::cstart
    int32_t cstart[5] = {0};
    std::vector<uint16_t> smask;  // position sets of 2..d-2 positions, by size then value
    std::vector<int32_t> gmap;    // staged slot -> s | flat << 10
    int32_t mstart[MAXD] = {0};   // first staged slot of each set size m (index m - 2)
    int lds_elems = 0;            // 0: the recursion reads lower orders from memory
    bool uploaded = false;
    DevBuf rows_d, cols_d, H_d, prank_d, tuples_d, parts_d, smask_d, gmap_d, terms_d, tpw_d;
};

// Cut points of the sorted rows (or columns) into 16-blocks.  A 16 x 16
// sub-block is computed when the smallest v of its rows is <= the largest w
// of its columns, so each row block costs as many sub-blocks as there are
// column blocks with w_max >= its smallest v, whatever number of real rows it
// holds; likewise for column blocks.  Given the other side's blocks, a
// dynamic program over the cut points (blocks of 1 to 16 consecutive
// features, the rest padding) minimises the computed sub-blocks.  cost[k] is
// the cost of a block whose key (the first feature's block index for rows,
// the last one's for columns) is k.  Returns the block sizes in order.
static std::vector<int> align_blocks(const std::vector<Feat> &f, const std::vector<int64_t> &cost, bool key_first) {
    const size_t N = f.size();
    std::vector<int64_t> best(N + 1, 0);
    std::vector<int> take(N + 1, 0);
    for (size_t i = 1; i <= N; ++i) {
        best[i] = INT64_MAX;
        for (int sz = 1; sz <= 16 && (size_t)sz <= i; ++sz) {
            const int key = key_first ? f[i - sz].blk : f[i - 1].blk;
            const int64_t c = best[i - sz] + cost[key];
            if (c < best[i]) {
                best[i] = c;
                take[i] = sz;
            }
        }
    }
    std::vector<int> sizes;
    for (size_t i = N; i > 0; i -= take[i]) sizes.push_back(take[i]);
    std::reverse(sizes.begin(), sizes.end());
    return sizes;
}

// Rows and columns laid out in 16-blocks of the given sizes, padded.
static std::vector<Feat> pad_blocks(const std::vector<Feat> &f, const std::vector<int> &sizes, const Feat &pad) {
    std::vector<Feat> out;
    out.reserve(sizes.size() * 16);
    size_t i = 0;
    for (int sz : sizes) {
        for (int k = 0; k < sz; ++k) out.push_back(f[i++]);
        for (int k = sz; k < 16; ++k) out.push_back(pad);
    }
    return out;
}

// Plain packing (full 16-blocks) when the dynamic program would take too long.
constexpr size_t ALIGN_MAX_FEATURES = 1 << 22;

// Digits per lane of the multi-entry first-position finalisation (orders
// >= 7): a lane takes the b^qe entries that differ only in their last qe
// digits, at most 4 of them.  Where the block's sub-blocks are staged in LDS
// (at b = 2 orders 7 and 8) one work-group of 64 lanes covers a block; where
// they are read from memory, qe is chosen so that a block still spreads over
// 256 or more lanes.  Other block sizes keep one entry per thread (qe = 0).
static int first_position_qe(int b, int d, bool staged) {
    if (b == 2) return staged ? (d >= 8 ? 2 : 1) : (d >= 10 ? 2 : 1);
    return (b == 3 || b == 4) ? 1 : 0;
}

// Group of a first-position term by its set A (holding position 0): which of
// the last qe positions A holds, as bits (position d-qe+i -> bit qe-1-i).
static int term_group(int mask, int d, int qe) {
    int c = 0;
    for (int i = 0; i < qe; ++i) c = c * 2 + (mask >> (d - qe + i) & 1);
    return c;
}

static cum_status build_order(int n, int b, int d, OrderPlan &o) {
    o.n = n;
    o.b = b;
    o.d = d;
    o.p = d / 2;
    o.q = d - o.p;
    o.nbar = (n + b - 1) / b;
    const int nbar = o.nbar, p = o.p, q = o.q;
    const int64_t bd = ipow64(b, d), bq = ipow64(b, q);
    o.nblocks = binom(nbar + d - 1, d);
    if (o.nblocks < 0) return fail(CUM_EINVAL, "order %d with %d blocks per mode overflows", d, nbar);
    o.elems = o.nblocks * bd;

    // rows: sorted prefixes ordered by their last block (then lexicographically)
    auto P = sorted_tuples(nbar, p);
    std::stable_sort(P.begin(), P.end(), [](const std::vector<int> &x, const std::vector<int> &y) {
        return x.back() < y.back();
    });
    const int64_t bp = ipow64(b, p);
    for (const auto &u : P) {
        int64_t part = 0;
        int prev = 0;
        for (int k = 0; k < p; ++k) {
            part += rank_term(nbar, d, k, prev, u[k]);
            prev = u[k];
        }
        for (int64_t ip = 0; ip < bp; ++ip) {
            Feat f;
            f.addr = part * bd + ip * bq;
            f.blk = u[p - 1];
            int64_t x = ip;
            int dig[MAXH] = {0};
            for (int k = p - 1; k >= 0; --k) {
                dig[k] = (int)(x % b);
                x /= b;
            }
            for (int k = 0; k < MAXH; ++k) {
                int v = k < p ? u[k] * b + dig[k] : n;
                f.var[k] = (uint8_t)(v < n ? v : n);
            }
            o.rows.push_back(f);
        }
    }
    // columns: sorted suffixes in lexicographic order (so by their first block)
    auto Q = sorted_tuples(nbar, q);
    for (const auto &u : Q) {
        int64_t part = 0;
        int prev = u[0];
        for (int k = p + 1; k < d; ++k) {
            part += rank_term(nbar, d, k, prev, u[k - p]);
            prev = u[k - p];
        }
        for (int64_t iq = 0; iq < bq; ++iq) {
            Feat f;
            f.addr = part * bd + iq;
            f.blk = u[0];
            int64_t x = iq;
            int dig[MAXH] = {0};
            for (int k = q - 1; k >= 0; --k) {
                dig[k] = (int)(x % b);
                x /= b;
            }
            for (int k = 0; k < MAXH; ++k) {
                int v = k < q ? u[k] * b + dig[k] : n;
                f.var[k] = (uint8_t)(v < n ? v : n);
            }
            o.cols.push_back(f);
        }
    }
    // padding rows and columns multiply the zero row only
    Feat padr, padc;
    memset(&padr, 0, sizeof padr);
    padr.blk = INT32_MAX;
    for (int k = 0; k < MAXH; ++k) padr.var[k] = (uint8_t)n;
    padc = padr;
    padc.blk = -1;
    // 16-blocks cut where they waste the fewest matrix products on unstored
    // entries (alternating between rows and columns, each pass optimal given
    // the other side; a pass never increases the count)
    if (o.rows.size() <= ALIGN_MAX_FEATURES && o.cols.size() <= ALIGN_MAX_FEATURES) {
        std::vector<int> rsz((o.rows.size() + 15) / 16, 16), csz((o.cols.size() + 15) / 16, 16);
        if (!rsz.empty()) rsz.back() = (int)(o.rows.size() - 16 * (rsz.size() - 1));
        if (!csz.empty()) csz.back() = (int)(o.cols.size() - 16 * (csz.size() - 1));
        auto keys = [](const std::vector<Feat> &f, const std::vector<int> &sz, bool first) {
            std::vector<int> k;
            size_t i = 0;
            for (int z : sz) {
                k.push_back(first ? f[i].blk : f[i + z - 1].blk);
                i += z;
            }
            return k;
        };
        for (int pass = 0; pass < 3; ++pass) {
            // rows: a block with smallest v costs the column blocks with w_max >= v
            std::vector<int64_t> cost(nbar + 1, 0);
            for (int w : keys(o.cols, csz, false)) ++cost[w];
            for (int v = nbar - 1; v >= 0; --v) cost[v] += cost[v + 1];
            rsz = align_blocks(o.rows, cost, true);
            // columns: a block with largest w costs the row blocks with v_min <= w
            std::vector<int64_t> cc(nbar, 0);
            for (int v : keys(o.rows, rsz, true)) ++cc[v];
            for (int w = 1; w < nbar; ++w) cc[w] += cc[w - 1];
            csz = align_blocks(o.cols, cc, false);
        }
        o.rows = pad_blocks(o.rows, rsz, padr);
        o.cols = pad_blocks(o.cols, csz, padc);
    }
    const int nr_real = (int)o.rows.size(), nc_real = (int)o.cols.size();
    o.nr = (nr_real + FEAT_BLOCK - 1) / FEAT_BLOCK * FEAT_BLOCK;
    o.nc = (nc_real + FEAT_BLOCK - 1) / FEAT_BLOCK * FEAT_BLOCK;
    o.rows.resize(o.nr, padr);
    o.cols.resize(o.nc, padc);
    for (int rb = 0; rb < o.nr / FEAT_BLOCK; ++rb) {
        int32_t v = INT32_MAX;
        for (int r = rb * FEAT_BLOCK; r < std::min(nr_real, (rb + 1) * FEAT_BLOCK); ++r) v = std::min(v, o.rows[r].blk);
        o.rb_vmin.push_back(v);
    }
    for (int cb = 0; cb < o.nc / FEAT_BLOCK; ++cb) {
        int32_t w = -1;
        for (int c = cb * FEAT_BLOCK; c < std::min(nc_real, (cb + 1) * FEAT_BLOCK); ++c) w = std::max(w, o.cols[c].blk);
        o.cb_wmax.push_back(w);
    }
    for (int rb = 0; rb < o.nr / 16; ++rb) {
        int32_t v = INT32_MAX;
        for (int r = rb * 16; r < std::min(nr_real, (rb + 1) * 16); ++r) v = std::min(v, o.rows[r].blk);
        o.rv16.push_back(v);
    }
    for (int cb = 0; cb < o.nc / 16; ++cb) {
        int32_t w = -1;
        for (int c = cb * 16; c < std::min(nc_real, (cb + 1) * 16); ++c) w = std::max(w, o.cols[c].blk);
        o.cw16.push_back(w);
    }
    o.H.assign((size_t)nbar * nbar, 0);
    for (int v = 0; v < nbar; ++v)
        for (int w = v; w < nbar; ++w) o.H[(size_t)v * nbar + w] = bd * rank_term(nbar, d, p, v, w);
    // rank terms of a whole sorted tuple (rank = sum_k prank[k][j_(k-1)] - prank[k][j_k], j_(-1) = 0)
    o.prank.assign((size_t)d * (nbar + 1), 0);
    for (int k = 0; k < d; ++k)
        for (int x = 0; x <= nbar; ++x) o.prank[(size_t)k * (nbar + 1) + x] = bd * binom(nbar - x + d - k - 1, d - k);

    // recursion tables
    auto T = sorted_tuples(nbar, d);
    for (const auto &u : T)
        for (int k = 0; k < d; ++k) o.tuples.push_back((uint8_t)u[k]);
    // the recursion of a block reads, for every set S of 2..d-2 positions,
    // the lower-order block j_S: the sets by size, and their sub-blocks'
    // slots in LDS when they all fit
    std::vector<int> sidx((size_t)1 << d, -1);
    std::vector<int64_t> soff;
    int64_t lds = 0;
    for (int m = 2; m <= d - 2; ++m) {
        o.mstart[m - 2] = (int32_t)std::min<int64_t>(lds, INT32_MAX);
        for (int mask = 0; mask < (1 << d); ++mask) {
            if (__builtin_popcount(mask) != m) continue;
            sidx[(size_t)mask] = (int)o.smask.size();
            o.smask.push_back((uint16_t)mask);
            soff.push_back(lds);
            lds += ipow64(b, m);
        }
    }
    if (d >= 4) o.mstart[d - 3] = (int32_t)std::min<int64_t>(lds, INT32_MAX);
    o.lds_elems = (d >= 4 && lds <= RED_LDS_MAX) ? (int)lds : 0;
    if (o.lds_elems)
        for (size_t si = 0; si < o.smask.size(); ++si) {
            const int64_t sz = ipow64(b, __builtin_popcount(o.smask[si]));
            for (int64_t f = 0; f < sz; ++f) o.gmap.push_back((int32_t)(si | (f << 10)));
        }
    auto parts = recursion_partitions(d);
    o.npart = (int)parts.size();
    const int per = d / 2;
    for (const auto &pm : parts)
        for (int k = 0; k < per; ++k) {
            int32_t v = 0;
            if (k < (int)pm.size()) {
                const int where = o.lds_elems ? (int)soff[(size_t)sidx[pm[k]]] : sidx[pm[k]];
                v = (int32_t)pm[k] | (int32_t)(where << 10);
            }
            o.parts.push_back(v);
        }
    // Orders >= 7 can also use the moment-cumulant relation split at the first
    // position: the sum over partitions equals the sum over sets A holding
    // position 0 (2 <= |A| <= d-2) of kappa_|A|(j_A) times the central moment
    // M_(d-|A|) of the complement (sets of one position drop out: kappa_1 = 0
    // and central M_1 = 0).  2^(d-1) - d - 1 terms of two factors, against
    // 162, 715, 3425 and 17722 partitions at d = 7..10.
    // The terms are grouped by which of the last qe positions A holds (see
    // term_group), so that a thread that takes the b^qe entries sharing all
    // other digits reads each factor's values for all of them as one run.
    if (d >= FIRST_POSITION_MIN_D) {
        const int full = (1 << d) - 1;
        o.qe = first_position_qe(b, d, o.lds_elems > 0);
        std::vector<int> group[5];
        for (int mask = 1; mask < (1 << d); mask += 2) {
            const int m = __builtin_popcount(mask);
            if (m < 2 || m > d - 2) continue;
            group[term_group(mask, d, o.qe)].push_back(mask);
        }
        for (int c = 0; c < 5; ++c) {
            o.cstart[c] = (int32_t)(o.terms.size() / 2);
            for (int mask : group[c]) {
                const int comp = full ^ mask;
                for (int f : {mask, comp}) {
                    const int where = o.lds_elems ? (int)soff[(size_t)sidx[f]] : sidx[f];
                    o.terms.push_back((int32_t)f | (int32_t)(where << 10));
                    o.tpw.push_back((int32_t)ipow64(b, __builtin_popcount((unsigned)f >> ((d + 1) / 2))));
                }
            }
        }
        o.nterm = (int)o.terms.size() / 2;
    }

    return CUM_OK;
}

static cum_status upload_order(OrderPlan &o) {
    if (o.uploaded) return CUM_OK;
    cum_status st;
    if ((st = upload(o.rows_d, o.rows)) || (st = upload(o.cols_d, o.cols)) || (st = upload(o.H_d, o.H)) || (st = upload(o.prank_d, o.prank)) ||
        (st = upload(o.tuples_d, o.tuples)) ||
        (st = upload(o.parts_d, o.parts)) || (st = upload(o.smask_d, o.smask)) ||
        (st = upload(o.gmap_d, o.gmap)) || (st = upload(o.terms_d, o.terms)) || (st = upload(o.tpw_d, o.tpw)))
        return st;
    o.uploaded = true;
    return CUM_OK;
}

static std::mutex g_mu;
static std::map<std::tuple<int, int, int>, std::unique_ptr<OrderPlan>> g_orders;

static cum_status get_order(int n, int b, int d, OrderPlan **out) {
    auto key = std::make_tuple(n, b, d);
    auto it = g_orders.find(key);
    if (it != g_orders.end()) {
        *out = it->second.get();
        return CUM_OK;
    }
    std::unique_ptr<OrderPlan> o(new OrderPlan);
    cum_status st = build_order(n, b, d, *o);
    if (st) return st;
    *out = o.get();
    g_orders[key] = std::move(o);
    return CUM_OK;
}

// Work-group tiles of one order.  A wave task is a 32-row block by WN
// consecutive 32-column blocks holding at least one stored entry; its cost
// is the number of stored 16 x 16 sub-blocks.  Tasks are sorted by cost and
// packed WG_WAVES to a work-group, so the waves of a work-group have nearly
// equal work and no wave sits idle except in the order's last tile.
struct HostTile {
    TileDev t;
    int cost;  // the largest task cost of the tile
};

static void order_tiles(const OrderPlan &o, int wn, int ord_index, std::vector<HostTile> &out) {
    struct Task {
        WaveTask w;
        int cost;
    };
    std::vector<Task> tasks;
    const int nrb = o.nr / 32, ncb = o.nc / 32;
    for (int rb = 0; rb < nrb; ++rb)
        for (int cb = 0; cb < ncb; cb += wn) {
            int mask = 0, cost = 0;
            for (int j = 0; j < wn && cb + j < ncb; ++j) {
                if (o.rb_vmin[rb] > o.cb_wmax[cb + j]) continue;
                for (int h = 0; h < 2; ++h)
                    for (int g = 0; g < 2; ++g)
                        if (o.rv16[2 * rb + h] <= o.cw16[2 * (cb + j) + g]) {
                            mask |= 1 << (j * 4 + h * 2 + g);
                            ++cost;
                        }
            }
            if (mask) tasks.push_back({{rb * 32, cb * 32, mask, 0}, cost});
        }
    std::stable_sort(tasks.begin(), tasks.end(), [](const Task &x, const Task &y) { return x.cost > y.cost; });
    for (size_t i = 0; i < tasks.size(); i += WG_WAVES) {
        HostTile ht;
        memset(&ht.t, 0, sizeof ht.t);
        ht.t.ord = ord_index;
        ht.cost = 0;
        for (size_t k = i; k < std::min(tasks.size(), i + (size_t)WG_WAVES); ++k) {
            ht.t.task[ht.t.ntask++] = tasks[k].w;
            ht.cost = std::max(ht.cost, tasks[k].cost);
        }
        out.push_back(ht);
    }
}

static int shape_wn(int shape) { return shape == TS_1x2 ? 2 : 1; }

// Contraction record of an order (device pointers once uploaded).
static OrderDev order_dev(const OrderPlan &o, int64_t off) {
    OrderDev od;
    od.rows = (const Feat *)o.rows_d.p;
    od.cols = (const Feat *)o.cols_d.p;
    od.H = (const int64_t *)o.H_d.p;
    od.out_off = off;
    od.elems = o.elems;
    od.d = o.d;
    od.p = o.p;
    od.q = o.q;
    od.nbar = o.nbar;
    od.b = o.b;
    od.nr = o.nr;
    od.nc = o.nc;
    od.pad = 0;
    return od;
}

// Reduction record of an order: output layout o, partial sums in layout po
// (the same plan, or the one of a smaller block size) at offset poff.
static RedOrder red_order(const OrderPlan &o, const OrderPlan &po, int64_t poff) {
    RedOrder ro;
    memset(&ro, 0, sizeof ro);
    ro.tuples = (const uint8_t *)o.tuples_d.p;
    ro.parts = (const int32_t *)o.parts_d.p;
    ro.smask = (const uint16_t *)o.smask_d.p;
    ro.gmap = (const int32_t *)o.gmap_d.p;
    ro.terms = (const int32_t *)o.terms_d.p;
    ro.tpw = (const int32_t *)o.tpw_d.p;
    ro.nterm = o.nterm;
    ro.qe = o.qe;
    for (int c = 0; c < 5; ++c) ro.cstart[c] = o.cstart[c];
    ro.prank = (const int64_t *)po.prank_d.p;
    ro.ns = (int32_t)o.smask.size();
    ro.lds_elems = o.lds_elems;
    for (int k = 0; k < MAXD; ++k) ro.mstart[k] = o.mstart[k];
    ro.nblocks = o.nblocks;
    ro.out_off = poff;
    ro.d = o.d;
    ro.npart = o.npart;
    ro.nbar = o.nbar;
    ro.b = o.b;
    ro.pb = po.b;
    ro.pnbar = po.nbar;
    ro.n = o.n;
    return ro;
}

// ---------------------------------------------------------------------------
// call plan: all orders dlo..dhi of one (n, b), one precision and tile shape,
// one sample count.
// ---------------------------------------------------------------------------
// The work items of one sample-chunk count: (tile, chunk) pairs in launch order.
struct ItemSet {
    std::vector<Item> items;
    bool uploaded = false;
    DevBuf items_d;
};

// Everything about a call that does not depend on its sample count: the
// orders' tables, the tiles, the finalisation records, and the work items of
// each chunk count met so far (at most one per chunk count, which the target
// item count bounds).
struct CallPlan {
    int n = 0, b = 0, bi = 0, dlo = 0, dhi = 0, prec = 0, shape = 0, target = 0;
    int64_t ntiles = 0;
    int64_t stride = 0;               // partial sums of all orders, block size bi
    int64_t kstride = 0;              // outputs of all orders, block size b
    std::vector<OrderPlan *> orders;  // output layout (block size b), index d - dlo
    std::vector<OrderPlan *> corders; // contraction layout (block size bi), index d - dlo
    std::vector<int64_t> out_off;     // output offsets in a contiguous buffer, index d - dlo
    std::vector<int64_t> pout_off;    // partial-sum offsets, index d - dlo
    std::vector<OrderDev> ods;
    std::vector<TileDev> tdev;
    std::vector<RedOrder> red;        // index d - dlo
    std::map<int64_t, std::unique_ptr<ItemSet>> itemsets;  // by chunk count
    bool uploaded = false;
    DevBuf ords_d, tiles_d, red_d;
};

// One call: its plan and the split of its t samples into chunks of whole stages.
struct Call {
    CallPlan *c = nullptr;
    ItemSet *is = nullptr;
    int64_t t = 0, nstages = 0, chunk_stages = 0, nchunks = 0;
};

// Upload the call's order tables (filling in their device pointers) and its
// tile, item and reduction records.
static cum_status upload_plan(CallPlan &c) {
    if (c.uploaded) return CUM_OK;
    cum_status st;
    c.ods.clear();
    c.red.clear();
    for (size_t i = 0; i < c.orders.size(); ++i) {
        if ((st = upload_order(*c.orders[i])) || (st = upload_order(*c.corders[i]))) return st;
        c.ods.push_back(order_dev(*c.corders[i], c.pout_off[i]));
        c.red.push_back(red_order(*c.orders[i], *c.corders[i], c.pout_off[i]));
    }
    if ((st = upload(c.ords_d, c.ods)) || (st = upload(c.tiles_d, c.tdev)) || (st = upload(c.red_d, c.red))) return st;
    c.uploaded = true;
    return CUM_OK;
}

static cum_status upload_call(const Call &k) {
    cum_status st;
    if ((st = upload_plan(*k.c))) return st;
    if (!k.is->uploaded) {
        if ((st = upload(k.is->items_d, k.is->items))) return st;
        k.is->uploaded = true;
    }
    return CUM_OK;
}

static std::map<std::tuple<int, int, int, int, int, int, int, int>, std::unique_ptr<CallPlan>> g_calls;

// Tuned choices: (n, b, dlo, dhi, prec, t) -> (shape, target items, inner block size).
struct Tuning {
    int shape;
    int target;
    int bi;
};
static std::map<std::tuple<int, int, int, int, int, int64_t>, Tuning> g_tuned;
static bool g_tune_loaded = false;

static const char *tune_file() {
    const char *f = getenv("CUM_TUNE_FILE");
    return (f && *f) ? f : nullptr;
}

// Cache file: one line per tuned shape, "n b dlo dhi prec t shape target bi";
// lines that do not parse, or name an invalid configuration, are skipped.
static void load_tune_file() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = tune_file();
    if (!f) return;
    FILE *fp = fopen(f, "r");
    if (!fp) return;
    char line[256];
    while (fgets(line, sizeof line, fp)) {
        int n, b, dlo, dhi, prec, shape, target, bi;
        long long t;
        if (sscanf(line, "%d %d %d %d %d %lld %d %d %d", &n, &b, &dlo, &dhi, &prec, &t, &shape, &target, &bi) != 9)
            continue;
        if ((shape != TS_1x1 && shape != TS_1x2) || target < 1 || bi < 1 || bi > b) continue;
        g_tuned[std::make_tuple(n, b, dlo, dhi, prec, (int64_t)t)] = Tuning{shape, target, bi};
    }
    fclose(fp);
}

static void save_tune_file() {
    const char *f = tune_file();
    if (!f) return;
    FILE *fp = fopen(f, "w");
    if (!fp) return;
    for (auto &kv : g_tuned) {
        auto &k = kv.first;
        fprintf(fp, "%d %d %d %d %d %lld %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                std::get<4>(k), (long long)std::get<5>(k), kv.second.shape, kv.second.target, kv.second.bi);
    }
    fclose(fp);
}

// 32 x 32 wave tasks for FP32 and FP64 (the autotuner chose them on every
// measured workload, orders 4 to 10) and the FP16 split; 32 x 64 for the BF16
// splits, whose operand arithmetic the wider task shares over twice the products.
static int default_shape(int prec) { return (prec == P_F32 || prec == P_F64 || prec == P_F16X2) ? TS_1x1 : TS_1x2; }
constexpr int DEFAULT_TARGET = 4096;
// The contraction computes each distinct sorted variable tuple once (inner
// block size 1) unless tuning chose otherwise.
static int default_inner(int) { return 1; }

// The work items of a plan for nck sample chunks: work-group i runs on XCD
// i % 8, and all items of one chunk share its stages, so a chunk goes to one
// XCD (8 or more chunks) or to a group of 8 / nck XCDs; otherwise tiles go
// round-robin.  Tiles are in cost order, so each XCD runs expensive ones first.
static ItemSet *plan_items(CallPlan &c, int64_t nck) {
    auto it = c.itemsets.find(nck);
    if (it != c.itemsets.end()) return it->second.get();
    std::vector<std::vector<Item>> per_xcd(8);
    for (int64_t ch = 0; ch < nck; ++ch)
        for (int64_t ti = 0; ti < c.ntiles; ++ti) {
            int x;
            if (nck >= 8)
                x = (int)(ch % 8);
            else if (8 % nck == 0)
                x = (int)(ch * (8 / nck) + ti % (8 / nck));
            else
                x = (int)(ti % 8);
            per_xcd[x].push_back({(int32_t)ti, (int32_t)ch, 0, 0});
        }
    size_t longest = 0;
    for (auto &v : per_xcd) longest = std::max(longest, v.size());
    std::unique_ptr<ItemSet> is(new ItemSet);
    for (size_t q = 0; q < longest; ++q)
        for (int x = 0; x < 8; ++x) is->items.push_back(q < per_xcd[x].size() ? per_xcd[x][q] : Item{-1, 0, 0, 0});
    while (!is->items.empty() && is->items.back().tile < 0) is->items.pop_back();
    ItemSet *r = is.get();
    c.itemsets[nck] = std::move(is);
    return r;
}

static cum_status get_call_cfg(int n, int b, int bi, int dlo, int dhi, int prec, int shape, int target, int64_t t,
                               Call *out, int min_stages = 4) {
    for (int d = dlo; d <= dhi; ++d)
        if (ipow64(b, d) > INT32_MAX)
            return fail(CUM_EUNSUPPORTED, "blocks of b^d = %d^%d entries (2^31 or more) are not supported", b, d);
    auto key = std::make_tuple(n, b, bi, dlo, dhi, prec, shape, target);
    auto it = g_calls.find(key);
    CallPlan *c;
    if (it != g_calls.end()) {
        c = it->second.get();
    } else {
        std::unique_ptr<CallPlan> cp(new CallPlan);
        cp->n = n;
        cp->b = b;
        cp->bi = bi;
        cp->dlo = dlo;
        cp->dhi = dhi;
        cp->prec = prec;
        cp->shape = shape;
        cp->target = target;
        const int wn = shape_wn(shape);
        std::vector<HostTile> tiles;
        int64_t off = 0, poff = 0;
        for (int d = dlo; d <= dhi; ++d) {
            OrderPlan *o, *co;
            cum_status st;
            if ((st = get_order(n, b, d, &o)) || (st = get_order(n, bi, d, &co))) return st;
            cp->orders.push_back(o);
            cp->corders.push_back(co);
            cp->out_off.push_back(off);
            cp->pout_off.push_back(poff);
            order_tiles(*co, wn, d - dlo, tiles);
            off += o->elems;
            poff += co->elems;
        }
        cp->kstride = off;
        cp->stride = poff;
        // expensive tiles first, so that the tail of each XCD's queue is short
        std::stable_sort(tiles.begin(), tiles.end(),
                         [](const HostTile &x, const HostTile &y) { return x.cost > y.cost; });
        cp->ntiles = (int64_t)tiles.size();
        for (auto &h : tiles) cp->tdev.push_back(h.t);
        c = cp.get();
        g_calls[key] = std::move(cp);
    }
    // sample chunks (whole stages): about `target` work items (1024 fill the
    // 256 CUs' four work-group slots once), chunks of >= min_stages stages
    Call k;
    k.c = c;
    k.t = t;
    k.nstages = (t + stage_kt(prec) - 1) / stage_kt(prec);
    const int64_t want = (target + std::max<int64_t>(c->ntiles, 1) - 1) / std::max<int64_t>(c->ntiles, 1);
    const int64_t maxch = std::max<int64_t>(1, k.nstages / min_stages);
    int64_t nch = std::max<int64_t>(1, std::min(want, maxch));
    if (nch >= 8) nch = (nch + 7) / 8 * 8;
    k.chunk_stages = (k.nstages + nch - 1) / nch;
    k.nchunks = (k.nstages + k.chunk_stages - 1) / k.chunk_stages;
    k.is = plan_items(*c, k.nchunks);
    *out = k;
    return CUM_OK;
}

// The call plan for a shape: the tuned choice if there is one, else the defaults.
static cum_status get_call(int n, int b, int dlo, int dhi, int prec, int64_t t, Call *out) {
    load_tune_file();
    auto it = g_tuned.find(std::make_tuple(n, b, dlo, dhi, prec, t));
    if (it != g_tuned.end())
        return get_call_cfg(n, b, it->second.bi, dlo, dhi, prec, it->second.shape, it->second.target, t, out);
    return get_call_cfg(n, b, default_inner(b), dlo, dhi, prec, default_shape(prec), DEFAULT_TARGET, t, out);
}

static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// The FP16 split's extra workspace: each centring group's column minima and
// maxima, and the n + 1 per-variable powers of two the staged data are
// divided by (0 for the other precisions).
static size_t f16_bytes(int prec, int groups, int n) {
    return prec == CUM_F16X2 ? align_up((size_t)groups * n * 2 * 8) + align_up((size_t)(n + 1) * 8) : 0;
}

static void center_groups(int64_t t, int &groups, int64_t &rows_per) {
    int64_t g = std::min<int64_t>(1024, (t + 255) / 256);
    if (g < 1) g = 1;
    rows_per = (t + g - 1) / g;
    groups = (int)((t + rows_per - 1) / rows_per);
}

static size_t staged_bytes(int64_t t, int n, int prec) {
    const int64_t nst = (t + stage_kt(prec) - 1) / stage_kt(prec);
    return align_up((size_t)nst * (n + 1) * stage_pitch(prec) * stage_esize(prec));
}

static cum_status check_common(int64_t t, int n, int b) {
    if (t < 1) return fail(CUM_EINVAL, "t must be >= 1 (got %lld)", (long long)t);
    if (n < 1 || n > MAXN) return fail(CUM_EINVAL, "n must be in 1..%d (got %d)", MAXN, n);
    if (b < 1 || b > n) return fail(CUM_EINVAL, "b must be in 1..n (got b=%d, n=%d)", b, n);
    return CUM_OK;
}

static cum_status check_prec(int prec) {
    if (prec < CUM_F64 || prec > CUM_F16X2) return fail(CUM_EUNSUPPORTED, "unknown precision %d", prec);
    return CUM_OK;
}

// The precision in which a call that centres its own data stages and
// contracts orders 2..d_max.  Rounding the centred samples to FP32 leaves up
// to 2^-24 relative error in every factor.  At orders of
// HIGH_F64_MIN_D and above, the cumulants of heavy-tailed data cancel most of
// moments that a few extreme samples carry, and that rounding alone puts the
// relative error of the cumulant above 1e-6 (1.4e-6 measured at order 8 on
// Laplace-mixed data with FP64 accumulation).  Those calls stage and contract
// in FP64 whatever precision was asked for.
static int staged_prec(int prec, int d_max) { return d_max >= HIGH_F64_MIN_D ? (int)CUM_F64 : prec; }

// Entries per lane of the finalisation of order ro in a launch with
// arguments ra: b^qe where the first-position formula runs in its
// multi-entry form, else 1.
static int32_t gather_entries(const RedOrder &ro, const RedArgs &ra) {
    if (!ra.recursion || !ra.subset || ro.d < FIRST_POSITION_MIN_D || ro.nterm == 0 || ro.qe <= 0) return 1;
    return (int32_t)ipow64(ro.b, ro.qe);
}

// q0, q1 and the staging bits of a launch of orders ro[0 .. ra.nords-1]
static void set_gather(const RedOrder *ro, RedArgs &ra) {
    ra.q0 = gather_entries(ro[0], ra);
    ra.q1 = ra.nords == 2 ? gather_entries(ro[1], ra) : 1;
    ra.gstaged = (ro[0].lds_elems > 0 ? 1 : 0) | (ra.nords == 2 && ro[1].lds_elems > 0 ? 2 : 0);
}

// Dynamic LDS of a finalisation launch over orders ro[0..nords-1]: the
// staged sub-blocks, the block's lower-order offsets and, when everything
// fits in 64 KiB, the partition table.  Fills the layout fields of ra and
// returns the bytes to allocate.
static int red_lds_layout(const RedOrder *ro, int nords, bool recursion, RedArgs &ra) {
    int64_t sub = 0, ns = 0, parts = 0;
    if (recursion)
        for (int i = 0; i < nords; ++i) {
            sub = std::max<int64_t>(sub, ro[i].lds_elems);
            ns = std::max<int64_t>(ns, ro[i].ns);
            const bool fp = ra.subset && ro[i].d >= FIRST_POSITION_MIN_D && ro[i].nterm > 0;
            parts = std::max<int64_t>(parts, fp ? (int64_t)ro[i].nterm * 2 : (int64_t)ro[i].npart * (ro[i].d / 2));
        }
    ra.base_off = (int32_t)((sub * 8 + 15) / 16 * 16);
    ra.parts_off = ra.base_off + (int32_t)((ns * 8 + 15) / 16 * 16);
    ra.parts_lds = (parts > 0 && ra.parts_off + parts * 4 <= 65536) ? 1 : 0;
    return ra.parts_off + (ra.parts_lds ? (int)(parts * 4) : 0);
}

// Partial sums up to this many (all chunks) are left for the finalisation to
// add up: a separate chunk-sum launch costs more than it saves there.
constexpr int64_t SMALL_PARTIALS = (int64_t)1 << 20;

// From this many sample chunks on, the contraction stores each chunk's sums
// in tile order (whole 64-lane rows, no addresses to work out) and one pass
// adds them over chunks and scatters them to block storage: the scatter's
// loads and scattered stores are then paid once, not once per chunk.
// (Calls whose contraction mixes the FP32 and FP64 accumulator layouts,
// FP32-staged with orders of HIGH_ACC64_MIN_D and up, keep the per-chunk
// scatter.)
constexpr int64_t RAW_MIN_CHUNKS = 4;
static int64_t raw_stride(const CallPlan *c) { return c->ntiles * WG_WAVES * (c->shape == TS_1x2 ? 2 : 1) * 1024; }
static bool raw_mode(const Call &k) {
    return k.nchunks >= RAW_MIN_CHUNKS && (k.c->prec == P_F64 || k.c->dhi < HIGH_ACC64_MIN_D);
}
// Bytes of the partial-sum region of a call: per-chunk block storage, or the
// tile-order chunks followed by one block-storage copy of their sum.
static size_t partial_bytes(const Call &k) {
    if (raw_mode(k)) return ((size_t)k.nchunks * raw_stride(k.c) + k.c->stride) * 8;
    return (size_t)k.nchunks * (size_t)k.c->stride * 8;
}

// The contraction of orders dlo..dhi over the staged data Xc into the
// per-chunk partial sums, then (if always_sum, or the partial sums are not
// small) their sum over chunks into chunk 0.  *summed tells which.
static cum_status run_contraction(const Call &k, const void *Xc, double *partial, bool always_sum, bool *summed,
                                  hipStream_t s, double **sums, const double *scale = nullptr) {
    cum_status st = upload_call(k);
    if (st) return st;
    const CallPlan *c = k.c;
    const int64_t nitems = (int64_t)k.is->items.size();
    MomentArgs ma;
    ma.ords = (const OrderDev *)c->ords_d.p;
    ma.tiles = (const TileDev *)c->tiles_d.p;
    ma.items = (const Item *)k.is->items_d.p;
    ma.nitems = nitems;
    ma.sets = nullptr;
    ma.set0.X = Xc;
    ma.set0.nstages = k.nstages;
    ma.set0.chunk_stages = k.chunk_stages;
    ma.set0.nchunks = k.nchunks;
    ma.set0.partial = partial;
    ma.set0.stride = c->stride;
    ma.n = c->n;
    ma.pad = 0;
    const bool raw = raw_mode(k);
    const int64_t rs = raw ? raw_stride(c) : 0;
    ma.raw = raw ? partial : nullptr;
    ma.rawstride = rs;
    ma.scale = scale;
    ma.set0.scale = scale;
    *sums = partial;
    if (nitems > 0)
        HIP_TRY(timed(CUM_KIND_MOMENT, s, [&] { return launch_moment(c->prec, c->shape, c->dhi, ma, (int)nitems, s); }));
    if (raw) {
        double *canon = partial + k.nchunks * rs;
        HIP_TRY(timed(CUM_KIND_REDUCE, s, [&] {
            return launch_rawsum(partial, rs, k.nchunks, (const TileDev *)c->tiles_d.p, (const OrderDev *)c->ords_d.p,
                                 canon, c->shape == TS_1x2 ? 2 : 1, c->prec == P_F64, s);
        }));
        *summed = true;
        *sums = canon;
        return CUM_OK;
    }
    *summed = k.nchunks == 1 || always_sum || k.nchunks * c->stride > SMALL_PARTIALS;
    if (k.nchunks > 1 && *summed) {
        SetRed sr0;
        memset(&sr0, 0, sizeof sr0);
        sr0.partial = partial;
        sr0.stride = c->stride;
        sr0.nchunks = k.nchunks;
        sr0.t = k.t;
        HIP_TRY(timed(CUM_KIND_REDUCE, s, [&] { return launch_chunksum(nullptr, sr0, 1, c->stride, s); }));
    }
    return CUM_OK;
}

// Finalisation of orders dlo..dhi from moment sums S (nchunks chunks in the
// call's partial-sum layout, added in chunk order): M = S / t and, with
// recursion, the cumulants, into outs (block storage of block size b).
// moms (or null): buffers in block storage for the central moments of
// orders 2..dhi-2 (moms[m-2]); with them, orders >= 7 use the first-position
// formula.
static cum_status run_finalize(CallPlan *c, double *sums, int64_t nchunks, int64_t t, double *const *outs,
                               bool recursion, hipStream_t s, double *const *moms = nullptr) {
    cum_status st = upload_plan(*c);
    if (st) return st;
    // in pairs of orders {d, d+1}: order d needs cumulants up to d-2 only, so
    // a pair depends only on earlier pairs
    const RedOrder *red_d = (const RedOrder *)c->red_d.p;
    for (int d = c->dlo; d <= c->dhi; d += 2) {
        RedArgs ra;
        memset(&ra, 0, sizeof ra);
        const int i0 = d - c->dlo;
        ra.ords = red_d + i0;
        ra.nords = (d + 1 <= c->dhi) ? 2 : 1;
        ra.d0 = d;
        ra.b = c->red[i0].b;
        ra.recursion = recursion ? 1 : 0;
        ra.presummed = 0;
        ra.nb0 = c->red[i0].nblocks;
        ra.nbtot = ra.nb0 + (ra.nords == 2 ? c->red[i0 + 1].nblocks : 0);
        ra.sets = nullptr;
        ra.set0.partial = sums;
        ra.set0.stride = c->stride;
        ra.set0.nchunks = nchunks;
        ra.set0.t = t;
        for (int k = 0; k < MAXD - 1; ++k) ra.set0.kappa[k] = ra.set0.mom[k] = nullptr;
        for (int dd = c->dlo; dd <= c->dhi; ++dd) ra.set0.kappa[dd - 2] = outs[dd - c->dlo];
        ra.subset = (recursion && moms && c->dlo == 2 && c->dhi >= FIRST_POSITION_MIN_D) ? 1 : 0;
        if (ra.subset)
            for (int m = 2; m <= c->dhi - 2; ++m) ra.set0.mom[m - 2] = moms[m - 2];
        ra.set0.stamp = nullptr;
        if (!recursion) {
            // plain moments: no order reads another, one launch for all
            ra.nords = 1;
            ra.nbtot = ra.nb0;
        }
        set_gather(&c->red[i0], ra);
        const int lds = red_lds_layout(&c->red[i0], ra.nords, recursion, ra);
        const int be0 = (int)ipow64(c->red[i0].b, d);
        HIP_TRY(timed(CUM_KIND_REDUCE, s, [&] { return launch_reduce(ra, 1, lds, be0, s); }));
        if (!recursion) {
            for (int dd = d + 1; dd <= c->dhi; ++dd) {
                RedArgs rb = ra;
                rb.ords = red_d + (dd - c->dlo);
                rb.d0 = dd;
                rb.nb0 = rb.nbtot = c->red[dd - c->dlo].nblocks;
                const int be = (int)ipow64(c->red[dd - c->dlo].b, dd);
                HIP_TRY(timed(CUM_KIND_REDUCE, s, [&] { return launch_reduce(rb, 1, 0, be, s); }));
            }
            break;
        }
    }
    return CUM_OK;
}

// moment contraction + reduction for orders dlo..dhi into outs (and the
// recursion for d >= 4 when recursion is set)
static cum_status run_orders(const Call &k, const void *Xc, double *partial, double *const *outs, bool recursion,
                             hipStream_t s, double *const *moms = nullptr, const double *scale = nullptr) {
    cum_status st;
    bool summed;
    double *sums = nullptr;
    if ((st = run_contraction(k, Xc, partial, false, &summed, s, &sums, scale))) return st;
    return run_finalize(k.c, sums, summed ? 1 : k.nchunks, k.t, outs, recursion, s, moms);
}

// Bytes of the central-moment buffers the first-position formula needs
// (orders 2..d_max-2 in block storage), 0 below order 7.
static size_t moment_bytes(int n, int b, int d_max) {
    if (d_max < FIRST_POSITION_MIN_D) return 0;
    size_t total = 0;
    const int64_t nbar = (n + b - 1) / b;
    for (int m = 2; m <= d_max - 2; ++m) total += align_up((size_t)(binom(nbar + m - 1, m) * ipow64(b, m)) * 8);
    return total;
}

}  // namespace cum

using namespace cum;

extern "C" {

const char *cum_status_str(cum_status s) {
    switch (s) {
        case CUM_OK: return "CUM_OK";
        case CUM_EINVAL: return "CUM_EINVAL: invalid argument";
        case CUM_ENOMEM: return "CUM_ENOMEM: workspace too small or allocation failed";
        case CUM_EHIP: return "CUM_EHIP: HIP runtime error";
        case CUM_EUNSUPPORTED: return "CUM_EUNSUPPORTED: unsupported combination";
    }
    return "unknown status";
}

const char *cum_last_error(void) { return g_last_error.c_str(); }

cum_status cum_layout_query(int n, int d, int b, cum_layout *out) {
    if (!out) return fail(CUM_EINVAL, "out is NULL");
    if (n < 1 || b < 1 || b > n) return fail(CUM_EINVAL, "need n >= 1 and 1 <= b <= n (n=%d, b=%d)", n, b);
    if (d < 1 || d > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d must be in 1..%d (got %d)", CUM_MAX_ORDER, d);
    const int nbar = (n + b - 1) / b;
    const int64_t nb = binom(nbar + d - 1, d);
    const int64_t be = ipow64(b, d);
    if (nb < 0 || be == INT64_MAX || nb > INT64_MAX / be)
        return fail(CUM_EUNSUPPORTED, "the layout of n=%d, d=%d, b=%d overflows 64-bit sizes", n, d, b);
    out->n = n;
    out->d = d;
    out->b = b;
    out->nbar = nbar;
    out->b_last = n - b * (nbar - 1);
    out->nblocks = nb;
    out->block_elems = be;
    out->elems = nb * out->block_elems;
    return CUM_OK;
}

cum_status cum_stored_offset(int n, int d, int b, const int32_t *idx, int64_t *offset) {
    cum_layout L;
    cum_status st = cum_layout_query(n, d, b, &L);
    if (st) return st;
    if (!idx || !offset) return fail(CUM_EINVAL, "NULL argument");
    int v[CUM_MAX_ORDER], j[CUM_MAX_ORDER];
    for (int k = 0; k < d; ++k) {
        if (idx[k] < 0 || idx[k] >= n) return fail(CUM_EINVAL, "index %d out of range", idx[k]);
        v[k] = idx[k];
    }
    std::sort(v, v + d);
    int64_t in = 0;
    for (int k = 0; k < d; ++k) {
        j[k] = v[k] / b;
        in = in * b + (v[k] - j[k] * b);
    }
    *offset = rank_sorted_host(j, d, L.nbar) * L.block_elems + in;
    return CUM_OK;
}

cum_status cum_workspace_size(int64_t t, int n, int d_max, int b, cum_prec prec, size_t *bytes) {
    if (!bytes) return fail(CUM_EINVAL, "bytes is NULL");
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    std::lock_guard<std::mutex> lk(g_mu);
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    size_t total = staged_bytes(t, n, prec) + align_up((size_t)groups * n * 2 * 8) + align_up((size_t)n * 8) +
                   f16_bytes(prec, groups, n);
    Call k;
    if ((st = get_call(n, b, 2, d_max, prec, t, &k))) return st;
    size_t part = partial_bytes(k);
    // a single-order moment call uses its own plan; cover the largest one
    for (int d = 2; d <= d_max; ++d) {
        Call k1;
        if ((st = get_call(n, b, d, d, prec, t, &k1))) return st;
        part = std::max(part, partial_bytes(k1));
    }
    *bytes = total + align_up(part) + moment_bytes(n, b, d_max);
    return CUM_OK;
}

static cum_status center_impl(const double *X, int64_t t, int n, int64_t ldx, int prec, double *mean, void *Xc,
                              char *ws, size_t ws_bytes, hipStream_t s);

// Centring and staging of a call that centres its own data: column sums and
// means, then the staged layout (FP16 split: also the per-variable scales,
// written to f16w + the minima / maxima part; returned in *scale).
static cum_status center_and_stage(const double *X, int64_t t, int n, int64_t ldx, int prec, double *mu, char *cw,
                                   size_t cbytes, char *Xst, char *f16w, const double **scale, hipStream_t s) {
    *scale = nullptr;
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    if (prec == CUM_F16X2) {
        if (cbytes < align_up((size_t)groups * n * 2 * 8) || !f16w) return fail(CUM_ENOMEM, "centring workspace");
        double *part = (double *)cw, *mm = (double *)f16w;
        double *sc = (double *)(f16w + align_up((size_t)groups * n * 2 * 8));
        HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_colsum(X, t, n, ldx, rows_per, groups, part, s, mm); }));
        HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_mean(part, groups, n, t, mu, s, mm, sc); }));
        HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_stage(X, t, n, ldx, mu, Xst, prec, true, true, s, sc); }));
        *scale = sc;
        return CUM_OK;
    }
    cum_status st = center_impl(X, t, n, ldx, prec, mu, nullptr, cw, cbytes, s);
    if (st) return st;
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_stage(X, t, n, ldx, mu, Xst, prec, true, true, s); }));
    return CUM_OK;
}

static cum_status center_impl(const double *X, int64_t t, int n, int64_t ldx, int prec, double *mean, void *Xc,
                              char *ws, size_t ws_bytes, hipStream_t s) {
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    size_t need = align_up((size_t)groups * n * 2 * 8);
    if (ws_bytes < need || !ws) return fail(CUM_ENOMEM, "centring needs %zu workspace bytes", need);
    double *part = (double *)ws;
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_colsum(X, t, n, ldx, rows_per, groups, part, s); }));
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_mean(part, groups, n, t, mean, s); }));
    if (Xc) HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_center(X, t, n, ldx, mean, Xc, prec, s); }));
    return CUM_OK;
}

cum_status cum_center(const double *X, int64_t t, int n, int64_t ldx, cum_prec prec, double *mean, void *Xc,
                      void *ws, size_t ws_bytes, void *stream) {
    cum_status st;
    if ((st = check_common(t, n, 1)) || (st = check_prec(prec))) return st;
    if (!X || !mean) return fail(CUM_EINVAL, "X and mean must not be NULL");
    if (ldx < n) return fail(CUM_EINVAL, "ldx (%lld) < n (%d)", (long long)ldx, n);
    return center_impl(X, t, n, ldx, prec, mean, Xc, (char *)ws, ws_bytes, (hipStream_t)stream);
}

cum_status cum_moment_blocks(const void *Xc, cum_prec prec, int64_t t, int n, int d, int b, double *M, void *ws,
                             size_t ws_bytes, void *stream) {
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d < 2 || d > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d must be in 2..%d", CUM_MAX_ORDER);
    if (prec == CUM_F16X2 && d > 6)
        return fail(CUM_EUNSUPPORTED, "the FP16 split contracts orders up to 6 (use CUM_F32 or CUM_F64)");
    if (!Xc || !M) return fail(CUM_EINVAL, "Xc and M must not be NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    Call k;
    if ((st = get_call(n, b, d, d, prec, t, &k))) return st;
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    const size_t xbytes = staged_bytes(t, n, prec), pbytes = align_up(partial_bytes(k));
    // FP16 split: each group's column sums (unused) beside its minima and maxima
    const size_t cbytes = prec == CUM_F16X2 ? align_up((size_t)groups * n * 2 * 8) : 0;
    const size_t need = xbytes + pbytes + cbytes + f16_bytes(prec, groups, n);
    if (!ws || ws_bytes < need) return fail(CUM_ENOMEM, "moment_blocks needs %zu workspace bytes", need);
    if ((st = upload_call(k))) return st;
    hipStream_t s = (hipStream_t)stream;
    char *Xst = (char *)ws;
    const double *scale = nullptr;
    if (prec == CUM_F16X2) {
        // the data as given, each variable divided by a power of two bounding it
        // about zero; undone in the contraction
        char *cw = Xst + xbytes + pbytes, *fw = cw + cbytes;
        double *mm = (double *)fw, *sc = (double *)(fw + align_up((size_t)groups * n * 2 * 8));
        HIP_TRY(timed(CUM_KIND_CENTER, s, [&] {
            return launch_scale_f32((const float *)Xc, t, n, rows_per, groups, (double *)cw, mm, sc, s);
        }));
        scale = sc;
    }
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] {
        return launch_stage(Xc, t, n, n, nullptr, Xst, prec, false, prec == CUM_F64, s, scale);
    }));
    double *outs[1] = {M};
    return run_orders(k, Xst, (double *)(Xst + xbytes), outs, false, s, nullptr, scale);
}

static_assert(NOALLOC_SCRATCH_BYTES == CUM_NOALLOC_SCRATCH_BYTES, "scratch size");

// The body of cum_cumulants and of its allocation-free variant.  With
// noalloc, ws is the fixed scratch (null until after the checks, which then
// look it up) and every device table must already exist: the call allocates
// nothing.
static cum_status cumulants_impl(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec,
                                 double *mean, double *const *kappa, void *ws, size_t ws_bytes, void *stream,
                                 bool noalloc) {
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    if (!X || !kappa) return fail(CUM_EINVAL, "X and kappa must not be NULL");
    if (ldx < n) return fail(CUM_EINVAL, "ldx (%lld) < n (%d)", (long long)ldx, n);
    for (int d = 2; d <= d_max; ++d)
        if (!kappa[d - 2]) return fail(CUM_EINVAL, "kappa[%d] is NULL", d - 2);
    std::lock_guard<std::mutex> lk(g_mu);
    Call k;
    if ((st = get_call(n, b, 2, d_max, prec, t, &k))) return st;
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    const size_t xbytes = staged_bytes(t, n, prec);
    const size_t cbytes = align_up((size_t)groups * n * 2 * 8);
    const size_t mbytes = align_up((size_t)n * 8);
    const size_t pbytes = align_up(partial_bytes(k));
    const size_t lbytes = moment_bytes(n, b, d_max);
    const size_t need = xbytes + cbytes + mbytes + pbytes + lbytes + f16_bytes(prec, groups, n);
    if (noalloc) {
        if (need > NOALLOC_SCRATCH_BYTES)
            return fail(CUM_ENOMEM, "this call needs %zu bytes of scratch; the fixed scratch holds %zu", need,
                        NOALLOC_SCRATCH_BYTES);
        if (!k.c->uploaded || !k.is->uploaded)
            return fail(CUM_EUNSUPPORTED,
                        "the device tables of this configuration (n, b, d_max, prec, tuning and the sample-chunk "
                        "count of t) do not exist yet: run cum_cumulants once with it first");
        HIP_TRY(noalloc_scratch(&ws));
        ws_bytes = NOALLOC_SCRATCH_BYTES;
    }
    // the benchmark's per-launch timing creates HIP events: off for this call
    struct TimingOff {
        bool was, on;
        ~TimingOff() { if (on) g_timing = was; }
    } toff{g_timing, noalloc};
    if (noalloc) g_timing = false;
    if (!ws || ws_bytes < need) return fail(CUM_ENOMEM, "cumulants needs %zu workspace bytes (got %zu)", need, ws_bytes);
    char *w = (char *)ws;
    char *Xst = w;
    char *cw = w + xbytes;
    double *mtmp = (double *)(w + xbytes + cbytes);
    double *partial = (double *)(w + xbytes + cbytes + mbytes);
    hipStream_t s = (hipStream_t)stream;
    double *mu = mean ? mean : mtmp;
    if ((st = upload_call(k))) return st;
    const double *scale = nullptr;
    if ((st = center_and_stage(X, t, n, ldx, prec, mu, cw, cbytes, Xst, w + xbytes + cbytes + mbytes + pbytes + lbytes,
                               &scale, s)))
        return st;
    // central moments of the lower orders for the first-position formula
    double *moms[MAXD - 1] = {nullptr};
    double *const *mp = nullptr;
    if (d_max >= FIRST_POSITION_MIN_D) {
        char *mw = w + xbytes + cbytes + mbytes + pbytes;
        const int64_t nbar = (n + b - 1) / b;
        for (int m = 2; m <= d_max - 2; ++m) {
            moms[m - 2] = (double *)mw;
            mw += align_up((size_t)(binom(nbar + m - 1, m) * ipow64(b, m)) * 8);
        }
        mp = moms;
    }
    return run_orders(k, Xst, partial, kappa, true, s, mp, scale);
}

cum_status cum_cumulants(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec,
                         double *mean, double *const *kappa, void *ws, size_t ws_bytes, void *stream) {
    return cumulants_impl(X, t, n, ldx, d_max, b, prec, mean, kappa, ws, ws_bytes, stream, false);
}

cum_status cum_cumulants_noalloc(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec,
                                 double *mean, double *const *kappa, void *stream) {
    return cumulants_impl(X, t, n, ldx, d_max, b, prec, mean, kappa, nullptr, 0, stream, true);
}

cum_status cum_unfold(const double *blocks, int n, int d, int b, double *dense, void *stream) {
    cum_layout L;
    cum_status st = cum_layout_query(n, d, b, &L);
    if (st) return st;
    if (!blocks || !dense) return fail(CUM_EINVAL, "NULL buffer");
    HIP_TRY(timed(CUM_KIND_UNFOLD, (hipStream_t)stream,
                  [&] { return launch_unfold(blocks, n, d, b, dense, (hipStream_t)stream); }));
    return CUM_OK;
}

cum_status cum_plan_check(int n, int d, int b) {
    cum_status st;
    if ((st = check_common(1, n, b))) return st;
    if (d < 2 || d > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d must be in 2..%d", CUM_MAX_ORDER);
    OrderPlan o;
    if ((st = build_order(n, b, d, o))) return st;  // host tables only, nothing uploaded
    const int64_t be = ipow64(b, d);
    auto T = sorted_tuples(o.nbar, d);
    // the rank terms the reduction uses to find a tuple's partial sums
    for (size_t i = 0; i < T.size(); ++i) {
        int64_t r = 0;
        int prev = 0;
        for (int k = 0; k < d; ++k) {
            r += o.prank[(size_t)k * (o.nbar + 1) + prev] - o.prank[(size_t)k * (o.nbar + 1) + T[i][k]];
            prev = T[i][k];
        }
        if (r != (int64_t)i * be) return fail(CUM_EINVAL, "d=%d: rank table gives %lld for tuple %zu", d, (long long)r, i);
    }
    // the general formula's table: every set partition once, as many as the
    // Bell number B(d) (Bell triangle), with weights (k-1)! (-1)^(k-1)
    {
        std::vector<std::vector<uint16_t>> ap;
        std::vector<double> w;
        all_partitions(d, ap, w);
        std::vector<int64_t> row{1};
        for (int m = 1; m < d; ++m) {
            std::vector<int64_t> nx{row.back()};
            for (int64_t v : row) nx.push_back(nx.back() + v);
            row = nx;
        }
        if ((int64_t)ap.size() != row.back())
            return fail(CUM_EINVAL, "d=%d: %zu set partitions, expected %lld", d, ap.size(), (long long)row.back());
        std::set<std::vector<uint16_t>> seen;
        for (size_t z = 0; z < ap.size(); ++z) {
            unsigned cover = 0;
            for (uint16_t m : ap[z]) {
                if (!m || (cover & m)) return fail(CUM_EINVAL, "d=%d: set partition %zu overlaps", d, z);
                cover |= m;
            }
            double f = 1.0;
            for (size_t q = 2; q < ap[z].size(); ++q) f *= (double)q;
            if (cover != (1u << d) - 1u || w[z] != ((ap[z].size() - 1) % 2 ? -f : f))
                return fail(CUM_EINVAL, "d=%d: set partition %zu", d, z);
            auto sorted = ap[z];
            std::sort(sorted.begin(), sorted.end());
            if (!seen.insert(sorted).second) return fail(CUM_EINVAL, "d=%d: set partition %zu repeated", d, z);
        }
    }
    // recursion tables: every partition splits the d positions into >= 2
    // disjoint parts of >= 2 positions, no partition twice, and as many as
    // there are (a(d) - 1, a(n) = sum_k C(n-1, k) a(n-1-k) counting the set
    // partitions without singletons by the part holding the first element)
    if (d >= 4) {
        const int per = d / 2;
        std::vector<int64_t> a(d + 1, 0);
        a[0] = 1;
        for (int m = 1; m <= d; ++m)
            for (int k = 1; k <= m - 1; ++k) a[m] += binom(m - 1, k) * a[m - 1 - k];
        if (o.npart != a[d] - 1) return fail(CUM_EINVAL, "d=%d: %d partitions, expected %lld", d, o.npart, (long long)(a[d] - 1));
        std::set<std::vector<int>> seen;
        for (int z = 0; z < o.npart; ++z) {
            std::vector<int> masks;
            unsigned cover = 0;
            for (int k = 0; k < per; ++k) {
                const int32_t v = o.parts[(size_t)z * per + k];
                if (!v) break;
                const unsigned mask = (unsigned)v & 1023u;
                const int where = v >> 10, m = __builtin_popcount(mask);
                if (m < 2 || m > d - 2 || (cover & mask)) return fail(CUM_EINVAL, "d=%d: bad part in partition %d", d, z);
                cover |= mask;
                masks.push_back((int)mask);
                // where: the staged sub-block's first slot, or the position set's index
                const size_t si = (size_t)(std::find(o.smask.begin(), o.smask.end(), (uint16_t)mask) - o.smask.begin());
                if (si >= o.smask.size()) return fail(CUM_EINVAL, "d=%d: part set missing from the set list", d);
                if (o.lds_elems) {
                    if (where < 0 || where >= o.lds_elems || (o.gmap[(size_t)where] & 1023) != (int32_t)si ||
                        (o.gmap[(size_t)where] >> 10) != 0)
                        return fail(CUM_EINVAL, "d=%d: staged offset of part %d of partition %d", d, k, z);
                } else if (where != (int)si) {
                    return fail(CUM_EINVAL, "d=%d: set index of part %d of partition %d", d, k, z);
                }
            }
            if (masks.size() < 2 || cover != (1u << d) - 1u)
                return fail(CUM_EINVAL, "d=%d: partition %d does not cover the positions", d, z);
            std::sort(masks.begin(), masks.end());
            if (!seen.insert(masks).second) return fail(CUM_EINVAL, "d=%d: partition %d repeated", d, z);
        }
        // first-position terms (orders >= 7): every set A holding position 0
        // with 2..d-2 positions once (2^(d-1) - d - 1 of them), each with its
        // complement, both located like the parts above
        const int want_terms = d >= FIRST_POSITION_MIN_D ? (1 << (d - 1)) - d - 1 : 0;
        if (o.nterm != want_terms || (int)o.terms.size() != 2 * want_terms)
            return fail(CUM_EINVAL, "d=%d: %d first-position terms, expected %d", d, o.nterm, want_terms);
        std::set<int> seen_a;
        for (int z = 0; z < o.nterm; ++z) {
            int masks2[2];
            for (int k = 0; k < 2; ++k) {
                const int32_t v = o.terms[(size_t)z * 2 + k];
                const unsigned mask = (unsigned)v & 1023u;
                const int where = v >> 10, m = __builtin_popcount(mask);
                if (m < 2 || m > d - 2) return fail(CUM_EINVAL, "d=%d: bad set in term %d", d, z);
                const size_t si = (size_t)(std::find(o.smask.begin(), o.smask.end(), (uint16_t)mask) - o.smask.begin());
                if (si >= o.smask.size()) return fail(CUM_EINVAL, "d=%d: term set missing from the set list", d);
                if (o.lds_elems) {
                    if (where < 0 || where >= o.lds_elems || (o.gmap[(size_t)where] & 1023) != (int32_t)si ||
                        (o.gmap[(size_t)where] >> 10) != 0)
                        return fail(CUM_EINVAL, "d=%d: staged offset of factor %d of term %d", d, k, z);
                } else if (where != (int)si) {
                    return fail(CUM_EINVAL, "d=%d: set index of factor %d of term %d", d, k, z);
                }
                masks2[k] = (int)mask;
                // the multiplier of the set's index: b^(positions from ceil(d/2) on)
                int64_t pw = 1;
                for (int k2 = (d + 1) / 2; k2 < d; ++k2)
                    if (mask >> k2 & 1u) pw *= b;
                if ((int)o.tpw.size() != 2 * o.nterm || o.tpw[(size_t)z * 2 + k] != pw)
                    return fail(CUM_EINVAL, "d=%d: multiplier of factor %d of term %d", d, k, z);
            }
            if (!(masks2[0] & 1) || (masks2[0] ^ masks2[1]) != (1 << d) - 1 || (masks2[0] & masks2[1]))
                return fail(CUM_EINVAL, "d=%d: term %d is not a set with position 0 and its complement", d, z);
            if (!seen_a.insert(masks2[0]).second) return fail(CUM_EINVAL, "d=%d: term %d repeated", d, z);
            // the term lies in the group of the last qe positions its set A holds
            const int grp = term_group(masks2[0], d, o.qe);
            if (z < o.cstart[grp] || z >= o.cstart[grp + 1])
                return fail(CUM_EINVAL, "d=%d: term %d outside its group %d", d, z, grp);
        }
        if (d >= FIRST_POSITION_MIN_D) {
            // groups 0 .. 2^qe - 1 in order, the rest empty
            if (o.qe != first_position_qe(b, d, o.lds_elems > 0) || o.cstart[0] != 0 || o.cstart[1 << o.qe] != o.nterm ||
                o.cstart[4] != o.nterm)
                return fail(CUM_EINVAL, "d=%d: term groups", d);
            for (int c = 0; c < 4; ++c)
                if (o.cstart[c] > o.cstart[c + 1]) return fail(CUM_EINVAL, "d=%d: term group %d bounds", d, c);
        }
        // staged slots: each set's sub-block in order, grouped by set size
        if (o.lds_elems) {
            size_t e = 0;
            for (int m = 2; m <= d - 2; ++m) {
                if (o.mstart[m - 2] != (int32_t)e) return fail(CUM_EINVAL, "d=%d: size-%d segment start", d, m);
                for (size_t si = 0; si < o.smask.size(); ++si) {
                    if (__builtin_popcount(o.smask[si]) != m) continue;
                    for (int64_t f = 0; f < ipow64(b, m); ++f, ++e)
                        if (e >= o.gmap.size() || o.gmap[e] != (int32_t)(si | (f << 10)))
                            return fail(CUM_EINVAL, "d=%d: gather map slot %zu", d, e);
                }
            }
            if (o.mstart[d - 3] != (int32_t)e || e != o.gmap.size() || (int)e != o.lds_elems)
                return fail(CUM_EINVAL, "d=%d: staged slot count", d);
        }
    }
    for (int shape : {TS_1x1, TS_1x2}) {
        const int wn = shape_wn(shape);
        std::vector<HostTile> tiles;
        order_tiles(o, wn, 0, tiles);
        std::vector<uint8_t> hits((size_t)o.elems, 0);
        for (const auto &ht : tiles)
            for (int w = 0; w < ht.t.ntask; ++w) {
                const WaveTask &wt = ht.t.task[w];
                if (wt.mask >> (4 * wn)) return fail(CUM_EINVAL, "d=%d: task mask 0x%x", d, wt.mask);
                for (int j = 0; j < wn; ++j) {
                    for (int r = wt.r0; r < wt.r0 + 32; ++r)
                        for (int c = wt.c0 + 32 * j; c < std::min(o.nc, wt.c0 + 32 * j + 32); ++c) {
                            const Feat &fr = o.rows[r], &fc = o.cols[c];
                            const bool stored = fr.blk <= fc.blk;
                            const int bit = j * 4 + (r - wt.r0) / 16 * 2 + (c - wt.c0 - 32 * j) / 16;
                            const bool computed = wt.mask >> bit & 1;
                            if (stored && !computed)
                                return fail(CUM_EINVAL, "d=%d: entry (%d,%d) lies in a skipped block", d, r, c);
                            if (!stored) continue;
                            const int64_t addr = fr.addr + fc.addr + o.H[(size_t)fr.blk * o.nbar + fc.blk];
                            if (addr < 0 || addr >= o.elems)
                                return fail(CUM_EINVAL, "d=%d: address %lld out of range", d, (long long)addr);
                            if (hits[(size_t)addr]++)
                                return fail(CUM_EINVAL, "d=%d: address %lld written twice", d, (long long)addr);
                            // the variables multiplied there must be the ones stored there
                            const auto &jt = T[(size_t)(addr / be)];
                            int64_t in = addr % be;
                            int dig[CUM_MAX_ORDER];
                            for (int k = d - 1; k >= 0; --k) {
                                dig[k] = (int)(in % b);
                                in /= b;
                            }
                            for (int k = 0; k < d; ++k) {
                                int v = jt[k] * b + dig[k];
                                if (v > n) v = n;
                                const int have = k < o.p ? fr.var[k] : fc.var[k - o.p];
                                if (have != v)
                                    return fail(CUM_EINVAL, "d=%d: variable mismatch at address %lld", d,
                                                (long long)addr);
                            }
                        }
                }
            }
        for (size_t e = 0; e < hits.size(); ++e)
            if (hits[e] != 1) return fail(CUM_EINVAL, "d=%d: address %zu never written", d, e);
    }
    return CUM_OK;
}

cum_status cum_set_tuning(int64_t t, int n, int d_max, int b, cum_prec prec, const cum_tuning *tune) {
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    std::lock_guard<std::mutex> lk(g_mu);
    load_tune_file();
    auto key = std::make_tuple(n, b, 2, d_max, (int)prec, t);
    if (!tune) {
        g_tuned.erase(key);
        return CUM_OK;
    }
    if (tune->shape != TS_1x1 && tune->shape != TS_1x2)
        return fail(CUM_EINVAL, "unknown tile shape %d", tune->shape);
    if (tune->target_items < 1) return fail(CUM_EINVAL, "target_items must be >= 1");
    if (tune->inner_b < 1 || tune->inner_b > b)
        return fail(CUM_EINVAL, "inner_b must be in 1..b (got %d, b=%d)", tune->inner_b, b);
    g_tuned[key] = Tuning{tune->shape, tune->target_items, tune->inner_b};
    return CUM_OK;
}

cum_status cum_get_plan_info(int64_t t, int n, int d_max, int b, cum_prec prec, cum_plan_info *info) {
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    if (!info) return fail(CUM_EINVAL, "info is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    Call k;
    if ((st = get_call(n, b, 2, d_max, prec, t, &k))) return st;
    info->nchunks = k.nchunks;
    info->work_items = (int64_t)k.is->items.size();
    info->tiles = k.c->ntiles;
    info->partial_entries = k.c->stride;
    info->stored_entries = k.c->kstride;
    return CUM_OK;
}

cum_status cum_get_tuning(int64_t t, int n, int d_max, int b, cum_prec prec, cum_tuning *tune) {
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    if (!tune) return fail(CUM_EINVAL, "tune is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    load_tune_file();
    auto it = g_tuned.find(std::make_tuple(n, b, 2, d_max, (int)prec, t));
    const bool have = it != g_tuned.end();
    tune->shape = have ? it->second.shape : default_shape(prec);
    tune->target_items = have ? it->second.target : DEFAULT_TARGET;
    tune->inner_b = have ? it->second.bi : default_inner(b);
    tune->ms = 0.f;
    return CUM_OK;
}

// Candidate inner block sizes: the caller's b, 2 and 1.
static std::vector<int> inner_candidates(int b) {
    std::vector<int> v{b};
    if (b > 2) v.push_back(2);
    if (b > 1) v.push_back(1);
    return v;
}

// Time every candidate (inner block size x tile shape x work-item target) on
// the caller's data and keep the fastest for this shape: the contraction plus
// the reduction and recursion, best of three after one warm-up, HIP events on
// the stream.
cum_status cum_autotune(const double *X, int64_t t, int n, int64_t ldx, int d_max, int b, cum_prec prec, void *stream,
                        cum_tuning *best) {
    cum_status st;
    if ((st = check_common(t, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    if (!X || ldx < n) return fail(CUM_EINVAL, "bad X / ldx");
    std::lock_guard<std::mutex> lk(g_mu);
    load_tune_file();  // so that saving the file keeps the entries it already holds
    hipStream_t s = (hipStream_t)stream;
    const int shapes[] = {TS_1x1, TS_1x2};
    const int targets[] = {1024, 2048, 4096, 8192, 16384};
    std::vector<Call> cands;
    size_t part_max = 0;
    for (int bi : inner_candidates(b))
        for (int sh : shapes) {
            int64_t ntiles = 0, nch = 0, nst = 0;
            for (int tg : targets) {
                Call k;
                if ((st = get_call_cfg(n, b, bi, 2, d_max, prec, sh, tg, t, &k))) return st;
                if ((st = upload_call(k))) return st;
                cands.push_back(k);
                part_max = std::max(part_max, align_up(partial_bytes(k)));
                ntiles = k.c->ntiles;
                nch = k.nchunks;
                nst = k.nstages;
            }
            // Many tiles: the largest target still leaves fewer than 8 chunks.
            // Eight put one chunk on each XCD, whose stages then fit its L2.
            if (nch < 8 && nst >= 8 * 4 && 8 * ntiles <= INT32_MAX) {
                Call k;
                if ((st = get_call_cfg(n, b, bi, 2, d_max, prec, sh, (int)(8 * ntiles), t, &k))) return st;
                if ((st = upload_call(k))) return st;
                cands.push_back(k);
                part_max = std::max(part_max, align_up(partial_bytes(k)));
            }
        }
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    const size_t xbytes = staged_bytes(t, n, prec), cbytes = align_up((size_t)groups * n * 2 * 8);
    const size_t mbytes = align_up((size_t)n * 8), kbytes = align_up((size_t)cands[0].c->kstride * 8);
    // the lower central moments, so that orders >= 7 are timed with the
    // finalisation cum_cumulants runs (the first-position form)
    const size_t lbytes = moment_bytes(n, b, d_max);
    DevBuf ws;
    const size_t fbytes = f16_bytes(prec, groups, n);
    HIP_TRY(hipMalloc(&ws.p, xbytes + cbytes + mbytes + kbytes + part_max + lbytes + fbytes));
    char *w = (char *)ws.p;
    char *Xst = w, *cw = w + xbytes;
    double *mu = (double *)(w + xbytes + cbytes), *kap = (double *)(w + xbytes + cbytes + mbytes);
    double *partial = (double *)(w + xbytes + cbytes + mbytes + kbytes);
    double *outs[CUM_MAX_ORDER];
    for (int d = 2; d <= d_max; ++d) outs[d - 2] = kap + cands[0].c->out_off[d - 2];
    double *moms[MAXD - 1] = {nullptr};
    double *const *mp = nullptr;
    if (lbytes) {
        char *mw = w + xbytes + cbytes + mbytes + kbytes + part_max;
        const int64_t nbar = (n + b - 1) / b;
        for (int m = 2; m <= d_max - 2; ++m) {
            moms[m - 2] = (double *)mw;
            mw += align_up((size_t)(binom(nbar + m - 1, m) * ipow64(b, m)) * 8);
        }
        mp = moms;
    }
    const double *scale = nullptr;
    if ((st = center_and_stage(X, t, n, ldx, prec, mu, cw, cbytes, Xst,
                               w + xbytes + cbytes + mbytes + kbytes + part_max + lbytes, &scale, s)))
        return st;
    // timing of the library's own launches is off while candidates run; the
    // events and that switch are restored on every way out
    struct Guard {
        bool was = g_timing;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Guard() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            g_timing = was;
        }
    } gd;
    g_timing = false;
    HIP_TRY(hipEventCreate(&gd.e0));
    HIP_TRY(hipEventCreate(&gd.e1));
    float best_ms = 1e30f;
    const CallPlan *best_c = nullptr;
    for (const Call &c : cands) {
        float cand_ms = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
            HIP_TRY(hipEventRecord(gd.e0, s));
            if ((st = run_orders(c, Xst, partial, outs, true, s, mp, scale))) return st;
            HIP_TRY(hipEventRecord(gd.e1, s));
            HIP_TRY(hipEventSynchronize(gd.e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, gd.e0, gd.e1));
            if (rep > 0) cand_ms = std::min(cand_ms, ms);
        }
        if (cand_ms < best_ms) {
            best_ms = cand_ms;
            best_c = c.c;
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    const int best_target = best_c->target;
    g_tuned[std::make_tuple(n, b, 2, d_max, (int)prec, t)] = Tuning{best_c->shape, best_target, best_c->bi};
    save_tune_file();
    if (best) {
        best->shape = best_c->shape;
        best->target_items = best_target;
        best->inner_b = best_c->bi;
        best->ms = best_ms;
    }
    return CUM_OK;
}

cum_status cum_timing_enable(int on) {
    g_timing = on != 0;
    return CUM_OK;
}

cum_status cum_timing_read(double *ms, int64_t *launches) {
    if (!ms || !launches) return fail(CUM_EINVAL, "NULL argument");
    for (int k = 0; k < CUM_NKINDS; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    cum_status st = CUM_OK;
    for (auto &tl : g_timed) {
        float x = 0.f;
        hipError_t e = hipEventSynchronize(tl.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&x, tl.a, tl.b);
        if (e != hipSuccess && st == CUM_OK) st = fail(CUM_EHIP, "timing events: %s", hipGetErrorString(e));
        ms[tl.kind] += x;
        launches[tl.kind] += 1;
        (void)hipEventDestroy(tl.a);
        (void)hipEventDestroy(tl.b);
    }
    g_timed.clear();
    return st;
}

// ---------------------------------------------------------------------------
// Batched cumulants.
// ---------------------------------------------------------------------------
// Dataset groups of a batch: one per BATCH_SETS_PER_GROUP datasets, at most
// BATCH_GROUPS (and up to BATCH_MAX_GROUPS when fixed by CUM_BATCH_GROUPS).
// On the 512-dataset workload (n = 32, d <= 4, 16384 target items), 4 groups
// left the batch time unchanged (5.37 against 5.33 ms) and took the median
// dataset's latency from 4.82 to 4.30 ms; 8 groups gave 3.89 ms but a 10 %
// longer batch (each group's contraction ends in a tail).
constexpr int BATCH_MAX_GROUPS = 8;
constexpr int BATCH_GROUPS = 4;
constexpr int BATCH_SETS_PER_GROUP = 128;

struct cum_batch {
    int nsets = 0, n = 0, d_max = 0, b = 0, bi = 0, prec = 0, shape = 0;
    int64_t chunk_stages = 0, nitems = 0;
    int64_t stride = 0;               // partial sums of all orders (block size bi)
    int64_t kstride = 0;              // outputs of all orders (block size b)
    std::vector<int64_t> t;
    std::vector<OrderPlan *> orders;  // output layout, d = 2..d_max
    std::vector<OrderPlan *> corders; // contraction layout (block size bi)
    std::vector<int64_t> out_off;     // output offsets in a contiguous buffer
    std::vector<OrderDev> ods;
    std::vector<RedOrder> red;
    std::vector<HostTile> tiles;
    std::vector<SetDev> sets;
    std::vector<SetRed> setred;
    std::vector<CenterSet> csets;
    int max_groups = 1, stage_blocks = 1;
    DevBuf ords_d, tiles_d, items_d, red_d, sets_d, setred_d, cset_d;
    DevBuf staged_d, partial_d, part_d, mean_d, stamps_d, mm_d, scale_d;
    CenterSet *h_cset = nullptr;  // pinned staging of the per-run pointer tables
    SetRed *h_setred = nullptr;
    hipEvent_t copied = nullptr, done = nullptr, ready = nullptr;
    hipStream_t stream = nullptr;     // the plan's own stream (graph capture and replay)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool pending_copy = false;
    // Datasets are finalised in groups: group g's datasets are seq[group_first[g]]
    // .. seq[group_first[g+1]-1], and its contraction items are items
    // group_item[g] .. group_item[g+1]-1.  The contraction of the groups runs
    // in group order on the plan's stream; each group's chunk sum and
    // finalisation run on the side stream as soon as its contraction is done,
    // beside the next group's contraction.
    int ngroups = 1;
    std::vector<int> group_first;
    // The datasets in group order: by sample count, smallest first (shortest
    // work first gives the least mean completion time), then by index.  The
    // device array of finalisation records (setred_d) is in this order.
    std::vector<int> seq;
    std::vector<int64_t> group_item;
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> group_done;  // capture-time fork events, one per group
    hipEvent_t side_done = nullptr;      // capture-time join event
    DevBuf mom_d;  // per-dataset central moments of orders 2..d_max-2 (first-position form, d_max >= 7)
};

static void batch_free(cum_batch *p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->h_cset) (void)hipHostFree(p->h_cset);
    if (p->h_setred) (void)hipHostFree(p->h_setred);
    if (p->copied) (void)hipEventDestroy(p->copied);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->ready) (void)hipEventDestroy(p->ready);
    for (hipEvent_t e : p->group_done)
        if (e) (void)hipEventDestroy(e);
    if (p->side_done) (void)hipEventDestroy(p->side_done);
    if (p->side) {
        (void)hipStreamSynchronize(p->side);
        (void)hipStreamDestroy(p->side);
    }
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

// Work items of one group of datasets (s0..s1-1) of a batch: datasets go to
// XCDs by longest-processing-time first (so each dataset's staged data stays
// in one XCD's L2); on each XCD the items run most expensive first; item i of
// the group's launch runs on XCD i % 8.
static std::vector<Item> batch_items(const cum_batch &p, int s0, int s1) {
    int64_t tile_cost = 0;
    for (auto &h : p.tiles) tile_cost += h.cost;
    std::vector<int> order;
    for (int i = s0; i < s1; ++i) order.push_back(p.seq[i]);
    std::vector<int64_t> nst(p.nsets);
    for (int s : order) nst[s] = p.sets[s].nstages;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nst[x] > nst[y]; });
    int64_t load[8] = {0};
    std::vector<std::vector<std::pair<int64_t, Item>>> per_xcd(8);
    for (int s : order) {
        int x = (int)(std::min_element(load, load + 8) - load);
        load[x] += nst[s] * tile_cost;
        for (int64_t ch = 0; ch < p.sets[s].nchunks; ++ch) {
            const int64_t len = std::min(p.chunk_stages, nst[s] - ch * p.chunk_stages);
            for (size_t ti = 0; ti < p.tiles.size(); ++ti)
                per_xcd[x].push_back({len * p.tiles[ti].cost, Item{(int32_t)ti, (int32_t)ch, (int32_t)s, 0}});
        }
    }
    size_t longest = 0;
    for (auto &v : per_xcd) {
        std::stable_sort(v.begin(), v.end(), [](const std::pair<int64_t, Item> &a, const std::pair<int64_t, Item> &b) {
            return a.first > b.first;
        });
        longest = std::max(longest, v.size());
    }
    std::vector<Item> items;
    for (size_t i = 0; i < longest; ++i)
        for (int x = 0; x < 8; ++x) items.push_back(i < per_xcd[x].size() ? per_xcd[x][i].second : Item{-1, 0, 0, 0});
    while (!items.empty() && items.back().tile < 0) items.pop_back();
    return items;
}

// (Re)build the contraction tables, tiles, chunking and items for an inner
// block size, shape and target, and the per-dataset records that depend on them.
static cum_status batch_layout(cum_batch &p, int bi, int shape, int target) {
    cum_status st;
    const int wn = shape_wn(shape);
    p.shape = shape;
    p.bi = bi;
    p.corders.clear();
    p.ods.clear();
    p.red.clear();
    int64_t poff_o = 0;
    for (size_t i = 0; i < p.orders.size(); ++i) {
        OrderPlan *co;
        if ((st = get_order(p.n, bi, p.orders[i]->d, &co)) || (st = upload_order(*co))) return st;
        p.corders.push_back(co);
        p.ods.push_back(order_dev(*co, poff_o));
        p.red.push_back(red_order(*p.orders[i], *co, poff_o));
        poff_o += co->elems;
    }
    p.stride = poff_o;
    if ((st = upload(p.ords_d, p.ods)) || (st = upload(p.red_d, p.red))) return st;
    p.tiles.clear();
    for (size_t i = 0; i < p.corders.size(); ++i) order_tiles(*p.corders[i], wn, (int)i, p.tiles);
    std::stable_sort(p.tiles.begin(), p.tiles.end(), [](const HostTile &x, const HostTile &y) { return x.cost > y.cost; });
    const int KT = stage_kt(p.prec);
    int64_t total_st = 0, max_st = 1;
    for (int s = 0; s < p.nsets; ++s) {
        const int64_t nst = (p.t[s] + KT - 1) / KT;
        total_st += nst;
        max_st = std::max(max_st, nst);
    }
    // chunk length: about `target` items overall, whole datasets when that is enough
    const int64_t ntiles = (int64_t)p.tiles.size();
    int64_t cs = std::max<int64_t>(4, (total_st * ntiles + target - 1) / std::max<int64_t>(target, 1));
    p.chunk_stages = std::min(cs, max_st);
    int64_t poff = 0;
    for (int s = 0; s < p.nsets; ++s) {
        SetDev &sd = p.sets[s];
        sd.nstages = (p.t[s] + KT - 1) / KT;
        sd.chunk_stages = p.chunk_stages;
        sd.nchunks = (sd.nstages + p.chunk_stages - 1) / p.chunk_stages;
        sd.stride = p.stride;
        sd.partial = reinterpret_cast<double *>(poff);  // offset; rebased after allocation
        poff += sd.nchunks * p.stride;
    }
    // groups of about equal contraction work, consecutive in the order of
    // increasing sample count
    p.seq.resize(p.nsets);
    for (int s = 0; s < p.nsets; ++s) p.seq[s] = s;
    std::stable_sort(p.seq.begin(), p.seq.end(),
                     [&](int x, int y) { return p.sets[x].nstages < p.sets[y].nstages; });
    int64_t tile_cost = 0, work = 0;
    for (auto &h : p.tiles) tile_cost += h.cost;
    std::vector<int64_t> cum_work(p.nsets + 1, 0);
    for (int i = 0; i < p.nsets; ++i) {
        work += p.sets[p.seq[i]].nstages * tile_cost;
        cum_work[i + 1] = work;
    }
    int64_t want_groups = std::min<int64_t>(BATCH_GROUPS, p.nsets / BATCH_SETS_PER_GROUP);
    if (const char *e = getenv("CUM_BATCH_GROUPS")) {  // a fixed group count (tests, experiments)
        const long v = strtol(e, nullptr, 10);
        if (v >= 1) want_groups = v;
    }
    p.ngroups = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)BATCH_MAX_GROUPS, (int64_t)p.nsets, want_groups}));
    p.group_first.assign(1, 0);
    for (int g = 1; g < p.ngroups; ++g) {
        const int64_t want = work * g / p.ngroups;
        int s = p.group_first.back() + 1;
        while (s < p.nsets - (p.ngroups - g) && cum_work[s] < want) ++s;
        p.group_first.push_back(s);
    }
    p.group_first.push_back(p.nsets);
    std::vector<Item> items;
    p.group_item.assign(1, 0);
    for (int g = 0; g < p.ngroups; ++g) {
        auto gi = batch_items(p, p.group_first[g], p.group_first[g + 1]);
        items.insert(items.end(), gi.begin(), gi.end());
        p.group_item.push_back((int64_t)items.size());
    }
    p.nitems = (int64_t)items.size();
    std::vector<TileDev> tdev;
    for (auto &h : p.tiles) tdev.push_back(h.t);
    if ((st = upload(p.tiles_d, tdev)) || (st = upload(p.items_d, items))) return st;
    if (p.partial_d.p) {
        (void)hipFree(p.partial_d.p);
        p.partial_d.p = nullptr;
    }
    HIP_TRY(hipMalloc(&p.partial_d.p, std::max<int64_t>(1, poff) * sizeof(double)));
    for (int s = 0; s < p.nsets; ++s) {
        p.sets[s].partial = (double *)p.partial_d.p + (int64_t)(intptr_t)p.sets[s].partial;
        p.setred[s].partial = p.sets[s].partial;
        p.setred[s].nchunks = p.sets[s].nchunks;
        p.setred[s].stride = p.stride;
    }
    if ((st = upload(p.sets_d, p.sets))) return st;
    if (p.exec) {
        (void)hipGraphExecDestroy(p.exec);
        p.exec = nullptr;
    }
    if (p.graph) {
        (void)hipGraphDestroy(p.graph);
        p.graph = nullptr;
    }
    return CUM_OK;
}

static cum_status batch_enqueue(cum_batch &p, hipStream_t s) {
    HIP_TRY(launch_batch_stamp((unsigned long long *)p.stamps_d.p, p.nsets, s));
    const CenterSet *cs = (const CenterSet *)p.cset_d.p;
    HIP_TRY(launch_batch_colsum(cs, p.nsets, p.max_groups, p.n, s, p.prec == CUM_F16X2));
    HIP_TRY(launch_batch_mean(cs, p.nsets, p.n, s, p.prec == CUM_F16X2));
    HIP_TRY(launch_batch_stage(cs, p.nsets, p.n, p.prec, p.stage_blocks, s));
    const RedOrder *red_d = (const RedOrder *)p.red_d.p;
    const SetRed *setred = (const SetRed *)p.setred_d.p;
    for (int g = 0; g < p.ngroups; ++g) {
        const int s0 = p.group_first[g], ns = p.group_first[g + 1] - s0;
        const int64_t i0 = p.group_item[g], ni = p.group_item[g + 1] - i0;
        MomentArgs ma;
        memset(&ma, 0, sizeof ma);
        ma.ords = (const OrderDev *)p.ords_d.p;
        ma.tiles = (const TileDev *)p.tiles_d.p;
        ma.items = (const Item *)p.items_d.p + i0;
        ma.nitems = ni;
        ma.sets = (const SetDev *)p.sets_d.p;
        ma.n = p.n;
        if (ni > 0) HIP_TRY(launch_moment(p.prec, p.shape, p.d_max, ma, (int)ni, s));
        // the group's finalisation on the side stream, once its contraction is done
        hipStream_t fs = p.side;
        HIP_TRY(hipEventRecord(p.group_done[g], s));
        HIP_TRY(hipStreamWaitEvent(p.side, p.group_done[g], 0));
        SetRed none;
        memset(&none, 0, sizeof none);
        HIP_TRY(launch_chunksum(setred + s0, none, ns, p.stride, fs));
        for (int d = 2; d <= p.d_max; d += 2) {
            RedArgs ra;
            memset(&ra, 0, sizeof ra);
            const int o0 = d - 2;
            ra.ords = red_d + o0;
            ra.nords = (d + 1 <= p.d_max) ? 2 : 1;
            ra.d0 = d;
            ra.b = p.b;
            ra.recursion = 1;
            ra.presummed = 1;
            ra.subset = p.d_max >= FIRST_POSITION_MIN_D ? 1 : 0;
            ra.nb0 = p.red[o0].nblocks;
            ra.nbtot = ra.nb0 + (ra.nords == 2 ? p.red[o0 + 1].nblocks : 0);
            ra.sets = setred + s0;
            set_gather(&p.red[o0], ra);
            const int lds = red_lds_layout(&p.red[o0], ra.nords, true, ra);
            HIP_TRY(launch_reduce(ra, ns, lds, (int)ipow64(p.b, d), fs));
        }
    }
    HIP_TRY(hipEventRecord(p.side_done, p.side));
    HIP_TRY(hipStreamWaitEvent(s, p.side_done, 0));
    return CUM_OK;
}

cum_status cum_batch_create(int n_sets, const int64_t *t_i, int n, int d_max, int b, cum_prec prec,
                            cum_batch **plan) {
    cum_status st;
    if (!plan || !t_i) return fail(CUM_EINVAL, "NULL argument");
    *plan = nullptr;
    if (n_sets < 1 || n_sets > 65535) return fail(CUM_EINVAL, "n_sets must be in 1..65535");
    if ((st = check_common(1, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    for (int s = 0; s < n_sets; ++s)
        if (t_i[s] < 1) return fail(CUM_EINVAL, "t_i[%d] = %lld < 1", s, (long long)t_i[s]);
    for (int d = 2; d <= d_max; ++d)
        if (ipow64(b, d) > INT32_MAX)
            return fail(CUM_EUNSUPPORTED, "blocks of b^d = %d^%d entries (2^31 or more) are not supported", b, d);
    std::lock_guard<std::mutex> lk(g_mu);
    std::unique_ptr<cum_batch, void (*)(cum_batch *)> p(new cum_batch, batch_free);
    p->nsets = n_sets;
    p->n = n;
    p->d_max = d_max;
    p->b = b;
    p->prec = prec;
    p->t.assign(t_i, t_i + n_sets);
    int64_t off = 0;
    for (int d = 2; d <= d_max; ++d) {
        OrderPlan *o;
        if (ipow64(b, d) > INT32_MAX)
            return fail(CUM_EUNSUPPORTED, "blocks of b^d = %d^%d entries (2^31 or more) are not supported", b, d);
        if ((st = get_order(n, b, d, &o)) || (st = upload_order(*o))) return st;
        p->orders.push_back(o);
        p->out_off.push_back(off);
        off += o->elems;
    }
    p->kstride = off;
    // per-dataset storage: staged data, centring partial sums, means scratch
    const int KT = stage_kt(prec), KTP = stage_pitch(prec);
    int64_t staged = 0, parts = 0;
    p->sets.resize(n_sets);
    p->setred.resize(n_sets);
    p->csets.resize(n_sets);
    std::vector<int64_t> st_off(n_sets), part_off(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        int groups;
        int64_t rows_per;
        center_groups(p->t[s], groups, rows_per);
        p->csets[s].groups = groups;
        p->csets[s].rows_per = rows_per;
        p->csets[s].t = p->t[s];
        p->max_groups = std::max(p->max_groups, groups);
        st_off[s] = staged;
        staged += (p->t[s] + KT - 1) / KT * (int64_t)(n + 1) * KTP * stage_esize(prec);
        staged = (int64_t)align_up((size_t)staged);
        part_off[s] = parts;
        parts += (int64_t)groups * n * 2;
    }
    HIP_TRY(hipMalloc(&p->staged_d.p, std::max<int64_t>(staged, 256)));
    HIP_TRY(hipMalloc(&p->part_d.p, std::max<int64_t>(parts, 1) * sizeof(double)));
    if (prec == CUM_F16X2) {
        // each dataset's column minima / maxima (laid out as its partial sums) and scales
        HIP_TRY(hipMalloc(&p->mm_d.p, std::max<int64_t>(parts, 1) * sizeof(double)));
        HIP_TRY(hipMalloc(&p->scale_d.p, (size_t)n_sets * (n + 1) * sizeof(double)));
    }
    HIP_TRY(hipMalloc(&p->mean_d.p, (size_t)n_sets * n * sizeof(double)));
    HIP_TRY(hipMalloc(&p->stamps_d.p, (size_t)(n_sets + 1) * sizeof(unsigned long long)));
    for (int s = 0; s < n_sets; ++s) {
        CenterSet &c = p->csets[s];
        c.X = nullptr;
        c.mean = (double *)p->mean_d.p + (int64_t)s * n;
        c.Xc = (char *)p->staged_d.p + st_off[s];
        c.part = (double *)p->part_d.p + part_off[s];
        c.pad = 0;
        c.mm = p->mm_d.p ? (double *)p->mm_d.p + part_off[s] : nullptr;
        c.scale = p->scale_d.p ? (double *)p->scale_d.p + (int64_t)s * (n + 1) : nullptr;
        p->sets[s].X = c.Xc;
        p->sets[s].scale = c.scale;
        SetRed &r = p->setred[s];
        r.t = p->t[s];
        for (int k = 0; k < MAXD - 1; ++k) r.kappa[k] = r.mom[k] = nullptr;
        r.stamp = (unsigned long long *)p->stamps_d.p + 1 + s;
    }
    // from d_max = 7 on, orders >= 7 are finalised by the first-position
    // formula, over each dataset's central moments of orders 2..d_max-2
    const size_t mom_set = moment_bytes(n, b, d_max);
    if (mom_set) {
        HIP_TRY(hipMalloc(&p->mom_d.p, mom_set * n_sets));
        const int64_t nbar = (n + b - 1) / b;
        for (int s = 0; s < n_sets; ++s) {
            char *mw = (char *)p->mom_d.p + mom_set * s;
            for (int m = 2; m <= d_max - 2; ++m) {
                p->setred[s].mom[m - 2] = (double *)mw;
                mw += align_up((size_t)(binom(nbar + m - 1, m) * ipow64(b, m)) * 8);
            }
        }
    }
    int64_t max_nst = 1;
    for (int s = 0; s < n_sets; ++s) max_nst = std::max(max_nst, (p->t[s] + KT - 1) / KT);
    p->stage_blocks = (int)std::min<int64_t>(max_nst, 64);
    load_tune_file();
    auto tk = g_tuned.find(std::make_tuple(n, b, 2, d_max, (int)prec, -(int64_t)n_sets));
    const int shape = tk != g_tuned.end() ? tk->second.shape : default_shape(prec);
    const int target = tk != g_tuned.end() ? tk->second.target : 16384;
    const int bi = tk != g_tuned.end() ? tk->second.bi : default_inner(b);
    if ((st = batch_layout(*p, bi, shape, target))) return st;
    HIP_TRY(hipMalloc(&p->cset_d.p, sizeof(CenterSet) * n_sets));
    HIP_TRY(hipMalloc(&p->setred_d.p, sizeof(SetRed) * n_sets));
    HIP_TRY(hipHostMalloc((void **)&p->h_cset, sizeof(CenterSet) * n_sets, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&p->h_setred, sizeof(SetRed) * n_sets, hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&p->copied, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->ready, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    p->group_done.assign(BATCH_MAX_GROUPS, nullptr);
    for (auto &e : p->group_done) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->side_done, hipEventDisableTiming));
    *plan = p.release();
    return CUM_OK;
}

cum_status cum_batch_run(cum_batch *p, const double *const *X_i, double *const *kappa, double *const *mean,
                         void *stream) {
    if (!p || !X_i || !kappa) return fail(CUM_EINVAL, "NULL argument");
    const int nk = p->d_max - 1;
    for (int s = 0; s < p->nsets; ++s) {
        if (!X_i[s]) return fail(CUM_EINVAL, "X_i[%d] is NULL", s);
        for (int k = 0; k < nk; ++k)
            if (!kappa[(int64_t)s * nk + k]) return fail(CUM_EINVAL, "kappa[%d] is NULL", s * nk + k);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t user = (hipStream_t)stream;
    // the pinned tables may still be read by the previous run's copies
    if (p->pending_copy) HIP_TRY(hipEventSynchronize(p->copied));
    for (int s = 0; s < p->nsets; ++s) {
        p->h_cset[s] = p->csets[s];
        p->h_cset[s].X = X_i[s];
        if (mean && mean[s]) p->h_cset[s].mean = mean[s];
    }
    for (int i = 0; i < p->nsets; ++i) {  // finalisation records in group order
        const int s = p->seq[i];
        p->h_setred[i] = p->setred[s];
        for (int k = 0; k < nk; ++k) p->h_setred[i].kappa[k] = kappa[(int64_t)s * nk + k];
    }
    // order after the caller's stream, run on the plan's stream, order the caller after it
    HIP_TRY(hipEventRecord(p->ready, user));
    HIP_TRY(hipStreamWaitEvent(p->stream, p->ready, 0));
    HIP_TRY(hipMemcpyAsync(p->cset_d.p, p->h_cset, sizeof(CenterSet) * p->nsets, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->setred_d.p, p->h_setred, sizeof(SetRed) * p->nsets, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipEventRecord(p->copied, p->stream));
    p->pending_copy = true;
    if (!p->exec) {
        HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
        cum_status st = batch_enqueue(*p, p->stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->stream, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(CUM_EHIP, "graph capture: %s", hipGetErrorString(e));
        p->graph = g;
        HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(timed(CUM_KIND_BATCH, p->stream, [&] { return hipGraphLaunch(p->exec, p->stream); }));
    HIP_TRY(hipEventRecord(p->done, p->stream));
    HIP_TRY(hipStreamWaitEvent(user, p->done, 0));
    return CUM_OK;
}

cum_status cum_batch_timestamps(cum_batch *p, uint64_t *start, uint64_t *ticks, double *hz) {
    if (!p || !start || !ticks || !hz) return fail(CUM_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(p->stream));
    std::vector<unsigned long long> h(p->nsets + 1);
    HIP_TRY(hipMemcpy(h.data(), p->stamps_d.p, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    *start = h[0];
    for (int s = 0; s < p->nsets; ++s) ticks[s] = h[1 + s];
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *hz = khz * 1000.0;
    return CUM_OK;
}

// Time the whole graph of every candidate (inner block size x tile shape x
// work-item target) on the batch's data and keep the fastest; the graph is
// captured again on the next run.
cum_status cum_batch_autotune(cum_batch *p, const double *const *X_i, cum_tuning *best) {
    if (!p || !X_i) return fail(CUM_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_tune_file();  // so that saving the file keeps the entries it already holds
    }
    std::vector<double *> kap((size_t)p->nsets * (p->d_max - 1));
    // outputs of the trial runs: a scratch buffer with every dataset's own
    // slice (the recursion of a dataset reads its own lower orders)
    DevBuf scratch;
    HIP_TRY(hipMalloc(&scratch.p, (size_t)p->nsets * p->kstride * sizeof(double)));
    for (int s = 0; s < p->nsets; ++s)
        for (int d = 2; d <= p->d_max; ++d)
            kap[(size_t)s * (p->d_max - 1) + d - 2] = (double *)scratch.p + (size_t)s * p->kstride + p->out_off[d - 2];
    const int shapes[] = {TS_1x1, TS_1x2};
    const int targets[] = {4096, 16384, 65536};
    float best_ms = 1e30f;
    int best_shape = p->shape, best_target = 16384, best_bi = p->bi;
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    HIP_TRY(hipEventCreate(&ev.e0));
    HIP_TRY(hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    struct Cand {
        int bi, sh, tg;
    };
    std::vector<Cand> cands;
    for (int bi : inner_candidates(p->b))
        for (int sh : shapes)
            for (int tg : targets) cands.push_back({bi, sh, tg});
    cum_status st = CUM_OK;
    for (const Cand &cd : cands) {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            if ((st = batch_layout(*p, cd.bi, cd.sh, cd.tg))) break;
        }
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3 && !st; ++rep) {
            if ((st = cum_batch_run(p, X_i, kap.data(), nullptr, nullptr))) break;
            HIP_TRY(hipStreamSynchronize(p->stream));
            HIP_TRY(hipEventRecord(e0, p->stream));
            HIP_TRY(hipGraphLaunch(p->exec, p->stream));
            HIP_TRY(hipEventRecord(e1, p->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            ms_best = std::min(ms_best, ms);
        }
        if (st) break;
        if (ms_best < best_ms) {
            best_ms = ms_best;
            best_shape = cd.sh;
            best_target = cd.tg;
            best_bi = cd.bi;
        }
    }
    HIP_TRY(hipDeviceSynchronize());
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((st = batch_layout(*p, best_bi, best_shape, best_target))) return st;
    g_tuned[std::make_tuple(p->n, p->b, 2, p->d_max, p->prec, -(int64_t)p->nsets)] =
        Tuning{best_shape, best_target, best_bi};
    save_tune_file();
    if (best) {
        best->shape = best_shape;
        best->target_items = best_target;
        best->inner_b = best_bi;
        best->ms = best_ms;
    }
    return CUM_OK;
}

cum_status cum_batch_destroy(cum_batch *plan) {
    batch_free(plan);
    return CUM_OK;
}

// ---------------------------------------------------------------------------
// Streaming windows: FP64 moment sums about a fixed shift, updated by adding
// and removing batches of samples, finalised on demand.
// ---------------------------------------------------------------------------
struct cum_stream {
    int n = 0, d_max = 0, b = 0, prec = 0;
    int64_t t = 0;          // samples in the window
    bool have_shift = false;
    int64_t stride = 0;     // sums of orders 2..d_max, each sorted variable tuple once
    std::vector<int64_t> off;  // offset of order d in the sums (index d - 2)
    CallPlan *last = nullptr;  // a plan of the window's shape (its finalisation records)
    DevBuf shift_d, s1_d, delta_d, bmean_d, sums_d, central_d, ws_d;
    DevBuf mom_d;           // central moments of orders 2..d_max-2 for the first-position formula (d_max >= 7)
    size_t ws_bytes = 0;
};

cum_status cum_stream_create(int n, int d_max, int b, cum_prec prec, const double *shift, cum_stream **out) {
    cum_status st;
    if (!out) return fail(CUM_EINVAL, "NULL argument");
    *out = nullptr;
    if ((st = check_common(1, n, b)) || (st = check_prec(prec))) return st;
    if (d_max < 2 || d_max > CUM_MAX_ORDER) return fail(CUM_EINVAL, "d_max must be in 2..%d", CUM_MAX_ORDER);
    prec = (cum_prec)staged_prec(prec, d_max);
    for (int d = 2; d <= d_max; ++d)
        if (ipow64(b, d) > INT32_MAX)
            return fail(CUM_EUNSUPPORTED, "blocks of b^d = %d^%d entries (2^31 or more) are not supported", b, d);
    std::lock_guard<std::mutex> lk(g_mu);
    std::unique_ptr<cum_stream> p(new cum_stream);
    p->n = n;
    p->d_max = d_max;
    p->b = b;
    p->prec = prec;
    for (int d = 2; d <= d_max; ++d) {
        OrderPlan *o;
        if ((st = get_order(n, 1, d, &o))) return st;
        p->off.push_back(p->stride);
        p->stride += o->elems;
    }
    const size_t sb = (size_t)std::max<int64_t>(p->stride, 1) * sizeof(double), nb = (size_t)n * sizeof(double);
    HIP_TRY(hipMalloc(&p->sums_d.p, sb));
    HIP_TRY(hipMalloc(&p->central_d.p, sb));
    HIP_TRY(hipMalloc(&p->shift_d.p, nb));
    HIP_TRY(hipMalloc(&p->s1_d.p, nb));
    HIP_TRY(hipMalloc(&p->delta_d.p, nb));
    HIP_TRY(hipMalloc(&p->bmean_d.p, nb));
    if (const size_t mb = moment_bytes(n, b, d_max)) HIP_TRY(hipMalloc(&p->mom_d.p, mb));
    HIP_TRY(hipMemset(p->sums_d.p, 0, sb));
    HIP_TRY(hipMemset(p->s1_d.p, 0, nb));
    if (shift) {
        HIP_TRY(hipMemcpy(p->shift_d.p, shift, nb, hipMemcpyHostToDevice));
        p->have_shift = true;
    }
    *out = p.release();
    return CUM_OK;
}

cum_status cum_stream_update(cum_stream *p, const double *X, int64_t t, int64_t ldx, int sign, void *stream) {
    cum_status st;
    if (!p || !X) return fail(CUM_EINVAL, "NULL argument");
    if (t < 1) return fail(CUM_EINVAL, "t must be >= 1 (got %lld)", (long long)t);
    if (ldx < p->n) return fail(CUM_EINVAL, "ldx (%lld) < n (%d)", (long long)ldx, p->n);
    if (sign != 1 && sign != -1) return fail(CUM_EINVAL, "sign must be +1 (add) or -1 (remove)");
    if (sign < 0 && p->t - t < 0)
        return fail(CUM_EINVAL, "removing %lld samples from a window of %lld", (long long)t, (long long)p->t);
    if (sign < 0 && !p->have_shift) return fail(CUM_EINVAL, "nothing has been added yet");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = (hipStream_t)stream;
    const int n = p->n;
    // the contraction fills the layout of block size 1 (each sorted tuple
    // once); a tuned task shape and item target for this sample count apply.
    // Untuned, chunks hold at least 16 stages: stream batches are often
    // small, and short work items spend much of their time on set-up
    Call k;
    int shape = default_shape(p->prec), target = DEFAULT_TARGET, min_stages = 16;
    load_tune_file();
    auto tu = g_tuned.find(std::make_tuple(n, p->b, 2, p->d_max, p->prec, t));
    if (tu != g_tuned.end()) {
        shape = tu->second.shape;
        target = tu->second.target;
        min_stages = 4;
    }
    if ((st = get_call_cfg(n, p->b, 1, 2, p->d_max, p->prec, shape, target, t, &k, min_stages))) return st;
    if ((st = upload_call(k))) return st;
    int groups;
    int64_t rows_per;
    center_groups(t, groups, rows_per);
    const size_t xbytes = staged_bytes(t, n, p->prec), cbytes = align_up((size_t)groups * n * 2 * 8);
    const size_t pbytes = align_up(partial_bytes(k));
    const size_t need = xbytes + cbytes + pbytes + f16_bytes(p->prec, groups, n);
    if (need > p->ws_bytes) {
        // the old workspace may still be read by work queued on the stream
        HIP_TRY(hipStreamSynchronize(s));
        if (p->ws_d.p) {
            (void)hipFree(p->ws_d.p);
            p->ws_d.p = nullptr;
            p->ws_bytes = 0;
        }
        HIP_TRY(hipMalloc(&p->ws_d.p, need));
        p->ws_bytes = need;
    }
    char *Xst = (char *)p->ws_d.p, *cw = Xst + xbytes;
    double *partial = (double *)(cw + cbytes);
    double *shift = (double *)p->shift_d.p, *bmean = (double *)p->bmean_d.p;
    // the batch's mean; the first batch's mean becomes the shift if none was given
    const double *scale = nullptr;
    if (p->prec == CUM_F16X2) {
        // this batch's own powers of two, bounding its values about the shift
        // (about its mean when that becomes the shift); undone in the
        // contraction, so the window's FP64 sums hold unscaled data
        char *fw = cw + cbytes + pbytes;
        double *mm = (double *)fw, *sc = (double *)(fw + align_up((size_t)groups * n * 2 * 8));
        const double *center = p->have_shift ? shift : nullptr;
        HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_colsum(X, t, n, ldx, rows_per, groups, (double *)cw, s, mm); }));
        HIP_TRY(timed(CUM_KIND_CENTER, s, [&] { return launch_mean((double *)cw, groups, n, t, bmean, s, mm, sc, center); }));
        scale = sc;
    } else if ((st = center_impl(X, t, n, ldx, p->prec, bmean, nullptr, cw, cbytes, s))) {
        return st;
    }
    if (!p->have_shift) {
        HIP_TRY(hipMemcpyAsync(shift, bmean, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
        p->have_shift = true;
    }
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] {
        return launch_stream_sum1((double *)p->s1_d.p, bmean, shift, (double)sign * (double)t, n, s);
    }));
    // the batch's sums of products of x - c, added into (or taken from) the window's
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] {
        return launch_stage(X, t, n, ldx, shift, Xst, p->prec, true, true, s, scale);
    }));
    bool summed;
    double *sums = nullptr;
    if ((st = run_contraction(k, Xst, partial, true, &summed, s, &sums, scale))) return st;
    HIP_TRY(timed(CUM_KIND_REDUCE, s,
                  [&] { return launch_axpy((double *)p->sums_d.p, sums, (double)sign, p->stride, s); }));
    p->t += sign * t;
    p->last = k.c;
    return CUM_OK;
}

cum_status cum_stream_cumulants(cum_stream *p, double *mean, double *const *kappa, void *stream) {
    cum_status st;
    if (!p || !kappa) return fail(CUM_EINVAL, "NULL argument");
    for (int d = 2; d <= p->d_max; ++d)
        if (!kappa[d - 2]) return fail(CUM_EINVAL, "kappa[%d] is NULL", d - 2);
    if (p->t < 1 || !p->last) return fail(CUM_EINVAL, "the window holds no samples");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = (hipStream_t)stream;
    const double tt = (double)p->t;
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] {
        return launch_stream_mean((const double *)p->s1_d.p, (const double *)p->shift_d.p, tt, p->n,
                                  (double *)p->delta_d.p, mean, s);
    }));
    RecArgs ra;
    memset(&ra, 0, sizeof ra);
    ra.sums = (const double *)p->sums_d.p;
    ra.central = (double *)p->central_d.p;
    ra.delta = (const double *)p->delta_d.p;
    for (int d = 2; d <= p->d_max; ++d) ra.off[d] = p->off[d - 2];
    ra.t = tt;
    ra.n = p->n;
    for (int d = 2; d <= p->d_max; ++d) {
        OrderPlan *o;
        if ((st = get_order(p->n, 1, d, &o)) || (st = upload_order(*o))) return st;
        ra.tuples = (const uint8_t *)o->tuples_d.p;
        ra.count = o->nblocks;
        ra.d = d;
        HIP_TRY(timed(CUM_KIND_REDUCE, s, [&] { return launch_recentre(ra, s); }));
    }
    // the central moments are already divided by t
    double *moms[MAXD - 1] = {nullptr};
    if (p->mom_d.p) {
        char *mw = (char *)p->mom_d.p;
        const int64_t nbar = (p->n + p->b - 1) / p->b;
        for (int m = 2; m <= p->d_max - 2; ++m) {
            moms[m - 2] = (double *)mw;
            mw += align_up((size_t)(binom(nbar + m - 1, m) * ipow64(p->b, m)) * 8);
        }
    }
    return run_finalize(p->last, (double *)p->central_d.p, 1, 1, kappa, true, s, p->mom_d.p ? moms : nullptr);
}

// device tables of all_partitions, per order
struct MoebTable {
    int npart = 0;
    DevBuf parts_d, weight_d;
};
static std::map<int, std::unique_ptr<MoebTable>> g_moeb;

static cum_status get_moebius(int d, MoebTable **out) {
    auto it = g_moeb.find(d);
    if (it != g_moeb.end()) {
        *out = it->second.get();
        return CUM_OK;
    }
    std::vector<std::vector<uint16_t>> ap;
    std::vector<double> w;
    all_partitions(d, ap, w);
    std::vector<uint16_t> flat;
    for (const auto &pm : ap)
        for (int k = 0; k < d; ++k) flat.push_back(k < (int)pm.size() ? pm[k] : 0);
    std::unique_ptr<MoebTable> t(new MoebTable);
    t->npart = (int)ap.size();
    cum_status st;
    if ((st = upload(t->parts_d, flat)) || (st = upload(t->weight_d, w))) return st;
    *out = t.get();
    g_moeb[d] = std::move(t);
    return CUM_OK;
}

cum_status cum_stream_cumulants_moebius(cum_stream *p, double *mean, double *const *kappa, void *stream) {
    cum_status st;
    if (!p || !kappa) return fail(CUM_EINVAL, "NULL argument");
    for (int d = 2; d <= p->d_max; ++d)
        if (!kappa[d - 2]) return fail(CUM_EINVAL, "kappa[%d] is NULL", d - 2);
    if (p->t < 1 || !p->last) return fail(CUM_EINVAL, "the window holds no samples");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = (hipStream_t)stream;
    const double tt = (double)p->t;
    HIP_TRY(timed(CUM_KIND_CENTER, s, [&] {
        return launch_stream_mean((const double *)p->s1_d.p, (const double *)p->shift_d.p, tt, p->n,
                                  (double *)p->delta_d.p, mean, s);
    }));
    MoebArgs ma;
    memset(&ma, 0, sizeof ma);
    ma.sums = (const double *)p->sums_d.p;
    ma.out = (double *)p->central_d.p;
    ma.delta = (const double *)p->delta_d.p;
    for (int d = 2; d <= p->d_max; ++d) ma.off[d] = p->off[d - 2];
    ma.t = tt;
    ma.n = p->n;
    for (int d = 2; d <= p->d_max; ++d) {
        OrderPlan *o;
        MoebTable *mt;
        if ((st = get_order(p->n, 1, d, &o)) || (st = upload_order(*o)) || (st = get_moebius(d, &mt))) return st;
        ma.tuples = (const uint8_t *)o->tuples_d.p;
        ma.count = o->nblocks;
        ma.parts = (const uint16_t *)mt->parts_d.p;
        ma.weight = (const double *)mt->weight_d.p;
        ma.npart = mt->npart;
        ma.d = d;
        HIP_TRY(timed(CUM_KIND_REDUCE, s, [&] { return launch_moebius(ma, s); }));
    }
    // expand each tuple's cumulant to every stored copy (t = 1: no division)
    return run_finalize(p->last, (double *)p->central_d.p, 1, 1, kappa, false, s);
}

cum_status cum_stream_count(cum_stream *p, int64_t *t) {
    if (!p || !t) return fail(CUM_EINVAL, "NULL argument");
    *t = p->t;
    return CUM_OK;
}

cum_status cum_stream_reset(cum_stream *p, void *stream) {
    if (!p) return fail(CUM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemsetAsync(p->sums_d.p, 0, (size_t)std::max<int64_t>(p->stride, 1) * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(p->s1_d.p, 0, (size_t)p->n * sizeof(double), s));
    p->t = 0;
    return CUM_OK;
}

cum_status cum_stream_destroy(cum_stream *p) {
    if (p && p->ws_d.p) (void)hipDeviceSynchronize();
    delete p;
    return CUM_OK;
}


}  // extern "C"
