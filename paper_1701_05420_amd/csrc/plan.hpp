// Host planner and the device-visible records it builds.
//
// The order-d moment tensor over sorted block tuples (Alg. 1, Alg. 2) is
// evaluated as one contraction per order: a tuple j_1 <= ... <= j_d is cut
// into a prefix (j_1..j_p, p = floor(d/2)) and a suffix (j_{p+1}..j_d).
// Rows enumerate (prefix tuple, in-block digits of the prefix), sorted by the
// prefix's last block v; columns enumerate (suffix tuple, in-block digits of
// the suffix), sorted by the suffix's first block w.  Entry (row, col) is a
// stored moment entry exactly when v <= w, and then
//   S[row, col] = sum_l  prod_{prefix vars} x_l  *  prod_{suffix vars} x_l ,
// a matrix product over samples whose operands are Khatri-Rao products of
// columns of X -- formed on the fly from samples staged in LDS, never stored.
// The lexicographic rank of a sorted tuple splits into a prefix part, a term
// that depends only on (v, w), and a suffix part, so the storage offset of
// (row, col) is row.addr + col.addr + H[v][w].
#pragma once

#include <cstdint>
#include <cstddef>

namespace cum {

constexpr int MAXD = 10;  // largest order
constexpr int MAXH = 5;   // longest prefix / suffix = ceil(MAXD / 2)
constexpr int MAXN = 112; // variables (index n is the zero row of the staged data)
constexpr int FEAT_BLOCK = 32;

// One row (prefix) or column (suffix) of an order's contraction.
struct Feat {
    int64_t addr;          // row: rank part of the prefix * b^d + prefix digits * b^q
                           // col: rank part of the suffix * b^d + suffix digits
    int32_t blk;           // row: last prefix block v (INT32_MAX for padding rows)
                           // col: first suffix block w (-1 for padding columns)
    uint8_t var[MAXH];     // variable of each position (n = the zero column)
    uint8_t pad[3];
};
static_assert(sizeof(Feat) == 24, "Feat layout");

// Everything a kernel needs to know about one order (device pointers).
struct OrderDev {
    const Feat *rows;
    const Feat *cols;
    const int64_t *H;        // nbar x nbar: (v, w) term of the rank, times b^d
    int64_t out_off;         // offset of this order in the per-chunk partial vector
    int64_t elems;           // stored entries of this order
    int32_t d, p, q, nbar, b, nr, nc, pad;
};

// One wave's share of a work item: rows r0..r0+31 by WN column blocks of 32
// starting at c0.  Bit j*4 + h*2 + g of mask: the 16 x 16 sub-block of rows
// r0+16h.. and columns c0+32j+16g.. holds a stored entry (the others are
// skipped).
struct WaveTask {
    int32_t r0;
    int32_t c0;
    int32_t mask;
    int32_t pad;
};

// Waves per work-group of the contraction: they share one staged copy of
// the samples in LDS (one DMA per stage for all of them).
#ifndef CUM_WG_WAVES
#define CUM_WG_WAVES 4
#endif
constexpr int WG_WAVES = CUM_WG_WAVES;

// A work-group tile: up to WG_WAVES wave tasks of one order.
struct TileDev {
    int32_t ord;   // index into the OrderDev array
    int32_t ntask;
    int32_t pad0, pad1;
    WaveTask task[WG_WAVES];
};

// One unit of the moment launch: a tile over one sample chunk of one dataset.
struct Item {
    int32_t tile;  // -1: no-op
    int32_t chunk;
    int32_t set;
    int32_t pad;
};

// Staged layout of the centred data, as the contraction reads it.  Samples
// are cut into stages of KT; stage s holds, for every variable v = 0..n
// (v = n is an all-zero row used by padding positions), the KT samples
// s*KT .. s*KT+KT-1 contiguously, followed by KTP - KT zeros:
//   Xst[(s * (n + 1) + v) * KTP + k],
// samples beyond t are zero.  One stage is one contiguous block of memory.
// The pitch is chosen for the LDS reads of the contraction: lanes in four
// groups of 16 read 16 bytes at (pitch * v + group * VEC) for a handful of
// variables v; a pitch of 16 (mod 32) 32-bit words (FP32, FP64) or 4 (mod 32)
// words (BF16 paths, two reads 32 bytes apart) spreads those reads over
// distinct banks.
constexpr int stage_kt(int prec) { return prec == 0 ? 32 : 64; }
constexpr int stage_pitch(int prec) { return prec == 0 ? 40 : (prec == 1 ? 80 : 68); }
constexpr int stage_esize(int prec) { return prec == 0 ? 8 : 4; }

// Per dataset: the staged centred data and its partial sums.
struct SetDev {
    const void *X;         // staged layout
    int64_t nstages;       // ceil(t / KT)
    int64_t chunk_stages;  // stages per sample chunk
    int64_t nchunks;
    double *partial;       // nchunks x stride
    int64_t stride;        // stored entries of all orders 2..d_max
    const double *scale;   // FP16 split: the powers of two the staged rows were divided by
                           // (n + 1), else null
};

// Reduction / recursion records.
constexpr int MAXPARTS = MAXD / 2;  // parts of size >= 2 in a partition of <= MAXD positions
struct RedOrder {
    const uint8_t *tuples;   // nblocks x d sorted block tuples (lexicographic order)
    const int32_t *parts;    // npart x (d/2) parts, packed mask | where << 10 (0 = no more parts);
                             // where = LDS offset of the staged sub-block (staged orders) or
                             // the index of the part's position set in smask (others)
    const uint16_t *smask;   // ns position sets S of 2..d-2 positions, by size then value
    const int32_t *gmap;     // lds_elems staged slots: s | flat << 10, grouped by |S|
    const int32_t *tpw;      // orders >= 7: nterm x 2 multipliers b^|S & ~(2^h - 1)|, h = ceil(d/2), of the
                             // factors' sets (the in-block index of a set is tlo * that + thi)
    const int32_t *terms;    // orders >= 7: nterm x 2 factors (a set A holding the first position
                             // and its complement C), packed mask | where << 10 like parts
    const int64_t *prank;    // d x (pnbar + 1) rank terms of the partial-sum layout:
                             // prank[k][x] = pb^d * C(pnbar - x + d - k - 1, d - k)
    int64_t nblocks;
    int64_t out_off;         // offset of this order in the per-chunk partial vector
    int32_t d, npart, nbar, b;
    int32_t nterm;           // terms of the first-position formula (orders >= 7), else 0
    int32_t qe;              // orders >= 7: a thread of the gathering finalisation takes b^qe
                             // consecutive entries (its last qe digits), 0: one entry
    int32_t cstart[5];       // orders >= 7: terms grouped by the last qe positions their set A
                             // holds; group c is terms cstart[c] .. cstart[c+1]-1
    int32_t pad2;
    int32_t ns;              // position sets of 2..d-2 positions
    int32_t lds_elems;       // doubles staged per block (0: lower orders read from memory)
    int32_t mstart[MAXD];    // staged slots of sets of size m start at mstart[m - 2]; mstart[d - 3] = lds_elems
    int32_t pb, pnbar;       // block size and blocks per mode of the partial-sum layout
    int32_t n;               // variables
    int32_t pad;
};
// Smallest order whose finalisation can use the first-position form of the
// moment-cumulant relation (when the central moments of lower orders are
// kept); lower orders keep the partition recursion.
constexpr int FIRST_POSITION_MIN_D = 7;
// Smallest order whose contraction sums in FP64 in every precision (the
// FP32-staged ones form FP32 operands and accumulate their products in FP64).
constexpr int HIGH_ACC64_MIN_D = 7;
// Smallest d_max at which a call that centres its own data stages it in FP64
// and runs its whole contraction in FP64, whatever precision was asked for.
constexpr int HIGH_F64_MIN_D = 7;
constexpr int RED_LDS_MAX = 6144;  // doubles of lower-order sub-blocks staged per block (48 KiB)

struct SetRed {
    double *partial;               // nchunks x stride; chunk 0 receives the sums
    int64_t stride;
    int64_t nchunks;
    int64_t t;
    double *kappa[MAXD - 1];       // kappa[d-2]
    double *mom[MAXD - 1];         // central moments of order d in block storage (mom[d-2]), or null:
                                   // written by the finalisation of order d, read as factors by
                                   // the first-position formula of orders d+2 and above
    unsigned long long *stamp;     // finalisation timestamp (or null)
};

}  // namespace cum
