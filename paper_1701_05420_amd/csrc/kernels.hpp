// Launch interface between the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace cum {

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16X2 = 2, P_BF16X3 = 3, P_F16X2 = 4 };

struct MomentArgs {
    const OrderDev *ords;
    const TileDev *tiles;
    const Item *items;
    int64_t nitems;
    const SetDev *sets;  // per-dataset records, or null: every item uses set0
    SetDev set0;
    int32_t n;           // variables; staged row n holds zeros
    int32_t pad;
    double *raw;         // or null: each chunk's sums in tile order (see launch_rawsum)
    int64_t rawstride;   // doubles per chunk in raw
    const double *scale; // FP16 split: the power of two each staged row was divided by
                         // (n + 1 entries, the zero row's 1), else null
};

struct RedArgs {
    const RedOrder *ords;  // the orders finalised by this launch (1 or 2: orders d0 and d0 + 1)
    int32_t nords;
    int32_t d0;         // order of ords[0]
    int32_t recursion;  // 0: plain moments (no cumulant recursion)
    int32_t presummed;  // 1: chunk 0 of the partial sums already holds their sum
    int32_t base_off;   // dynamic LDS layout: staged sub-blocks at 0, the block's
    int32_t parts_off;  // lower-order offsets at base_off, the partition table at
    int32_t parts_lds;  // parts_off when parts_lds (else it is read from memory)
    int32_t subset;     // 1: orders >= 7 use the first-position formula (the sets hold the
                        // central moments of every order they need)
    int32_t b;          // block size (a block of order d holds b^d entries)
    int32_t sl0, sl1;   // work-groups per block of each order (set by the launch)
    int32_t q0, q1;     // entries per lane of each order: b^qe where the first-position
                        // formula runs in its multi-entry form, else 1
    int32_t gstaged;    // bit i: order d0 + i has its sub-blocks staged in LDS
    int32_t pad;
    int64_t nb0;   // blocks of the first order
    int64_t nbtot; // blocks of all orders of the launch
    const SetRed *sets;  // per-dataset records (grid.y), or null: set0
    SetRed set0;
};

// Re-centring of one order: raw moment sums of shifted data (each sorted
// variable tuple once) to central moments.
struct RecArgs {
    const double *sums;      // sums of products of shifted data, order m at off[m]
    double *central;         // central moments (already divided by t), same layout
    const double *delta;     // n: mean of the shifted data
    const uint8_t *tuples;   // count x d sorted variable tuples of order d
    int64_t off[MAXD + 1];   // layout offset of order m (m = 2..d)
    int64_t count;           // tuples of order d
    double t;                // samples (moments are sums / t)
    int32_t n, d;
};

// Cumulants of one order directly from the moments of shifted data by the
// Moebius-weighted sum over all set partitions of the positions.
struct MoebArgs {
    const double *sums;      // sums of products of shifted data, order m at off[m]
    double *out;             // cumulants of order d, each sorted tuple once, at off[d]
    const double *delta;     // n: mean of the shifted data (the order-1 moment)
    const uint8_t *tuples;   // count x d sorted variable tuples of order d
    const uint16_t *parts;   // npart x d position masks (0 = no more parts)
    const double *weight;    // npart: (k-1)! (-1)^(k-1) for a partition of k parts
    int64_t off[MAXD + 1];
    int64_t count;
    double t;
    int32_t n, d, npart, pad;
};

// Wave task shapes: one 32-row block by WN 32-column blocks.
enum TileShape { TS_1x1 = 0, TS_1x2 = 2 };

int lds_bytes_moment(int prec, int n);
// row-major data (FP64 with ldx, or FP32 with ldx) -> staged layout, optionally centred;
// with scale (FP16 split: centred FP64 input, or FP32 input taken as given),
// variable v is divided by scale[v]
hipError_t launch_stage(const void *X, int64_t t, int n, int64_t ldx, const double *mean, void *Xst, int prec,
                        bool center, bool in_f64, hipStream_t s, const double *scale = nullptr);
hipError_t launch_moment(int prec, int shape, int dmax, const MomentArgs &a, int grid, hipStream_t s);
// block_elems: b^d of the launch's first order (it picks the work-group size)
hipError_t launch_reduce(const RedArgs &a, int nsets, int lds_bytes, int block_elems, hipStream_t s);
hipError_t launch_chunksum(const SetRed *sets, const SetRed &set0, int nsets, int64_t entries, hipStream_t s);
// Chunk sums kept in tile order (raw[chunk * rawstride + p], p = position of a
// wave task's accumulator register): add them over chunks, in chunk order,
// and write each stored entry's sum at its block-storage offset in canon.
hipError_t launch_rawsum(const double *raw, int64_t rawstride, int64_t nchunks, const TileDev *tiles,
                         const OrderDev *ords, double *canon, int wn, bool acc64, hipStream_t s);
hipError_t launch_axpy(double *y, const double *x, double a, int64_t count, hipStream_t s);
hipError_t launch_stream_sum1(double *s1, const double *bmean, const double *shift, double tb, int n, hipStream_t s);
hipError_t launch_stream_mean(const double *s1, const double *shift, double t, int n, double *delta, double *mean,
                              hipStream_t s);
hipError_t launch_recentre(const RecArgs &a, hipStream_t s);
hipError_t launch_moebius(const MoebArgs &a, hipStream_t s);
// With mm (groups x n x 2 doubles), the column sums also record each
// group's column minima and maxima; launch_mean then also writes scale
// (n + 1 doubles) for the FP16 split, bounding the values about center
// (n doubles) when given, else about the mean: see mean_body.
hipError_t launch_colsum(const double *X, int64_t t, int n, int64_t ldx, int64_t rows_per, int groups, double *part,
                         hipStream_t s, double *mm = nullptr);
hipError_t launch_mean(const double *part, int groups, int n, int64_t t, double *mean, hipStream_t s,
                       const double *mm = nullptr, double *scale = nullptr, const double *center = nullptr);
// FP16 split of FP32 data taken as given (t x n, ld n): each group's column
// sums (part) and minima / maxima (mm, groups x n x 2 each), then scale
// (n + 1): per variable the power of two bounding its values about zero below
// 32 (see mean_body), and scale[n] = 1.
hipError_t launch_scale_f32(const float *X, int64_t t, int n, int64_t rows_per, int groups, double *part, double *mm,
                            double *scale, hipStream_t s);
hipError_t launch_center(const double *X, int64_t t, int n, int64_t ldx, const double *mean, void *Xc, int prec,
                         hipStream_t s);
hipError_t launch_unfold(const double *blocks, int n, int d, int b, double *dense, hipStream_t s);

// Batched centring: one launch for many datasets (same n).
struct CenterSet {
    const double *X;   // t x n, ld n
    int64_t t;
    double *mean;      // n
    void *Xc;          // staged layout (FP32, or FP64 for the FP64 path)
    double *part;      // groups x n x 2 partial sums
    int32_t groups;
    int32_t pad;
    int64_t rows_per;
    double *mm;        // FP16 split: groups x n x 2 column minima and maxima, else null
    double *scale;     // FP16 split: n + 1 powers of two (see launch_mean), else null
};
hipError_t launch_batch_colsum(const CenterSet *sets, int nsets, int max_groups, int n, hipStream_t s, bool mm = false);
hipError_t launch_batch_mean(const CenterSet *sets, int nsets, int n, hipStream_t s, bool mm = false);
hipError_t launch_batch_stage(const CenterSet *sets, int nsets, int n, int prec, int blocks_per_set, hipStream_t s);
hipError_t launch_batch_stamp(unsigned long long *stamps, int nsets, hipStream_t s);
hipError_t launch_stamp(unsigned long long *where, hipStream_t s);

// Fixed device scratch of the allocation-free entry point
// (CUM_NOALLOC_SCRATCH_BYTES on each of devices 0..NOALLOC_MAX_DEVICES-1).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(void **out);

}  // namespace cum
