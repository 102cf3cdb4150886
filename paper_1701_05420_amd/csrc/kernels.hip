// gfx950 kernels: centring, block moment contraction on matrix cores,
// fixed-order chunk reduction fused with the cumulant recursion, unfold.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace cum {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
    double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__device__ __forceinline__ int64_t binom_dev(int a, int r) {
    if (r < 0 || a < r) return 0;
    int64_t v = 1;
    for (int i = 1; i <= r; ++i) v = v * (a - r + i) / i;
    return v;
}

// Lexicographic rank of a sorted tuple u[0..m-1] over 0..nbar-1: for each
// position, the number of sorted tuples that agree before it and are smaller
// at it, summed in closed form (hockey-stick identity).
__device__ __forceinline__ int64_t rank_sorted(const int *u, int m, int nbar) {
    int64_t s = 0;
    int prev = 0;
    for (int k = 0; k < m; ++k) {
        s += binom_dev(nbar - prev + m - k - 1, m - k) - binom_dev(nbar - u[k] + m - k - 1, m - k);
        prev = u[k];
    }
    return s;
}

__device__ __forceinline__ int64_t ipow_dev(int b, int e) {
    int64_t r = 1;
    for (int k = 0; k < e; ++k) r *= b;
    return r;
}

// ---------------------------------------------------------------------------
// centring (Def. of the centred variable): FP64 column sums in a fixed order,
// Neumaier-compensated; then x - mean in FP64, stored in the device precision.
// ---------------------------------------------------------------------------
// MM: also each column's minimum and maximum over the group (mm)
template <bool MM = false, typename TI = double>
__device__ __forceinline__ void colsum_body(const TI *X, int64_t t, int n, int64_t ldx, int64_t rows_per, int g,
                                            double *part, double *mm = nullptr) {
    __shared__ double ss[256], cs[256];
    __shared__ double lo_s[MM ? 256 : 1], hi_s[MM ? 256 : 1];
    const int tid = threadIdx.x;
    const int R = 256 / n;
    const int col = tid % n, rl = tid / n;
    double s = 0.0, c = 0.0, lo = INFINITY, hi = -INFINITY;
    const int64_t r0 = (int64_t)g * rows_per;
    const int64_t r1 = min(t, r0 + rows_per);
    if (rl < R) {
        int64_t r = r0 + rl;
        // eight independent loads in flight, added in row order
        for (; r + 7 * R < r1; r += 8 * R) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = (double)X[(r + u * R) * ldx + col];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                neumaier(s, c, x[u]);
                if constexpr (MM) {
                    lo = fmin(lo, x[u]);
                    hi = fmax(hi, x[u]);
                }
            }
        }
        for (; r < r1; r += R) {
            const double x = (double)X[r * ldx + col];
            neumaier(s, c, x);
            if constexpr (MM) {
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
        }
    }
    ss[tid] = s;
    cs[tid] = c;
    if constexpr (MM) {
        lo_s[tid] = lo;
        hi_s[tid] = hi;
    }
    __syncthreads();
    if (tid < n) {
        double S = 0.0, C = 0.0, L = INFINITY, H = -INFINITY;
        for (int k = 0; k < R; ++k) {
            neumaier(S, C, ss[k * n + tid]);
            neumaier(S, C, cs[k * n + tid]);
            if constexpr (MM) {
                L = fmin(L, lo_s[k * n + tid]);
                H = fmax(H, hi_s[k * n + tid]);
            }
        }
        part[((int64_t)g * n + tid) * 2] = S;
        part[((int64_t)g * n + tid) * 2 + 1] = C;
        if constexpr (MM) {
            mm[((int64_t)g * n + tid) * 2] = L;
            mm[((int64_t)g * n + tid) * 2 + 1] = H;
        }
    }
}

template <bool MM>
__global__ __launch_bounds__(256) void colsum_kernel(const double *X, int64_t t, int n, int64_t ldx,
                                                     int64_t rows_per, double *part, double *mm) {
    colsum_body<MM>(X, t, n, ldx, rows_per, blockIdx.x, part, mm);
}

// One work-group per column: thread k sums groups k, k+256, ...; the 256
// compensated partials are then combined pairwise in a fixed tree.
// The FP16 split's power of two for values in [lo, hi] staged about c:
// 2^(e - 5), where a = max |x - c| lies in [2^(e-1), 2^e) (1 where a = 0).
__device__ __forceinline__ double f16_scale(double lo, double hi, double c) {
    const double a = fmax(hi - c, c - lo);
    int e = 0;
    if (a > 0.0) (void)frexp(a, &e);  // a = f * 2^e, f in [0.5, 1): 2^e > a
    return a > 0.0 ? ldexp(1.0, e - 5) : 1.0;
}

// MM (the FP16 split): from the groups' minima and maxima, also the power of
// two scale[i] = 2^(e - 5), where a = max |x - c| over the column lies in
// [2^(e-1), 2^e), c being center[i] if given (the fixed shift a stream stages
// about) and the mean otherwise (scale 1 where a = 0), and scale[n] = 1.
// Divided by it, every staged value is below 32 in magnitude, so a product
// of up to three of them stays below the FP16 maximum (65504).
template <bool MM = false>
__device__ __forceinline__ void mean_body(const double *part, int groups, int n, int64_t t, double *mean, int i,
                                          const double *mm = nullptr, double *scale = nullptr,
                                          const double *center = nullptr) {
    __shared__ double ss[256], cs[256];
    __shared__ double lo_s[MM ? 256 : 1], hi_s[MM ? 256 : 1];
    const int tid = threadIdx.x;
    double S = 0.0, C = 0.0, L = INFINITY, H = -INFINITY;
    for (int g = tid; g < groups; g += 256) {
        neumaier(S, C, part[((int64_t)g * n + i) * 2]);
        neumaier(S, C, part[((int64_t)g * n + i) * 2 + 1]);
        if constexpr (MM) {
            L = fmin(L, mm[((int64_t)g * n + i) * 2]);
            H = fmax(H, mm[((int64_t)g * n + i) * 2 + 1]);
        }
    }
    ss[tid] = S;
    cs[tid] = C;
    if constexpr (MM) {
        lo_s[tid] = L;
        hi_s[tid] = H;
    }
    for (int w = 128; w > 0; w >>= 1) {
        __syncthreads();
        if (tid < w) {
            double S2 = ss[tid], C2 = cs[tid];
            neumaier(S2, C2, ss[tid + w]);
            neumaier(S2, C2, cs[tid + w]);
            ss[tid] = S2;
            cs[tid] = C2;
            if constexpr (MM) {
                lo_s[tid] = fmin(lo_s[tid], lo_s[tid + w]);
                hi_s[tid] = fmax(hi_s[tid], hi_s[tid + w]);
            }
        }
    }
    if (tid == 0) {
        const double mu = (ss[0] + cs[0]) / (double)t;
        mean[i] = mu;
        if constexpr (MM) {
            // the values are staged about center (a stream's fixed shift) when given
            scale[i] = f16_scale(lo_s[0], hi_s[0], center ? center[i] : mu);
            if (i == 0) scale[n] = 1.0;
        }
    }
}

// The FP16 split of FP32 data taken as given (cum_moment_blocks): each
// group's column sums (unused) and minima / maxima, then per column the
// power of two bounding the values about zero.
__global__ __launch_bounds__(256) void colminmax_f32_kernel(const float *X, int64_t t, int n, int64_t rows_per,
                                                            double *part, double *mm) {
    colsum_body<true, float>(X, t, n, n, rows_per, blockIdx.x, part, mm);
}

__global__ __launch_bounds__(256) void scale_about_zero_kernel(const double *mm, int groups, int n, double *scale) {
    __shared__ double lo_s[256], hi_s[256];
    const int tid = threadIdx.x, i = blockIdx.x;
    double L = INFINITY, H = -INFINITY;
    for (int g = tid; g < groups; g += 256) {
        L = fmin(L, mm[((int64_t)g * n + i) * 2]);
        H = fmax(H, mm[((int64_t)g * n + i) * 2 + 1]);
    }
    lo_s[tid] = L;
    hi_s[tid] = H;
    for (int w = 128; w > 0; w >>= 1) {
        __syncthreads();
        if (tid < w) {
            lo_s[tid] = fmin(lo_s[tid], lo_s[tid + w]);
            hi_s[tid] = fmax(hi_s[tid], hi_s[tid + w]);
        }
    }
    if (tid == 0) {
        scale[i] = f16_scale(lo_s[0], hi_s[0], 0.0);
        if (i == 0) scale[n] = 1.0;
    }
}

template <bool MM>
__global__ __launch_bounds__(256) void mean_kernel(const double *part, int groups, int n, int64_t t,
                                                   double *mean, const double *mm, double *scale,
                                                   const double *center) {
    mean_body<MM>(part, groups, n, t, mean, blockIdx.x, mm, scale, center);
}

template <typename T>
__global__ __launch_bounds__(256) void center_kernel(const double *X, int64_t t, int n, int64_t ldx,
                                                     const double *mean, T *Xc) {
    const int64_t total = t * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t l = e / n;
        const int i = (int)(e - l * n);
        Xc[e] = (T)(X[l * ldx + i] - mean[i]);
    }
}

template <bool MM>
__global__ __launch_bounds__(256) void batch_colsum_kernel(const CenterSet *sets, int n) {
    const CenterSet cs = sets[blockIdx.y];
    if ((int)blockIdx.x >= cs.groups) return;
    colsum_body<MM>(cs.X, cs.t, n, n, cs.rows_per, blockIdx.x, cs.part, cs.mm);
}

template <bool MM>
__global__ __launch_bounds__(256) void batch_mean_kernel(const CenterSet *sets, int n) {
    const CenterSet cs = sets[blockIdx.y];
    mean_body<MM>(cs.part, cs.groups, n, cs.t, cs.mean, blockIdx.x, cs.mm, cs.scale);
}

__global__ void stamp_kernel(unsigned long long *where) {
    if (threadIdx.x == 0) *where = wall_clock64();
}

// ---------------------------------------------------------------------------
// Staged layout writers: row-major data -> the staged layout of plan.hpp.
// One work-group per stage; variables are moved through LDS in groups of 32
// so that both the row-major reads and the stage writes are contiguous.
// ---------------------------------------------------------------------------
template <typename TI, typename TO, bool CENTER, bool SCALED = false>
__device__ __forceinline__ void stage_body(const TI *X, int64_t t, int n, int64_t ldx, const double *mean, TO *Xst,
                                           int KT, int KTP, int64_t s, const double *scale = nullptr) {
    __shared__ double tile[64][33];
    const int tid = threadIdx.x;
    const int64_t l0 = s * KT;
    TO *dst = Xst + s * (int64_t)(n + 1) * KTP;
    for (int v0 = 0; v0 <= n; v0 += 32) {
        __syncthreads();
        for (int e = tid; e < KT * 32; e += 256) {
            const int k = e >> 5, v = v0 + (e & 31);
            double x = 0.0;
            if (v < n && l0 + k < t) {
                x = (double)X[(l0 + k) * ldx + v];
                if (CENTER) x -= mean[v];
                if constexpr (SCALED) x /= scale[v];  // a power of two: exact
            }
            tile[k][e & 31] = x;
        }
        __syncthreads();
        const int nv = min(32, n + 1 - v0);
        for (int e = tid; e < nv * KTP; e += 256) {
            const int vv = e / KTP, k = e - vv * KTP;
            dst[(int64_t)(v0 + vv) * KTP + k] = (k < KT) ? (TO)tile[k][vv] : TO(0);
        }
    }
}

template <typename TI, typename TO, bool CENTER>
__global__ __launch_bounds__(256) void stage_kernel(const TI *X, int64_t t, int n, int64_t ldx, const double *mean,
                                                    TO *Xst, int KT, int KTP, int64_t nstages) {
    for (int64_t s = blockIdx.x; s < nstages; s += gridDim.x) stage_body<TI, TO, CENTER>(X, t, n, ldx, mean, Xst, KT, KTP, s);
}

// centred FP64 data divided by per-variable powers of two, to FP32 (FP16 split)
__global__ __launch_bounds__(256) void stage_scaled_kernel(const double *X, int64_t t, int n, int64_t ldx,
                                                           const double *mean, const double *scale, float *Xst,
                                                           int KT, int KTP, int64_t nstages) {
    for (int64_t s = blockIdx.x; s < nstages; s += gridDim.x)
        stage_body<double, float, true, true>(X, t, n, ldx, mean, Xst, KT, KTP, s, scale);
}

// FP32 data taken as given, divided by per-variable powers of two (FP16 split)
__global__ __launch_bounds__(256) void stage_scaled_f32_kernel(const float *X, int64_t t, int n, int64_t ldx,
                                                               const double *scale, float *Xst, int KT, int KTP,
                                                               int64_t nstages) {
    for (int64_t s = blockIdx.x; s < nstages; s += gridDim.x)
        stage_body<float, float, false, true>(X, t, n, ldx, nullptr, Xst, KT, KTP, s, scale);
}

hipError_t launch_stage(const void *X, int64_t t, int n, int64_t ldx, const double *mean, void *Xst, int prec,
                        bool center, bool in_f64, hipStream_t s, const double *scale) {
    const int KT = stage_kt(prec), KTP = stage_pitch(prec);
    const int64_t nst = (t + KT - 1) / KT;
    const unsigned grid = (unsigned)std::min<int64_t>(nst, 65535);
    if (scale && !center && !in_f64 && prec != P_F64) {
        hipLaunchKernelGGL(stage_scaled_f32_kernel, dim3(grid), dim3(256), 0, s, (const float *)X, t, n, ldx, scale,
                           (float *)Xst, KT, KTP, nst);
        return hipGetLastError();
    }
    if (scale) {
        if (!center || !in_f64 || prec == P_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL(stage_scaled_kernel, dim3(grid), dim3(256), 0, s, (const double *)X, t, n, ldx, mean, scale,
                           (float *)Xst, KT, KTP, nst);
        return hipGetLastError();
    }
    if (center) {
        if (prec == P_F64)
            hipLaunchKernelGGL((stage_kernel<double, double, true>), dim3(grid), dim3(256), 0, s, (const double *)X, t,
                               n, ldx, mean, (double *)Xst, KT, KTP, nst);
        else
            hipLaunchKernelGGL((stage_kernel<double, float, true>), dim3(grid), dim3(256), 0, s, (const double *)X, t,
                               n, ldx, mean, (float *)Xst, KT, KTP, nst);
    } else {
        if (prec == P_F64)
            hipLaunchKernelGGL((stage_kernel<double, double, false>), dim3(grid), dim3(256), 0, s, (const double *)X,
                               t, n, ldx, nullptr, (double *)Xst, KT, KTP, nst);
        else if (in_f64)
            hipLaunchKernelGGL((stage_kernel<double, float, false>), dim3(grid), dim3(256), 0, s, (const double *)X,
                               t, n, ldx, nullptr, (float *)Xst, KT, KTP, nst);
        else
            hipLaunchKernelGGL((stage_kernel<float, float, false>), dim3(grid), dim3(256), 0, s, (const float *)X, t,
                               n, ldx, nullptr, (float *)Xst, KT, KTP, nst);
    }
    return hipGetLastError();
}

// Batched: grid (blocks per dataset, datasets); each block walks its
// dataset's stages with stride gridDim.x.
template <typename TO, bool SCALED = false>
__global__ __launch_bounds__(256) void batch_stage_kernel(const CenterSet *sets, int n, int KT, int KTP) {
    const CenterSet cs = sets[blockIdx.y];
    const int64_t nst = (cs.t + KT - 1) / KT;
    for (int64_t st = blockIdx.x; st < nst; st += gridDim.x)
        stage_body<double, TO, true, SCALED>(cs.X, cs.t, n, n, cs.mean, reinterpret_cast<TO *>(cs.Xc), KT, KTP, st,
                                             cs.scale);
}

hipError_t launch_batch_stage(const CenterSet *sets, int nsets, int n, int prec, int blocks_per_set, hipStream_t s) {
    const int KT = stage_kt(prec), KTP = stage_pitch(prec);
    if (prec == P_F16X2)
        hipLaunchKernelGGL((batch_stage_kernel<float, true>), dim3(blocks_per_set, nsets), dim3(256), 0, s, sets, n, KT,
                           KTP);
    else if (prec == P_F64)
        hipLaunchKernelGGL(batch_stage_kernel<double>, dim3(blocks_per_set, nsets), dim3(256), 0, s, sets, n, KT, KTP);
    else
        hipLaunchKernelGGL(batch_stage_kernel<float>, dim3(blocks_per_set, nsets), dim3(256), 0, s, sets, n, KT, KTP);
    return hipGetLastError();
}

// Zero the per-dataset finalisation stamps and record the start time.
__global__ void batch_stamp_kernel(unsigned long long *stamps, int nsets) {
    for (int i = threadIdx.x; i < nsets; i += blockDim.x) stamps[1 + i] = 0ull;
    if (threadIdx.x == 0) stamps[0] = wall_clock64();
}

hipError_t launch_batch_stamp(unsigned long long *stamps, int nsets, hipStream_t s) {
    hipLaunchKernelGGL(batch_stamp_kernel, dim3(1), dim3(256), 0, s, stamps, nsets);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block moment contraction.
//
// A work item is one work-group of WG_WAVES wave tasks (each a 32-row block by
// WN 32-column blocks of one order's (prefix rows) x (suffix columns)
// product, packed on the host so that no wave is idle) over one chunk of
// stages of one dataset.  Each stage is copied from HBM to
// LDS by the DMA path (global_load_lds, 16 bytes per lane, no registers),
// double-buffered.  Every lane forms its Khatri-Rao operand values from the
// staged samples -- the product of the prefix (or suffix) variables of its
// row (or column) -- reading VEC consecutive samples per variable with one
// 16-byte LDS read.  The sample order inside a stage is a free choice of the
// sum, so lane group g of an MFMA takes samples g*VEC .. g*VEC+VEC-1 of each
// group of steps.  16 x 16 sub-blocks with no stored entry (v > w everywhere)
// are skipped per wave, as the task's mask (built on the host) says.  The
// chunk's sums go, in FP64, to the chunk's slice of the partial buffer, at
// each entry's offset in the block storage of the inner block size.
// ---------------------------------------------------------------------------
template <int PREC>
struct PT;
template <>
struct PT<P_F64> {
    typedef double T;
    enum { KT = 32, KTP = 40 };
};
template <>
struct PT<P_F32> {
    typedef float T;
    enum { KT = 64, KTP = 80 };
};
template <>
struct PT<P_BF16X2> {
    typedef float T;
    enum { KT = 64, KTP = 68 };
};
template <>
struct PT<P_BF16X3> {
    typedef float T;
    enum { KT = 64, KTP = 68 };
};
template <>
struct PT<P_F16X2> {
    typedef float T;
    enum { KT = 64, KTP = 68 };
};

int lds_bytes_moment(int prec, int n) { return 2 * (n + 1) * stage_pitch(prec) * stage_esize(prec); }
static_assert(PT<P_F64>::KTP == stage_pitch(P_F64) && PT<P_F32>::KTP == stage_pitch(P_F32) &&
                  PT<P_BF16X2>::KTP == stage_pitch(P_BF16X2) && PT<P_F64>::KT == stage_kt(P_F64) &&
                  PT<P_F32>::KT == stage_kt(P_F32) && PT<P_BF16X2>::KT == stage_kt(P_BF16X2) &&
                  PT<P_F16X2>::KTP == stage_pitch(P_F16X2) && PT<P_F16X2>::KT == stage_kt(P_F16X2),
              "stage constants");

typedef __attribute__((address_space(3))) void lds_void;

// Copy one stage (bytes, a multiple of 16) from global to LDS with the DMA
// path: each wave moves 1 KiB per instruction, lane l its 16-byte piece.
__device__ __forceinline__ void stage_dma(const char *src, char *lds, int bytes, int wave, int lane) {
    for (int c = wave * 1024; c < bytes; c += WG_WAVES * 1024) {
        const int off = c + lane * 16;
        if (off < bytes)
            __builtin_amdgcn_global_load_lds((const void *)(src + off), (lds_void *)(lds + c), 16, 0, 0);
    }
}

__device__ __forceinline__ void wait_dma() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// The BF16 splits of eight FP32 values, two at a time: each rounding to
// nearest even converts a pair with one packed conversion.
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf2 to_bf2(f2 x) { return __builtin_convertvector(x, bf2); }
__device__ __forceinline__ f2 to_f2(bf2 x) { return __builtin_convertvector(x, f2); }

// Two terms: hi, and lo = x - hi rounded (the compiler may form x - hi from
// the unrounded product with one fused multiply-add, which only helps lo).
// FP16 split of eight FP32 values: hi = fp16(v) (nearest even) and
// lo = fp16((v - hi) * 2^11).  v - hi is exact in FP32 and 2^11 times it is
// of the order of v, so lo keeps FP16's full 11 bits where (v - hi) itself
// would fall into FP16's subnormal range; hi + lo / 2^11 carries 22 bits of v.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_f16(const float *v, h8 &hi, h8 &lo) {
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        const f2 x = {v[k], v[k + 1]};
        const h2 h = __builtin_convertvector(x, h2);
        const f2 r = (x - __builtin_convertvector(h, f2)) * 2048.f;
        const h2 l = __builtin_convertvector(r, h2);
        hi[k] = h[0];
        hi[k + 1] = h[1];
        lo[k] = l[0];
        lo[k + 1] = l[1];
    }
}

__device__ __forceinline__ void split2(const float *v, bf8 &hi, bf8 &lo) {
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        const f2 x = {v[k], v[k + 1]};
        const bf2 h = to_bf2(x);
        const bf2 l = to_bf2(x - to_f2(h));
        hi[k] = h[0];
        hi[k + 1] = h[1];
        lo[k] = l[0];
        lo[k + 1] = l[1];
    }
}

// Two FP32 values whose low 16 bits are zero (exact in BF16), packed by
// moving bits: no conversion instruction.
__device__ __forceinline__ bf2 pack_exact(f2 x) {
    // (the whole vector is cast: a cast of one element reads element 0)
    const u2 u = __builtin_bit_cast(u2, x);
    return __builtin_bit_cast(bf2, (u[0] >> 16) | (u[1] & 0xffff0000u));
}

// The third term: x - hi is a multiple of x's FP32 ulp no larger than half a
// BF16 ulp of x, so it holds at most 16 significant bits; less its own
// rounding to BF16 (mid) at most 8 remain, and the FP32 value is exact in
// BF16 (below the FP32 normal range, packing truncates where a conversion
// would round, a difference under 2^-133).  This needs x to be the FP32
// value of the product: contraction is off here, so that x - hi is not
// fused with the multiplication into a residual of the exact product.
__device__ __forceinline__ void split3(const float *v, bf8 &hi, bf8 &mid, bf8 &lo) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        const f2 x = {v[k], v[k + 1]};
        const bf2 h = to_bf2(x);
        const f2 r = x - to_f2(h);
        const bf2 m = to_bf2(r);
        const bf2 l = pack_exact(r - to_f2(m));
        hi[k] = h[0];
        hi[k + 1] = h[1];
        mid[k] = m[0];
        mid[k + 1] = m[1];
        lo[k] = l[0];
        lo[k + 1] = l[1];
    }
}

typedef double d2 __attribute__((ext_vector_type(2)));

template <int PREC, int WN, int P, int Q>
__device__ __forceinline__ void moment_item(const Item &item, const TileDev *tile, const OrderDev &od,
                                            const SetDev &sd, char *lds, int n, int wave, double *raw,
                                            int64_t rawstride, const double *scale) {
    typedef typename PT<PREC>::T T;
    constexpr int KT = PT<PREC>::KT, KTP = PT<PREC>::KTP;
    // Orders of HIGH_ACC64_MIN_D and above in the FP32-staged precisions: the
    // operands are FP32 products of the staged samples as in the FP32 path,
    // but each product of two operands is summed in FP64 on the matrix unit
    // (exact product, FP64 accumulation).  At these orders the moments of
    // heavy-tailed data are carried by a few extreme samples whose products
    // nearly cancel, and an FP32 sum over a stage loses the digits the
    // cumulant keeps.
    constexpr bool HI = PREC != P_F64 && P + Q >= HIGH_ACC64_MIN_D;
    constexpr bool ACC64 = PREC == P_F64 || HI;  // FP64 accumulators (FP64 16x16 output layout)
    constexpr bool BF = PREC >= P_BF16X2 && !HI;
    constexpr bool F16 = PREC == P_F16X2 && !HI;     // FP16 hi and scaled lo (split_f16)
    constexpr int NS = (PREC == P_BF16X3) ? 3 : 2;  // split terms (BF16 and FP16 paths)
    // samples per step group: lane group g (= lane / 16) holds VEC consecutive samples
    constexpr int VEC = (PREC == P_F64) ? 2 : (PREC == P_F32 || HI ? 4 : 8);
    constexpr int STEP = 4 * VEC;
    const int tid = threadIdx.x, lane = tid & 63;
    const int stage_bytes = (n + 1) * KTP * (int)sizeof(T);
    const bool active = wave < tile->ntask;
    const WaveTask wt = tile->task[active ? wave : 0];
    const int rbase = wt.r0, cbase = wt.c0;
    const int soff = VEC * (lane >> 4);

    // which 16 x 16 sub-blocks of this wave's 32 x (32*WN) task hold stored
    // entries: bit (j*4 + h*2 + g).  The mask is the same in every lane; say
    // so, so that the per-sub-block tests below are scalar branches and not
    // exec-mask regions
    const unsigned vmask = __builtin_amdgcn_readfirstlane(active ? (unsigned)wt.mask : 0u);

    // LDS offsets (in T) of this lane's operand variables, plus its sample offset
    int roff[2][P], coff[WN][2][Q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const Feat f = od.rows[rbase + 16 * h + (lane & 15)];
#pragma unroll
        for (int q = 0; q < P; ++q) roff[h][q] = f.var[q] * KTP + soff;
    }
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            Feat f;
            const int c = cbase + 32 * j + 16 * g + (lane & 15);
            if (c < od.nc)
                f = od.cols[c];
            else
                for (int q = 0; q < MAXH; ++q) f.var[q] = (uint8_t)n;
#pragma unroll
            for (int q = 0; q < Q; ++q) coff[j][g][q] = f.var[q] * KTP + soff;
        }

    d4 acc64[WN][2][2];
    f4 acc[WN][2][2], acc2[WN][2][2];
    double dacc[WN][2][2][4];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    acc64[j][h][g][k] = 0.0;
                    acc[j][h][g][k] = 0.f;
                    acc2[j][h][g][k] = 0.f;
                    dacc[j][h][g][k] = 0.0;
                }

    const int64_t st0 = (int64_t)item.chunk * sd.chunk_stages;
    const int nst = (int)(min(sd.nstages, st0 + sd.chunk_stages) - st0);
    const char *src = reinterpret_cast<const char *>(sd.X) + st0 * (int64_t)stage_bytes;

    // the first stage's copy was issued before the tile's records were read
    wait_dma();
    __syncthreads();

    for (int k = 0; k < nst; ++k) {
        const T *xb = reinterpret_cast<const T *>(lds + (k & 1) * stage_bytes);
        if (k + 1 < nst)
            stage_dma(src + (int64_t)(k + 1) * stage_bytes, lds + ((k + 1) & 1) * stage_bytes, stage_bytes, wave,
                      lane);
        // one stage of products; `all` (a compile-time flag) drops the per-sub-block
        // tests when every sub-block of the task holds stored entries
        auto stage = [&](auto all_t) {
            constexpr bool all = decltype(all_t)::value;
#pragma unroll
            for (int kk = 0; kk < KT; kk += STEP) {
                if constexpr (!BF) {
                    typedef typename std::conditional<PREC == P_F64, d2, f4>::type V;
                    // every factor of the step is read before any is used, so the
                    // reads are in flight together
                    V fa[2][P], fb[WN][2][Q];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int q = 0; q < P; ++q) fa[h][q] = *reinterpret_cast<const V *>(xb + roff[h][q] + kk);
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int g = 0; g < 2; ++g)
#pragma unroll
                            for (int q = 0; q < Q; ++q)
                                fb[j][g][q] = *reinterpret_cast<const V *>(xb + coff[j][g][q] + kk);
                    V A[2], B[WN][2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        V v = fa[h][0];
#pragma unroll
                        for (int q = 1; q < P; ++q) v *= fa[h][q];
                        A[h] = v;
                    }
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int g = 0; g < 2; ++g) {
                            V v = fb[j][g][0];
#pragma unroll
                            for (int q = 1; q < Q; ++q) v *= fb[j][g][q];
                            B[j][g] = v;
                        }
                    // each accumulator's products of the step back to back (the
                    // scheduling barrier keeps the compiler from interleaving them)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int g = 0; g < 2; ++g) {
                                if (all || (vmask >> (j * 4 + h * 2 + g) & 1u)) {
#pragma unroll
                                    for (int u = 0; u < VEC; ++u) {
                                        if constexpr (ACC64)
                                            acc64[j][h][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                                (double)A[h][u], (double)B[j][g][u], acc64[j][h][g], 0, 0, 0);
                                        else
                                            acc[j][h][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                                A[h][u], B[j][g][u], acc[j][h][g], 0, 0, 0);
                                    }
                                }
                                __builtin_amdgcn_sched_barrier(0);
                            }
                } else {
                    bf8 As[2][NS], Bs[WN][2][NS];
                    h8 Ah[2][2], Bh[WN][2][2];  // FP16 split: hi, 2^11-scaled lo
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        f4 v0 = *reinterpret_cast<const f4 *>(xb + roff[h][0] + kk);
                        f4 v1 = *reinterpret_cast<const f4 *>(xb + roff[h][0] + kk + 4);
#pragma unroll
                        for (int q = 1; q < P; ++q) {
                            v0 *= *reinterpret_cast<const f4 *>(xb + roff[h][q] + kk);
                            v1 *= *reinterpret_cast<const f4 *>(xb + roff[h][q] + kk + 4);
                        }
                        float v[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
                        if constexpr (F16)
                            split_f16(v, Ah[h][0], Ah[h][1]);
                        else if constexpr (NS == 3)
                            split3(v, As[h][0], As[h][1], As[h][2]);
                        else
                            split2(v, As[h][0], As[h][1]);
                    }
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int g = 0; g < 2; ++g) {
                            f4 v0 = *reinterpret_cast<const f4 *>(xb + coff[j][g][0] + kk);
                            f4 v1 = *reinterpret_cast<const f4 *>(xb + coff[j][g][0] + kk + 4);
#pragma unroll
                            for (int q = 1; q < Q; ++q) {
                                v0 *= *reinterpret_cast<const f4 *>(xb + coff[j][g][q] + kk);
                                v1 *= *reinterpret_cast<const f4 *>(xb + coff[j][g][q] + kk + 4);
                            }
                            float v[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
                            if constexpr (F16)
                                split_f16(v, Bh[j][g][0], Bh[j][g][1]);
                            else if constexpr (NS == 3)
                                split3(v, Bs[j][g][0], Bs[j][g][1], Bs[j][g][2]);
                            else
                                split2(v, Bs[j][g][0], Bs[j][g][1]);
                        }
                    // FP16 split: hh in acc; hl and lh (each 2^11 times its weight) in
                    // acc2; ll (weight 2^-22) is left out
                    if constexpr (F16) {
#pragma unroll
                        for (int pr = 2; pr >= 0; --pr)
#pragma unroll
                            for (int j = 0; j < WN; ++j)
#pragma unroll
                                for (int h = 0; h < 2; ++h)
#pragma unroll
                                    for (int g = 0; g < 2; ++g)
                                        if (all || (vmask >> (j * 4 + h * 2 + g) & 1u)) {
                                            if (pr == 0)
                                                acc[j][h][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                                    Ah[h][0], Bh[j][g][0], acc[j][h][g], 0, 0, 0);
                                            else
                                                acc2[j][h][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                                    Ah[h][pr == 1 ? 0 : 1], Bh[j][g][pr == 1 ? 1 : 0],
                                                    acc2[j][h][g], 0, 0, 0);
                                        }
                    } else {
                    // cross products of the split terms: all 4 for two terms; for three
                    // terms the 6 of combined weight >= 2^-16 (hh, hm, mh, hl, lh, mm),
                    // hh in its own accumulator so that the five small products do not
                    // add roundings at the full magnitude; smallest first
                    constexpr int NP = (NS == 3) ? 6 : 4;
                    constexpr int PA[4] = {0, 0, 1, 1};        // hh, hl, lh, ll
                    constexpr int PB[4] = {0, 1, 0, 1};
                    constexpr int PA3[6] = {0, 0, 1, 0, 2, 1};  // hh, hm, mh, hl, lh, mm
                    constexpr int PB3[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
                    for (int pr = NP - 1; pr >= 0; --pr)
#pragma unroll
                        for (int j = 0; j < WN; ++j)
#pragma unroll
                            for (int h = 0; h < 2; ++h)
#pragma unroll
                                for (int g = 0; g < 2; ++g)
                                    if (all || (vmask >> (j * 4 + h * 2 + g) & 1u)) {
                                        const int ia = (NS == 3) ? PA3[pr] : PA[pr & 3];
                                        const int ib = (NS == 3) ? PB3[pr] : PB[pr & 3];
                                        if (NS == 3 && pr > 0)
                                            acc2[j][h][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                                As[h][ia], Bs[j][g][ib], acc2[j][h][g], 0, 0, 0);
                                        else
                                            acc[j][h][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                                As[h][ia], Bs[j][g][ib], acc[j][h][g], 0, 0, 0);
                                    }
                    }
                }
            }
                };
        // The three-term BF16 path is bound by its operand arithmetic, not by
        // the matrix unit, and runs one branch-free copy (computing, and then
        // not storing, the sub-blocks without stored entries) to keep its
        // registers down; the others have a test-free copy for full tasks and
        // a tested one for tasks on the edge of the stored region.
        if constexpr (PREC == P_BF16X3 && !HI) {
            if (vmask) stage(std::true_type());
        } else {
            if (vmask == (1u << (4 * WN)) - 1u)
                stage(std::true_type());
            else if (vmask)
                stage(std::false_type());
        }
        wait_dma();
        __syncthreads();
        if constexpr (!ACC64) {
            // Carry the FP32 sums into FP64.  The leading products of the FP32
            // and three-term paths are carried after every stage.  The
            // three-term path's small products (2^-8 of the leading ones and
            // smaller) and the two-term path's sums, whose error is set by its
            // 16-bit operands, are carried every fourth stage: their FP32
            // roundings stay far below the path's own error, and the
            // conversions saved are a sizeable part of the vector work.
            const bool fourth = (k & 3) == 3 || k + 1 == nst;
            if (PREC != P_BF16X2 || fourth) {
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int g = 0; g < 2; ++g)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                dacc[j][h][g][q] += (double)acc[j][h][g][q];
                                acc[j][h][g][q] = 0.f;
                            }
            }
            if ((PREC == P_BF16X3 || PREC == P_F16X2) && fourth) {
                // the FP16 split's hl + lh sums carry the factor 2^11 of its lo terms
                constexpr double w2 = PREC == P_F16X2 ? 0x1p-11 : 1.0;
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int g = 0; g < 2; ++g)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                dacc[j][h][g][q] += (double)acc2[j][h][g][q] * w2;
                                acc2[j][h][g][q] = 0.f;
                            }
            }
        }
    }

    if constexpr (F16) {
        // undo the staging's per-variable powers of two (exact): each sum of
        // products of row and column operands times the scales of their variables
        if (!scale) scale = sd.scale;  // batches: each dataset's own
        double cs[WN][2], rs[2][4];
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int c = cbase + 32 * j + 16 * g + (lane & 15);
                double v = 1.0;
                if (c < od.nc) {
                    const Feat fc = od.cols[c];
#pragma unroll
                    for (int q = 0; q < Q; ++q) v *= scale[fc.var[q]];
                }
                cs[j][g] = v;
            }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const Feat fr = od.rows[rbase + 16 * h + 4 * (lane >> 4) + q];
                double v = 1.0;
#pragma unroll
                for (int p = 0; p < P; ++p) v *= scale[fr.var[p]];
                rs[h][q] = v;
            }
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int g = 0; g < 2; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) dacc[j][h][g][q] *= rs[h][q] * cs[j][g];
    }
    if (raw) {
        // this chunk's sums in tile order: wave task (item.tile, wave), then
        // (j, g, h) sub-block, register q, lane; 64 consecutive doubles per store
        double *rb = raw + (int64_t)item.chunk * rawstride + ((int64_t)item.tile * WG_WAVES + wave) * (WN * 1024) + lane;
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (!(vmask >> (j * 4 + h * 2 + g) & 1u)) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        rb[((j * 2 + g) * 2 + h) * 256 + q * 64] = ACC64 ? acc64[j][h][g][q] : dacc[j][h][g][q];
                }
        return;
    }
    // epilogue: write this chunk's sums at their block-storage offsets
    double *dst = sd.partial + (int64_t)item.chunk * sd.stride + od.out_off;
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            if (!(vmask >> (j * 4 + g) & 5u)) continue;  // neither h = 0 nor h = 1 stored
            const int c = cbase + 32 * j + 16 * g + (lane & 15);
            if (c >= od.nc) continue;
            const Feat fc = od.cols[c];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (!(vmask >> (j * 4 + h * 2 + g) & 1u)) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // 16 x 16 accumulator layouts: FP64 rows 4q + lane/16, FP32 rows 4*(lane/16) + q
                    const int r = rbase + 16 * h + (ACC64 ? 4 * q + (lane >> 4) : 4 * (lane >> 4) + q);
                    const Feat fr = od.rows[r];
                    if (fr.blk <= fc.blk) {
                        const double val = ACC64 ? acc64[j][h][g][q] : dacc[j][h][g][q];
                        dst[fr.addr + fc.addr + od.H[(int64_t)fr.blk * od.nbar + fc.blk]] = val;
                    }
                }
            }
        }
}

// DMAX: the largest order the launch holds (4, 6, 8 or 10).  Only the prefix /
// suffix lengths up to it are compiled in, so a launch of low orders gets
// the register allocation of its own bodies.
// Waves per SIMD the register allocation must allow: more resident waves
// hide the LDS latency between the matrix instructions of any one wave.  A
// work-group puts WG_WAVES / 4 waves on each SIMD, so the count is rounded
// down to a multiple of that.  FP64 launches holding orders 8 or more keep
// three: at four, their operand registers spill inside the stage loop
// (324 bytes per lane at order 10), which took the n = 8, d <= 10
// contraction from 0.155 to 0.254 ms.
template <int PREC, int WN, int DMAX>
constexpr int moment_occupancy() {
    constexpr int want = WN == 2 ? 2 : (PREC == P_F64 ? (DMAX <= 6 ? 4 : 3) : (PREC == P_F32 ? (DMAX <= 4 ? 4 : 3) : (PREC == P_BF16X2 || PREC == P_F16X2 ? 3 : 2)));
    constexpr int per = WG_WAVES / 4;
    return want / per * per > 0 ? want / per * per : per;
}

template <int PREC, int WN, int DMAX>
__global__ __launch_bounds__(64 * WG_WAVES, (moment_occupancy<PREC, WN, DMAX>())) void moment_kernel(MomentArgs a) {
    extern __shared__ __align__(16) char lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const Item item = a.items[it];
        if (item.tile < 0) continue;
        const SetDev sd = a.sets ? a.sets[item.set] : a.set0;
        // Copy the chunk's first stage to LDS before reading the tile's
        // records, so that the two latencies overlap.  No wave reads LDS
        // after the last barrier of a previous item, so the buffer is free.
        {
            const int stage_bytes = (a.n + 1) * PT<PREC>::KTP * (int)sizeof(typename PT<PREC>::T);
            stage_dma(reinterpret_cast<const char *>(sd.X) + (int64_t)item.chunk * sd.chunk_stages * stage_bytes, lds,
                      stage_bytes, wave, threadIdx.x & 63);
        }
        const TileDev *tile = a.tiles + item.tile;
        const OrderDev od = a.ords[tile->ord];
        switch (od.p * 8 + od.q) {
            case 1 * 8 + 1: moment_item<PREC, WN, 1, 1>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale); break;
            case 1 * 8 + 2: moment_item<PREC, WN, 1, 2>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale); break;
            case 2 * 8 + 2: moment_item<PREC, WN, 2, 2>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale); break;
            case 2 * 8 + 3:
                if constexpr (DMAX >= 5)
                    moment_item<PREC, WN, 2, 3>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale);
                else
                    wait_dma();
                break;
            case 3 * 8 + 3:
                if constexpr (DMAX >= 6)
                    moment_item<PREC, WN, 3, 3>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale);
                else
                    wait_dma();
                break;
            case 3 * 8 + 4:
                if constexpr (DMAX >= 7)
                    moment_item<PREC, WN, 3, 4>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale);
                else
                    wait_dma();
                break;
            case 4 * 8 + 4:
                if constexpr (DMAX >= 8)
                    moment_item<PREC, WN, 4, 4>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale);
                else
                    wait_dma();
                break;
            case 4 * 8 + 5:
                if constexpr (DMAX >= 9)
                    moment_item<PREC, WN, 4, 5>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale);
                else
                    wait_dma();
                break;
            case 5 * 8 + 5:
                if constexpr (DMAX >= 10)
                    moment_item<PREC, WN, 5, 5>(item, tile, od, sd, lds, a.n, wave, a.raw, a.rawstride, a.scale);
                else
                    wait_dma();
                break;
            default:
                // not a split of this launch's orders (the plans never ask for
                // one): let the first stage's copy land before the wave ends
                wait_dma();
                break;
        }
    }
}

template <int PREC, int WN>
static void launch_moment_dmax(int dmax, const MomentArgs &a, int grid, int lds, hipStream_t s) {
    if (dmax <= 4)
        hipLaunchKernelGGL((moment_kernel<PREC, WN, 4>), dim3(grid), dim3(64 * WG_WAVES), lds, s, a);
    else if (dmax <= 6)
        hipLaunchKernelGGL((moment_kernel<PREC, WN, 6>), dim3(grid), dim3(64 * WG_WAVES), lds, s, a);
    else if constexpr (PREC == P_F16X2)
        return;  // orders >= 7 stage in FP64 (the host refuses the FP16 split there)
    else if (dmax <= 8)
        hipLaunchKernelGGL((moment_kernel<PREC, WN, 8>), dim3(grid), dim3(64 * WG_WAVES), lds, s, a);
    else
        hipLaunchKernelGGL((moment_kernel<PREC, WN, 10>), dim3(grid), dim3(64 * WG_WAVES), lds, s, a);
}

template <int PREC>
static hipError_t launch_moment_prec(int shape, int dmax, const MomentArgs &a, int grid, hipStream_t s) {
    const int lds = lds_bytes_moment(PREC, a.n);
    switch (shape) {
        case TS_1x1: launch_moment_dmax<PREC, 1>(dmax, a, grid, lds, s); break;
        case TS_1x2: launch_moment_dmax<PREC, 2>(dmax, a, grid, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_moment(int prec, int shape, int dmax, const MomentArgs &a, int grid, hipStream_t s) {
    switch (prec) {
        case P_F64: return launch_moment_prec<P_F64>(shape, dmax, a, grid, s);
        case P_F32: return launch_moment_prec<P_F32>(shape, dmax, a, grid, s);
        case P_BF16X2: return launch_moment_prec<P_BF16X2>(shape, dmax, a, grid, s);
        case P_F16X2:
            if (dmax > 6 || (!a.scale && !a.sets)) return hipErrorInvalidValue;
            return launch_moment_prec<P_F16X2>(shape, dmax, a, grid, s);
        default: return launch_moment_prec<P_BF16X3>(shape, dmax, a, grid, s);
    }
}

// ---------------------------------------------------------------------------
// Finalisation: M_d = S_d / t and the cumulant recursion (Alg. 4 and Alg. 5;
// eq. cum_r of Section 3.2), all FP64.  One work-group per stored block j of
// one dataset.  Per block: the block tuple, the lower-order block offset of
// every sub-tuple j_S (S = a set of 2..d-2 positions; j_S is sorted because
// j is) and, when they fit, those lower-order sub-blocks, all in LDS.  Then
// each entry reads its chunk sum, divides by t and subtracts the sum over
// partitions of products of lower cumulants read at (j_S, i_S).  Each thread
// takes EPT entries at a time, so that one read of a partition's parts
// serves all of them.  A block's entries can be cut into slices of NT * EPT
// entries, each taken by its own work-group (which stages the block's
// lower-order sub-blocks for itself): at high orders there are few blocks of
// many entries, each with hundreds of terms, and one work-group per block
// leaves most of the chip idle.
// ---------------------------------------------------------------------------
// Binomial coefficients C(a, r), a < MAXN + MAXD + 1, r <= MAXD, built at
// compile time (Pascal's rule).
struct BinomTable {
    int64_t c[MAXN + MAXD + 1][MAXD + 1];
};
constexpr BinomTable make_binom_table() {
    BinomTable t{};
    for (int a = 0; a <= MAXN + MAXD; ++a)
        for (int r = 0; r <= MAXD; ++r)
            t.c[a][r] = r == 0 ? 1 : (a == 0 ? 0 : t.c[a - 1][r - 1] + t.c[a - 1][r]);
    return t;
}
__constant__ BinomTable c_binom = make_binom_table();

static_assert(MAXD <= 10, "the 24-bit sub-block index products of the finalisation assume orders up to 10");
constexpr int RED_EPT = 4;  // entries per thread of launches below order 7 (one work-group per block)

// Pointers read from memory are generic; these say which ones address
// global memory, so that their accesses are global (not flat) instructions.
#define CUM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ CUM_GLOBAL T *gmem(T *p) {
    return (CUM_GLOBAL T *)p;
}
// Read-only tables that every lane reads at the same index: constant address
// space, so that those reads are scalar loads and a wait for them is not a
// wait for the vector loads in flight.
#define CUM_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const CUM_CONST T *cmem(const T *p) {
    return (const CUM_CONST T *)p;
}

// kappa[m - 2] for a wave-uniform m, by constant indices (no dynamic
// indexing of the record)
__device__ __forceinline__ double *kappa_of(const SetRed &sr, int m) {
    switch (m) {
        case 2: return sr.kappa[0];
        case 3: return sr.kappa[1];
        case 4: return sr.kappa[2];
        case 5: return sr.kappa[3];
        case 6: return sr.kappa[4];
        case 7: return sr.kappa[5];
        default: return sr.kappa[6];
    }
}

// mom[m - 2] likewise
__device__ __forceinline__ double *mom_of(const SetRed &sr, int m) {
    switch (m) {
        case 2: return sr.mom[0];
        case 3: return sr.mom[1];
        case 4: return sr.mom[2];
        case 5: return sr.mom[3];
        case 6: return sr.mom[4];
        case 7: return sr.mom[5];
        default: return sr.mom[6];
    }
}

// Index, in the run of b^|last positions in the set| consecutive values a
// factor holds for a thread's entries, of entry q's value (the thread's
// entries differ in their last E digits, q = those digits in base BB).  The
// term group C has bit E-1-i set when the set A holds position D-E+i; the
// side is A's (A_SIDE) or its complement's.
template <unsigned BB, int E, int C, bool A_SIDE>
__device__ constexpr unsigned run_index(unsigned q) {
    unsigned j = 0;
    for (int i = 0; i < E; ++i) {
        if ((((C >> (E - 1 - i)) & 1) != 0) != A_SIDE) continue;
        unsigned dig = q;
        for (int k = 0; k < E - 1 - i; ++k) dig /= BB;
        j = j * BB + dig % BB;
    }
    return j;
}

// GB > 0: the multi-entry form of the first-position formula with block
// size GB, GE digits per lane, factors read from the LDS-staged sub-blocks
// (GST) or from memory (a kernel of its own, see below).
template <int D, int NT, int EPT, int GB = 0, int GE = 0, bool GST = false>
__device__ __forceinline__ void finalize_block(const RedArgs &a, const RedOrder &ro, const SetRed &sr, int64_t B,
                                               int slice, int nslice, char *dyn, int *tup, double *gred = nullptr,
                                               const unsigned char *ptab = nullptr, unsigned short *ftab = nullptr) {
    constexpr int PARTS = D / 2;  // parts per partition slot
    const int tid = threadIdx.x;
    const unsigned b = (unsigned)ro.b;
    unsigned be = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) be *= b;
    const bool rec = a.recursion && D >= 4;
    const bool staged = rec && ro.lds_elems > 0;
    // orders >= 7 with the lower central moments at hand: the first-position
    // formula (two factors per term, a set A holding position 0 and its
    // complement); the staged slots of sets without position 0 then hold
    // moments, the others cumulants
    const bool first_pos = D >= FIRST_POSITION_MIN_D && rec && a.subset && ro.nterm > 0;
    double *sub = reinterpret_cast<double *>(dyn);
    const double **base = reinterpret_cast<const double **>(dyn + a.base_off);
    int32_t *parts_l = reinterpret_cast<int32_t *>(dyn + a.parts_off);
    const bool parts_in_lds = rec && a.parts_lds;
    const CUM_CONST int32_t *parts_g = cmem(ro.parts);
    const CUM_GLOBAL int64_t *prank = gmem(ro.prank);

    __syncthreads();  // the previous block's readers are done with the LDS tables
    if (tid < D) tup[tid] = gmem(ro.tuples)[B * D + tid];
    const CUM_CONST int32_t *terms_g = cmem(ro.terms);
    const CUM_CONST int32_t *tpw_g = cmem(ro.tpw);
    if (parts_in_lds) {
        if (first_pos)
            for (int i = tid; i < ro.nterm * 2; i += NT) parts_l[i] = terms_g[i];
        else
            for (int i = tid; i < ro.npart * PARTS; i += NT) parts_l[i] = parts_g[i];
    }
    __syncthreads();
    if (rec) {
        // address of the sub-block j_S: in the order-|S| buffer (the cumulants,
        // or the central moments for a first-position factor without position
        // 0) at the rank of the sorted tuple j_S (sum of the hockey-stick rank
        // terms) times b^|S|
        for (int s = tid; s < ro.ns; s += NT) {
            const unsigned mask = gmem(ro.smask)[s];
            const int m = __popc(mask);
            int64_t rank = 0, bm = 1;
            int prev = 0, k2 = 0;
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (mask >> k & 1u) {
                    rank += c_binom.c[ro.nbar - prev + m - k2 - 1][m - k2] -
                            c_binom.c[ro.nbar - tup[k] + m - k2 - 1][m - k2];
                    prev = tup[k];
                    ++k2;
                    bm *= b;
                }
            const bool moment = first_pos && !(mask & 1u);
            base[s] = (moment ? mom_of(sr, m) : kappa_of(sr, m)) + rank * bm;
        }
        __syncthreads();
    }
    if (staged) {
        // the block's lower-order sub-blocks into LDS, eight slots per thread
        // at a time so that their loads are in flight together
        // (slots past the end repeat the last one, so that no load is
        // conditional; only the stores are)
        const CUM_GLOBAL int32_t *gm = gmem(ro.gmap);
        const int le = ro.lds_elems;
        for (int e0 = tid; e0 < le; e0 += 8 * NT) {
            int g[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) g[i] = gm[min(e0 + i * NT, le - 1)];
            const double *bp[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) bp[i] = base[g[i] & 1023];
            double v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = gmem(bp[i])[g[i] >> 10];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (e0 + i * NT < le) sub[e0 + i * NT] = v[i];
        }
        __syncthreads();
    }

    CUM_GLOBAL double *out = gmem(sr.kappa[D - 2]);
    const CUM_GLOBAL double *partial = gmem(sr.partial + ro.out_off);
    const int64_t stride = sr.stride, nchunks = a.presummed ? 1 : sr.nchunks;
    const double tt = (double)sr.t;
    // The partial sums are either in this layout (one per stored copy) or in
    // the layout of block size pb, which holds each sorted variable tuple
    // once; then every stored copy reads that tuple's sums.
    const bool canon = ro.pb != ro.b;
    bool need_sort = false;  // equal adjacent blocks: the variables need sorting
#pragma unroll
    for (int k = 0; k + 1 < D; ++k) need_sort |= tup[k] == tup[k + 1];

    // M = S / t of the entry with in-block index oo and digits rr, from the
    // partial sums (0 for an entry past the block's end)
    auto moment_at = [&](const int (&rr)[D], unsigned oo, bool valid) -> double {
        int64_t poff = (int64_t)B * be + oo;
        bool pad = !valid;
        if (canon && valid) {
            int u[D];
#pragma unroll
            for (int k = 0; k < D; ++k) u[k] = tup[k] * ro.b + rr[k];
            if (need_sort) {
                // odd-even transposition network: D rounds sort D keys
#pragma unroll
                for (int rd = 0; rd < D; ++rd)
#pragma unroll
                    for (int k = rd & 1; k + 1 < D; k += 2) {
                        const int lo = min(u[k], u[k + 1]), hi = max(u[k], u[k + 1]);
                        u[k] = lo;
                        u[k + 1] = hi;
                    }
            }
            int umax = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) umax = max(umax, u[k]);
            pad = umax >= ro.n;  // a padded position of a ragged block: M = 0
            if (!pad) {
                const int pb = ro.pb, w = ro.pnbar + 1;
                int64_t rank = 0, in = 0;
                int prev = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int jb = pb == 1 ? u[k] : u[k] / pb;
                    rank += prank[k * w + prev] - prank[k * w + jb];
                    in = in * pb + (u[k] - jb * pb);
                    prev = jb;
                }
                poff = rank + in;
            }
        }
        double S = 0.0;
        if (!pad) {
            const CUM_GLOBAL double *pp = partial + poff;
            int64_t c = 0;
            // eight independent loads in flight, summed in chunk order
            for (; c + 8 <= nchunks; c += 8) {
                double v[8];
#pragma unroll
                for (int x = 0; x < 8; ++x) v[x] = pp[(c + x) * stride];
#pragma unroll
                for (int x = 0; x < 8; ++x) S += v[x];
            }
            for (; c < nchunks; ++c) S += pp[c * stride];
        }
        return S / tt;
    };

    // Orders >= 7 in the multi-entry form (launched on their own, GB = b):
    // the first-position formula with factors read from the staged
    // sub-blocks in LDS (GST) or from memory.  Each lane takes the BB^E
    // entries that differ only in their last E digits: a factor's values for
    // them are one run of consecutive values of its sub-block (its digits on
    // the last E positions are the least significant), a single value when
    // the set holds none of those positions.  The terms come grouped by which of them A holds, so each
    // group's run lengths are known at compile time.  The four waves of the
    // work-group take the same 64 lanes' entries and a quarter of the terms
    // each; wave 0 adds the other waves' sums to its own, in wave order.
    if constexpr (GB > 0) {
        auto gather_multi = [&](auto b_t, auto e_t) {
            constexpr unsigned BB = decltype(b_t)::value;
            constexpr int E = decltype(e_t)::value;
            constexpr unsigned Q = E == 2 ? BB * BB : BB;
            constexpr int DP = D - E;  // digits of the lane's entry group u
            constexpr int HL = (DP + 1) / 2, HH = DP - HL;
            constexpr int TW = NT / 64;  // waves sharing the terms
            static_assert(Q <= 4 && TW >= 1, "gathering layout");
            const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
            const CUM_CONST int32_t *terms_c = cmem(ro.terms);
            CUM_GLOBAL double *out_m = gmem(sr.kappa[D - 2]);
            CUM_GLOBAL double *mo = sr.mom[D - 2] ? gmem(sr.mom[D - 2]) : nullptr;
            const unsigned bu = be / Q;
            const int zlo = (int)((int64_t)ro.nterm * wave / TW), zhi = (int)((int64_t)ro.nterm * (wave + 1) / TW);
            // the loop bounds are the same in every lane (barriers inside)
            for (unsigned u0 = (unsigned)slice * 64u; u0 < bu; u0 += 64u * (unsigned)nslice) {
                const bool valid = u0 + (unsigned)lane < bu;
                const unsigned u = valid ? u0 + (unsigned)lane : u0;
                int rr[D];
                unsigned x = u;
#pragma unroll
                for (int k = DP - 1; k >= 0; --k) {
                    rr[k] = (int)(x % BB);
                    x /= BB;
                }
                // index of u's digits at the positions of any set: for b = 2
                // a bit extraction (below), else from two tables over
                // positions 0..HL-1 and HL..DP-1 (as in the one-entry form)
                constexpr bool BITS = BB == 2;
                constexpr int TL = BITS ? 1 : (1 << HL), TH = BITS ? 1 : (1 << HH);
                unsigned tlo[TL], thi[TH];
                tlo[0] = thi[0] = 0;
                if constexpr (!BITS) {
#pragma unroll
                    for (int m = 1; m < TL; ++m) {
                        const int k = 31 - __builtin_clz((unsigned)m);
                        tlo[m] = tlo[m & ~(1 << k)] * BB + (unsigned)rr[k];
                    }
#pragma unroll
                    for (int m = 1; m < TH; ++m) {
                        const int k = 31 - __builtin_clz((unsigned)m);
                        thi[m] = thi[m & ~(1 << k)] * BB + (unsigned)rr[HL + k];
                    }
                }
                // b = 2: u's bit DP-1-k is the digit of position k, and its low
                // six bits are the lane; the wave's high bits are uniform
                const unsigned uh = u0 >> 6;
                double sum[Q];
#pragma unroll
                for (unsigned q = 0; q < Q; ++q) sum[q] = 0.0;
                // the N values of factor pk (mask | set index << 10) for the
                // lane's entries
                auto load = [&](int pk0, auto n_t, double *v) {
                    constexpr unsigned N = decltype(n_t)::value;
                    const int pk = __builtin_amdgcn_readfirstlane(pk0);
                    const unsigned mask = (unsigned)pk & 1023u;
                    unsigned flat;
                    if constexpr (BITS) {
                        // the set's bits of u, in u's order: the uniform high
                        // part, then the lane's six bits from the table
                        static_assert(DP >= 6 && DP <= 8, "bit layout");
                        const unsigned rm = __builtin_bitreverse32(mask & ((1u << DP) - 1u)) >> (32 - DP);
                        const unsigned ml = rm & 63u, mh = rm >> 6;
                        unsigned hp = 0, k = 0;
#pragma unroll
                        for (int i = 0; i < DP - 6; ++i)
                            if (mh >> i & 1u) hp |= ((uh >> i) & 1u) << k++;
                        flat = ((hp << __builtin_popcount(ml)) | ptab[ml * 64 + lane]) * N;
                    } else {
                        const unsigned lo = mask & ((1u << HL) - 1u), hi = (mask >> HL) & ((1u << HH) - 1u);
                        const unsigned c = __builtin_popcount(hi);
                        unsigned pw = 1;
                        for (unsigned i = 0; i < c; ++i) pw *= BB;
                        flat = (tlo[lo] * pw + thi[hi]) * N;
                    }
                    if constexpr (GST) {
                        const double *p = sub + (pk >> 10) + flat;
#pragma unroll
                        for (unsigned j = 0; j < N; ++j) v[j] = p[j];
                    } else {
                        const CUM_GLOBAL double *p = gmem(base[pk >> 10]) + flat;
#pragma unroll
                        for (unsigned j = 0; j < N; ++j) v[j] = p[j];
                    }
                };
                auto group = [&](auto c_t) {
                    constexpr int C = decltype(c_t)::value;
                    constexpr int KA = (C & 1) + ((C >> 1) & 1);  // last positions A holds
                    constexpr unsigned NA = KA == 0 ? 1u : (KA == 1 ? BB : BB * BB), NC = Q / NA;
                    const int z1 = min(ro.cstart[C + 1], zhi);
                    int z = max(ro.cstart[C], zlo);
                    // four terms' factors in flight at once (eight need more registers
                    // than three waves per SIMD allow)
                    for (; z + 4 <= z1; z += 4) {
                        int pk[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) pk[i] = terms_c[z * 2 + i];
                        double va[4][NA], vc[4][NC];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            load(pk[2 * i], std::integral_constant<unsigned, NA>(), va[i]);
                            load(pk[2 * i + 1], std::integral_constant<unsigned, NC>(), vc[i]);
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (unsigned q = 0; q < Q; ++q)
                                sum[q] += va[i][run_index<BB, E, C, true>(q)] * vc[i][run_index<BB, E, C, false>(q)];
                    }
                    for (; z < z1; ++z) {
                        double va[NA], vc[NC];
                        load(terms_c[z * 2], std::integral_constant<unsigned, NA>(), va);
                        load(terms_c[z * 2 + 1], std::integral_constant<unsigned, NC>(), vc);
#pragma unroll
                        for (unsigned q = 0; q < Q; ++q)
                            sum[q] += va[run_index<BB, E, C, true>(q)] * vc[run_index<BB, E, C, false>(q)];
                    }
                };
                group(std::integral_constant<int, 0>());
                group(std::integral_constant<int, 1>());
                if constexpr (E == 2) {
                    group(std::integral_constant<int, 2>());
                    group(std::integral_constant<int, 3>());
                }
                // the other waves' sums go to LDS: into the staged sub-blocks
                // once every wave is done reading them, else into gred
                double *gr = gred;
                if constexpr (GST) {
                    __syncthreads();
                    gr = sub;
                }
                if (wave > 0) {
#pragma unroll
                    for (unsigned q = 0; q < Q; ++q) gr[((wave - 1) * 4 + (int)q) * 64 + lane] = sum[q];
                }
                // the moments after the terms, so that their registers are
                // free during the term loop
                double M[Q];
                if (wave == 0) {
                    x = u;
#pragma unroll
                    for (int k = DP - 1; k >= 0; --k) {
                        rr[k] = (int)(x % BB);
                        x /= BB;
                    }
#pragma unroll
                    for (unsigned q = 0; q < Q; ++q) {
                        unsigned y = q;
#pragma unroll
                        for (int k = D - 1; k >= DP; --k) {
                            rr[k] = (int)(y % BB);
                            y /= BB;
                        }
                        M[q] = moment_at(rr, u * Q + q, valid);
                    }
                }
                __syncthreads();
                if (wave == 0 && valid) {
                    const int64_t e0 = (int64_t)B * be + (int64_t)u * Q;
#pragma unroll
                    for (unsigned q = 0; q < Q; ++q) {
                        double sq = sum[q];
                        for (int w = 1; w < TW; ++w) sq += gr[((w - 1) * 4 + (int)q) * 64 + lane];
                        if (mo) mo[e0 + q] = M[q];
                        out_m[e0 + q] = M[q] - sq;
                    }
                }
                __syncthreads();  // gr is free again
            }
        };
        // (the host launches this kernel only for b = GB, qe = GE)
        gather_multi(std::integral_constant<unsigned, (unsigned)GB>(), std::integral_constant<int, GE>());
        if (sr.stamp && tid == 0) atomicMax(sr.stamp, (unsigned long long)wall_clock64());
        return;
    } else {
        // Orders 4 to 6 by the partition recursion, sub-blocks staged, b in
        // {2, 3, 4}: each thread takes the b entries that differ only in the
        // last digit.  In each partition exactly one part holds the last
        // position: its values for the b entries are one run of consecutive
        // values of its sub-block, and each other part has one value for all
        // of them, so a partition costs one run and one value per other
        // part.  The in-block index of every set of the first D - 1
        // positions comes from a per-thread LDS table (ftab), built once per
        // entry group by one Horner step per set.
        if constexpr (EPT > 1 && D >= 4 && D <= 6) {
            auto rec_multi = [&](auto b_t) {
                constexpr unsigned BB = decltype(b_t)::value, Q = BB;
                constexpr int DP = D - 1, NS = 1 << DP;
                constexpr int PARTS_ = D / 2;
                unsigned short *tb = ftab + tid;  // set S at tb[S * NT]
                const unsigned bu = be / Q;
                for (unsigned u = (unsigned)(slice * NT + tid); u < bu; u += (unsigned)(NT * nslice)) {
                    int rr[D];
                    unsigned x = u;
#pragma unroll
                    for (int k = DP - 1; k >= 0; --k) {
                        rr[k] = (int)(x % BB);
                        x /= BB;
                    }
                    {
                        unsigned t[NS];
                        t[0] = 0;
#pragma unroll
                        for (int m = 1; m < NS; ++m) {
                            const int k = 31 - __builtin_clz((unsigned)m);
                            t[m] = t[m & ~(1 << k)] * BB + (unsigned)rr[k];
                        }
#pragma unroll
                        for (int m = 0; m < NS; ++m) tb[m * NT] = (unsigned short)t[m];
                    }
                    double M[Q], sum[Q];
#pragma unroll
                    for (unsigned q = 0; q < Q; ++q) {
                        rr[D - 1] = (int)q;
                        M[q] = moment_at(rr, u * Q + q, true);
                        sum[q] = 0.0;
                    }
                    const int64_t e0 = (int64_t)B * be + (int64_t)u * Q;
                    if (sr.mom[D - 2]) {
                        CUM_GLOBAL double *mo = gmem(sr.mom[D - 2]);
#pragma unroll
                        for (unsigned q = 0; q < Q; ++q) mo[e0 + q] = M[q];
                    }
                    // one partition's product for each entry, its parts
                    // multiplied left to right as in the one-entry form: the
                    // parts before the one holding the last position (pre),
                    // that part's run, then the parts after it
                    auto partition = [&](const int *pks, double (&prod)[Q]) {
                        double pre = 1.0;
                        bool held = false;
#pragma unroll
                        for (unsigned j = 0; j < Q; ++j) prod[j] = 0.0;
#pragma unroll
                        for (int pt = 0; pt < PARTS_; ++pt) {
                            const int pk = __builtin_amdgcn_readfirstlane(pks[pt]);
                            if (!pk) break;
                            const unsigned mask = (unsigned)pk & 1023u;
                            const int where = pk >> 10;
                            const unsigned f = tb[(mask & (unsigned)(NS - 1)) * NT];
                            if (mask >> DP & 1u) {
#pragma unroll
                                for (unsigned j = 0; j < Q; ++j) prod[j] = pre * sub[where + f * Q + j];
                                held = true;
                            } else {
                                const double v = sub[where + f];
                                if (held) {
#pragma unroll
                                    for (unsigned j = 0; j < Q; ++j) prod[j] *= v;
                                } else {
                                    pre *= v;
                                }
                            }
                        }
                    };
                    int z = 0;
                    // four partitions' factors in flight at once, added in order
                    for (; z + 4 <= ro.npart; z += 4) {
                        int pks[4 * PARTS_];
#pragma unroll
                        for (int i = 0; i < 4 * PARTS_; ++i) pks[i] = parts_g[z * PARTS_ + i];
                        double prod[4][Q];
#pragma unroll
                        for (int w = 0; w < 4; ++w) partition(pks + w * PARTS_, prod[w]);
#pragma unroll
                        for (int w = 0; w < 4; ++w)
#pragma unroll
                            for (unsigned q = 0; q < Q; ++q) sum[q] += prod[w][q];
                    }
                    for (; z < ro.npart; ++z) {
                        int pks[PARTS_];
#pragma unroll
                        for (int i = 0; i < PARTS_; ++i) pks[i] = parts_g[z * PARTS_ + i];
                        double prod[Q];
                        partition(pks, prod);
#pragma unroll
                        for (unsigned q = 0; q < Q; ++q) sum[q] += prod[q];
                    }
#pragma unroll
                    for (unsigned q = 0; q < Q; ++q) out[e0 + q] = M[q] - sum[q];
                }
            };
            if (ftab && staged && b >= 2 && b <= 4) {
                if (b == 2)
                    rec_multi(std::integral_constant<unsigned, 2>());
                else if (b == 3)
                    rec_multi(std::integral_constant<unsigned, 3>());
                else
                    rec_multi(std::integral_constant<unsigned, 4>());
                if (sr.stamp && tid == 0) atomicMax(sr.stamp, (unsigned long long)wall_clock64());
                return;
            }
        }
        for (unsigned o0 = (unsigned)(slice * NT * EPT + tid); o0 < be; o0 += (unsigned)(NT * EPT * nslice)) {
            int r[EPT][D];  // in-block digits, first position most significant
            double M[EPT];
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                unsigned oo = o0 + (unsigned)NT * q;
                const bool valid = oo < be;
                if (!valid) oo = 0;
                unsigned x = oo;
#pragma unroll
                for (int k = D - 1; k >= 0; --k) {
                    r[q][k] = (int)(x % b);
                    x /= b;
                }
                M[q] = moment_at(r[q], oo, valid);
            }
            // One entry per thread: the in-block index of the entry's digits at
            // the positions of any set, from two tables built once per entry.
            // Positions 0..HL-1 index tlo, positions HL..D-1 index thi (by the set
            // mask shifted down by HL); each table entry follows from the one
            // without its last position by one step of Horner's rule, and a set's
            // index is tlo[low part] * b^|high part| + thi[high part].
            constexpr int HL = (D + 1) / 2, HH = D - HL;
            unsigned tlo[1 << HL], thi[1 << HH];
            const unsigned b2 = b * b, b4 = b2 * b2;  // b^|high part| = b^(c&1) b2^(c>>1&1) b4^(c>>2), c <= 5
            if constexpr (EPT == 1) {
                tlo[0] = 0;
#pragma unroll
                for (int m = 1; m < (1 << HL); ++m) {
                    const int k = 31 - __builtin_clz((unsigned)m);
                    tlo[m] = __umul24(tlo[m & ~(1 << k)], b) + (unsigned)r[0][k];
                }
                thi[0] = 0;
#pragma unroll
                for (int m = 1; m < (1 << HH); ++m) {
                    const int k = 31 - __builtin_clz((unsigned)m);
                    thi[m] = __umul24(thi[m & ~(1 << k)], b) + (unsigned)r[0][HL + k];
                }
            }
            // One factor of a term for every entry of the thread: the lower-order
            // sub-block of part pk (position mask | where << 10), read in LDS
            // (staged) or in memory, where first-position formula factors without
            // position 0 are central moments.  The part is the same for every lane:
            // readfirstlane makes that explicit, so that the position tests are
            // scalar.
            // pw0: the set's multiplier b^|high part| when the table gives it (the
            // first-position terms), else negative
            auto factor = [&](auto staged_t, int pk0, double (&v)[EPT], int pw0 = -1) {
                constexpr bool ST = decltype(staged_t)::value;
                const int pk = __builtin_amdgcn_readfirstlane(pk0);
                const unsigned mask = (unsigned)pk & 1023u;
                const int where = pk >> 10;
                if constexpr (EPT == 1) {
                    const unsigned lo = mask & ((1u << HL) - 1u), hi = mask >> HL;
                    unsigned pw;
                    if (pw0 >= 0) {
                        pw = (unsigned)__builtin_amdgcn_readfirstlane(pw0);
                    } else {
                        const unsigned c = __builtin_popcount(hi);
                        pw = ((c & 1u) ? b : 1u) * ((c & 2u) ? b2 : 1u) * ((c & 4u) ? b4 : 1u);
                    }
                    const unsigned flat = __umul24(tlo[lo], pw) + thi[hi];
                    if constexpr (ST)
                        v[0] = sub[where + flat];
                    else
                        v[0] = gmem(base[where])[flat];
                    return;
                }
                // In-block index of the sub-block entry, by Horner's rule over the
                // digits of the set's positions.  A set has at most D - 2
                // positions, so every product below is of a value under b^(D-3)
                // by b; with blocks under 2^31 entries (b^D < 2^31, D <= 10)
                // b^(D-3) stays under 2^24, and the 24-bit multiply-add, a full
                // rate vector instruction, is exact.
#pragma unroll
                for (int q = 0; q < EPT; ++q) {
                    unsigned flat = 0;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        if (mask >> k & 1u) flat = __umul24(flat, b) + (unsigned)r[q][k];
                    if constexpr (ST)
                        v[q] = sub[where + flat];
                    else
                        v[q] = gmem(base[where])[flat];
                }
            };
            auto part_at = [&](const CUM_CONST int32_t *table, int i) {
                return __builtin_amdgcn_readfirstlane(parts_in_lds ? parts_l[i] : table[i]);
            };
            // the first-position formula: sum over sets A holding position 0 of
            // kappa(A) times the central moment of the complement, in term order
            auto first_position = [&](auto staged_t) {
                double sum[EPT];
#pragma unroll
                for (int q = 0; q < EPT; ++q) sum[q] = 0.0;
                int z = 0;
                if constexpr (EPT == 1) {
                    // one entry per thread: eight terms' parts in one scalar read,
                    // then their sixteen loads in flight at once
                    for (; z + 8 <= ro.nterm; z += 8) {
                        int pk[16], pw[16];
#pragma unroll
                        for (int i = 0; i < 16; ++i) pk[i] = terms_g[z * 2 + i];
#pragma unroll
                        for (int i = 0; i < 16; ++i) pw[i] = tpw_g[z * 2 + i];
                        double v[16][EPT];
#pragma unroll
                        for (int i = 0; i < 16; ++i) factor(staged_t, pk[i], v[i], pw[i]);
#pragma unroll
                        for (int u = 0; u < 8; ++u) sum[0] += v[2 * u][0] * v[2 * u + 1][0];
                    }
                }
                for (; z < ro.nterm; ++z) {
                    double v0[EPT], v1[EPT];
                    factor(staged_t, part_at(terms_g, z * 2), v0);
                    factor(staged_t, part_at(terms_g, z * 2 + 1), v1);
#pragma unroll
                    for (int q = 0; q < EPT; ++q) sum[q] += v0[q] * v1[q];
                }
#pragma unroll
                for (int q = 0; q < EPT; ++q) M[q] -= sum[q];
            };
            // sum over partitions of products of lower cumulants, in partition
            // order; a partition's row ends at its first zero part
            auto recursion = [&](auto staged_t) {
                double sum[EPT];
#pragma unroll
                for (int q = 0; q < EPT; ++q) sum[q] = 0.0;
                int z = 0;
                if constexpr (EPT == 1) {
                    for (; z + 4 <= ro.npart; z += 4) {
                        int pks[4 * PARTS];
#pragma unroll
                        for (int i = 0; i < 4 * PARTS; ++i) pks[i] = parts_g[z * PARTS + i];
                        double prod[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            double v[PARTS][EPT];
                            bool live = true;
#pragma unroll
                            for (int pt = 0; pt < PARTS; ++pt) {
                                const int pk = __builtin_amdgcn_readfirstlane(pks[u * PARTS + pt]);
                                live = live && pk != 0;
                                if (live)
                                    factor(staged_t, pk, v[pt]);
                                else
                                    v[pt][0] = 1.0;
                            }
                            prod[u] = 1.0;
#pragma unroll
                            for (int pt = 0; pt < PARTS; ++pt) prod[u] *= v[pt][0];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) sum[0] += prod[u];
                    }
                }
                for (; z < ro.npart; ++z) {
                    double prod[EPT];
#pragma unroll
                    for (int q = 0; q < EPT; ++q) prod[q] = 1.0;
#pragma unroll
                    for (int pt = 0; pt < PARTS; ++pt) {
                        const int pk = part_at(parts_g, z * PARTS + pt);
                        if (!pk) break;
                        double v[EPT];
                        factor(staged_t, pk, v);
#pragma unroll
                        for (int q = 0; q < EPT; ++q) prod[q] *= v[q];
                    }
#pragma unroll
                    for (int q = 0; q < EPT; ++q) sum[q] += prod[q];
                }
#pragma unroll
                for (int q = 0; q < EPT; ++q) M[q] -= sum[q];
            };
            // the central moments of this order, for the first-position formula of
            // higher orders
            if (sr.mom[D - 2]) {
                CUM_GLOBAL double *mo = gmem(sr.mom[D - 2]);
#pragma unroll
                for (int q = 0; q < EPT; ++q) {
                    const unsigned o = o0 + (unsigned)NT * q;
                    if (o < be) mo[B * be + o] = M[q];
                }
            }
            if constexpr (D >= FIRST_POSITION_MIN_D) {
                if (first_pos) {
                    if (staged)
                        first_position(std::true_type());
                    else
                        first_position(std::false_type());
                } else if (staged) {
                    recursion(std::true_type());
                } else if (rec) {
                    recursion(std::false_type());
                }
            } else {
                if (staged)
                    recursion(std::true_type());
                else if (rec)
                    recursion(std::false_type());
            }
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const unsigned o = o0 + (unsigned)NT * q;
                if (o < be) out[B * be + o] = M[q];
            }
        }
        if (sr.stamp && tid == 0) atomicMax(sr.stamp, (unsigned long long)wall_clock64());
    }
}

// NT threads per work-group: 256, or one wave (64) when the blocks are small,
// so that more blocks are in flight per compute unit.  Work-group g takes
// slice g % sl of block g / sl of its order (sl0 or sl1 slices per block).
template <int D0, int NT, int EPT>
__global__ __launch_bounds__(NT) void reduce_kernel(RedArgs a) {
    extern __shared__ __align__(16) char dyn[];
    __shared__ int tup[MAXD];
    // launches of several entries per thread over orders 4..6: the in-block
    // index tables of the recursion's multi-entry form, 2^(D-1) per thread
    constexpr bool FT = EPT > 1 && D0 >= 4 && D0 <= 6;
    constexpr int FTN = FT ? NT << (D0 + 1 >= 6 ? 5 : D0) : 1;
    __shared__ unsigned short ftab[FTN];
    SetRed sr = a.set0;
    if (a.sets) sr = a.sets[blockIdx.y];
    const int64_t n0 = a.nb0 * a.sl0, ntot = n0 + (a.nbtot - a.nb0) * a.sl1;
    for (int64_t g = blockIdx.x; g < ntot; g += gridDim.x) {
        if (g < n0) {
            const RedOrder ro = a.ords[0];
            finalize_block<D0, NT, EPT>(a, ro, sr, g / a.sl0, (int)(g % a.sl0), a.sl0, dyn, tup, nullptr, nullptr,
                                        FT ? ftab : nullptr);
        } else {
            if constexpr (D0 < MAXD) {
                const RedOrder ro = a.ords[1];
                const int64_t h = g - n0;
                finalize_block<D0 + 1, NT, EPT>(a, ro, sr, h / a.sl1, (int)(h % a.sl1), a.sl1, dyn, tup, nullptr,
                                                nullptr, (FT && D0 + 1 <= 6) ? ftab : nullptr);
            }
        }
    }
}

// One order D in the multi-entry form (block size GB, GE digits per lane,
// factors in LDS when ST), a kernel of its own so that its registers do not
// weigh on the other finalisation kernels.
template <int D, int GB, int GE, bool ST>
__global__ __launch_bounds__(256) void gather_kernel(RedArgs a) {
    extern __shared__ __align__(16) char dyn[];
    __shared__ int tup[MAXD];
    SetRed sr = a.set0;
    if (a.sets) sr = a.sets[blockIdx.y];
    // the sums of waves 1..3, 4 entries per lane (staged launches use the
    // staged sub-blocks' LDS, which holds at least as much, once read)
    __shared__ double gred[ST ? 1 : 3 * 4 * 64];
    // b = 2: ptab[m * 64 + l] = the bits of lane l selected by mask m, packed
    // in order (made visible by the first barrier of the block loop)
    __shared__ unsigned char ptab[GB == 2 ? 64 * 64 : 1];
    if constexpr (GB == 2) {
        for (int i = threadIdx.x; i < 64 * 64; i += 256) {
            const unsigned m = (unsigned)i >> 6, l = (unsigned)i & 63u;
            unsigned r = 0, k = 0;
            for (int j = 0; j < 6; ++j)
                if (m >> j & 1u) r |= ((l >> j) & 1u) << k++;
            ptab[i] = (unsigned char)r;
        }
    }
    const RedOrder ro = a.ords[0];
    const int64_t ntot = a.nb0 * a.sl0;
    for (int64_t g = blockIdx.x; g < ntot; g += gridDim.x)
        finalize_block<D, 256, 1, GB, GE, ST>(a, ro, sr, g / a.sl0, (int)(g % a.sl0), a.sl0, dyn, tup, gred, ptab);
}

// Sum of the per-chunk partial sums of every entry, in chunk order (Alg. 3's
// reduction), into the entry's chunk-0 slot: one coalesced pass, so that the
// finalisation reads one value per entry.
__global__ __launch_bounds__(256) void chunksum_kernel(const SetRed *sets, SetRed set0, int64_t entries) {
    const SetRed sr = sets ? sets[blockIdx.y] : set0;
    const int64_t stride = sr.stride, nchunks = sr.nchunks;
    if (nchunks <= 1) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < entries; e += (int64_t)gridDim.x * 256) {
        const double *pp = sr.partial + e;
        double S = 0.0;
        int64_t c = 0;
        // eight independent loads in flight, summed in chunk order
        for (; c + 8 <= nchunks; c += 8) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = pp[(c + q) * stride];
#pragma unroll
            for (int q = 0; q < 8; ++q) S += v[q];
        }
        for (; c < nchunks; ++c) S += pp[c * stride];
        sr.partial[e] = S;
    }
}

// The chunk sums in tile order, added over chunks and scattered once to block
// storage: the same additions in the same order as chunksum_kernel, with the
// address of each entry (row and column records, the (v, w) rank term)
// worked out once instead of once per chunk in the contraction's epilogue.
template <int WN, bool ACC64>
__global__ __launch_bounds__(256) void rawsum_kernel(const double *raw, int64_t rawstride, int64_t nchunks,
                                                     const TileDev *tiles, const OrderDev *ords, double *canon) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < rawstride; p += (int64_t)gridDim.x * 256) {
        const int64_t wb = p / (WN * 1024);
        const int rem = (int)(p - wb * (WN * 1024));
        const int64_t ti = wb / WG_WAVES;
        const int wave = (int)(wb - ti * WG_WAVES);
        const TileDev *tile = tiles + ti;
        if (wave >= tile->ntask) continue;
        const WaveTask wt = tile->task[wave];
        const int k3 = rem >> 8, q = (rem >> 6) & 3, lane = rem & 63;
        const int j = k3 >> 2, g = (k3 >> 1) & 1, h = k3 & 1;
        if (!((unsigned)wt.mask >> (j * 4 + h * 2 + g) & 1u)) continue;
        const OrderDev od = ords[tile->ord];
        const int c = wt.c0 + 32 * j + 16 * g + (lane & 15);
        if (c >= od.nc) continue;
        const int r = wt.r0 + 16 * h + (ACC64 ? 4 * q + (lane >> 4) : 4 * (lane >> 4) + q);
        const Feat fr = od.rows[r], fc = od.cols[c];
        if (fr.blk > fc.blk) continue;
        const double *pp = raw + p;
        double S = 0.0;
        int64_t ch = 0;
        for (; ch + 8 <= nchunks; ch += 8) {
            double v[8];
#pragma unroll
            for (int x = 0; x < 8; ++x) v[x] = pp[(ch + x) * rawstride];
#pragma unroll
            for (int x = 0; x < 8; ++x) S += v[x];
        }
        for (; ch < nchunks; ++ch) S += pp[ch * rawstride];
        canon[od.out_off + fr.addr + fc.addr + od.H[(int64_t)fr.blk * od.nbar + fc.blk]] = S;
    }
}

hipError_t launch_rawsum(const double *raw, int64_t rawstride, int64_t nchunks, const TileDev *tiles,
                         const OrderDev *ords, double *canon, int wn, bool acc64, hipStream_t s) {
    int64_t gx = (rawstride + 255) / 256;
    if (gx > 65535) gx = 65535;
    if (gx < 1) gx = 1;
    if (wn == 1 && !acc64)
        hipLaunchKernelGGL((rawsum_kernel<1, false>), dim3((unsigned)gx), dim3(256), 0, s, raw, rawstride, nchunks, tiles, ords, canon);
    else if (wn == 1)
        hipLaunchKernelGGL((rawsum_kernel<1, true>), dim3((unsigned)gx), dim3(256), 0, s, raw, rawstride, nchunks, tiles, ords, canon);
    else if (!acc64)
        hipLaunchKernelGGL((rawsum_kernel<2, false>), dim3((unsigned)gx), dim3(256), 0, s, raw, rawstride, nchunks, tiles, ords, canon);
    else
        hipLaunchKernelGGL((rawsum_kernel<2, true>), dim3((unsigned)gx), dim3(256), 0, s, raw, rawstride, nchunks, tiles, ords, canon);
    return hipGetLastError();
}

hipError_t launch_chunksum(const SetRed *sets, const SetRed &set0, int nsets, int64_t entries, hipStream_t s) {
    int64_t gx = (entries + 255) / 256;
    if (gx > 16384) gx = 16384;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(chunksum_kernel, dim3((unsigned)gx, (unsigned)nsets), dim3(256), 0, s, sets, set0, entries);
    return hipGetLastError();
}

template <int NT, int EPT>
static void launch_reduce_nt(const RedArgs &a, dim3 grid, int lds_bytes, hipStream_t s) {
    const dim3 block(NT);
    if constexpr (EPT == 1) {
        // launches whose top order is 7 or more
        switch (a.d0) {
            case 6: hipLaunchKernelGGL((reduce_kernel<6, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
            case 7: hipLaunchKernelGGL((reduce_kernel<7, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
            case 8: hipLaunchKernelGGL((reduce_kernel<8, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
            case 9: hipLaunchKernelGGL((reduce_kernel<9, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
            default: hipLaunchKernelGGL((reduce_kernel<10, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        }
        return;
    }
    switch (a.d0) {
        case 2: hipLaunchKernelGGL((reduce_kernel<2, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 3: hipLaunchKernelGGL((reduce_kernel<3, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 4: hipLaunchKernelGGL((reduce_kernel<4, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 5: hipLaunchKernelGGL((reduce_kernel<5, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 6: hipLaunchKernelGGL((reduce_kernel<6, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 7: hipLaunchKernelGGL((reduce_kernel<7, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 8: hipLaunchKernelGGL((reduce_kernel<8, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        case 9: hipLaunchKernelGGL((reduce_kernel<9, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
        default: hipLaunchKernelGGL((reduce_kernel<10, NT, EPT>), grid, block, (size_t)lds_bytes, s, a); break;
    }
}

// With the recursion up to order 7 and beyond, every entry runs 56 to 501
// terms, and the blocks are few: one entry per thread, and a block's entries
// over as many work-groups as it fills.  Elsewhere four entries per thread
// and one work-group per block.
// wide_in: -1 to decide from the launch's orders, else the layout of the
// pair of orders this launch was split from
static hipError_t launch_reduce_impl(const RedArgs &a0, int nsets, int lds_bytes, int block_elems, int wide_in,
                                     hipStream_t s) {
    if (a0.d0 < 2 || a0.d0 > MAXD || block_elems < 1) return hipErrorInvalidValue;
    RedArgs a = a0;
    const int top = a.d0 + (a.nords == 2 ? 1 : 0);
    const bool wide = wide_in >= 0 ? wide_in != 0 : (a.recursion && top >= FIRST_POSITION_MIN_D && a.d0 >= 6);
    const int nt = wide ? (block_elems >= 256 ? 256 : 64) : (block_elems <= 64 * RED_EPT ? 64 : 256);
    const int64_t be1 = (int64_t)block_elems * a.b;  // entries per block of order d0 + 1
    // several entries per lane only in launches whose top order is 7 or more
    if (!wide || a.q0 < 1) a.q0 = 1;
    if (!wide || a.q1 < 1) a.q1 = 1;
    if (a.nords == 2 && (a.q0 > 1 || a.q1 > 1)) {
        // an order in the multi-entry form is a launch of its own
        RedArgs a1 = a, a2 = a;
        a1.nords = 1;
        a1.nbtot = a1.nb0;
        a1.q1 = 1;
        a1.gstaged = a.gstaged & 1;
        a2.ords = a.ords + 1;
        a2.nords = 1;
        a2.d0 = a.d0 + 1;
        a2.nb0 = a2.nbtot = a.nbtot - a.nb0;
        a2.q0 = a.q1;
        a2.q1 = 1;
        a2.gstaged = (a.gstaged >> 1) & 1;
        // the other order keeps the pair's one-entry-per-thread layout, or,
        // at order 6 and below, takes the layout of its own order
        const hipError_t e = launch_reduce_impl(a1, nsets, lds_bytes, block_elems, a1.d0 <= 6 ? -1 : (wide ? 1 : 0), s);
        if (e != hipSuccess) return e;
        return launch_reduce_impl(a2, nsets, lds_bytes, (int)be1, wide ? 1 : 0, s);
    }
    if (a.q0 > 1) {
        // b^qe entries per lane: qe = 2 only for b = 2 (4 entries), else 1;
        // staged sub-blocks only at b = 2, orders 7 and 8
        if (block_elems % a.q0) return hipErrorInvalidValue;
        const int ge = (a.q0 == a.b) ? 1 : (a.b == 2 && a.q0 == 4 ? 2 : 0);
        const int st = a.gstaged & 1;
        if (!ge || a.b < 2 || a.b > 4 || a.d0 < FIRST_POSITION_MIN_D) return hipErrorInvalidValue;
        // a staged launch keeps three waves' sums in its staged sub-blocks' LDS
        if (st && a.base_off < 3 * 4 * 64 * (int)sizeof(double)) return hipErrorInvalidValue;
        const int64_t per = 64 * (int64_t)a.q0;  // 64 lanes' entries per work-group
        a.sl0 = (int32_t)((block_elems + per - 1) / per);
        int64_t gg = a.nb0 * a.sl0;
        if (gg > 65535) gg = 65535;
        if (gg < 1) gg = 1;
        const dim3 ggrid((unsigned)gg, (unsigned)nsets);
        const int key = a.d0 * 1000 + a.b * 100 + ge * 10 + st;
        switch (key) {
#define CUM_GATHER(D, B, E, ST) \
    case D * 1000 + B * 100 + E * 10 + ST: \
        hipLaunchKernelGGL((gather_kernel<D, B, E, ST != 0>), ggrid, dim3(256), (size_t)lds_bytes, s, a); \
        break;
            CUM_GATHER(7, 2, 1, 1) CUM_GATHER(8, 2, 2, 1)
            CUM_GATHER(9, 2, 1, 0) CUM_GATHER(10, 2, 2, 0)
            CUM_GATHER(7, 3, 1, 0) CUM_GATHER(8, 3, 1, 0) CUM_GATHER(9, 3, 1, 0) CUM_GATHER(10, 3, 1, 0)
            CUM_GATHER(7, 4, 1, 0) CUM_GATHER(8, 4, 1, 0) CUM_GATHER(9, 4, 1, 0) CUM_GATHER(10, 4, 1, 0)
#undef CUM_GATHER
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    a.sl0 = wide ? (int32_t)((block_elems + nt - 1) / nt) : 1;
    a.sl1 = wide ? (int32_t)((be1 + nt - 1) / nt) : 1;
    int64_t gx = a.nb0 * a.sl0 + (a.nbtot - a.nb0) * a.sl1;
    if (gx > 65535) gx = 65535;
    if (gx < 1) gx = 1;
    const dim3 grid((unsigned)gx, (unsigned)nsets);
    if (wide) {
        if (nt == 64)
            launch_reduce_nt<64, 1>(a, grid, lds_bytes, s);
        else
            launch_reduce_nt<256, 1>(a, grid, lds_bytes, s);
    } else if (nt == 64) {
        launch_reduce_nt<64, RED_EPT>(a, grid, lds_bytes, s);
    } else {
        launch_reduce_nt<256, RED_EPT>(a, grid, lds_bytes, s);
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const RedArgs &a, int nsets, int lds_bytes, int block_elems, hipStream_t s) {
    return launch_reduce_impl(a, nsets, lds_bytes, block_elems, -1, s);
}

// ---------------------------------------------------------------------------
// Streaming sums.  Sums over samples are additive over disjoint sample ranges
// (the chunk decomposition of Alg. 3, eq. mapred), so a window's moment sums
// are the sum of its batches' sums, and a batch leaves the window by
// subtracting its sums again.  Sums are kept about a fixed shift c; the
// central moments follow by expanding prod_k (y_k - delta_k), y = x - c,
// delta = mean(y), over the subsets of positions.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void axpy_kernel(double *y, const double *x, double a, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        y[e] += a * x[e];
}

hipError_t launch_axpy(double *y, const double *x, double a, int64_t count, hipStream_t s) {
    int64_t g = (count + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)g), dim3(256), 0, s, y, x, a, count);
    return hipGetLastError();
}

// s1 += tb * (batch mean - c): the batch's sum of shifted samples (tb = +-t_B)
__global__ void stream_sum1_kernel(double *s1, const double *bmean, const double *shift, double tb, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) s1[i] += tb * (bmean[i] - shift[i]);
}

hipError_t launch_stream_sum1(double *s1, const double *bmean, const double *shift, double tb, int n, hipStream_t s) {
    hipLaunchKernelGGL(stream_sum1_kernel, dim3((n + 255) / 256), dim3(256), 0, s, s1, bmean, shift, tb, n);
    return hipGetLastError();
}

// delta = s1 / t (mean of the shifted data), mean = c + delta
__global__ void stream_mean_kernel(const double *s1, const double *shift, double t, int n, double *delta,
                                   double *mean) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double dl = s1[i] / t;
        delta[i] = dl;
        if (mean) mean[i] = shift[i] + dl;
    }
}

hipError_t launch_stream_mean(const double *s1, const double *shift, double t, int n, double *delta, double *mean,
                              hipStream_t s) {
    hipLaunchKernelGGL(stream_mean_kernel, dim3((n + 255) / 256), dim3(256), 0, s, s1, shift, t, n, delta, mean);
    return hipGetLastError();
}

// Central moment of the sorted variable tuple u (order D): the sum over
// position subsets A of prod_{k not in A} (-delta_{u_k}) times the moment of
// the shifted data at u_A (1 for A empty, delta for one position, the summed
// products / t otherwise, read at the rank of the sorted sub-tuple).  The
// subsets run in increasing mask order.
template <int D>
__global__ __launch_bounds__(256) void recentre_kernel(RecArgs a) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.count; e += (int64_t)gridDim.x * 256) {
        int u[D];
        double dl[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            u[k] = a.tuples[e * D + k];
            dl[k] = a.delta[u[k]];
        }
        double acc = 0.0;
        for (unsigned mask = 0; mask < (1u << D); ++mask) {
            const int m = __popc(mask);
            double coef = 1.0;
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (!(mask >> k & 1u)) coef *= -dl[k];
            double v;
            if (m == 0) {
                v = 1.0;
            } else if (m == 1) {
                v = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (mask >> k & 1u) v = dl[k];
            } else {
                int64_t rank = 0;
                int prev = 0, k2 = 0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (mask >> k & 1u) {
                        rank += c_binom.c[a.n - prev + m - k2 - 1][m - k2] - c_binom.c[a.n - u[k] + m - k2 - 1][m - k2];
                        prev = u[k];
                        ++k2;
                    }
                v = a.sums[a.off[m] + rank] / a.t;
            }
            acc += coef * v;
        }
        a.central[a.off[D] + e] = acc;
    }
}

hipError_t launch_recentre(const RecArgs &a, hipStream_t s) {
    int64_t g = (a.count + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    const dim3 grid((unsigned)g), block(256);
    switch (a.d) {
        case 2: hipLaunchKernelGGL(recentre_kernel<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(recentre_kernel<3>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(recentre_kernel<4>, grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL(recentre_kernel<5>, grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL(recentre_kernel<6>, grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL(recentre_kernel<7>, grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL(recentre_kernel<8>, grid, block, 0, s, a); break;
        case 9: hipLaunchKernelGGL(recentre_kernel<9>, grid, block, 0, s, a); break;
        case 10: hipLaunchKernelGGL(recentre_kernel<10>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Cumulant of the sorted variable tuple u (order D) from the moments of the
// shifted data (eq. cumfmom, the general formula of Section 5.3): the sum
// over every set partition of the D positions, in table order, of its weight
// (k-1)! (-1)^(k-1) (k parts) times the product over its parts B of the
// moment at u_B (delta for one position, the summed products / t otherwise).
// Cumulants of order >= 2 do not depend on the shift.
template <int D>
__global__ __launch_bounds__(256) void moebius_kernel(MoebArgs a) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.count; e += (int64_t)gridDim.x * 256) {
        int u[D];
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = a.tuples[e * D + k];
        double acc = 0.0;
        for (int z = 0; z < a.npart; ++z) {
            double prod = a.weight[z];
            for (int pt = 0; pt < D; ++pt) {
                const unsigned mask = __builtin_amdgcn_readfirstlane((int)a.parts[z * D + pt]);
                if (!mask) break;
                const int m = __popc(mask);
                double v;
                if (m == 1) {
                    v = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        if (mask >> k & 1u) v = a.delta[u[k]];
                } else {
                    int64_t rank = 0;
                    int prev = 0, k2 = 0;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        if (mask >> k & 1u) {
                            rank += c_binom.c[a.n - prev + m - k2 - 1][m - k2] -
                                    c_binom.c[a.n - u[k] + m - k2 - 1][m - k2];
                            prev = u[k];
                            ++k2;
                        }
                    v = a.sums[a.off[m] + rank] / a.t;
                }
                prod *= v;
            }
            acc += prod;
        }
        a.out[a.off[D] + e] = acc;
    }
}

hipError_t launch_moebius(const MoebArgs &a, hipStream_t s) {
    int64_t g = (a.count + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    const dim3 grid((unsigned)g), block(256);
    switch (a.d) {
        case 2: hipLaunchKernelGGL(moebius_kernel<2>, grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL(moebius_kernel<3>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(moebius_kernel<4>, grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL(moebius_kernel<5>, grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL(moebius_kernel<6>, grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL(moebius_kernel<7>, grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL(moebius_kernel<8>, grid, block, 0, s, a); break;
        case 9: hipLaunchKernelGGL(moebius_kernel<9>, grid, block, 0, s, a); break;
        case 10: hipLaunchKernelGGL(moebius_kernel<10>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unfold to dense: entry i is read at the stored position of sorted(i).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void unfold_kernel(const double *blocks, int n, int d, int b, int nbar,
                                                     int64_t total, double *dense) {
    const int64_t be = ipow_dev(b, d);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int idx[MAXD];
        int64_t x = e;
        for (int k = d - 1; k >= 0; --k) {
            idx[k] = (int)(x % n);
            x /= n;
        }
        for (int k = 1; k < d; ++k) {  // insertion sort, ascending
            const int v = idx[k];
            int m = k - 1;
            while (m >= 0 && idx[m] > v) {
                idx[m + 1] = idx[m];
                --m;
            }
            idx[m + 1] = v;
        }
        int j[MAXD];
        int64_t in = 0;
        for (int k = 0; k < d; ++k) {
            j[k] = idx[k] / b;
            in = in * b + (idx[k] - j[k] * b);
        }
        dense[e] = blocks[rank_sorted(j, d, nbar) * be + in];
    }
}

hipError_t launch_unfold(const double *blocks, int n, int d, int b, double *dense, hipStream_t s) {
    int64_t total = 1;
    for (int k = 0; k < d; ++k) total *= n;
    int64_t grid = (total + 255) / 256;
    if (grid > 16384) grid = 16384;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(unfold_kernel, dim3((unsigned)grid), dim3(256), 0, s, blocks, n, d, b, (n + b - 1) / b,
                       total, dense);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// centring launchers
// ---------------------------------------------------------------------------
hipError_t launch_colsum(const double *X, int64_t t, int n, int64_t ldx, int64_t rows_per, int groups, double *part,
                         hipStream_t s, double *mm) {
    if (mm)
        hipLaunchKernelGGL(colsum_kernel<true>, dim3(groups), dim3(256), 0, s, X, t, n, ldx, rows_per, part, mm);
    else
        hipLaunchKernelGGL(colsum_kernel<false>, dim3(groups), dim3(256), 0, s, X, t, n, ldx, rows_per, part, mm);
    return hipGetLastError();
}

hipError_t launch_scale_f32(const float *X, int64_t t, int n, int64_t rows_per, int groups, double *part, double *mm,
                            double *scale, hipStream_t s) {
    hipLaunchKernelGGL(colminmax_f32_kernel, dim3(groups), dim3(256), 0, s, X, t, n, rows_per, part, mm);
    hipLaunchKernelGGL(scale_about_zero_kernel, dim3(n), dim3(256), 0, s, mm, groups, n, scale);
    return hipGetLastError();
}

hipError_t launch_mean(const double *part, int groups, int n, int64_t t, double *mean, hipStream_t s,
                       const double *mm, double *scale, const double *center) {
    if (mm && scale)
        hipLaunchKernelGGL(mean_kernel<true>, dim3(n), dim3(256), 0, s, part, groups, n, t, mean, mm, scale, center);
    else
        hipLaunchKernelGGL(mean_kernel<false>, dim3(n), dim3(256), 0, s, part, groups, n, t, mean, nullptr, nullptr,
                           nullptr);
    return hipGetLastError();
}

hipError_t launch_center(const double *X, int64_t t, int n, int64_t ldx, const double *mean, void *Xc, int prec,
                         hipStream_t s) {
    int64_t grid = (t * n + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (prec == P_F64)
        hipLaunchKernelGGL(center_kernel<double>, dim3((unsigned)grid), dim3(256), 0, s, X, t, n, ldx, mean,
                           (double *)Xc);
    else
        hipLaunchKernelGGL(center_kernel<float>, dim3((unsigned)grid), dim3(256), 0, s, X, t, n, ldx, mean,
                           (float *)Xc);
    return hipGetLastError();
}

hipError_t launch_batch_colsum(const CenterSet *sets, int nsets, int max_groups, int n, hipStream_t s, bool mm) {
    if (mm)
        hipLaunchKernelGGL(batch_colsum_kernel<true>, dim3(max_groups, nsets), dim3(256), 0, s, sets, n);
    else
        hipLaunchKernelGGL(batch_colsum_kernel<false>, dim3(max_groups, nsets), dim3(256), 0, s, sets, n);
    return hipGetLastError();
}

hipError_t launch_batch_mean(const CenterSet *sets, int nsets, int n, hipStream_t s, bool mm) {
    if (mm)
        hipLaunchKernelGGL(batch_mean_kernel<true>, dim3(n, nsets), dim3(256), 0, s, sets, n);
    else
        hipLaunchKernelGGL(batch_mean_kernel<false>, dim3(n, nsets), dim3(256), 0, s, sets, n);
    return hipGetLastError();
}

hipError_t launch_stamp(unsigned long long *where, hipStream_t s) {
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, s, where);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch memory of the allocation-free entry point: an array in each
// GPU's copy of the code object, held until the process ends.  Host code
// never uses the array's name as an address (on the host it only stands for
// the symbol); it uses the device address looked up below.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// The device address of the current GPU's copy of `scratch`, looked up once
// per device with that device current and kept.  Callers hold the library's
// lock.  Returns the HIP status of the lookup.
hipError_t noalloc_scratch(void **out) {
    static void *ptr[NOALLOC_MAX_DEVICES] = {nullptr};
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace cum
