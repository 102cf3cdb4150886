// gfx950 kernels: centring, block moment contraction on matrix cores,
// fixed-order chunk reduction fused with the cumulant recursion, unfold.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

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
__device__ __forceinline__ void colsum_body(const double *X, int64_t t, int n, int64_t ldx, int64_t rows_per, int g,
                                            double *part) {
    __shared__ double ss[256], cs[256];
    const int tid = threadIdx.x;
    const int R = 256 / n;
    const int col = tid % n, rl = tid / n;
    double s = 0.0, c = 0.0;
    const int64_t r0 = (int64_t)g * rows_per;
    const int64_t r1 = min(t, r0 + rows_per);
    if (rl < R)
        for (int64_t r = r0 + rl; r < r1; r += R) neumaier(s, c, X[r * ldx + col]);
    ss[tid] = s;
    cs[tid] = c;
    __syncthreads();
    if (tid < n) {
        double S = 0.0, C = 0.0;
        for (int k = 0; k < R; ++k) {
            neumaier(S, C, ss[k * n + tid]);
            neumaier(S, C, cs[k * n + tid]);
        }
        part[((int64_t)g * n + tid) * 2] = S;
        part[((int64_t)g * n + tid) * 2 + 1] = C;
    }
}

__global__ __launch_bounds__(256) void colsum_kernel(const double *X, int64_t t, int n, int64_t ldx,
                                                     int64_t rows_per, double *part) {
    colsum_body(X, t, n, ldx, rows_per, blockIdx.x, part);
}

__device__ __forceinline__ void mean_body(const double *part, int groups, int n, int64_t t, double *mean) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double S = 0.0, C = 0.0;
        for (int g = 0; g < groups; ++g) {
            neumaier(S, C, part[((int64_t)g * n + i) * 2]);
            neumaier(S, C, part[((int64_t)g * n + i) * 2 + 1]);
        }
        mean[i] = (S + C) / (double)t;
    }
}

__global__ __launch_bounds__(256) void mean_kernel(const double *part, int groups, int n, int64_t t,
                                                   double *mean) {
    mean_body(part, groups, n, t, mean);
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

__global__ __launch_bounds__(256) void batch_colsum_kernel(const CenterSet *sets, int n) {
    const CenterSet cs = sets[blockIdx.y];
    if ((int)blockIdx.x >= cs.groups) return;
    colsum_body(cs.X, cs.t, n, n, cs.rows_per, blockIdx.x, cs.part);
}

__global__ __launch_bounds__(256) void batch_mean_kernel(const CenterSet *sets, int n) {
    const CenterSet cs = sets[blockIdx.x];
    mean_body(cs.part, cs.groups, n, cs.t, cs.mean);
}

template <typename T>
__global__ __launch_bounds__(256) void batch_center_kernel(const CenterSet *sets, int n) {
    const CenterSet cs = sets[blockIdx.y];
    const int64_t total = cs.t * n;
    T *Xc = reinterpret_cast<T *>(cs.Xc);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t l = e / n;
        const int i = (int)(e - l * n);
        Xc[e] = (T)(cs.X[l * n + i] - cs.mean[i]);
    }
}

__global__ void stamp_kernel(unsigned long long *where) {
    if (threadIdx.x == 0) *where = wall_clock64();
}

// ---------------------------------------------------------------------------
// Block moment contraction.
//
// A work item is one work-group tile (2 x 2 waves, each WM x WN blocks of
// 32 x 32 entries) of one order's (prefix rows) x (suffix columns) product,
// over one chunk of samples.  Samples are staged through LDS in stages of kt
// samples (double-buffered, register prefetch, contiguous global reads of the
// row-major data); every lane forms its Khatri-Rao operand values from the
// staged samples: the product of the prefix (or suffix) variables of its row
// (or column).  32 x 32 blocks with no stored entry (v > w everywhere) are
// skipped per wave.  The chunk's sums go, in FP64, to the chunk's slice of
// the partial buffer at each entry's block-storage offset.
// ---------------------------------------------------------------------------
template <int PREC>
struct PT;
template <>
struct PT<P_F64> {
    typedef double T;
    enum { KSTEP = 4, UMAX = 16, FLUSH = 0 };
};
template <>
struct PT<P_F32> {
    typedef float T;
    enum { KSTEP = 2, UMAX = 16, FLUSH = 64 };
};
template <>
struct PT<P_BF16X2> {
    typedef float T;
    enum { KSTEP = 16, UMAX = 16, FLUSH = 256 };
};
template <>
struct PT<P_BF16X3> {
    typedef float T;
    enum { KSTEP = 16, UMAX = 16, FLUSH = 256 };
};

int lds_bytes_moment(int prec, int n, int kt) {
    if (prec >= P_BF16X2) return 2 * (n + 1) * (kt + 4) * 4;
    return 2 * kt * (n + 1) * (prec == P_F64 ? 8 : 4);
}

__device__ __forceinline__ void split2(const float *v, bf8 &hi, bf8 &lo) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const __bf16 h = (__bf16)v[k];
        hi[k] = h;
        lo[k] = (__bf16)(v[k] - (float)h);
    }
}

__device__ __forceinline__ void split3(const float *v, bf8 &hi, bf8 &mid, bf8 &lo) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const __bf16 h = (__bf16)v[k];
        const float r = v[k] - (float)h;
        const __bf16 m = (__bf16)r;
        hi[k] = h;
        mid[k] = m;
        lo[k] = (__bf16)(r - (float)m);
    }
}

template <int PREC, int WM, int WN, int P, int Q>
__device__ __forceinline__ void moment_item(const MomentArgs &a, const Item &item, const TileDev &tile,
                                            const OrderDev &od, const SetDev &sd, typename PT<PREC>::T *xs,
                                            const int *lpos, int wave) {
    typedef typename PT<PREC>::T T;
    constexpr bool TRANS = PREC >= P_BF16X2;  // LDS as [variable][sample]
    constexpr int RH = (PREC == P_F64) ? 2 : 1; // operand rows per lane per 32-block
    constexpr int UMAX = PT<PREC>::UMAX;
    const int n = a.n, kt = a.kt, tid = threadIdx.x, lane = tid & 63;
    const int wy = wave >> 1, wx = wave & 1;
    const int ld = n + 1, ldt = kt + 4;
    const int buf_elems = TRANS ? (n + 1) * ldt : kt * ld;
    const int rbase = tile.row0 + wy * (WM * 32), cbase = tile.col0 + wx * (WN * 32);

    // which of this wave's 32 x 32 blocks hold stored entries (wave-uniform)
    unsigned vmask = 0;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int r0 = rbase + i * 32, c0 = cbase + j * 32;
            if (r0 < od.nr && c0 < od.nc && od.rb_vmin[r0 >> 5] <= od.cb_wmax[c0 >> 5]) vmask |= 1u << (i * WN + j);
        }

    // operand offsets into LDS of this lane's rows and columns
    int roff[WM][RH][P], coff[WN][RH][Q];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            const int r = rbase + i * 32 + (PREC == P_F64 ? h * 16 + (lane & 15) : (lane & 31));
            Feat f;
            if (r < od.nr)
                f = od.rows[r];
            else
                for (int q = 0; q < MAXH; ++q) f.var[q] = (uint8_t)n;
#pragma unroll
            for (int q = 0; q < P; ++q) roff[i][h][q] = TRANS ? f.var[q] * ldt : f.var[q];
        }
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            const int c = cbase + j * 32 + (PREC == P_F64 ? h * 16 + (lane & 15) : (lane & 31));
            Feat f;
            if (c < od.nc)
                f = od.cols[c];
            else
                for (int q = 0; q < MAXH; ++q) f.var[q] = (uint8_t)n;
#pragma unroll
            for (int q = 0; q < Q; ++q) coff[j][h][q] = TRANS ? f.var[q] * ldt : f.var[q];
        }

    // accumulators
    d4 acc64[WM][WN][RH][RH];
    f16v acc[WM][WN];
    double dacc[WM][WN][16];
    if constexpr (PREC == P_F64) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int h = 0; h < RH; ++h)
#pragma unroll
                    for (int g = 0; g < RH; ++g) acc64[i][j][h][g] = d4{0.0, 0.0, 0.0, 0.0};
    } else {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) {
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    acc[i][j][k] = 0.f;
                    dacc[i][j][k] = 0.0;
                }
            }
    }

    const int64_t s0 = (int64_t)item.chunk * sd.chunk_len;
    const int64_t s1 = min(sd.t, s0 + sd.chunk_len);
    const int nk = (int)((s1 - s0 + kt - 1) / kt);
    const T *X = reinterpret_cast<const T *>(sd.X);

    T pf[UMAX];
    auto gload = [&](int k) {
        const int64_t sb = s0 + (int64_t)k * kt;
        const T *src = X + sb * n;
        const int64_t left = s1 - sb;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
            pf[u] = T(0);
            if (lpos[u] >= 0 && (lpos[u] >> 20) < left) pf[u] = src[tid + 256 * u];
        }
    };
    auto lstore = [&](int buf) {
        T *dst = xs + buf * buf_elems;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (lpos[u] >= 0) dst[lpos[u] & 0xFFFFF] = pf[u];
    };

    __syncthreads();  // the previous item's readers are done with both buffers
    gload(0);
    lstore(0);
    __syncthreads();

    const int flush_every = (PT<PREC>::FLUSH > 0) ? max(1, (int)PT<PREC>::FLUSH / kt) : 0;
    int since_flush = 0;

    for (int k = 0; k < nk; ++k) {
        const int buf = k & 1;
        if (k + 1 < nk) gload(k + 1);
        const T *xb = xs + buf * buf_elems;
        if (vmask) {
            if constexpr (PREC == P_F64) {
                for (int kk = 0; kk < kt; kk += 4) {
                    const double *xr = xb + (kk + (lane >> 4)) * ld;
                    double A[WM][2], B[WN][2];
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            double v = xr[roff[i][h][0]];
#pragma unroll
                            for (int q = 1; q < P; ++q) v *= xr[roff[i][h][q]];
                            A[i][h] = v;
                        }
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            double v = xr[coff[j][h][0]];
#pragma unroll
                            for (int q = 1; q < Q; ++q) v *= xr[coff[j][h][q]];
                            B[j][h] = v;
                        }
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int j = 0; j < WN; ++j)
                            if (vmask >> (i * WN + j) & 1u) {
#pragma unroll
                                for (int h = 0; h < 2; ++h)
#pragma unroll
                                    for (int g = 0; g < 2; ++g)
                                        acc64[i][j][h][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                            A[i][h], B[j][g], acc64[i][j][h][g], 0, 0, 0);
                            }
                }
            } else if constexpr (PREC == P_F32) {
                for (int kk = 0; kk < kt; kk += 2) {
                    const float *xr = xb + (kk + (lane >> 5)) * ld;
                    float A[WM], B[WN];
#pragma unroll
                    for (int i = 0; i < WM; ++i) {
                        float v = xr[roff[i][0][0]];
#pragma unroll
                        for (int q = 1; q < P; ++q) v *= xr[roff[i][0][q]];
                        A[i] = v;
                    }
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        float v = xr[coff[j][0][0]];
#pragma unroll
                        for (int q = 1; q < Q; ++q) v *= xr[coff[j][0][q]];
                        B[j] = v;
                    }
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int j = 0; j < WN; ++j)
                            if (vmask >> (i * WN + j) & 1u)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[i], B[j], acc[i][j], 0, 0, 0);
                }
            } else {
                for (int kk = 0; kk < kt; kk += 16) {
                    const float *xr = xb + kk + 8 * (lane >> 5);
                    constexpr int NS = (PREC == P_BF16X3) ? 3 : 2;
                    bf8 As[WM][NS], Bs[WN][NS];
#pragma unroll
                    for (int i = 0; i < WM; ++i) {
                        f4 v0 = *reinterpret_cast<const f4 *>(xr + roff[i][0][0]);
                        f4 v1 = *reinterpret_cast<const f4 *>(xr + roff[i][0][0] + 4);
#pragma unroll
                        for (int q = 1; q < P; ++q) {
                            v0 *= *reinterpret_cast<const f4 *>(xr + roff[i][0][q]);
                            v1 *= *reinterpret_cast<const f4 *>(xr + roff[i][0][q] + 4);
                        }
                        float v[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
                        if constexpr (NS == 3)
                            split3(v, As[i][0], As[i][1], As[i][2]);
                        else
                            split2(v, As[i][0], As[i][1]);
                    }
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        f4 v0 = *reinterpret_cast<const f4 *>(xr + coff[j][0][0]);
                        f4 v1 = *reinterpret_cast<const f4 *>(xr + coff[j][0][0] + 4);
#pragma unroll
                        for (int q = 1; q < Q; ++q) {
                            v0 *= *reinterpret_cast<const f4 *>(xr + coff[j][0][q]);
                            v1 *= *reinterpret_cast<const f4 *>(xr + coff[j][0][q] + 4);
                        }
                        float v[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
                        if constexpr (NS == 3)
                            split3(v, Bs[j][0], Bs[j][1], Bs[j][2]);
                        else
                            split2(v, Bs[j][0], Bs[j][1]);
                    }
                    // cross products of the split terms: all 4 for two terms; for three
                    // terms the 6 of combined weight >= 2^-16 (hh, hm, mh, hl, lh, mm)
                    constexpr int NP = (NS == 3) ? 6 : 4;
                    constexpr int PA[4] = {0, 0, 1, 1};          // hh, hl, lh, ll
                    constexpr int PB[4] = {0, 1, 0, 1};
                    constexpr int PA3[6] = {0, 0, 1, 0, 2, 1};    // hh, hm, mh, hl, lh, mm
                    constexpr int PB3[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
                    for (int pr = NP - 1; pr >= 0; --pr) {
#pragma unroll
                        for (int i = 0; i < WM; ++i)
#pragma unroll
                            for (int j = 0; j < WN; ++j)
                                if (vmask >> (i * WN + j) & 1u) {
                                    const int ia = (NS == 3) ? PA3[pr] : PA[pr & 3];
                                    const int ib = (NS == 3) ? PB3[pr] : PB[pr & 3];
                                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(As[i][ia], Bs[j][ib],
                                                                                        acc[i][j], 0, 0, 0);
                                }
                    }
                }
            }
        }
        if (k + 1 < nk) lstore(buf ^ 1);
        __syncthreads();
        if constexpr (PREC != P_F64) {
            if (++since_flush >= flush_every || k + 1 == nk) {
                since_flush = 0;
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            dacc[i][j][q] += (double)acc[i][j][q];
                            acc[i][j][q] = 0.f;
                        }
            }
        }
    }

    // epilogue: write this chunk's sums at their block-storage offsets
    double *dst = sd.partial + (int64_t)item.chunk * sd.stride + od.out_off;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (!(vmask >> (i * WN + j) & 1u)) continue;
            if constexpr (PREC == P_F64) {
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const int c = cbase + j * 32 + g * 16 + (lane & 15);
                    if (c >= od.nc) continue;
                    const Feat fc = od.cols[c];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int r = rbase + i * 32 + h * 16 + 4 * q + (lane >> 4);
                            if (r >= od.nr) continue;
                            const Feat fr = od.rows[r];
                            if (fr.blk <= fc.blk)
                                dst[fr.addr + fc.addr + od.H[(int64_t)fr.blk * od.nbar + fc.blk]] =
                                    acc64[i][j][h][g][q];
                        }
                }
            } else {
                const int c = cbase + j * 32 + (lane & 31);
                if (c >= od.nc) continue;
                const Feat fc = od.cols[c];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int r = rbase + i * 32 + (q >> 2) * 8 + (lane >> 5) * 4 + (q & 3);
                    if (r >= od.nr) continue;
                    const Feat fr = od.rows[r];
                    if (fr.blk <= fc.blk)
                        dst[fr.addr + fc.addr + od.H[(int64_t)fr.blk * od.nbar + fc.blk]] = dacc[i][j][q];
                }
            }
        }
}

template <int PREC, int WM, int WN>
__global__ __launch_bounds__(256, 2) void moment_kernel(MomentArgs a) {
    typedef typename PT<PREC>::T T;
    constexpr bool TRANS = PREC >= P_BF16X2;
    constexpr int UMAX = PT<PREC>::UMAX;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    const int n = a.n, kt = a.kt, tid = threadIdx.x;
    const int ld = n + 1, ldt = kt + 4;
    const int buf_elems = TRANS ? (n + 1) * ldt : kt * ld;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // the zero column (row, transposed) of both stages is never overwritten
    if (TRANS) {
        for (int i = tid; i < 2 * ldt; i += 256) xs[(i / ldt) * buf_elems + n * ldt + (i % ldt)] = T(0);
    } else {
        for (int i = tid; i < 2 * kt; i += 256) xs[(i / kt) * buf_elems + (i % kt) * ld + n] = T(0);
    }
    // this thread's share of one LDS stage: (sample row << 20) | LDS offset
    int lpos[UMAX];
    const int tile_elems = kt * n;
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
        const int e = tid + 256 * u;
        if (e < tile_elems) {
            const int row = e / n, col = e - (e / n) * n;
            lpos[u] = (row << 20) | (TRANS ? col * ldt + row : row * ld + col);
        } else {
            lpos[u] = -1;
        }
    }

    for (int64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const Item item = a.items[it];
        if (item.tile < 0) continue;
        const TileDev tile = a.tiles[item.tile];
        const OrderDev od = a.ords[tile.ord];
        const SetDev sd = a.sets ? a.sets[item.set] : a.set0;
        switch (od.p * 8 + od.q) {
            case 1 * 8 + 1: moment_item<PREC, WM, WN, 1, 1>(a, item, tile, od, sd, xs, lpos, wave); break;
            case 1 * 8 + 2: moment_item<PREC, WM, WN, 1, 2>(a, item, tile, od, sd, xs, lpos, wave); break;
            case 2 * 8 + 2: moment_item<PREC, WM, WN, 2, 2>(a, item, tile, od, sd, xs, lpos, wave); break;
            case 2 * 8 + 3: moment_item<PREC, WM, WN, 2, 3>(a, item, tile, od, sd, xs, lpos, wave); break;
            case 3 * 8 + 3: moment_item<PREC, WM, WN, 3, 3>(a, item, tile, od, sd, xs, lpos, wave); break;
            case 3 * 8 + 4: moment_item<PREC, WM, WN, 3, 4>(a, item, tile, od, sd, xs, lpos, wave); break;
            case 4 * 8 + 4: moment_item<PREC, WM, WN, 4, 4>(a, item, tile, od, sd, xs, lpos, wave); break;
            default: break;
        }
    }
}

template <int PREC>
static hipError_t launch_moment_prec(int shape, const MomentArgs &a, int grid, hipStream_t s) {
    const int lds = lds_bytes_moment(PREC, a.n, a.kt);
    switch (shape) {
        case TS_1x1:
            hipLaunchKernelGGL((moment_kernel<PREC, 1, 1>), dim3(grid), dim3(256), lds, s, a);
            break;
        case TS_2x1:
            hipLaunchKernelGGL((moment_kernel<PREC, 2, 1>), dim3(grid), dim3(256), lds, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_moment(int prec, int shape, const MomentArgs &a, int grid, hipStream_t s) {
    switch (prec) {
        case P_F64: return launch_moment_prec<P_F64>(shape, a, grid, s);
        case P_F32: return launch_moment_prec<P_F32>(shape, a, grid, s);
        case P_BF16X2: return launch_moment_prec<P_BF16X2>(shape, a, grid, s);
        default: return launch_moment_prec<P_BF16X3>(shape, a, grid, s);
    }
}

// ---------------------------------------------------------------------------
// Chunk reduction fused with the cumulant recursion (Alg. 3's reduce; Alg. 4
// and Alg. 5; eq. cum_r of Section 3.2).  One work-group per stored block j
// of one dataset: the block's sub-tuples j_S (S = a set of 2..d-2 positions,
// sorted because j is) get their lower-order block offsets once, in LDS;
// then each entry sums its chunk partials in chunk order, divides by t, and
// subtracts the sum over partitions of products of lower cumulants read at
// (j_S, i_S).  All FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(RedArgs a) {
    __shared__ int64_t base[1 << MAXD];
    __shared__ int tup[MAXD];
    __shared__ double *kap[MAXD - 1];
    const int tid = threadIdx.x;
    const SetRed sr = a.sets ? a.sets[blockIdx.y] : a.set0;
#pragma unroll
    for (int k = 0; k < MAXD - 1; ++k)
        if (tid == k) kap[k] = sr.kappa[k];
    const double *partial = sr.partial;
    const int64_t stride = sr.stride, nchunks = sr.nchunks;
    const double tt = (double)sr.t;
    for (int64_t gb = blockIdx.x; gb < a.nbtot; gb += gridDim.x) {
        const int oi = gb < a.nb0 ? 0 : 1;
        const int64_t B = oi ? gb - a.nb0 : gb;
        const RedOrder ro = a.ords[oi];
        const int d = ro.d, b = ro.b;
        const int64_t be = ipow_dev(b, d);
        __syncthreads();
        if (tid < d) tup[tid] = ro.tuples[B * d + tid];
        __syncthreads();
        const bool rec = a.recursion && d >= 4;
        if (rec) {
            for (int mask = tid; mask < (1 << d); mask += 256) {
                const int m = __popc(mask);
                if (m < 2 || m > d - 2) continue;
                int u[MAXD], mm = 0;
                for (int k = 0; k < d; ++k)
                    if (mask >> k & 1) u[mm++] = tup[k];
                base[mask] = rank_sorted(u, m, ro.nbar) * ipow_dev(b, m);
            }
        }
        __syncthreads();
        double *out = kap[d - 2];
        for (int64_t o = tid; o < be; o += 256) {
            const int64_t e = B * be + o;
            const double *pp = partial + ro.out_off + e;
            double S = 0.0;
            for (int64_t c = 0; c < nchunks; ++c) S += pp[c * stride];
            const double M = S / tt;
            double res = M;
            if (rec) {
                int r[MAXD];
                int64_t oo = o;
                for (int k = d - 1; k >= 0; --k) {
                    r[k] = (int)(oo % b);
                    oo /= b;
                }
                double sum = 0.0;
                for (int z = 0; z < ro.npart; ++z) {
                    double prod = 1.0;
                    for (int pt = 0; pt < MAXPARTS; ++pt) {
                        const int mask = ro.parts[z * MAXPARTS + pt];
                        if (!mask) break;
                        int64_t flat = 0;
                        for (int k = 0; k < d; ++k)
                            if (mask >> k & 1) flat = flat * b + r[k];
                        prod *= kap[__popc(mask) - 2][base[mask] + flat];
                    }
                    sum += prod;
                }
                res = M - sum;
            }
            out[e] = res;
        }
        if (sr.stamp && tid == 0) atomicMax(sr.stamp, (unsigned long long)wall_clock64());
    }
}

hipError_t launch_reduce(const RedArgs &a, int nsets, hipStream_t s) {
    int64_t gx = a.nbtot;
    if (gx > 65535) gx = 65535;
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)gx, (unsigned)nsets), dim3(256), 0, s, a);
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
                         hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3(groups), dim3(256), 0, s, X, t, n, ldx, rows_per, part);
    return hipGetLastError();
}

hipError_t launch_mean(const double *part, int groups, int n, int64_t t, double *mean, hipStream_t s) {
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, part, groups, n, t, mean);
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

hipError_t launch_batch_colsum(const CenterSet *sets, int nsets, int max_groups, int n, hipStream_t s) {
    hipLaunchKernelGGL(batch_colsum_kernel, dim3(max_groups, nsets), dim3(256), 0, s, sets, n);
    return hipGetLastError();
}

hipError_t launch_batch_mean(const CenterSet *sets, int nsets, int n, hipStream_t s) {
    hipLaunchKernelGGL(batch_mean_kernel, dim3(nsets), dim3(256), 0, s, sets, n);
    return hipGetLastError();
}

hipError_t launch_batch_center(const CenterSet *sets, int nsets, int n, int prec, int blocks_per_set, hipStream_t s) {
    if (prec == P_F64)
        hipLaunchKernelGGL(batch_center_kernel<double>, dim3(blocks_per_set, nsets), dim3(256), 0, s, sets, n);
    else
        hipLaunchKernelGGL(batch_center_kernel<float>, dim3(blocks_per_set, nsets), dim3(256), 0, s, sets, n);
    return hipGetLastError();
}

hipError_t launch_stamp(unsigned long long *where, hipStream_t s) {
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, s, where);
    return hipGetLastError();
}

}  // namespace cum
