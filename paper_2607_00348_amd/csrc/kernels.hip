// HIP kernels of the TLS search for gfx950 (MI355X) and their launchers.
//
// Per trial period P (Sect. 2.3 of the GTLS paper):
//   k_fold_sort   one 1024-thread workgroup per period: phase fold on raw
//                 times (Sect. 2.3.1), 32-bit fixed-point phase keys, a
//                 4-pass stable LSD radix sort with wave-ballot ranking, a
//                 tie-fix of equal keys by full FP64 phase then input index,
//                 then the cyclic padding (Sect. 2.3.2): the folded weights
//                 and residuals gathered in phase order for n + D_max
//                 positions, and (moving-average depth only) exact integer
//                 prefix sums of 1 - y over the padded curve (Sect. 2.3.3).
//   k_slide       one 256-thread workgroup per (period, duration): the
//                 transit template resampled to D points is slid over the
//                 padded curve (Sect. 2.3.4, in-transit term); each lane owns
//                 16 consecutive windows whose correlation sums run in
//                 registers over a padded, bank-conflict-free LDS tile.  The
//                 per-window depth and chi2 improvement are reduced to the
//                 first best window.
//   k_reduce      per period: first best over durations -> chi2(P), depth, T0.
//   k_sde_*       SR, SDE_raw, running-median detrend, argmax (Sect. 2.4).
//
// Every floating-point expression that decides a result is written to give
// the same IEEE operations in the same order as a plain sequential
// evaluation (the library is compiled with -ffp-contract=off): each window's
// correlation is one fused multiply-add per template point in ascending
// order, so FP64 results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "gtls_impl.hpp"

namespace gtls {
namespace {

constexpr double kDay = 86400.0;
constexpr double kTwo53 = 9007199254740992.0;
constexpr double kTwo32 = 4294967296.0;

// Layout of the per-curve scalar block (uint64 slots).
enum MiscSlot { kChi2Null = 0, kTminOrd = 1, kWminBits = 2, kWmaxBits = 3, kEvals = 4, kMacs = 5, kMiscSlots = 8 };

__device__ __forceinline__ uint64_t ordered_bits(double x) {
    uint64_t b = __double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered(uint64_t o) {
    uint64_t b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ double phase_of(double t, double period) {
    double x = t / period;
    return x - floor(x);
}

// Duration envelope (Sect. 2.2.2) evaluated cubed: q^3 P_s^2 against k^3.
__device__ __forceinline__ bool duration_valid(double period, double dur, const gtls_params& p) {
    double q = dur / period;
    if (q > p.q_cap) return false;
    if (p.envelope) {
        double ps = period * kDay;
        double lhs = (q * q * q) * (ps * ps);
        if (lhs < p.k_min * p.k_min * p.k_min) return false;
        if (lhs > p.k_max * p.k_max * p.k_max) return false;
    }
    return true;
}

// Points inside one duration: n T/P rounded half up, clamped to [1, n].
__device__ __forceinline__ int64_t points_in(int64_t n, double period, double dur) {
    double q = dur / period;
    double d = floor((double)n * q + 0.5);
    if (d < 1.0) return 1;
    if (d > (double)n) return n;
    return (int64_t)d;
}

// T0 step (Sect. 2.5): floor(dt0 * D), at least 1; dt0 = 0 -> every offset.
__device__ __forceinline__ int64_t t0_stride(int64_t d, double dt0) {
    if (!(dt0 > 0.0)) return 1;
    double s = floor(dt0 * (double)d);
    return s < 1.0 ? 1 : (int64_t)s;
}

// Template point k of D: linear interpolation at x = (k + 1/2)/D of the m
// samples taken at (j + 1/2)/m.
__device__ __forceinline__ double resample(const double* __restrict__ tm, int m, int64_t d, int64_t k) {
    double u = ((double)k + 0.5) * (double)m / (double)d - 0.5;
    double fl = floor(u);
    int64_t m0 = (int64_t)fl;
    if (m0 < 0) m0 = 0;
    if (m0 > m - 2) m0 = m - 2;
    double f = u - (double)m0;
    if (f < 0.0) f = 0.0;
    if (f > 1.0) f = 1.0;
    double a = tm[m0] * (1.0 - f);
    double b = tm[m0 + 1] * f;
    return a + b;
}

// Round-to-nearest-even conversion of a 128-bit integer to double.
__device__ __forceinline__ double i128_to_double(__int128 v) {
    if (v == 0) return 0.0;
    const bool neg = v < 0;
    unsigned __int128 a = neg ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
    uint64_t hi = (uint64_t)(a >> 64), lo = (uint64_t)a;
    int msb = hi ? 127 - __clzll((long long)hi) : 63 - __clzll((long long)lo);
    double r;
    if (msb <= 52) {
        r = (double)lo;
    } else {
        int shift = msb - 52;
        unsigned __int128 mant = a >> shift;
        unsigned __int128 rem = a - (mant << shift);
        unsigned __int128 half = (unsigned __int128)1 << (shift - 1);
        if (rem > half || (rem == half && (mant & 1))) mant += 1;
        if (mant == ((unsigned __int128)1 << 53)) {
            mant >>= 1;
            shift += 1;
        }
        r = ldexp((double)(uint64_t)mant, shift);
    }
    return neg ? -r : r;
}

// ------------------------------------------------------------------------
// Per-point preparation: weights, residuals w (1 - y), exact deficits
// (1 - y) 2^53, and the block-reduced min/max of w and min of t.

__global__ void k_init_misc(uint64_t* misc) {
    if (threadIdx.x == 0) {
        misc[kChi2Null] = 0;
        misc[kTminOrd] = ~0ull;
        misc[kWminBits] = ~0ull;
        misc[kWmaxBits] = 0;
        misc[kEvals] = 0;
        misc[kMacs] = 0;
    }
}

__global__ __launch_bounds__(256) void k_prep(const double* __restrict__ t, const double* __restrict__ y,
                                              const double* __restrict__ dy, int64_t n, double* __restrict__ w,
                                              double* __restrict__ r, int64_t* __restrict__ u, uint64_t* misc) {
    __shared__ uint64_t red[3][256];
    const int tid = threadIdx.x;
    int64_t i = (int64_t)blockIdx.x * 256 + tid;
    uint64_t wmin = ~0ull, wmax = 0, tmin = ~0ull;
    if (i < n) {
        double wi = 1.0 / (dy[i] * dy[i]);
        w[i] = wi;
        r[i] = wi * (1.0 - y[i]);
        u[i] = (int64_t)((1.0 - y[i]) * kTwo53);
        wmin = wmax = (uint64_t)__double_as_longlong(wi);
        tmin = ordered_bits(t[i]);
    }
    red[0][tid] = wmin;
    red[1][tid] = wmax;
    red[2][tid] = tmin;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] = min(red[0][tid], red[0][tid + s]);
            red[1][tid] = max(red[1][tid], red[1][tid + s]);
            red[2][tid] = min(red[2][tid], red[2][tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        atomicMin((unsigned long long*)&misc[kWminBits], (unsigned long long)red[0][0]);
        atomicMax((unsigned long long*)&misc[kWmaxBits], (unsigned long long)red[1][0]);
        atomicMin((unsigned long long*)&misc[kTminOrd], (unsigned long long)red[2][0]);
    }
}

// chi2_0 = sum w (y-1)^2 in input order, Neumaier-compensated.  The terms are
// formed in parallel into LDS and summed by one lane in index order.
__global__ __launch_bounds__(256) void k_chi2_null(const double* __restrict__ y, const double* __restrict__ dy,
                                                   int64_t n, uint64_t* misc) {
    constexpr int CH = 2048;
    __shared__ double xs[CH];
    double sum = 0.0, comp = 0.0;
    for (int64_t base = 0; base < n; base += CH) {
        for (int k = threadIdx.x; k < CH; k += 256) {
            int64_t i = base + k;
            if (i < n) {
                double wi = 1.0 / (dy[i] * dy[i]);
                double d = y[i] - 1.0;
                xs[k] = wi * (d * d);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t m = min((int64_t)CH, n - base);
            for (int64_t k = 0; k < m; ++k) {
                double x = xs[k];
                double t = sum + x;
                if (fabs(sum) >= fabs(x))
                    comp += (sum - t) + x;
                else
                    comp += (x - t) + sum;
                sum = t;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) misc[kChi2Null] = (uint64_t)__double_as_longlong(sum + comp);
}

// ------------------------------------------------------------------------
// Fold + stable radix sort + tie fix + padding, one workgroup per period.

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;

struct SortArgs {
    const double* t;
    const double* r;
    const double* w;
    const int64_t* u;
    int64_t n;
    const double* periods;   // already offset to the batch's first period
    const double* durations;
    int32_t nd;
    gtls_params prm;
    uint64_t* keys_a;        // [bp][n] sorted (phase key << 32 | index)
    uint64_t* keys_b;        // [bp][n] ping-pong
    void* rpad;              // [bp][pstride] double (FP64) or float (FP32C)
    void* wpad;              // [bp][pstride] or null
    void* pfx;               // [bp][pstride + 1] __int128 (FP64) or float2 (FP32C), or null
    int64_t pstride;
    int32_t* perm_out;       // optional [bp][n] copy of the permutation
    int32_t f32;             // 1: FP32C storage of the padded curve and prefix sums
};

// Error-free sum of two floats (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ bool key_less(uint64_t a, uint64_t b, const double* __restrict__ t, double period) {
    double pa = phase_of(t[(uint32_t)a], period);
    double pb = phase_of(t[(uint32_t)b], period);
    if (pa < pb) return true;
    if (pa > pb) return false;
    return (uint32_t)a < (uint32_t)b;
}

__global__ __launch_bounds__(kSortThreads) void k_fold_sort(SortArgs a) {
    __shared__ uint32_t hist[4][256];
    __shared__ uint32_t wcnt[kSortWaves][256];
    __shared__ uint32_t dbase[256];
    __shared__ int64_t sh_dpad;
    __shared__ __int128 sh_part[kSortThreads];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int pl = blockIdx.x;
    const double period = a.periods[pl];
    const int64_t n = a.n;
    uint64_t* A = a.keys_a + (size_t)pl * n;
    uint64_t* B = a.keys_b + (size_t)pl * n;

    for (int k = tid; k < 4 * 256; k += kSortThreads) (&hist[0][0])[k] = 0;
    for (int k = tid; k < kSortWaves * 256; k += kSortThreads) (&wcnt[0][0])[k] = 0;
    __syncthreads();

    // Phase keys: floor(phi 2^32); phi < 1 so the key fits 32 bits.
    for (int64_t i = tid; i < n; i += kSortThreads) {
        double ph = phase_of(a.t[i], period);
        uint32_t key = (uint32_t)(ph * kTwo32);
        A[i] = ((uint64_t)key << 32) | (uint32_t)i;
        atomicAdd(&hist[0][key & 255u], 1u);
        atomicAdd(&hist[1][(key >> 8) & 255u], 1u);
        atomicAdd(&hist[2][(key >> 16) & 255u], 1u);
        atomicAdd(&hist[3][key >> 24], 1u);
    }
    __syncthreads();
    if (tid < 4) {
        uint32_t run = 0;
        for (int d = 0; d < 256; ++d) {
            uint32_t c = hist[tid][d];
            hist[tid][d] = run;
            run += c;
        }
    }
    __syncthreads();

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t* src = A;
    uint64_t* dst = B;
    for (int pass = 0; pass < 4; ++pass) {
        if (tid < 256) dbase[tid] = hist[pass][tid];
        __syncthreads();
        const int shift = 32 + 8 * pass;
        for (int64_t tile0 = 0; tile0 < n; tile0 += kSortTile) {
            const int64_t seg0 = tile0 + (int64_t)wave * 64 * kSortItems;
            uint64_t item[kSortItems];
            uint32_t dig[kSortItems], rnk[kSortItems];
#pragma unroll
            for (int e = 0; e < kSortItems; ++e) {
                const int64_t idx = seg0 + e * 64 + lane;
                const bool active = idx < n;
                item[e] = active ? src[idx] : 0ull;
                const uint32_t d = active ? (uint32_t)(item[e] >> shift) & 255u : 0u;
                uint64_t peers = __ballot(active);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t m = __ballot(bit);
                    peers &= bit ? m : ~m;
                }
                const uint32_t before = __popcll(peers & lt_mask);
                uint32_t cnt = 0;
                if (active) cnt = wcnt[wave][d];
                __builtin_amdgcn_wave_barrier();
                if (active && before == 0) wcnt[wave][d] = cnt + (uint32_t)__popcll(peers);
                __builtin_amdgcn_wave_barrier();
                rnk[e] = cnt + before;
                dig[e] = d;
            }
            __syncthreads();
            if (tid < 256) {
                uint32_t run = dbase[tid];
                for (int w2 = 0; w2 < kSortWaves; ++w2) {
                    uint32_t c = wcnt[w2][tid];
                    wcnt[w2][tid] = run;
                    run += c;
                }
                dbase[tid] = run;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < kSortItems; ++e) {
                const int64_t idx = seg0 + e * 64 + lane;
                const uint32_t pos = wcnt[wave][dig[e]] + rnk[e];
                if (idx < n && pos < (uint32_t)n) dst[pos] = item[e];
            }
            __syncthreads();
            for (int k = tid; k < kSortWaves * 256; k += kSortThreads) (&wcnt[0][0])[k] = 0;
            __syncthreads();
        }
        uint64_t* tmp = src;
        src = dst;
        dst = tmp;
    }
    // src == A holds the order by 32-bit key, equal keys in input order.
    // Equal 32-bit keys may hide different phases: order each run by the full
    // FP64 phase, then input index (insertion sort; runs are rare and short).
    for (int64_t k = tid; k + 1 < n; k += kSortThreads) {
        const uint32_t kk = (uint32_t)(A[k] >> 32);
        if (kk == (uint32_t)(A[k + 1] >> 32) && (k == 0 || (uint32_t)(A[k - 1] >> 32) != kk)) {
            int64_t e = k + 1;
            while (e + 1 < n && (uint32_t)(A[e + 1] >> 32) == kk) ++e;
            for (int64_t x = k + 1; x <= e; ++x) {
                uint64_t v = A[x];
                int64_t y = x;
                while (y > k && key_less(v, A[y - 1], a.t, period)) {
                    A[y] = A[y - 1];
                    --y;
                }
                A[y] = v;
            }
        }
    }
    if (tid == 0) {
        int64_t dp = 0;
        for (int j = 0; j < a.nd; ++j)
            if (duration_valid(period, a.durations[j], a.prm)) dp = max(dp, points_in(n, period, a.durations[j]));
        sh_dpad = dp;
    }
    __syncthreads();
    const int64_t npad = n + sh_dpad;
    if (a.f32) {
        float* rp = (float*)a.rpad + (size_t)pl * a.pstride;
        float* wp = a.wpad ? (float*)a.wpad + (size_t)pl * a.pstride : nullptr;
        for (int64_t k = tid; k < npad; k += kSortThreads) {
            const uint32_t idx = (uint32_t)A[k < n ? k : k - n];
            rp[k] = (float)a.r[idx];
            if (wp) wp[k] = (float)a.w[idx];
        }
    } else {
        double* rp = (double*)a.rpad + (size_t)pl * a.pstride;
        double* wp = a.wpad ? (double*)a.wpad + (size_t)pl * a.pstride : nullptr;
        for (int64_t k = tid; k < npad; k += kSortThreads) {
            const uint32_t idx = (uint32_t)A[k < n ? k : k - n];
            rp[k] = a.r[idx];
            if (wp) wp[k] = a.w[idx];
        }
    }
    if (a.perm_out) {
        int32_t* po = a.perm_out + (size_t)pl * n;
        for (int64_t k = tid; k < n; k += kSortThreads) po[k] = (int32_t)(uint32_t)A[k];
    }
    if (a.pfx && !a.f32) {
        // Exact prefix sums of the integer deficits over the padded curve:
        // pfx[k] = sum_{m<k} u[perm[m mod n]].
        __int128* pf = (__int128*)a.pfx + (size_t)pl * (a.pstride + 1);
        const int64_t chunk = (npad + kSortThreads - 1) / kSortThreads;
        const int64_t c0 = (int64_t)tid * chunk, c1 = min(npad, c0 + chunk);
        __int128 s = 0;
        for (int64_t k = c0; k < c1; ++k) s += (__int128)a.u[(uint32_t)A[k < n ? k : k - n]];
        sh_part[tid] = s;
        __syncthreads();
        if (tid == 0) {
            __int128 run = 0;
            for (int q = 0; q < kSortThreads; ++q) {
                __int128 c = sh_part[q];
                sh_part[q] = run;
                run += c;
            }
        }
        __syncthreads();
        __int128 run = sh_part[tid];
        if (tid == 0) pf[0] = 0;
        for (int64_t k = c0; k < c1; ++k) {
            run += (__int128)a.u[(uint32_t)A[k < n ? k : k - n]];
            pf[k + 1] = run;
        }
    } else if (a.pfx) {
        // FP32C: Kahan-compensated prefix sums of (float)(1 - y): each
        // position stores an unevaluated (hi, lo) pair; chunk totals are
        // combined by one thread with the same compensation.
        float2* pf = (float2*)a.pfx + (size_t)pl * (a.pstride + 1);
        float2* part = (float2*)sh_part;
        const int64_t chunk = (npad + kSortThreads - 1) / kSortThreads;
        const int64_t c0 = (int64_t)tid * chunk, c1 = min(npad, c0 + chunk);
        float hi = 0.f, lo = 0.f;
        for (int64_t k = c0; k < c1; ++k) {
            const float x = (float)ldexp((double)a.u[(uint32_t)A[k < n ? k : k - n]], -53);
            float sum, err;
            two_sum(hi, x, sum, err);
            hi = sum;
            lo += err;
        }
        part[tid] = make_float2(hi, lo);
        __syncthreads();
        if (tid == 0) {
            float rh = 0.f, rl = 0.f;
            for (int q = 0; q < kSortThreads; ++q) {
                const float2 c = part[q];
                part[q] = make_float2(rh, rl);
                float sum, err;
                two_sum(rh, c.x, sum, err);
                rh = sum;
                rl += err + c.y;
            }
        }
        __syncthreads();
        hi = part[tid].x;
        lo = part[tid].y;
        if (tid == 0) pf[0] = make_float2(0.f, 0.f);
        for (int64_t k = c0; k < c1; ++k) {
            const float x = (float)ldexp((double)a.u[(uint32_t)A[k < n ? k : k - n]], -53);
            float sum, err;
            two_sum(hi, x, sum, err);
            hi = sum;
            lo += err;
            pf[k + 1] = make_float2(hi, lo);
        }
    }
}

// ------------------------------------------------------------------------
// Template table: row D holds the D-point ideal transit, zero-padded to a
// multiple of 32, so any (period, duration) item reads its template as a
// uniform stream through the scalar cache.  FP32C keeps a float copy.  With
// constant weights the per-window b = sum_k w s_k^2 and the template sum
// s1 = sum_k s_k depend on D only; they are summed once per D, in FP64 and
// in the same sequential order as a per-window evaluation.

__host__ __device__ __forceinline__ int64_t trow_off(int64_t d) {
    const int64_t m = d - 1, a = m / 32, b = m % 32;
    return 32 * (16 * a * (a + 1) + (a + 1) * b);
}
__host__ __device__ __forceinline__ int64_t rup32(int64_t d) { return (d + 31) & ~(int64_t)31; }

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__global__ __launch_bounds__(256) void k_tmpl_table(const double* __restrict__ tm, int32_t nt, T* __restrict__ table) {
    const int64_t d = (int64_t)blockIdx.x + 1;
    T* row = table + trow_off(d);
    const int64_t w = rup32(d);
    for (int64_t k = threadIdx.x; k < w; k += 256) row[k] = (k < d) ? (T)resample(tm, nt, d, k) : (T)0;
}

__global__ __launch_bounds__(64) void k_tmpl_sums(const double* __restrict__ tm, int32_t nt, int64_t dmax,
                                                  const uint64_t* misc, double* __restrict__ bsum,
                                                  double* __restrict__ s1sum) {
    const int64_t d = (int64_t)blockIdx.x * 64 + threadIdx.x + 1;
    if (d > dmax) return;
    const double wc = __longlong_as_double((long long)misc[kWminBits]);
    double b = 0.0, s1 = 0.0;
    for (int64_t k = 0; k < d; ++k) {
        const double sv = resample(tm, nt, d, k);
        b = fma(wc, sv * sv, b);
        s1 = s1 + sv;
    }
    bsum[d] = b;
    s1sum[d] = s1;
}

// ------------------------------------------------------------------------
// Slide: one workgroup per (period, duration) item, or per window tile of
// it.

constexpr int kSlideThreads = 256;
constexpr int kR = 16;                              // consecutive windows per lane (unit stride)
constexpr int kTile = kSlideThreads * kR;           // windows per tile
constexpr int kKC = 256;                            // template points per staged chunk
constexpr int kXs = kTile + kKC + kR;               // staged curve points
// Padded LDS index: every 16 points get 16 bytes of padding, so the 64 lanes'
// 16-point groups start on distinct bank quads.
template <typename T>
__host__ __device__ constexpr int xpad(int e) { return e + (int)(16 / sizeof(T)) * (e >> 4); }

struct SlideArgs {
    const double* periods;   // batch-offset
    const double* durations;
    int32_t nd;
    int32_t bp;
    int64_t n;
    gtls_params prm;
    const void* rpad;        // T [bp][pstride]
    const void* wpad;
    const void* pfx;         // __int128 (FP64) or float2 (FP32C) [bp][pstride + 1]
    int64_t pstride;
    const uint64_t* misc;
    const void* table;       // T template rows
    const double* bsum;      // [D] constant-weight b
    const double* s1sum;     // [D] template sums
    ItemBest* items;         // [bp][nd][ntiles]
    int32_t ntiles;          // window tiles per unit-stride item
};

struct Best {
    double dchi2;
    double depth;
    int64_t start;
};

__device__ __forceinline__ void consider(Best& b, double dchi2, double depth, int64_t i) {
    if (dchi2 > b.dchi2) {
        b.dchi2 = dchi2;
        b.depth = depth;
        b.start = i;
    }
}

// Window fit: WLS depth c/b or moving-average depth usum/s1, clamped at 0.
template <bool MEAN>
__device__ __forceinline__ void fit(double c, double b, double usum, double s1, double& dchi2, double& depth) {
    if (MEAN) {
        double md = usum / s1;
        depth = (md > 0.0) ? md : 0.0;
        dchi2 = (2.0 * depth) * c - (depth * depth) * b;
    } else {
        depth = (c > 0.0) ? c / b : 0.0;
        dchi2 = depth * c;
    }
}

// Sum of 1 - y over the window [i, i + d): exact from 128-bit prefix sums
// (FP64), or from the compensated (hi, lo) float pairs (FP32C).
template <typename T, bool MEAN>
__device__ __forceinline__ double window_deficit(const void* pf_base, int64_t i, int64_t d) {
    if constexpr (!MEAN) {
        return 0.0;
    } else if constexpr (sizeof(T) == 8) {
        const __int128* pf = (const __int128*)pf_base;
        return ldexp(i128_to_double(pf[i + d] - pf[i]), -53);
    } else {
        const float2* pf = (const float2*)pf_base;
        const float2 e = pf[i + d], s = pf[i];
        return ((double)e.x - (double)s.x) + ((double)e.y - (double)s.y);
    }
}

struct ItemInfo {
    bool valid;
    int pl, j, tile;
    double period;
    int64_t d, stride;
};

// Work units in launch order: longest durations first, then window tile,
// then period, so the costliest units start earliest.
__device__ __forceinline__ ItemInfo item_info(const SlideArgs& a, int tiles) {
    ItemInfo it;
    const int per_j = tiles * a.bp;
    const int jrev = blockIdx.x / per_j;
    const int rem = blockIdx.x - jrev * per_j;
    it.tile = rem / a.bp;
    it.pl = rem - it.tile * a.bp;
    it.j = a.nd - 1 - jrev;
    it.period = a.periods[it.pl];
    const double dur = a.durations[it.j];
    it.valid = duration_valid(it.period, dur, a.prm);
    it.d = it.valid ? points_in(a.n, it.period, dur) : 0;
    it.stride = it.valid ? t0_stride(it.d, a.prm.dt0) : 1;
    return it;
}

__device__ __forceinline__ ItemBest* item_slot(const SlideArgs& a, const ItemInfo& it) {
    return a.items + ((size_t)it.pl * a.nd + it.j) * a.ntiles + it.tile;
}

// Block-wide first-best (largest dchi2, then smallest start) -> item slot.
__device__ __forceinline__ void store_best(Best best, const SlideArgs& a, const ItemInfo& it, Best* red,
                                           int64_t evals, int ntiles) {
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        const double od = __shfl_xor(best.dchi2, off);
        const double op = __shfl_xor(best.depth, off);
        const long long oi = __shfl_xor((long long)best.start, off);
        const bool take = (od > best.dchi2) || (od == best.dchi2 && oi >= 0 && (best.start < 0 || oi < best.start));
        if (take) {
            best.dchi2 = od;
            best.depth = op;
            best.start = oi;
        }
    }
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        Best b = red[0];
        for (int q = 1; q < kSlideThreads / 64; ++q) {
            const Best o = red[q];
            if (o.dchi2 > b.dchi2 || (o.dchi2 == b.dchi2 && o.start >= 0 && (b.start < 0 || o.start < b.start)))
                b = o;
        }
        ItemBest* out = item_slot(a, it);
        out->dchi2 = b.dchi2;
        out->depth = b.depth;
        out->start = (int32_t)b.start;
        out->d = (int32_t)it.d;
        out->evals = (int32_t)evals;
        if (it.tile == 0) out->ntiles = ntiles;
    }
}

__device__ __forceinline__ void store_invalid(const SlideArgs& a, const ItemInfo& it) {
    if (threadIdx.x == 0 && it.tile == 0) {
        ItemBest* out = item_slot(a, it);
        out->dchi2 = -INFINITY;
        out->depth = 0.0;
        out->start = -1;
        out->d = 0;
        out->evals = 0;
        out->ntiles = 1;
    }
}

// 16 template steps on 16 windows: window m at step u reads lo[u+m] (or
// hi[u+m-16]); one fused multiply-add per step in ascending template order.
// SQ squares the template value (the b = sum w s^2 sums of varying weights).
template <typename T, bool SQ>
__device__ __forceinline__ void block16(T (&acc)[kR], const T (&lo)[kR], const T (&hi)[kR], cptr<T> t) {
#pragma unroll
    for (int u = 0; u < kR; ++u) {
        const T sv = SQ ? t[u] * t[u] : t[u];
#pragma unroll
        for (int m = 0; m < kR; ++m) acc[m] = fma((u + m < kR) ? lo[u + m] : hi[u + m - kR], sv, acc[m]);
    }
}

template <typename T>
__device__ __forceinline__ void ld16(T (&x)[kR], const T* p) {
#pragma unroll
    for (int m = 0; m < kR; ++m) x[m] = p[m];
}

// Correlation of the 16 windows of this lane over one staged chunk of kc
// template points.  FP64 accumulates straight into acc; FP32 accumulates
// each 32-point block in float and adds it to the FP64 accumulator.
template <typename T, bool SQ>
__device__ __forceinline__ void chunk_correlate(double (&acc)[kR], const T* xs, int base, int kc, cptr<T> t) {
    T xa[kR], xb[kR];
    ld16(xa, xs + xpad<T>(base));
    for (int kb = 0; kb < kc; kb += 2 * kR) {
        if constexpr (sizeof(T) == 8) {
            ld16(xb, xs + xpad<T>(base + kb + kR));
            block16<T, SQ>(acc, xa, xb, t + kb);
            ld16(xa, xs + xpad<T>(base + kb + 2 * kR));
            block16<T, SQ>(acc, xb, xa, t + kb + kR);
        } else {
            T a32[kR];
#pragma unroll
            for (int m = 0; m < kR; ++m) a32[m] = (T)0;
            ld16(xb, xs + xpad<T>(base + kb + kR));
            block16<T, SQ>(a32, xa, xb, t + kb);
            ld16(xa, xs + xpad<T>(base + kb + 2 * kR));
            block16<T, SQ>(a32, xb, xa, t + kb + kR);
#pragma unroll
            for (int m = 0; m < kR; ++m) acc[m] += (double)a32[m];
        }
    }
}

// Every T0 offset (stride 1): each lane owns 16 consecutive windows; their
// correlation sums advance together over a padded LDS copy of the curve,
// with the template streamed from the table into scalar registers.
template <typename T, bool VARW, bool MEAN>
__global__ __launch_bounds__(kSlideThreads) void k_slide_unit(SlideArgs a) {
    __shared__ T x_sh[xpad<T>(kXs)];
    __shared__ T xw_sh[VARW ? xpad<T>(kXs) : 1];
    __shared__ Best red[kSlideThreads / 64];
    const ItemInfo it = item_info(a, a.ntiles);
    if (!it.valid) {
        store_invalid(a, it);
        return;
    }
    if (it.stride != 1) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int64_t n = a.n, D = it.d;
    const T* __restrict__ rp = (const T*)a.rpad + (size_t)it.pl * a.pstride;
    const T* __restrict__ wp = VARW ? (const T*)a.wpad + (size_t)it.pl * a.pstride : nullptr;
    const void* pf = MEAN ? (const void*)((const char*)a.pfx + (size_t)it.pl * (a.pstride + 1) *
                                          (sizeof(T) == 8 ? sizeof(__int128) : sizeof(float2)))
                          : nullptr;
    const cptr<T> trow = (cptr<T>)((const T*)a.table + trow_off(D));
    const double bconst = VARW ? 0.0 : a.bsum[D];
    const double s1 = MEAN ? a.s1sum[D] : 0.0;
    const int64_t limit = n + D;
    const int64_t dpad = rup32(D);
    const int base = tid * kR;
    const int64_t i0 = (int64_t)it.tile * kTile;
    Best best{-INFINITY, 0.0, -1};

    const bool busy = i0 + (int64_t)wave * 64 * kR < n;     // wave has at least one window
    double acc[kR], bacc[VARW ? kR : 1];
#pragma unroll
    for (int m = 0; m < kR; ++m) acc[m] = 0.0;
#pragma unroll
    for (int m = 0; m < (VARW ? kR : 1); ++m) bacc[m] = 0.0;
    for (int64_t k0 = 0; k0 < dpad; k0 += kKC) {
        const int kc = (int)min((int64_t)kKC, dpad - k0);
        if (k0 > 0) __syncthreads();
        const int nx = kTile + kc + kR;
        for (int e = tid; e < nx; e += kSlideThreads) {
            const int64_t g = i0 + k0 + e;
            x_sh[xpad<T>(e)] = (g < limit) ? rp[g] : (T)0;
            if (VARW) xw_sh[xpad<T>(e)] = (g < limit) ? wp[g] : (T)0;
        }
        __syncthreads();
        if (!busy) continue;
        chunk_correlate<T, false>(acc, x_sh, base, kc, trow + k0);
        if constexpr (VARW) chunk_correlate<T, true>(bacc, xw_sh, base, kc, trow + k0);
    }
#pragma unroll
    for (int m = 0; m < kR; ++m) {
        const int64_t i = i0 + base + m;
        if (i < n) {
            double dchi2, depth;
            fit<MEAN>(acc[m], VARW ? bacc[m] : bconst, window_deficit<T, MEAN>(pf, i, D), s1, dchi2, depth);
            consider(best, dchi2, depth, i);
        }
    }
    store_best(best, a, it, red, min((int64_t)kTile, n - i0), a.ntiles);
}

// Strided T0 grid (stride >= 2): one window per lane, each wave working on
// its own 64 windows through a wave-private LDS tile.  Small strides stage
// the contiguous span the 64 windows cover (each point read once); large
// strides stage each window's next 32 points as a transposed 64 x 32 tile
// (coalesced reads of 32-point runs).  The template is a uniform stream.
constexpr int kSTC = 32;                            // template points per tile step (transposed mode)
constexpr int kSPitch = kSTC + 1;
constexpr int kSTile = 64 * kSPitch;                // elements per wave tile

template <typename T, bool VARW, bool MEAN>
__global__ __launch_bounds__(kSlideThreads) void k_slide_strided(SlideArgs a) {
    __shared__ T tile[kSlideThreads / 64][kSTile];
    __shared__ T tilew[VARW ? kSlideThreads / 64 : 1][VARW ? kSTile : 1];
    __shared__ Best red[kSlideThreads / 64];
    const ItemInfo it = item_info(a, 1);
    if (!it.valid || it.stride == 1) return;     // the unit-stride kernel writes those items
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t n = a.n, D = it.d, s = it.stride;
    const int64_t nw = (n + s - 1) / s;
    const T* __restrict__ rp = (const T*)a.rpad + (size_t)it.pl * a.pstride;
    const T* __restrict__ wp = VARW ? (const T*)a.wpad + (size_t)it.pl * a.pstride : nullptr;
    const void* pf = MEAN ? (const void*)((const char*)a.pfx + (size_t)it.pl * (a.pstride + 1) *
                                          (sizeof(T) == 8 ? sizeof(__int128) : sizeof(float2)))
                          : nullptr;
    const cptr<T> trow = (cptr<T>)((const T*)a.table + trow_off(D));
    const double bconst = VARW ? 0.0 : a.bsum[D];
    const double s1 = MEAN ? a.s1sum[D] : 0.0;
    const int64_t limit = n + D;
    const int64_t dpad = rup32(D);
    T* tl = tile[wave];
    T* tw = VARW ? tilew[wave] : nullptr;
    // Contiguous mode: the 64 windows of a group span 63 s + TCu points.
    const int64_t tcu = (kSTile - 63 * s) & ~(int64_t)31;
    const bool contiguous = tcu >= 32;
    const int64_t tc = contiguous ? tcu : kSTC;
    Best best{-INFINITY, 0.0, -1};

    for (int64_t g0 = (int64_t)wave * 64; g0 < nw; g0 += kSlideThreads) {
        const int64_t m = g0 + lane;
        const bool active = m < nw;
        const int64_t i = m * s;
        const int64_t ibase = g0 * s;
        double c = 0.0, bv = 0.0;
        for (int64_t k0 = 0; k0 < dpad; k0 += tc) {
            const int kc = (int)min(tc, dpad - k0);
            if (contiguous) {
                const int64_t span = 63 * s + kc;
                for (int64_t e = lane; e < span; e += 64) {
                    const int64_t gsrc = ibase + k0 + e;
                    tl[e] = (gsrc < limit) ? rp[gsrc] : (T)0;
                    if (VARW) tw[e] = (gsrc < limit) ? wp[gsrc] : (T)0;
                }
            } else {
                const int e = lane & 31;
                for (int r = 0; r < 32; ++r) {
                    const int seg = 2 * r + (lane >> 5);
                    const int64_t mm = g0 + seg;
                    const int64_t gsrc = mm * s + k0 + e;
                    const bool ok = mm < nw && gsrc < limit;
                    tl[seg * kSPitch + e] = ok ? rp[gsrc] : (T)0;
                    if (VARW) tw[seg * kSPitch + e] = ok ? wp[gsrc] : (T)0;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const T* xl = contiguous ? tl + lane * s : tl + lane * kSPitch;
            const T* xw = VARW ? (contiguous ? tw + lane * s : tw + lane * kSPitch) : nullptr;
            const cptr<T> t = trow + k0;
            for (int kb = 0; kb < kc; kb += kSTC) {
                T cb = (sizeof(T) == 8) ? (T)c : (T)0;
                T bb = (sizeof(T) == 8) ? (T)bv : (T)0;
#pragma unroll
                for (int kk = 0; kk < kSTC; ++kk) {
                    const T sv = t[kb + kk];
                    cb = fma(xl[kb + kk], sv, cb);
                    if (VARW) bb = fma(xw[kb + kk], sv * sv, bb);
                }
                if constexpr (sizeof(T) == 8) {
                    c = cb;
                    bv = bb;
                } else {
                    c += (double)cb;
                    bv += (double)bb;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (active) {
            double dchi2, depth;
            fit<MEAN>(c, VARW ? bv : bconst, window_deficit<T, MEAN>(pf, i, D), s1, dchi2, depth);
            consider(best, dchi2, depth, i);
        }
    }
    store_best(best, a, it, red, nw, 1);
}

// ------------------------------------------------------------------------
// Per-period reduction over durations and the T0 of the best window.

struct ReduceArgs {
    const double* t;
    int64_t n;
    const double* periods;   // batch-offset
    int32_t bp;
    int32_t nd;
    const ItemBest* items;
    int32_t ntiles;
    const uint64_t* keys_a;
    const uint64_t* misc;
    uint64_t* misc_rw;
    double* chi2;            // batch-offset outputs
    int32_t* best_dur;
    int32_t* best_start;
    double* depth;
    double* t0;
};

__global__ __launch_bounds__(64) void k_reduce(ReduceArgs a) {
    const int pl = blockIdx.x * 64 + threadIdx.x;
    uint64_t evals = 0, macs = 0;
    if (pl < a.bp) {
        const double chi2_0 = __longlong_as_double((long long)a.misc[kChi2Null]);
        const double tmin = from_ordered(a.misc[kTminOrd]);
        double best = -INFINITY, bdepth = 0.0;
        int bj = -1, bi = -1, bd = 0;
        for (int j = 0; j < a.nd; ++j) {
            const ItemBest* slots = a.items + ((size_t)pl * a.nd + j) * a.ntiles;
            const int nt = min(max(slots[0].ntiles, 0), a.ntiles);
            for (int t = 0; t < nt; ++t) {
                const ItemBest b = slots[t];
                if (b.start < 0) continue;
                evals += (uint64_t)b.evals;
                macs += (uint64_t)b.evals * (uint64_t)b.d;
                if (b.dchi2 > best) {
                    best = b.dchi2;
                    bdepth = b.depth;
                    bj = j;
                    bi = b.start;
                    bd = b.d;
                }
            }
        }
        if (bj < 0) {
            a.chi2[pl] = chi2_0;
            a.best_dur[pl] = -1;
            a.best_start[pl] = -1;
            a.depth[pl] = 0.0;
            a.t0[pl] = NAN;
        } else {
            const double period = a.periods[pl];
            a.chi2[pl] = chi2_0 - best;
            a.best_dur[pl] = bj;
            a.best_start[pl] = bi;
            a.depth[pl] = bdepth;
            const int64_t mid = ((int64_t)bi + bd / 2) % a.n;
            const uint32_t idx = (uint32_t)a.keys_a[(size_t)pl * a.n + mid];
            const double phic = phase_of(a.t[idx], period);
            const double x = phic * period;
            a.t0[pl] = x + period * ceil((tmin - x) / period);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        evals += __shfl_xor(evals, off);
        macs += __shfl_xor(macs, off);
    }
    if (threadIdx.x == 0 && evals) {
        atomicAdd((unsigned long long*)&a.misc_rw[kEvals], (unsigned long long)evals);
        atomicAdd((unsigned long long*)&a.misc_rw[kMacs], (unsigned long long)macs);
    }
}

// ------------------------------------------------------------------------
// Periodogram statistics.

// SR, the sequential mean and population standard deviation, SDE_raw.
__global__ __launch_bounds__(256) void k_sde_stats(const double* __restrict__ chi2, int32_t n, double* __restrict__ sr,
                                                   double* __restrict__ raw) {
    constexpr int CH = 2048;
    __shared__ double xs[CH];
    __shared__ double red[256];
    __shared__ double sh_mean, sh_sd, sh_min;
    const int tid = threadIdx.x;
    double mn = INFINITY;
    for (int i = tid; i < n; i += 256) mn = fmin(mn, chi2[i]);
    red[tid] = mn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmin(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) sh_min = red[0];
    __syncthreads();
    const double cmin = sh_min;
    for (int i = tid; i < n; i += 256) sr[i] = (chi2[i] == 0.0) ? 1.0 : cmin / chi2[i];
    __syncthreads();
    double sum = 0.0;
    for (int base = 0; base < n; base += CH) {
        for (int k = tid; k < CH && base + k < n; k += 256) xs[k] = sr[base + k];
        __syncthreads();
        if (tid == 0) {
            const int m = min(CH, n - base);
            for (int k = 0; k < m; ++k) sum += xs[k];
        }
        __syncthreads();
    }
    if (tid == 0) sh_mean = sum / (double)n;
    __syncthreads();
    const double mean = sh_mean;
    double var = 0.0;
    for (int base = 0; base < n; base += CH) {
        for (int k = tid; k < CH && base + k < n; k += 256) xs[k] = sr[base + k];
        __syncthreads();
        if (tid == 0) {
            const int m = min(CH, n - base);
            for (int k = 0; k < m; ++k) {
                const double d = xs[k] - mean;
                var += d * d;
            }
        }
        __syncthreads();
    }
    if (tid == 0) sh_sd = sqrt(var / (double)n);
    __syncthreads();
    const double sd = sh_sd;
    for (int i = tid; i < n; i += 256) raw[i] = (sd > 0.0) ? (sr[i] - mean) / sd : 0.0;
}

// SDE = SDE_raw - running median over `window` points, ends replicated.
// The median is selected by rank, so it is an input element exactly.
constexpr int kMedThreads = 256;
constexpr int kMedMaxWindow = 1023;

__global__ __launch_bounds__(kMedThreads) void k_sde_median(const double* __restrict__ raw, int32_t n, int32_t window,
                                                            double* __restrict__ sde) {
    __shared__ double v[kMedThreads + kMedMaxWindow];
    const int half = window / 2;
    const int i0 = blockIdx.x * kMedThreads;
    const int span = kMedThreads + 2 * half;
    for (int k = threadIdx.x; k < span; k += kMedThreads) {
        int idx = i0 - half + k;
        idx = idx < 0 ? 0 : (idx > n - 1 ? n - 1 : idx);
        v[k] = raw[idx];
    }
    __syncthreads();
    const int i = i0 + threadIdx.x;
    if (i >= n) return;
    const double* w = v + threadIdx.x;
    double med = w[0];
    for (int aidx = 0; aidx < window; ++aidx) {
        const double x = w[aidx];
        int lt = 0, le_before = 0;
        for (int b = 0; b < window; ++b) {
            const double y = w[b];
            lt += (y < x);
            le_before += (y == x) & (b < aidx);
        }
        if (lt + le_before == half) {
            med = x;
            break;
        }
    }
    sde[i] = raw[i] - med;
}

__global__ __launch_bounds__(1024) void k_sde_argmax(const double* __restrict__ sde, int32_t n, gtls_summary* summary,
                                                     const uint64_t* misc) {
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    const int tid = threadIdx.x;
    double v = -INFINITY;
    int idx = -1;
    for (int i = tid; i < n; i += 1024) {
        if (sde[i] > v) {
            v = sde[i];
            idx = i;
        }
    }
    bv[tid] = v;
    bi[tid] = idx;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (tid < s) {
            const double ov = bv[tid + s];
            const int oi = bi[tid + s];
            if (oi >= 0 && (ov > bv[tid] || (ov == bv[tid] && (bi[tid] < 0 || oi < bi[tid])))) {
                bv[tid] = ov;
                bi[tid] = oi;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && summary) {
        summary->best_period = bi[0];
        summary->sde_max = bv[0];
        if (misc) {
            summary->chi2_null = __longlong_as_double((long long)misc[kChi2Null]);
            summary->n_evals = (int64_t)misc[kEvals];
            summary->n_macs = (int64_t)misc[kMacs];
        }
    }
}

}  // namespace

// ------------------------------------------------------------------------
// Launchers

hipError_t ensure(gtls_ctx* ctx, DeviceBuffer& b, size_t bytes) {
    if (b.bytes >= bytes) return hipSuccess;
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return e;
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return e;
    }
    b.bytes = bytes;
    return hipSuccess;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static hipEvent_t pool_event(gtls_ctx* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

StageTimer::StageTimer(gtls_ctx* ctx, int stage) : ctx_(ctx), stage_(stage) {
    if (!ctx_->profiling) return;
    start_ = pool_event(ctx_);
    stop_ = pool_event(ctx_);
    if (start_) (void)hipEventRecord(start_, ctx_->stream);
}

StageTimer::~StageTimer() {
    if (!ctx_->profiling || !start_ || !stop_) return;
    (void)hipEventRecord(stop_, ctx_->stream);
    ctx_->pending.push_back({stage_, start_, stop_});
}

hipError_t profile_collect(gtls_ctx* ctx) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    for (auto& p : ctx->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            ctx->prof_ms[p.stage] += ms;
            ctx->prof_launches[p.stage] += 1;
        }
        ctx->event_pool.push_back(p.start);
        ctx->event_pool.push_back(p.stop);
    }
    ctx->pending.clear();
    return hipSuccess;
}

hipError_t run_sde(gtls_ctx* ctx, const double* chi2, int32_t n, int32_t window, double* sr, double* raw,
                   double* sde, gtls_summary* summary, const uint64_t* misc) {
    hipStream_t s = ctx->stream;
    StageTimer tm(ctx, kStageSde);
    k_sde_stats<<<1, 256, 0, s>>>(chi2, n, sr, raw);
    k_sde_median<<<(n + kMedThreads - 1) / kMedThreads, kMedThreads, 0, s>>>(raw, n, window, sde);
    k_sde_argmax<<<1, 1024, 0, s>>>(sde, n, summary, misc);
    return hipGetLastError();
}

hipError_t run_sde(gtls_ctx* ctx, const double* chi2, int32_t n, int32_t window, double* sr, double* raw,
                   double* sde, gtls_summary* summary) {
    return run_sde(ctx, chi2, n, window, sr, raw, sde, summary, nullptr);
}

namespace {

struct Plan {
    int64_t n, pstride, dcap;
    int32_t bp, ntiles;
    bool varw, mean, f32;
    size_t esize, psize;     // bytes per padded-curve element and per prefix element
    size_t off_a, off_b, off_r, off_w, off_pf, off_items, per_batch;
};

Plan make_plan(int64_t n, int32_t n_periods, int32_t nd, const gtls_params& prm, bool varw) {
    Plan p{};
    p.n = n;
    p.varw = varw;
    p.mean = prm.depth_mode == GTLS_DEPTH_MEAN;
    p.f32 = prm.precision == GTLS_FP32C;
    p.esize = p.f32 ? sizeof(float) : sizeof(double);
    p.psize = p.f32 ? sizeof(float2) : sizeof(__int128);
    int64_t dcap = (int64_t)std::floor((double)n * prm.q_cap + 0.5);
    dcap = std::max<int64_t>(1, std::min<int64_t>(n, dcap));
    p.dcap = dcap;
    p.ntiles = (int32_t)((n + kTile - 1) / kTile);
    p.pstride = ((n + dcap + 63) / 64) * 64;
    size_t per = 2 * sizeof(uint64_t) * (size_t)n + p.esize * (size_t)p.pstride +
                 (varw ? p.esize * (size_t)p.pstride : 0) + (p.mean ? p.psize * (size_t)(p.pstride + 1) : 0) +
                 sizeof(ItemBest) * (size_t)nd * (size_t)p.ntiles + 1024;
    const size_t budget = (size_t)24 << 30;
    int64_t bp = (int64_t)(budget / per);
    bp = std::max<int64_t>(1, std::min<int64_t>(bp, 8192));
    bp = std::min<int64_t>(bp, n_periods);
    // one-dimensional grids of bp * nd * ntiles work units
    const int64_t units = std::max<int64_t>(1, (int64_t)nd * p.ntiles);
    bp = std::max<int64_t>(1, std::min<int64_t>(bp, 0x7fffffffLL / units));
    p.bp = (int32_t)bp;
    size_t o = 0;
    p.off_a = o;
    o = align256(o + sizeof(uint64_t) * (size_t)n * bp);
    p.off_b = o;
    o = align256(o + sizeof(uint64_t) * (size_t)n * bp);
    p.off_r = o;
    o = align256(o + p.esize * (size_t)p.pstride * bp);
    p.off_w = o;
    if (varw) o = align256(o + p.esize * (size_t)p.pstride * bp);
    p.off_pf = o;
    if (p.mean) o = align256(o + p.psize * (size_t)(p.pstride + 1) * bp);
    p.off_items = o;
    o = align256(o + sizeof(ItemBest) * (size_t)nd * (size_t)p.ntiles * bp);
    p.per_batch = o;
    return p;
}

template <typename T, bool VARW, bool MEAN>
void launch_slides(const SlideArgs& la, unsigned grid, unsigned grid_items, bool strided, hipStream_t s) {
    k_slide_unit<T, VARW, MEAN><<<grid, kSlideThreads, 0, s>>>(la);
    if (strided) k_slide_strided<T, VARW, MEAN><<<grid_items, kSlideThreads, 0, s>>>(la);
}

template <typename T>
void launch_slides(const SlideArgs& la, unsigned grid, unsigned grid_items, bool strided, bool varw, bool mean,
                   hipStream_t s) {
    if (varw) {
        if (mean) launch_slides<T, true, true>(la, grid, grid_items, strided, s);
        else launch_slides<T, true, false>(la, grid, grid_items, strided, s);
    } else {
        if (mean) launch_slides<T, false, true>(la, grid, grid_items, strided, s);
        else launch_slides<T, false, false>(la, grid, grid_items, strided, s);
    }
}

}  // namespace

hipError_t run_search(gtls_ctx* ctx, const SearchArgs& a) {
    hipStream_t s = ctx->stream;
    const int64_t n = a.n;
    // Per-curve arrays: misc | w | r | u
    const size_t off_w = 256, off_r = align256(off_w + 8 * (size_t)n), off_u = align256(off_r + 8 * (size_t)n);
    hipError_t e = ensure(ctx, ctx->curve, align256(off_u + 8 * (size_t)n));
    if (e != hipSuccess) return e;
    char* cb = (char*)ctx->curve.ptr;
    uint64_t* misc = (uint64_t*)cb;
    double* w = (double*)(cb + off_w);
    double* r = (double*)(cb + off_r);
    int64_t* u = (int64_t*)(cb + off_u);
    {
        StageTimer tm(ctx, kStagePrep);
        k_init_misc<<<1, 64, 0, s>>>(misc);
        k_prep<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a.t, a.y, a.dy, n, w, r, u, misc);
        k_chi2_null<<<1, 256, 0, s>>>(a.y, a.dy, n, misc);
    }
    uint64_t hmisc[kMiscSlots];
    e = hipMemcpyAsync(hmisc, misc, sizeof(hmisc), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const bool varw = hmisc[kWminBits] != hmisc[kWmaxBits];

    const Plan pl = make_plan(n, a.n_periods, a.n_durations, a.prm, varw);
    // Template rows for every D in [1, dcap] and the per-D sums.
    const size_t tab_elems = (size_t)trow_off(pl.dcap + 1);
    const size_t off_bsum = align256(pl.esize * tab_elems), off_s1 = align256(off_bsum + 8 * (size_t)(pl.dcap + 1));
    e = ensure(ctx, ctx->table, align256(off_s1 + 8 * (size_t)(pl.dcap + 1)));
    if (e != hipSuccess) return e;
    void* table = ctx->table.ptr;
    double* bsum = (double*)((char*)ctx->table.ptr + off_bsum);
    double* s1sum = (double*)((char*)ctx->table.ptr + off_s1);
    {
        StageTimer tm(ctx, kStagePrep);
        if (pl.f32) k_tmpl_table<float><<<(unsigned)pl.dcap, 256, 0, s>>>(a.tmpl, a.n_tmpl, (float*)table);
        else k_tmpl_table<double><<<(unsigned)pl.dcap, 256, 0, s>>>(a.tmpl, a.n_tmpl, (double*)table);
        k_tmpl_sums<<<(unsigned)((pl.dcap + 63) / 64), 64, 0, s>>>(a.tmpl, a.n_tmpl, pl.dcap, misc, bsum, s1sum);
    }
    e = ensure(ctx, ctx->batch, pl.per_batch);
    if (e != hipSuccess) return e;
    char* bb = (char*)ctx->batch.ptr;
    uint64_t* keys_a = (uint64_t*)(bb + pl.off_a);
    uint64_t* keys_b = (uint64_t*)(bb + pl.off_b);
    void* rpad = bb + pl.off_r;
    void* wpad = varw ? (void*)(bb + pl.off_w) : nullptr;
    void* pfx = pl.mean ? (void*)(bb + pl.off_pf) : nullptr;
    ItemBest* items = (ItemBest*)(bb + pl.off_items);
    const bool strided = a.prm.dt0 > 0.0;

    for (int32_t p0 = 0; p0 < a.n_periods; p0 += pl.bp) {
        const int32_t bp = std::min(pl.bp, a.n_periods - p0);
        SortArgs sa{a.t, r, w, u, n, a.periods + p0, a.durations, a.n_durations, a.prm, keys_a, keys_b,
                    rpad, wpad, pfx, pl.pstride, nullptr, pl.f32 ? 1 : 0};
        {
            StageTimer tm(ctx, kStageSort);
            k_fold_sort<<<bp, kSortThreads, 0, s>>>(sa);
        }
        SlideArgs la{a.periods + p0, a.durations, a.n_durations, bp, n, a.prm, rpad, wpad, pfx, pl.pstride,
                     misc, table, bsum, s1sum, items, pl.ntiles};
        const unsigned grid = (unsigned)bp * (unsigned)a.n_durations * (unsigned)pl.ntiles;
        const unsigned grid_items = (unsigned)bp * (unsigned)a.n_durations;
        {
            StageTimer tm(ctx, kStageSlide);
            if (pl.f32) launch_slides<float>(la, grid, grid_items, strided, varw, pl.mean, s);
            else launch_slides<double>(la, grid, grid_items, strided, varw, pl.mean, s);
        }
        ReduceArgs ra{a.t, n, a.periods + p0, bp, a.n_durations, items, pl.ntiles, keys_a, misc, misc,
                      a.chi2 + p0, a.best_dur + p0, a.best_start + p0, a.depth + p0, a.t0 + p0};
        {
            StageTimer tm(ctx, kStageReduce);
            k_reduce<<<(bp + 63) / 64, 64, 0, s>>>(ra);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return run_sde(ctx, a.chi2, a.n_periods, a.prm.median_window, a.sr, a.sde_raw, a.sde, a.summary, misc);
}

hipError_t run_fold_sort(gtls_ctx* ctx, const double* t, int64_t n, const double* periods, int32_t n_periods,
                         int32_t* perm) {
    hipStream_t s = ctx->stream;
    gtls_params prm;
    gtls_params_default(&prm);
    const Plan pl = make_plan(n, n_periods, 1, prm, false);
    // r/w/u are read by the padding step; give it a zeroed dummy curve.
    const size_t off_r = 256, off_u = align256(off_r + 8 * (size_t)n);
    hipError_t e = ensure(ctx, ctx->curve, align256(off_u + 8 * (size_t)n));
    if (e != hipSuccess) return e;
    char* cb = (char*)ctx->curve.ptr;
    double* r = (double*)(cb + off_r);
    int64_t* u = (int64_t*)(cb + off_u);
    e = ensure(ctx, ctx->batch, pl.per_batch);
    if (e != hipSuccess) return e;
    char* bb = (char*)ctx->batch.ptr;
    for (int32_t p0 = 0; p0 < n_periods; p0 += pl.bp) {
        const int32_t bp = std::min(pl.bp, n_periods - p0);
        SortArgs sa{t, r, r, u, n, periods + p0, periods, 0, prm, (uint64_t*)(bb + pl.off_a),
                    (uint64_t*)(bb + pl.off_b), bb + pl.off_r, nullptr, nullptr, pl.pstride,
                    perm + (size_t)p0 * n, 0};
        k_fold_sort<<<bp, kSortThreads, 0, s>>>(sa);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gtls
