// HIP kernels of the TLS search for gfx950 (MI355X) and their launchers.
//
// Per trial period P (Sect. 2.3 of the GTLS paper):
//   k_fold_sort   one 512-thread workgroup per period, two per CU: phase fold on raw
//                 times (Sect. 2.3.1) and the order of the points by (FP64
//                 phase, index), in two phases over 32-bit fixed-point phase
//                 keys: one counting pass over HBM by the top 8 key bits,
//                 then LDS tiles of whole top-digit buckets ordered by the
//                 next 9 bits and, within those bins, by rank; periods whose
//                 phases bunch too tightly for the LDS tiles take a 3-pass
//                 stable LSD radix sort over 24-bit keys (wave-ballot
//                 ranking, equal keys fixed by FP64 phase then index).  Then
//                 the cyclic padding (Sect. 2.3.2): the folded residuals (and
//                 weights) gathered in phase order for n + D_max positions,
//                 and (moving-average depth only) exact integer prefix sums
//                 of 1 - y over the padded curve (Sect. 2.3.3).
//   k_plan_*      per launch: the every-offset items and the wave tasks of
//                 the items with a T0 step of two or more points.
//   k_slide_unit  every T0 offset (Sect. 2.3.4, in-transit term): work units
//                 of 4096 windows of one (period, duration) item; each lane
//                 owns 16 consecutive windows whose correlation sums run in
//                 registers over a padded, bank-conflict-free LDS tile.
//   k_slide_rows  T0 step s >= 2 (Sect. 2.5): persistent waves pop wave
//                 tasks of four 16-lane rows, each row on one (period,
//                 duration) item; each lane owns R windows s points apart and
//                 streams its run of the padded curve once for all of them.
//   k_reduce      per period: first best over durations -> chi2(P), depth, T0.
//   k_sde_*       SR, SDE_raw, running-median detrend, argmax (Sect. 2.4).
//   k_batch       many curves: one persistent kernel over (curve, period)
//                 items, each folded, sorted, padded and slid by one
//                 workgroup.
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
#include <cstring>
#include <utility>

#include "gtls_impl.hpp"

#include <mutex>

// Scratch of the allocation-free search entry point (tls_search_dev_noalloc):
// one array per GPU, alive until the process ends.  Host code never passes
// this name to a kernel: it uses the device address resolved per device by
// gtls::static_scratch_address.
static __device__ __align__(256) char scratch[(size_t)256 << 20];

namespace gtls {
namespace {

constexpr double kDay = 86400.0;
constexpr double kTwo53 = 9007199254740992.0;

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
// Fold + stable radix sort + tie fix + padding.  The steps are device
// functions parameterised by the workgroup size NT, shared by the
// one-period-per-workgroup kernel (NT = 1024) and the batched persistent
// kernel (NT = 256).

constexpr int kSortThreads = 512;
constexpr int kSortItems = 8;

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

constexpr int kTieCap = 2048;   // equal-key neighbours listed during the last pass

template <int NT, int ITEMS = kSortItems>
struct SortShared {
    uint32_t lastkey[256];       // last pass: key of the last word written per digit (0xffffffff: none yet)
    uint32_t tie_n;              // last pass: output positions whose key equals the previous position's
    uint32_t tie_pos[kTieCap];
    uint32_t hist[3][256];
    uint32_t wcnt[NT / 64][256];
    uint32_t dbase[256];
    uint32_t tcount[256];        // this tile's count per digit
    uint32_t tstart[256];        // ... and its first slot in the tile's digit order
    uint32_t wtot[4];
    union {
        uint64_t buf[NT * ITEMS];        // a tile in digit order (sort passes)
        __int128 part[NT];               // per-thread partial sums (prefix sums)
    };
    int64_t dpad;
};

constexpr double kTwo24 = 16777216.0;
constexpr uint32_t kKeyMax = (1u << 24) - 1;

// 24-bit sort key floor(phi 2^24), monotone in phi; a phase that rounds up
// to 1.0 (tiny negative t / P) takes the largest key, and the tie fix
// places it by its FP64 value.
__device__ __forceinline__ uint32_t phase_key(double ph) {
    const double x = ph * kTwo24;
    return x >= kTwo24 ? kKeyMax : (uint32_t)x;
}

// 32-bit key floor(phi 2^32) of the two-phase sort, monotone in phi (equal
// keys: phases within 2^-32 of each other).
__device__ __forceinline__ uint32_t phase_key32(double ph) {
    const double x = ph * 4294967296.0;
    return x >= 4294967296.0 ? 0xffffffffu : (uint32_t)x;
}

// Zeros kept after every padded curve of the single-curve search: the
// strided slide reads 16-byte pieces that start at most at the end of the
// padded curve.
constexpr int64_t kOverRead = 16;

// Where the sorted order goes: the padded residual / weight copies (npad
// positions, position k holding sorted point k mod n), or nothing (rpad
// null: permutation only).
struct PadOut {
    const double* r;
    const double* w;
    void* rpad;
    void* wpad;
    int64_t npad;
    bool f32;
};

// Writes a residual rv (and weight wv) at padded position pos and, when
// pos + n is still inside the padding, at pos + n.
__device__ __forceinline__ void pad_put(const PadOut& po, int64_t n, int64_t pos, double rv, double wv) {
    const bool twice = pos + n < po.npad;
    if (po.f32) {
        float* rp = (float*)po.rpad;
        rp[pos] = (float)rv;
        if (twice) rp[pos + n] = (float)rv;
        if (po.wpad) {
            float* wp = (float*)po.wpad;
            wp[pos] = (float)wv;
            if (twice) wp[pos + n] = (float)wv;
        }
    } else {
        double* rp = (double*)po.rpad;
        rp[pos] = rv;
        if (twice) rp[pos + n] = rv;
        if (po.wpad) {
            double* wp = (double*)po.wpad;
            wp[pos] = wv;
            if (twice) wp[pos + n] = wv;
        }
    }
}

// The residual (and weight) of input point idx at padded position pos.
__device__ __forceinline__ void pad_store(const PadOut& po, int64_t n, int64_t pos, uint32_t idx) {
    pad_put(po, n, pos, po.r[idx], po.wpad ? po.w[idx] : 0.0);
}

// Stable rank of each item's 8-bit digit (bits shift..shift+7) among the
// items of this wave that precede it: items are in (item, lane) order, item
// e of lane l at segment position e*64 + l, and the first `valid` positions
// hold items.  wcnt is this wave's per-digit count, advanced by the wave's
// items.
template <int ITEMS>
__device__ __forceinline__ void wave_rank(const uint64_t (&item)[ITEMS], int valid, int shift, uint32_t* wcnt,
                                          uint32_t (&dig)[ITEMS], uint32_t (&rnk)[ITEMS]) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) {
        const bool active = e * 64 + lane < valid;
        const uint32_t d = active ? (uint32_t)(item[e] >> shift) & 255u : 0u;
        // lanes whose digit differs in some bit: ballot(bit) XOR this
        // lane's bit spread over 32 bits, OR-ed over the 8 bits
        uint32_t dlo = 0u, dhi = 0u;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t sb = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
            const uint64_t m = __ballot(sb != 0u);
            dlo |= (uint32_t)m ^ sb;
            dhi |= (uint32_t)(m >> 32) ^ sb;
        }
        const uint64_t peers = __ballot(active) & ~(((uint64_t)dhi << 32) | dlo);
        const uint32_t before = __popcll(peers & lt_mask);
        uint32_t cnt = 0;
        if (active) cnt = wcnt[d];
        __builtin_amdgcn_wave_barrier();
        if (active && before == 0) wcnt[d] = cnt + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rnk[e] = cnt + before;
        dig[e] = d;
    }
}

// cnt[d] += 1 for every active lane, aggregated over runs of equal d in
// consecutive lanes (neighbouring points of a curve often fall into the same
// bucket, and same-address LDS atomics serialise): the first lane of a run
// adds the run's length.  Returns each lane's count before it (its rank
// among the lanes counted so far with its d).  The inactive lanes are a
// suffix of the wave; every lane of the wave calls it.
__device__ __forceinline__ uint32_t run_atomic_add(uint32_t* cnt, uint32_t d, bool active) {
    const int lane = threadIdx.x & 63;
    const uint32_t dk = active ? d : 0xffffffffu;
    const uint32_t prev = __shfl_up(dk, 1);
    const bool head = active && (lane == 0 || prev != dk);
    const uint64_t heads = __ballot(head);
    const int nact = __popcll(__ballot(active));                             // all lanes vote: outside the branch
    const uint64_t below = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);     // lanes 0..lane
    uint32_t base = 0;
    if (head) {
        const uint64_t above = heads & ~below;
        const int next = above ? __ffsll((long long)above) - 1 : nact;
        base = atomicAdd(&cnt[d], (uint32_t)(next - lane));
    }
    const uint64_t upto = heads & below;
    const int h = (active && upto) ? 63 - __clzll((long long)upto) : lane;
    return __shfl(base, h) + (uint32_t)(lane - h);
}

// Items of a wave segment that starts at seg0 when lim items exist.
template <int ITEMS>
__device__ __forceinline__ int seg_valid(int64_t seg0, int64_t lim) {
    const int64_t v = lim - seg0;
    return v <= 0 ? 0 : (v >= 64 * ITEMS ? 64 * ITEMS : (int)v);
}

// After every wave has ranked a tile (and a barrier): per digit, the waves'
// exclusive offsets within the digit (wcnt), the tile's count (tcount) and
// the digit's first slot in the tile's digit order (tstart).  Ends with a
// barrier.
template <int NT, int ITEMS>
__device__ __forceinline__ void tile_offsets(SortShared<NT, ITEMS>& sh) {
    constexpr int W = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (tid < 256) {
        uint32_t run = 0;
        for (int w2 = 0; w2 < W; ++w2) {
            const uint32_t c = sh.wcnt[w2][tid];
            sh.wcnt[w2][tid] = run;
            run += c;
        }
        sh.tcount[tid] = run;
        // inclusive scan of the counts over the 256 digits: per wave, then across waves
        uint32_t v = run;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(v, off);
            if (lane >= off) v += o;
        }
        if (lane == 63) sh.wtot[tid >> 6] = v;
        sh.tstart[tid] = v - run;
    }
    __syncthreads();
    if (tid >= 64 && tid < 256) {
        uint32_t add = 0;
        for (int w2 = 0; w2 < (tid >> 6); ++w2) add += sh.wtot[w2];
        sh.tstart[tid] += add;
    }
    __syncthreads();
}

// Phase order of n points at `period`: A[k] = (phase key << 32 | index) of
// the k-th point, and (Sect. 2.3.2) the padded residuals in that order.
// Three stable 8-bit LSD passes over 24-bit keys, ranked with wave ballots:
// the first computes the keys from t (t -> A), the second moves A -> B, the
// last B -> A and writes the padded copies.  Each run of equal keys is then
// reordered by the full FP64 phase and the input index (and its padded
// copies rewritten).  With PREFETCH every pass loads its next tile before
// ranking the current one.
template <int NT, bool PREFETCH, int ITEMS = kSortItems>
__device__ void fold_sort_core(const double* __restrict__ t, int64_t n, double period, uint64_t* A, uint64_t* B,
                               const PadOut& po, SortShared<NT, ITEMS>& sh) {
    constexpr int W = NT / 64;
    constexpr int TILE = NT * ITEMS;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    for (int k = tid; k < 3 * 256; k += NT) (&sh.hist[0][0])[k] = 0;
    for (int k = tid; k < W * 256; k += NT) (&sh.wcnt[0][0])[k] = 0;
    for (int k = tid; k < 256; k += NT) sh.lastkey[k] = 0xffffffffu;   // keys are < 2^24
    if (tid == 0) sh.tie_n = 0;
    __syncthreads();
    for (int64_t i = tid; i < n; i += NT) {
        const uint32_t key = phase_key(phase_of(t[i], period));
        atomicAdd(&sh.hist[0][key & 255u], 1u);
        atomicAdd(&sh.hist[1][(key >> 8) & 255u], 1u);
        atomicAdd(&sh.hist[2][key >> 16], 1u);
    }
    __syncthreads();
    if (tid < 3) {
        uint32_t run = 0;
        for (int d = 0; d < 256; ++d) {
            const uint32_t c = sh.hist[tid][d];
            sh.hist[tid][d] = run;
            run += c;
        }
    }
    __syncthreads();

    const bool gather = po.rpad != nullptr;
    for (int pass = 0; pass < 3; ++pass) {
        const uint64_t* src = (pass == 2) ? B : A;
        uint64_t* dst = (pass == 1) ? B : A;
        if (tid < 256) sh.dbase[tid] = sh.hist[pass][tid];
        __syncthreads();
        const int shift = 32 + 8 * pass;
        // tile items: the fold itself on the first pass, the previous pass's output after
        auto fetch = [&](int64_t tile0, uint64_t (&it)[ITEMS]) {
            const int64_t seg0 = tile0 + (int64_t)wave * 64 * ITEMS;
#pragma unroll
            for (int e = 0; e < ITEMS; ++e) {
                const int64_t idx = seg0 + e * 64 + lane;
                if (idx < n) {
                    it[e] = (pass == 0) ? (((uint64_t)phase_key(phase_of(t[idx], period)) << 32) | (uint32_t)idx)
                                        : src[idx];
                } else {
                    it[e] = 0ull;
                }
            }
        };
        uint64_t item[ITEMS], nxt[PREFETCH ? ITEMS : 1];
        fetch(0, item);
        for (int64_t tile0 = 0; tile0 < n; tile0 += TILE) {
            if constexpr (!PREFETCH) {
                if (tile0 > 0) fetch(tile0, item);
            }
            const int64_t seg0 = tile0 + (int64_t)wave * 64 * ITEMS;
            uint32_t dig[ITEMS], rnk[ITEMS];
            wave_rank<ITEMS>(item, seg_valid<ITEMS>(seg0, n), shift, sh.wcnt[wave], dig, rnk);
            if constexpr (PREFETCH) {
                if (tile0 + TILE < n) fetch(tile0 + TILE, nxt);
            }
            __syncthreads();
            tile_offsets(sh);
            // the tile in digit order (stable: waves, then items, then lanes, follow input order) ...
#pragma unroll
            for (int e = 0; e < ITEMS; ++e) {
                const int64_t idx = seg0 + e * 64 + lane;
                if (idx < n) sh.buf[sh.tstart[dig[e]] + sh.wcnt[wave][dig[e]] + rnk[e]] = item[e];
            }
            __syncthreads();
            // ... written out by consecutive threads: each digit's run lands contiguously
            const int tn = (int)min((int64_t)TILE, n - tile0);
            for (int i = tid; i < tn; i += NT) {
                const uint64_t it = sh.buf[i];
                const uint32_t d = (uint32_t)(it >> shift) & 255u;
                const uint32_t pos = sh.dbase[d] + (uint32_t)i - sh.tstart[d];
                if (pos < (uint32_t)n) {
                    dst[pos] = it;
                    if (pass == 2) {
                        if (gather) pad_store(po, n, pos, (uint32_t)it);
                        // the word before it in the output: the previous one of its digit's run in this
                        // tile, or the last one an earlier tile wrote for the digit
                        const uint32_t key = (uint32_t)(it >> 32);
                        const uint32_t prev = (uint32_t)i > sh.tstart[d] ? (uint32_t)(sh.buf[i - 1] >> 32)
                                                                         : sh.lastkey[d];
                        if (key == prev) {
                            const uint32_t slot = atomicAdd(&sh.tie_n, 1u);
                            if (slot < (uint32_t)kTieCap) sh.tie_pos[slot] = pos;
                        }
                    }
                }
            }
            __syncthreads();
            if (tid < 256) {
                sh.dbase[tid] += sh.tcount[tid];
                if (pass == 2 && sh.tcount[tid] > 0)
                    sh.lastkey[tid] = (uint32_t)(sh.buf[sh.tstart[tid] + sh.tcount[tid] - 1] >> 32);
            }
            for (int k = tid; k < W * 256; k += NT) (&sh.wcnt[0][0])[k] = 0;
            __syncthreads();
            if constexpr (PREFETCH) {
#pragma unroll
                for (int e = 0; e < ITEMS; ++e) item[e] = nxt[e];
            }
        }
    }
    // A: order by 24-bit key, equal keys in input order.  Equal keys may hide
    // different phases: order each run by the full FP64 phase, then input
    // index (insertion sort; runs are short), and rewrite its padded copies.
    // The last pass listed every position whose key equals its predecessor's;
    // a run is fixed by the thread holding its first pair.  When the list
    // overflowed, every position is checked instead (8 consecutive positions
    // per thread and trip, their 10 keys loaded at once).
    auto fix_run = [&](int64_t k, uint32_t kk) {
        int64_t e = k + 1;
        while (e + 1 < n && (uint32_t)(A[e + 1] >> 32) == kk) ++e;
        for (int64_t x = k + 1; x <= e; ++x) {
            const uint64_t v = A[x];
            int64_t y = x;
            while (y > k && key_less(v, A[y - 1], t, period)) {
                A[y] = A[y - 1];
                --y;
            }
            A[y] = v;
        }
        if (gather)
            for (int64_t x = k; x <= e; ++x) pad_store(po, n, x, (uint32_t)A[x]);
    };
    const uint32_t nties = sh.tie_n;
    if (nties <= (uint32_t)kTieCap) {
        for (uint32_t q = tid; q < nties; q += NT) {
            const int64_t k = (int64_t)sh.tie_pos[q] - 1;
            const uint32_t kk = (uint32_t)(A[k] >> 32);
            if (k > 0 && (uint32_t)(A[k - 1] >> 32) == kk) continue;   // not its run's first pair
            fix_run(k, kk);
        }
    } else {
        for (int64_t k0 = (int64_t)tid * 8; k0 + 1 < n; k0 += (int64_t)NT * 8) {
            uint32_t kv[10];
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const int64_t p = k0 - 1 + q;
                kv[q] = (p >= 0 && p < n) ? (uint32_t)(A[p] >> 32) : 0xffffffffu;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t k = k0 + j;
                const uint32_t kk = kv[j + 1];
                if (k + 1 >= n || kk != kv[j + 2] || kv[j] == kk) continue;
                fix_run(k, kk);
            }
        }
    }
    __syncthreads();
}

// The same order in two phases over 32-bit keys floor(phi 2^32), with
// atomic (unstable) counting; the order is still unique, since each group of
// equal 16-bit key prefixes is finally ranked by (key, FP64 phase, index).
//   1. the top 8 key bits: a histogram of the buckets, then per tile of
//      input points a rank of each point within its bucket (LDS atomics),
//      the tile gathered in bucket order in LDS and written to the buckets'
//      runs of A (t -> A);
//   2. LDS tiles of whole buckets (at most NT * ITEMS points and
//      kTileBuckets buckets): the same counting step over the next kSubBits
//      key bits of each bucket (kBins bins); each word's place in its bin
//      is the number of the bin's words that precede it in (key, phase,
//      index) order; the tile is written back to A in place with its padded
//      copies.
// A then holds (32-bit key << 32 | index) in phase order; its indices are
// those of the three-pass sort.  Returns false, leaving A and the padded
// copies to be rewritten, when a bucket holds more than NT * ITEMS points or
// a bin more than kBinCap (more than kBinCap phases within 2^-17 of a
// period); the caller then runs fold_sort_core.
constexpr int kTileBuckets = 8;
constexpr int kSubBits = 9;                          // key bits below the bucket that pick a bin
constexpr int kBins = kTileBuckets << kSubBits;
constexpr uint32_t kBinCap = 1024;

template <int NT>
struct SortTwoPhase {
    uint32_t bins[kBins];        // per tile: counts, then first slots, of (bucket, next digit) bins
    uint32_t wsum[NT / 64];
    int32_t tiles[257];          // first bucket of each LDS tile, then 256
    int32_t ntiles;
    int32_t fallback;
};

template <int NT, int ITEMS>
__device__ bool fold_sort_twophase(const double* __restrict__ t, int64_t n, double period, uint64_t* A,
                                   const PadOut& po, SortShared<NT, ITEMS>& sh, SortTwoPhase<NT>& sx) {
    constexpr int TILE = NT * ITEMS;
    constexpr int BPT = kBins / NT;      // bins per thread in the scan
    static_assert(kBins % NT == 0 && ITEMS % 2 == 0 && TILE < 65536, "bins per thread, halves of a tile, slots");
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    uint32_t* const off = sh.hist[2];    // bucket d: first position in A
    for (int k = tid; k < 256; k += NT) {
        off[k] = 0;
        sh.tcount[k] = 0;
    }
    if (tid == 0) sx.fallback = 0;
    __syncthreads();
    // ITEMS loads in flight per thread before the keys are counted
    for (int64_t i0 = 0; i0 < n; i0 += (int64_t)NT * ITEMS) {
        double tv[ITEMS];
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) {
            const int64_t i = i0 + (int64_t)e * NT + tid;
            tv[e] = i < n ? t[i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < ITEMS; ++e)
            (void)run_atomic_add(off, phase_key32(phase_of(tv[e], period)) >> 24, i0 + (int64_t)e * NT + tid < n);
    }
    __syncthreads();
    // wave 0: exclusive offsets of 256 counts (four per lane) into dst, and
    // whether any count exceeds cap
    auto scan256 = [&](const uint32_t* cnt, uint32_t* dst, uint32_t cap) {
        uint32_t c[4], sum = 0, mx = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = cnt[4 * lane + q];
            sum += c[q];
            mx = max(mx, c[q]);
        }
        uint32_t v = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(v, o);
            if (lane >= o) v += u;
        }
        uint32_t run = v - sum;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dst[4 * lane + q] = run;
            run += c[q];
        }
        return __ballot(mx > cap) != 0ull;
    };
    if (wave == 0) {
        const bool big = scan256(off, off, (uint32_t)TILE);
        if (lane == 0 && big) sx.fallback = 1;
    }
    __syncthreads();
    if (sx.fallback) return false;
    if (wave == 0) {
        // LDS tiles: greedy runs of whole buckets, at most TILE points and
        // kTileBuckets buckets.  Bucket d joins the tile opened at bucket b
        // while off[d + 1] <= off[b] + TILE and d - b < kTileBuckets; both
        // hold for a prefix of the lanes, whose count is the step.
        auto end_of = [&](int d) -> uint32_t { return d + 1 < 256 ? off[d + 1] : (uint32_t)n; };
        int b = 0, nt = 0;
        while (b < 256) {
            if (lane == 0) sx.tiles[nt] = b;
            ++nt;
            const uint32_t lim = off[b] + (uint32_t)TILE;
            const int b0 = b;
            for (;;) {
                const int d = b + lane;
                const uint64_t acc = __ballot(d < 256 && d - b0 < kTileBuckets && end_of(d) <= lim);
                const int cnt = __popcll(acc);
                b += cnt;
                if (cnt < 64) break;
            }
        }
        if (lane == 0) {
            sx.tiles[nt] = 256;
            sx.ntiles = nt;
        }
    }
    for (int k = tid; k < 256; k += NT) sh.dbase[k] = off[k];
    __syncthreads();

    // 1. the top-digit pass, t -> A; the next tile's times are loaded while
    // the current tile is ranked and written
    double tv[ITEMS];
    auto fetch = [&](int64_t tile0) {
        const int64_t seg0 = tile0 + (int64_t)wave * 64 * ITEMS;
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) {
            const int64_t idx = seg0 + e * 64 + lane;
            tv[e] = idx < n ? t[idx] : 0.0;
        }
    };
    uint64_t item[ITEMS];
    uint32_t rk[ITEMS];
    fetch(0);
    for (int64_t tile0 = 0; tile0 < n; tile0 += TILE) {
        {
            const int64_t seg0 = tile0 + (int64_t)wave * 64 * ITEMS;
#pragma unroll
            for (int e = 0; e < ITEMS; ++e)
                item[e] = ((uint64_t)phase_key32(phase_of(tv[e], period)) << 32) | (uint32_t)(seg0 + e * 64 + lane);
        }
        const int valid = seg_valid<ITEMS>(tile0 + (int64_t)wave * 64 * ITEMS, n);
#pragma unroll
        for (int e = 0; e < ITEMS; ++e)
            rk[e] = run_atomic_add(sh.tcount, (uint32_t)(item[e] >> 56), e * 64 + lane < valid);
        if (tile0 + TILE < n) fetch(tile0 + TILE);
        __syncthreads();
        if (wave == 0) (void)scan256(sh.tcount, sh.tstart, 0xffffffffu);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < ITEMS; ++e)
            if (e * 64 + lane < valid) sh.buf[sh.tstart[(uint32_t)(item[e] >> 56)] + rk[e]] = item[e];
        __syncthreads();
        const int tn = (int)min((int64_t)TILE, n - tile0);
        for (int i = tid; i < tn; i += NT) {
            const uint64_t it = sh.buf[i];
            const uint32_t d = (uint32_t)(it >> 56);
            const uint32_t pos = sh.dbase[d] + (uint32_t)i - sh.tstart[d];
            if (pos < (uint32_t)n) A[pos] = it;
        }
        __syncthreads();
        if (tid < 256) {
            sh.dbase[tid] += sh.tcount[tid];
            sh.tcount[tid] = 0;
        }
        __syncthreads();
    }

    // 2. LDS tiles of whole buckets (no prefetch of the next tile: its
    // registers would push the kernel into spills)
    const bool gather = po.rpad != nullptr;
    const int ntiles = sx.ntiles;
    const int wseg = wave * 64 * ITEMS + lane;           // this lane's first position in a tile
    auto tile_base = [&](int j) -> uint32_t { return off[sx.tiles[j]]; };
    auto tile_end = [&](int j) -> uint32_t { return sx.tiles[j + 1] < 256 ? off[sx.tiles[j + 1]] : (uint32_t)n; };
    auto load = [&](int j, uint64_t (&it)[ITEMS]) {
        const uint32_t base = tile_base(j);
        const int m = (int)(tile_end(j) - base);
        const uint64_t* src = A + base + wseg;
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) it[e] = wseg + e * 64 < m ? src[e * 64] : 0ull;
    };
    for (int j = 0; j < ntiles; ++j) {
        load(j, item);
        const uint32_t base = tile_base(j);
        const int m = (int)(tile_end(j) - base);
        const uint32_t bin0 = (uint32_t)sx.tiles[j] << kSubBits;
        const int nbins = (sx.tiles[j + 1] - sx.tiles[j]) << kSubBits;
        const int valid = seg_valid<ITEMS>(wave * 64 * ITEMS, m);
        for (int k = tid; k < nbins; k += NT) sx.bins[k] = 0;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < ITEMS; ++e)
            if (e * 64 + lane < valid) rk[e] = atomicAdd(&sx.bins[(uint32_t)(item[e] >> (56 - kSubBits)) - bin0], 1u);
        __syncthreads();
        // exclusive scan of the nbins counts: BPT consecutive bins per thread
        uint32_t c[BPT], sum = 0;
        bool big = false;
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int k = tid * BPT + q;
            c[q] = k < nbins ? sx.bins[k] : 0u;
            sum += c[q];
            big |= c[q] > kBinCap;
        }
        uint32_t v = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(v, o);
            if (lane >= o) v += u;
        }
        if (lane == 63) sx.wsum[wave] = v;
        if (big) sx.fallback = 1;
        __syncthreads();
        if (sx.fallback) return false;
        uint32_t run = v - sum;
        for (int w2 = 0; w2 < wave; ++w2) run += sx.wsum[w2];
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int k = tid * BPT + q;
            if (k < nbins) sx.bins[k] = run;
            run += c[q];
        }
        __syncthreads();
        // each word into its bin's run, then its place within the run: the
        // number of the run's words ordered before it (the runs are short;
        // the ITEMS words of a thread step through their runs together)
        uint32_t span[ITEMS];                 // the bin's first slot | its end << 16 (slots < 2^16)
        int steps = 0;
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) {
            span[e] = 0u;
            if (e * 64 + lane < valid) {
                const uint32_t b = (uint32_t)(item[e] >> (56 - kSubBits)) - bin0;
                const uint32_t r0 = sx.bins[b];
                const uint32_t r1 = (int)b + 1 < nbins ? sx.bins[b + 1] : (uint32_t)m;
                span[e] = r0 | (r1 << 16);
                sh.buf[r0 + rk[e]] = item[e];
                steps = max(steps, (int)(r1 - r0));
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) rk[e] = 0u;
        // keys first; a word that meets an equal key in its run (phases
        // within 2^-32) is recounted with the full order
        uint32_t ties = 0u;
        for (int q = 0; q < steps; ++q) {
#pragma unroll
            for (int e = 0; e < ITEMS; ++e) {
                const uint32_t x = (span[e] & 0xffffu) + (uint32_t)q;
                if (x < (span[e] >> 16)) {
                    const uint64_t o = sh.buf[x];
                    const uint32_t ko = (uint32_t)(o >> 32), ki = (uint32_t)(item[e] >> 32);
                    rk[e] += ko < ki ? 1u : 0u;
                    if (ko == ki && o != item[e]) ties |= 1u << e;
                }
            }
        }
        if (ties) {
#pragma unroll
            for (int e = 0; e < ITEMS; ++e) {
                if (ties & (1u << e)) {
                    // (key, FP64 phase, index) order; this word's phase computed once
                    const uint64_t me = item[e];
                    const uint32_t kme = (uint32_t)(me >> 32);
                    const double pme = phase_of(t[(uint32_t)me], period);
                    uint32_t r = 0u;
                    for (uint32_t x = span[e] & 0xffffu; x < (span[e] >> 16); ++x) {
                        const uint64_t o = sh.buf[x];
                        const uint32_t ko = (uint32_t)(o >> 32);
                        if (ko < kme) {
                            ++r;
                        } else if (ko == kme && o != me) {
                            const double po = phase_of(t[(uint32_t)o], period);
                            if (po < pme || (po == pme && (uint32_t)o < (uint32_t)me)) ++r;
                        }
                    }
                    rk[e] = r;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < ITEMS; ++e)
            if (e * 64 + lane < valid) sh.buf[(span[e] & 0xffffu) + rk[e]] = item[e];
        __syncthreads();
        // the sorted tile to A and its padded copies, in two halves: every
        // residual (and weight) of a half gathered before any is stored
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            constexpr int HI = ITEMS / 2;
            uint64_t wd[HI];
            double rv[HI], wv[HI];
#pragma unroll
            for (int e = 0; e < HI; ++e) {
                const int i = (h * HI + e) * NT + tid;
                wd[e] = i < m ? sh.buf[i] : 0ull;
            }
            if (gather) {
#pragma unroll
                for (int e = 0; e < HI; ++e) {
                    const bool in = (h * HI + e) * NT + tid < m;
                    const uint32_t idx = (uint32_t)wd[e];
                    rv[e] = in ? po.r[idx] : 0.0;
                    wv[e] = in && po.wpad ? po.w[idx] : 0.0;
                }
            }
#pragma unroll
            for (int e = 0; e < HI; ++e) {
                const int i = (h * HI + e) * NT + tid;
                if (i < m) {
                    A[base + i] = wd[e];
                    if (gather) pad_put(po, n, (int64_t)base + i, rv[e], wv[e]);
                }
            }
        }
        __syncthreads();
    }
    return true;
}

// Moving-average depth: prefix sums of 1 - y over the npad padded positions
// (position k holding sorted point k mod n), from the final order in A.
template <int NT, int ITEMS = kSortItems>
__device__ void pad_prefix(const uint64_t* __restrict__ A, int64_t n, int64_t npad, const int64_t* __restrict__ u,
                           void* pfx, bool f32, SortShared<NT, ITEMS>& sh) {
    const int tid = threadIdx.x;
    if (!pfx) return;
    const int64_t chunk = (npad + NT - 1) / NT;
    const int64_t c0 = (int64_t)tid * chunk, c1 = min(npad, c0 + chunk);
    if (!f32) {
        // Exact prefix sums of the integer deficits: pfx[k] = sum_{m<k} u[perm[m mod n]].
        __int128* pf = (__int128*)pfx;
        __int128 s = 0;
        for (int64_t k = c0; k < c1; ++k) s += (__int128)u[(uint32_t)A[k < n ? k : k - n]];
        sh.part[tid] = s;
        __syncthreads();
        if (tid == 0) {
            __int128 run = 0;
            for (int q = 0; q < NT; ++q) {
                const __int128 c = sh.part[q];
                sh.part[q] = run;
                run += c;
            }
        }
        __syncthreads();
        __int128 run = sh.part[tid];
        if (tid == 0) pf[0] = 0;
        for (int64_t k = c0; k < c1; ++k) {
            run += (__int128)u[(uint32_t)A[k < n ? k : k - n]];
            pf[k + 1] = run;
        }
    } else {
        // FP32C: Kahan-compensated prefix sums of (float)(1 - y), stored as
        // unevaluated (hi, lo) pairs; chunk totals combined the same way.
        float2* pf = (float2*)pfx;
        float2* part = (float2*)sh.part;
        float hi = 0.f, lo = 0.f;
        for (int64_t k = c0; k < c1; ++k) {
            const float x = (float)ldexp((double)u[(uint32_t)A[k < n ? k : k - n]], -53);
            float sum, err;
            two_sum(hi, x, sum, err);
            hi = sum;
            lo += err;
        }
        part[tid] = make_float2(hi, lo);
        __syncthreads();
        if (tid == 0) {
            float rh = 0.f, rl = 0.f;
            for (int q = 0; q < NT; ++q) {
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
            const float x = (float)ldexp((double)u[(uint32_t)A[k < n ? k : k - n]], -53);
            float sum, err;
            two_sum(hi, x, sum, err);
            hi = sum;
            lo += err;
            pf[k + 1] = make_float2(hi, lo);
        }
    }
    __syncthreads();
}

// Largest D over the durations valid at `period`.
__device__ __forceinline__ int64_t max_points(int64_t n, double period, const double* __restrict__ durs, int nd,
                                              const gtls_params& prm) {
    int64_t dp = 0;
    for (int j = 0; j < nd; ++j)
        if (duration_valid(period, durs[j], prm)) dp = max(dp, points_in(n, period, durs[j]));
    return dp;
}

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

// One workgroup per period of the batch.
__global__ __launch_bounds__(kSortThreads, 4) void k_fold_sort(SortArgs a) {
    __shared__ SortShared<kSortThreads> sh;
    __shared__ SortTwoPhase<kSortThreads> sx;
    const int pl = blockIdx.x;
    const double period = a.periods[pl];
    const int64_t n = a.n;
    uint64_t* A = a.keys_a + (size_t)pl * n;
    uint64_t* B = a.keys_b + (size_t)pl * n;
    if (threadIdx.x == 0) sh.dpad = max_points(n, period, a.durations, a.nd, a.prm);
    __syncthreads();
    const int64_t npad = n + sh.dpad;
    const size_t es = a.f32 ? sizeof(float) : sizeof(double);
    const size_t ps = a.f32 ? sizeof(float2) : sizeof(__int128);
    PadOut po{a.r, a.w, a.rpad ? (char*)a.rpad + (size_t)pl * a.pstride * es : nullptr,
              a.wpad ? (char*)a.wpad + (size_t)pl * a.pstride * es : nullptr, npad, a.f32 != 0};
    if (!fold_sort_twophase<kSortThreads, kSortItems>(a.t, n, period, A, po, sh, sx))
        fold_sort_core<kSortThreads, true>(a.t, n, period, A, B, po, sh);
    pad_prefix<kSortThreads>(A, n, npad, a.u, a.pfx ? (char*)a.pfx + (size_t)pl * (a.pstride + 1) * ps : nullptr,
                             a.f32 != 0, sh);
    if (po.rpad) {
        for (int64_t k = npad + threadIdx.x; k < npad + kOverRead; k += kSortThreads) {
            if (a.f32) {
                ((float*)po.rpad)[k] = 0.0f;
                if (po.wpad) ((float*)po.wpad)[k] = 0.0f;
            } else {
                ((double*)po.rpad)[k] = 0.0;
                if (po.wpad) ((double*)po.wpad)[k] = 0.0;
            }
        }
    }
    if (a.perm_out) {
        int32_t* po = a.perm_out + (size_t)pl * n;
        for (int64_t k = threadIdx.x; k < n; k += kSortThreads) po[k] = (int32_t)(uint32_t)A[k];
    }
}

// ------------------------------------------------------------------------
// Template table: row D holds the D-point ideal transit, zero-padded to a
// multiple of 32 and preceded by 32 zeros (the last row is followed by 32
// more), so any (period, duration) item reads its template as a uniform
// stream through the scalar cache, and a 16-point read that starts up to 31
// points before the row or ends up to 31 points after it sees zeros there.  FP32C keeps a float copy.  With
// constant weights the per-window b = sum_k w s_k^2 and the template sum
// s1 = sum_k s_k depend on D only; they are summed once per D, in FP64 and
// in the same sequential order as a per-window evaluation.

constexpr int kTGuard = 32;
__host__ __device__ __forceinline__ int64_t trow_off(int64_t d) {
    const int64_t m = d - 1, a = m / 32, b = m % 32;
    return 32 * (16 * a * (a + 1) + (a + 1) * b) + kTGuard * d;
}
__host__ __device__ __forceinline__ int64_t rup32(int64_t d) { return (d + 31) & ~(int64_t)31; }

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// One block per D in [1, dcap]; table holds trow_off(dcap + 1) elements.
template <typename T>
__global__ __launch_bounds__(256) void k_tmpl_table(const double* __restrict__ tm, int32_t nt, int64_t dcap,
                                                    T* __restrict__ table) {
    const int64_t d = (int64_t)blockIdx.x + 1;
    T* row = table + trow_off(d);
    const int64_t w = rup32(d);
    for (int64_t k = threadIdx.x; k < w; k += 256) row[k] = (k < d) ? (T)resample(tm, nt, d, k) : (T)0;
    if (threadIdx.x < kTGuard) {
        row[(int)threadIdx.x - kTGuard] = (T)0;
        if (d == dcap) row[w + threadIdx.x] = (T)0;
    }
}

// b_D = sum_k fma(w, s_k^2, .) and s1_D = sum_k s_k, sequential in k, over
// the table's template values (FP32C sums its float template in FP64).
template <typename T>
__global__ __launch_bounds__(64) void k_tmpl_sums(const T* __restrict__ table, int64_t dmax, const uint64_t* misc,
                                                  double* __restrict__ bsum, double* __restrict__ s1sum) {
    const int64_t d = (int64_t)blockIdx.x * 64 + threadIdx.x + 1;
    if (d > dmax) return;
    const double wc = __longlong_as_double((long long)misc[kWminBits]);
    const T* row = table + trow_off(d);
    double b = 0.0, s1 = 0.0;
    for (int64_t k = 0; k < d; ++k) {
        const double sv = (double)row[k];
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
    // Strided items: row tasks (16 lanes each) packed four to a wave task.
    int32_t* toff;           // [bp nd] first row slot of item (queue index)
    int32_t* tcnt;           // [bp nd] row slots of item (0: not strided)
    int32_t* rowmap;         // [row slots] item of the slot (queue index), -1: empty
    int32_t* wfirst;         // [waves] first row slot of the wave task
    int32_t* cell_s;         // [cells + 1] planner: row slots per cell, then their exclusive scan
    int32_t* cell_w;         // [cells + 1] planner: wave tasks per cell, then their exclusive scan
    ItemBest* sb;            // [row slots] best of each row
    uint32_t* queue;         // [2 kXcds + 2] pop counters, queue starts, total, unit-item count
    int32_t rmax;            // most windows per lane (the FP32C rule keeps it at 4)
    int32_t rcost;           // 1: windows per lane by the wave-chunk count (FP64), 0: the FP32C rule
    // Every-offset items (stride 1), listed by the planner: item pl nd + j,
    // longest durations first, then period.
    int32_t* ulist;          // [bp nd]
    int32_t* ucnt;           // [bp nd] planner scratch: 1 per every-offset item in list order
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

__device__ __forceinline__ ItemBest* item_slot(const SlideArgs& a, const ItemInfo& it) {
    return a.items + ((size_t)it.pl * a.nd + it.j) * a.ntiles + it.tile;
}

// Writes a (block-reduced) best into the item's slot.
__device__ __forceinline__ void store_best(const Best& b, const SlideArgs& a, const ItemInfo& it, int64_t evals,
                                           int ntiles) {
    if (threadIdx.x == 0) {
        ItemBest* out = item_slot(a, it);
        out->dchi2 = b.dchi2;
        out->depth = b.depth;
        out->start = (int32_t)b.start;
        out->d = (int32_t)it.d;
        out->evals = (int32_t)evals;
        if (it.tile == 0) out->ntiles = ntiles;
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

// Geometry of one (period, duration) item on its padded curve.
struct SlideItem {
    int64_t n, D, stride, limit, dpad;
    const void* rp;          // T padded residuals of this period
    const void* wp;          // T padded weights (varying weights only)
    const void* pf;          // prefix sums of this period (moving-average depth only)
    const void* trow;        // T template row of D
    double bconst, s1;       // constant-weight b and template sum for D
};

// Block-wide first-best (largest dchi2, then smallest start), returned to
// every thread.
__device__ __forceinline__ Best block_best(Best best, Best* red) {
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
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    Best b = red[0];
    for (int q = 1; q < kSlideThreads / 64; ++q) {
        const Best o = red[q];
        if (o.dchi2 > b.dchi2 || (o.dchi2 == b.dchi2 && o.start >= 0 && (b.start < 0 || o.start < b.start))) b = o;
    }
    return b;
}

// Every T0 offset (stride 1), windows [i0, i0 + 4096): each lane owns 16
// consecutive windows; their correlation sums advance together over a
// padded LDS copy of the curve, with the template streamed from the table
// into scalar registers.  Returns the lane's first best window.
template <typename T, bool VARW, bool MEAN>
__device__ Best slide_unit_tile(const SlideItem& si, int64_t i0, T* x_sh, T* xw_sh) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int64_t n = si.n, D = si.D;
    const T* __restrict__ rp = (const T*)si.rp;
    const T* __restrict__ wp = (const T*)si.wp;
    const cptr<T> trow = (cptr<T>)si.trow;
    const int base = tid * kR;
    const bool busy = i0 + (int64_t)wave * 64 * kR < n;     // wave has at least one window
    double acc[kR], bacc[VARW ? kR : 1];
#pragma unroll
    for (int m = 0; m < kR; ++m) acc[m] = 0.0;
#pragma unroll
    for (int m = 0; m < (VARW ? kR : 1); ++m) bacc[m] = 0.0;
    for (int64_t k0 = 0; k0 < si.dpad; k0 += kKC) {
        const int kc = (int)min((int64_t)kKC, si.dpad - k0);
        __syncthreads();
        const int nx = kTile + kc + kR;
        {
            // all of this lane's loads in flight before the first LDS write
            constexpr int kPer = (kXs + kSlideThreads - 1) / kSlideThreads;
            T v[kPer], vw[VARW ? kPer : 1];
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int e = tid + q * kSlideThreads;
                const int64_t g = i0 + k0 + e;
                const bool ok = e < nx && g < si.limit;
                v[q] = ok ? rp[g] : (T)0;
                if constexpr (VARW) vw[q] = ok ? wp[g] : (T)0;
            }
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int e = tid + q * kSlideThreads;
                if (e < nx) {
                    x_sh[xpad<T>(e)] = v[q];
                    if constexpr (VARW) xw_sh[xpad<T>(e)] = vw[q];
                }
            }
        }
        __syncthreads();
        if (!busy) continue;
        chunk_correlate<T, false>(acc, x_sh, base, kc, trow + k0);
        if constexpr (VARW) chunk_correlate<T, true>(bacc, xw_sh, base, kc, trow + k0);
    }
    Best best{-INFINITY, 0.0, -1};
#pragma unroll
    for (int m = 0; m < kR; ++m) {
        const int64_t i = i0 + base + m;
        if (i < n) {
            double dchi2, depth;
            fit<MEAN>(acc[m], VARW ? bacc[m] : si.bconst, window_deficit<T, MEAN>(si.pf, i, D), si.s1, dchi2,
                      depth);
            consider(best, dchi2, depth, i);
        }
    }
    return best;
}

// Strided T0 grid (stride s >= 2).  A wave works on a run of windows; each
// lane owns R consecutive windows m, m + 1, ..., m + R - 1, which start s
// points apart, so one curve point x[m s + j] serves all of them: window r
// takes it with template point j - r s.  The lane walks j upward over its
// own contiguous run of the padded curve in chunks of 16 points.
constexpr int kSC = 16;                             // j steps per chunk
constexpr int kRunCap = 1024;                       // FP32C rule: (R - 1) s + 32 <= kRunCap

// Windows per lane for FP32C, the rule the single-curve and batched searches
// share (their float partial sums depend on R): the largest of 8, 4, 2 (at
// most rmax) that still gives `fill` lanes a window each and keeps a lane's
// run within kRunCap points beyond D, when consecutive windows overlap
// (s < D); else 1.
__host__ __device__ __forceinline__ int strided_r(int64_t nw, int64_t s, int64_t d, int64_t fill, int rmax) {
    if (s >= d) return 1;
    auto fits = [&](int r) { return nw >= r * fill && (r - 1) * s + 2 * kSC <= kRunCap; };
    if (rmax >= 8 && fits(8)) return 8;
    if (rmax >= 4 && fits(4)) return 4;
    if (fits(2)) return 2;
    return 1;
}

// First-best over the 64 lanes (largest dchi2, then smallest start).
__device__ __forceinline__ Best wave_best(Best best) {
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
    return best;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Windows [m_lo, m_hi) of one strided item on one wave (the persistent
// single-curve kernel and the batched megakernel); returns the wave's first
// best on every lane.  Operands:
//  - each 16-point chunk of the 64 lanes' runs is loaded cooperatively: 8
//    lanes (FP64) or 4 lanes (FP32) read one lane's chunk as 16-byte pieces,
//    so one load instruction touches 8 or 16 runs instead of 64; the pieces
//    go to a per-wave LDS buffer of 64 padded rows and every lane reads its
//    own row back;
//  - the template block of window r (16 points from c0 - r s) is loaded from
//    the table with lane l holding point l mod 16, and each multiply-add takes
//    its template point by a DPP row broadcast from lane u of the 16-lane row,
//    so no template value passes through LDS.
// Windows outside their span in a chunk multiply template zeros (the row
// guards), which leaves their sums unchanged exactly (every curve value is
// finite), so every window sums its D products in ascending template order.
template <typename T>
constexpr int kPiece = 16 / (int)sizeof(T);                  // points per 16-byte piece
template <typename T>
constexpr int kStRow = kSC + kPiece<T>;                      // staging row stride (points), 16-byte pad
template <typename T>
constexpr int kStage = 64 * kStRow<T>;                       // staging points per wave and array

template <typename T>
struct Piece {
    T v[kPiece<T>];
};

template <typename T>
__device__ __forceinline__ Piece<T> load_piece(const T* p) {
    Piece<T> r;
    __builtin_memcpy(&r, p, 16);
    return r;
}

// acc[r] = fma(t, x, acc[r]) for every window r, with t the value of tv[r]
// in lane (l & ~15) + U of the lane's 16-lane row (a DPP row broadcast).  One
// fused multiply-add instruction per window, so the broadcast values are never
// materialised in registers.  The leading s_nop 1 gives the two wait states a
// DPP read needs after a vector ALU write of any of its registers; inside the
// block every instruction writes a different accumulator, so the next block's
// read of an accumulator is at least two wait states after its write as well.
#define GTLS_DPP(OP, A, T, X, U) OP " %" #A ", %" #T ", %" #X " row_newbcast:%" #U " row_mask:0xf bank_mask:0xf\n\t"
#define GTLS_DPP_FMAC_SET(TY, OP)                                                                                  \
    template <int U>                                                                                               \
    __device__ __forceinline__ void dpp_fmac(TY(&acc)[1], const TY(&tv)[1], TY x) {                                \
        asm volatile("s_nop 1\n\t" GTLS_DPP(OP, 0, 1, 2, 3) : "+v"(acc[0]) : "v"(tv[0]), "v"(x), "i"(U));        \
    }                                                                                                              \
    template <int U>                                                                                               \
    __device__ __forceinline__ void dpp_fmac(TY(&acc)[2], const TY(&tv)[2], TY x) {                                \
        asm volatile("s_nop 1\n\t" GTLS_DPP(OP, 0, 2, 4, 5) GTLS_DPP(OP, 1, 3, 4, 5)                             \
                     : "+v"(acc[0]), "+v"(acc[1])                                                                  \
                     : "v"(tv[0]), "v"(tv[1]), "v"(x), "i"(U));                                                    \
    }                                                                                                              \
    template <int U>                                                                                               \
    __device__ __forceinline__ void dpp_fmac(TY(&acc)[4], const TY(&tv)[4], TY x) {                                \
        asm volatile("s_nop 1\n\t" GTLS_DPP(OP, 0, 4, 8, 9) GTLS_DPP(OP, 1, 5, 8, 9) GTLS_DPP(OP, 2, 6, 8, 9)      \
                         GTLS_DPP(OP, 3, 7, 8, 9)                                                                  \
                     : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])                                      \
                     : "v"(tv[0]), "v"(tv[1]), "v"(tv[2]), "v"(tv[3]), "v"(x), "i"(U));                            \
    }                                                                                                              \
    template <int U>                                                                                               \
    __device__ __forceinline__ void dpp_fmac(TY(&acc)[8], const TY(&tv)[8], TY x) {                                \
        asm volatile("s_nop 1\n\t" GTLS_DPP(OP, 0, 8, 16, 17) GTLS_DPP(OP, 1, 9, 16, 17)                          \
                         GTLS_DPP(OP, 2, 10, 16, 17) GTLS_DPP(OP, 3, 11, 16, 17) GTLS_DPP(OP, 4, 12, 16, 17)       \
                             GTLS_DPP(OP, 5, 13, 16, 17) GTLS_DPP(OP, 6, 14, 16, 17) GTLS_DPP(OP, 7, 15, 16, 17)   \
                     : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),         \
                       "+v"(acc[6]), "+v"(acc[7])                                                                  \
                     : "v"(tv[0]), "v"(tv[1]), "v"(tv[2]), "v"(tv[3]), "v"(tv[4]), "v"(tv[5]), "v"(tv[6]),         \
                       "v"(tv[7]), "v"(x), "i"(U));                                                                \
    }
GTLS_DPP_FMAC_SET(double, "v_fmac_f64_dpp")
GTLS_DPP_FMAC_SET(float, "v_fmac_f32_dpp")
#undef GTLS_DPP_FMAC_SET
#undef GTLS_DPP

// f(integral_constant<int, k>) for k = 0 .. N - 1, in order.
template <int N, typename F, int... K>
__device__ __forceinline__ void unrolled_impl(F&& f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void unrolled(F&& f) {
    unrolled_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// The 16 template steps of one chunk in ascending order.  The template
// block covers two chunks, two points per lane: point j of chunk H sits in
// lane 8 H + j / 2 of every row, in tlo for even j and thi for odd j.
template <typename T, int R, int H, int J>
__device__ __forceinline__ void dpp_step(T (&acc)[R], const T (&tlo)[R], const T (&thi)[R], const T (&x)[kSC]) {
    if constexpr (J % 2 == 0) dpp_fmac<8 * H + J / 2>(acc, tlo, x[J]);
    else dpp_fmac<8 * H + J / 2>(acc, thi, x[J]);
}
template <typename T, int R, int H, int... J>
__device__ __forceinline__ void dpp_chunk(T (&acc)[R], const T (&tlo)[R], const T (&thi)[R], const T (&x)[kSC],
                                          std::integer_sequence<int, J...>) {
    (dpp_step<T, R, H, J>(acc, tlo, thi, x), ...);
}

// Loads sizeof(V) bytes at a 32-bit byte offset from a wave-uniform base
// (one address register per lane; the base stays in scalar registers).
template <typename V>
__device__ __forceinline__ V load_at(const void* base, uint32_t byte_off) {
    V v;
    __builtin_memcpy(&v, (const char*)base + byte_off, sizeof(V));
    return v;
}

template <typename T, bool VARW, bool MEAN, int R>
__device__ Best strided_windows_coop(const SlideItem& si, int64_t m_lo, int64_t m_hi, T* stage, T* stage_w) {
    constexpr int P = kPiece<T>;
    constexpr int NP = kSC / P;                     // pieces per row = load instructions per chunk
    constexpr int OPI = 64 / NP;                    // runs per load instruction
    const int lane = threadIdx.x & 63;
    const int a = lane / NP, q = lane % NP;
    const int64_t s = si.stride, D = si.D;
    const T* __restrict__ rp = (const T*)si.rp;
    const T* __restrict__ wp = (const T*)si.wp;
    const T* __restrict__ tbase = (const T*)si.trow - 2 * kSC;   // the row's 32 leading zeros
    const int64_t J = D + (R - 1) * s;              // points of a lane's run
    const int64_t nch = (J + kSC - 1) / kSC;
    const uint32_t tl = (uint32_t)(lane & 15) * 2 * sizeof(T);
    T* const srow = stage + lane * kStRow<T>;
    T* const srow_w = VARW ? stage_w + lane * kStRow<T> : nullptr;

    // Template block of window r for the two chunks from c0: lane l holds
    // points c0 - r s + 2 (l mod 16) and the next (one load per window per
    // two chunks).  Blocks wholly before the row read its 32 leading zeros,
    // blocks at or past its end the zeros that follow it, so no branch is
    // needed.
    struct TPair {
        T lo, hi;
    };
    auto tload = [&](int64_t c0, TPair (&tv)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t klo = c0 - (int64_t)r * s;
            const int64_t kc = klo <= -2 * kSC ? -2 * kSC : (klo >= D ? D : klo);
            tv[r] = load_at<TPair>(tbase, (uint32_t)(kc + 2 * kSC) * (uint32_t)sizeof(T) + tl);
        }
    };
    auto stage_get = [&](const T* row, T (&x)[kSC]) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const Piece<T> pc = *reinterpret_cast<const Piece<T>*>(row + i * P);
#pragma unroll
            for (int e = 0; e < P; ++e) x[i * P + e] = pc.v[e];
        }
    };
    // products of chunk H (0: the first of the template block's two chunks)
    auto products = [&](auto hc, double (&acc)[R], double (&bacc)[VARW ? R : 1], const T (&x)[kSC],
                        const T (&xw)[VARW ? kSC : 1], const TPair (&tv)[R]) {
        constexpr int H = decltype(hc)::value;
        T tlo[R], thi[R], qlo[VARW ? R : 1], qhi[VARW ? R : 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            tlo[r] = tv[r].lo;
            thi[r] = tv[r].hi;
            if constexpr (VARW) {
                qlo[r] = tv[r].lo * tv[r].lo;
                qhi[r] = tv[r].hi * tv[r].hi;
            }
        }
        if constexpr (sizeof(T) == 8) {
            dpp_chunk<T, R, H>(acc, tlo, thi, x, std::make_integer_sequence<int, kSC>{});
            if constexpr (VARW) dpp_chunk<T, R, H>(bacc, qlo, qhi, xw, std::make_integer_sequence<int, kSC>{});
        } else {
            T ca[R], cq[R];
#pragma unroll
            for (int r = 0; r < R; ++r) ca[r] = cq[r] = (T)0;
            dpp_chunk<T, R, H>(ca, tlo, thi, x, std::make_integer_sequence<int, kSC>{});
            if constexpr (VARW) dpp_chunk<T, R, H>(cq, qlo, qhi, xw, std::make_integer_sequence<int, kSC>{});
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] += (double)ca[r];
                if constexpr (VARW) bacc[r] += (double)cq[r];
            }
        }
    };

    Best best{-INFINITY, 0.0, -1};
    for (int64_t g0 = m_lo; g0 < m_hi; g0 += 64 * R) {
        const int64_t ml = g0 + (int64_t)lane * R;
        // Byte offset of this lane's piece in the run it loads (lanes past the
        // range re-read a valid run).  A piece that starts at or past the end
        // of the padded curve (n + D points) is read from that end instead:
        // the row holds at least kOverRead finite points there, and such
        // points meet only template zeros or windows past the task's range.
        uint32_t cb[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i)
            cb[i] = (uint32_t)((min(g0 + (int64_t)(i * OPI + a) * R, m_hi - 1) * s + q * P) * (int64_t)sizeof(T));
        const uint32_t cend = (uint32_t)(si.limit * (int64_t)sizeof(T));
        auto xload = [&](const T* __restrict__ src, int64_t c0, Piece<T> (&nx)[NP]) {
            const uint32_t co = (uint32_t)c0 * (uint32_t)sizeof(T);
#pragma unroll
            for (int i = 0; i < NP; ++i) nx[i] = load_at<Piece<T>>(src, min(cb[i] + co, cend));
        };
        auto stage_put = [&](T* buf, const Piece<T> (&nx)[NP]) {
#pragma unroll
            for (int i = 0; i < NP; ++i)
                *reinterpret_cast<Piece<T>*>(buf + (i * OPI + a) * kStRow<T> + q * P) = nx[i];
        };
        // chunk c0 from the loads in flight to this lane's registers, via LDS
        auto restage = [&](Piece<T> (&nx)[NP], Piece<T> (&nw)[VARW ? NP : 1], T (&x)[kSC],
                           T (&xw)[VARW ? kSC : 1]) {
            wave_sync();
            stage_put(stage, nx);
            if constexpr (VARW) stage_put(stage_w, nw);
            wave_sync();
            stage_get(srow, x);
            if constexpr (VARW) stage_get(srow_w, xw);
        };

        double acc[R], bacc[VARW ? R : 1];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
        for (int r = 0; r < (VARW ? R : 1); ++r) bacc[r] = 0.0;
        // Chunks go two by two (j even), one template block per window for
        // both.  Chunk j's curve pieces are requested while chunk j - 2 is
        // being computed, written to LDS and read back into the other half of
        // x while chunk j - 1 is computed; the block for chunks j and j + 1 is
        // requested right after the products of chunks j - 4 and j - 3.  So
        // no product waits on a load.  Two pairs per trip keep the template
        // slot indices constant.  Chunks past the run (at most one) are
        // computed too, on clamped addresses and template zeros, so every
        // register is written every trip.
        T x[2][kSC], xw[2][VARW ? kSC : 1];
        TPair tv[2][R];
        Piece<T> nx[NP], nw[VARW ? NP : 1];
        auto pieces = [&](int64_t j) {
            xload(rp, j * kSC, nx);
            if constexpr (VARW) xload(wp, j * kSC, nw);
        };
        pieces(0);
        tload(0, tv[0]);
        tload(2 * kSC, tv[1]);
        restage(nx, nw, x[0], xw[0]);
        pieces(1);
        auto pair = [&](auto slotc, int64_t j) {
            constexpr int sl = decltype(slotc)::value;
            restage(nx, nw, x[1], xw[1]);
            pieces(j + 2);
            products(std::integral_constant<int, 0>{}, acc, bacc, x[0], xw[0], tv[sl]);
            restage(nx, nw, x[0], xw[0]);
            pieces(j + 3);
            products(std::integral_constant<int, 1>{}, acc, bacc, x[1], xw[1], tv[sl]);
            tload((j + 4) * kSC, tv[sl]);
        };
        const int64_t npair = (nch + 1) / 2;
        int64_t c = 0;
        for (; c + 2 <= npair; c += 2) {
            pair(std::integral_constant<int, 0>{}, 2 * c);
            pair(std::integral_constant<int, 1>{}, 2 * c + 2);
        }
        if (c < npair) pair(std::integral_constant<int, 0>{}, 2 * c);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t m = ml + r;
            if (m < m_hi) {
                const int64_t i = m * s;
                double dchi2, depth;
                fit<MEAN>(acc[r], VARW ? bacc[r] : si.bconst, window_deficit<T, MEAN>(si.pf, i, D), si.s1, dchi2,
                          depth);
                consider(best, dchi2, depth, i);
            }
        }
    }
    return wave_best(best);
}

// FP64 takes R in {4, 8} (strided_r_cost; RMAX = 4 for the batched
// megakernel, whose other phases hold many registers), FP32C R in {1, 2, 4}
// (strided_r with at most 4, the rule both searches share).
template <typename T, bool VARW, bool MEAN, int RMAX = 8>
__device__ Best strided_windows_coop_r(int R, const SlideItem& si, int64_t m_lo, int64_t m_hi, T* stage,
                                       T* stage_w) {
    if constexpr (sizeof(T) == 8) {
        if constexpr (RMAX >= 8) {
            if (R == 8) return strided_windows_coop<T, VARW, MEAN, 8>(si, m_lo, m_hi, stage, stage_w);
        }
        return strided_windows_coop<T, VARW, MEAN, 4>(si, m_lo, m_hi, stage, stage_w);
    } else {
        switch (R) {
            case 4: return strided_windows_coop<T, VARW, MEAN, 4>(si, m_lo, m_hi, stage, stage_w);
            case 2: return strided_windows_coop<T, VARW, MEAN, 2>(si, m_lo, m_hi, stage, stage_w);
            default: return strided_windows_coop<T, VARW, MEAN, 1>(si, m_lo, m_hi, stage, stage_w);
        }
    }
}

// ------------------------------------------------------------------------
// Row-packed strided slide (single-curve search).  A wave is four rows of 16
// lanes; each row works on windows of one strided item (period, duration),
// so small items (the same duration at neighbouring periods of an XCD's
// list) share a wave instead of leaving most of its lanes idle, while an
// item with many windows fills all four rows itself.  Within a row the
// template points are broadcast from a lane of the row (DPP row broadcast),
// so each row follows its own item's stride and duration.  The wave's loop
// runs over the longest run of its rows; a shorter row meets template zeros
// past its run, which leaves its sums unchanged.
constexpr int kRowLanes = 16;
constexpr int kRowMax = 64;          // rows per strided item
constexpr int kCellItems = 2;        // neighbouring periods whose rows share waves

struct RowItem {
    const void* rp;                  // T padded residuals of the row's period
    const void* wp;                  // T padded weights (varying weights only)
    const void* pf;                  // prefix sums (moving-average depth only)
    const void* trow;                // T template row of D
    int64_t D, s, limit;             // points, T0 step, end of the padded curve
    int64_t m_lo, m_hi;              // windows of this pass
    double bconst, s1;
    bool active;                     // the row has windows in this pass
};

template <typename V>
__device__ __forceinline__ V pick4(int k, V v0, V v1, V v2, V v3) {
    return k == 0 ? v0 : (k == 1 ? v1 : (k == 2 ? v2 : v3));
}

// Windows [m_lo, m_hi) of each active row on one wave, R windows per lane
// (lane l of row k owns windows m_lo + l R .. + R - 1, s points apart);
// returns the lane's first best over its windows, merged into `best`.
template <typename T, bool VARW, bool MEAN, int R>
__device__ void strided_rows(const RowItem (&ri)[4], Best& best, int64_t& evals, T* stage, T* stage_w) {
    constexpr int P = kPiece<T>;
    constexpr int NP = kSC / P;                     // pieces per run chunk = load instructions per chunk
    constexpr int OPI = 64 / NP;                    // runs per load instruction
    const int lane = threadIdx.x & 63;
    const int row = lane >> 4, lp = lane & 15;
    const int a = lane / NP, q = lane % NP;
    // this lane's row
    const bool act = pick4(row, ri[0].active, ri[1].active, ri[2].active, ri[3].active);
    const int64_t s = pick4(row, ri[0].s, ri[1].s, ri[2].s, ri[3].s);
    const int64_t D = pick4(row, ri[0].D, ri[1].D, ri[2].D, ri[3].D);
    const int64_t m_lo = pick4(row, ri[0].m_lo, ri[1].m_lo, ri[2].m_lo, ri[3].m_lo);
    const int64_t m_hi = pick4(row, ri[0].m_hi, ri[1].m_hi, ri[2].m_hi, ri[3].m_hi);
    const T* __restrict__ tbase = (const T*)pick4(row, ri[0].trow, ri[1].trow, ri[2].trow, ri[3].trow) - 2 * kSC;
    const uint32_t tl = (uint32_t)(lane & 15) * 2 * sizeof(T);
    T* const srow = stage + lane * kStRow<T>;
    T* const srow_w = VARW ? stage_w + lane * kStRow<T> : nullptr;
    // the longest run over the active rows (a row with no windows in this
    // pass loads the first active row's curve and contributes nothing)
    int64_t J = 0;
    int first = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (ri[k].active) {
            J = max(J, ri[k].D + (int64_t)(R - 1) * ri[k].s);
            if (first < 0) first = k;
        }
    const int64_t nch = (J + kSC - 1) / kSC;

    struct TPair {
        T lo, hi;
    };
    auto tload = [&](int64_t c0, TPair (&tv)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t klo = c0 - (int64_t)r * s;
            // a block wholly before or after the window is zeros: not loaded
            if (klo > -2 * kSC && klo < D)
                tv[r] = load_at<TPair>(tbase, (uint32_t)(klo + 2 * kSC) * (uint32_t)sizeof(T) + tl);
            else
                tv[r] = TPair{(T)0, (T)0};
        }
    };
    auto stage_get = [&](const T* rowp, T (&x)[kSC]) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const Piece<T> pc = *reinterpret_cast<const Piece<T>*>(rowp + i * P);
#pragma unroll
            for (int e = 0; e < P; ++e) x[i * P + e] = pc.v[e];
        }
    };
    auto products = [&](auto hc, double (&acc)[R], double (&bacc)[VARW ? R : 1], const T (&x)[kSC],
                        const T (&xw)[VARW ? kSC : 1], const TPair (&tv)[R]) {
        constexpr int H = decltype(hc)::value;
        T tlo[R], thi[R], qlo[VARW ? R : 1], qhi[VARW ? R : 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            tlo[r] = tv[r].lo;
            thi[r] = tv[r].hi;
            if constexpr (VARW) {
                qlo[r] = tv[r].lo * tv[r].lo;
                qhi[r] = tv[r].hi * tv[r].hi;
            }
        }
        if constexpr (sizeof(T) == 8) {
            dpp_chunk<T, R, H>(acc, tlo, thi, x, std::make_integer_sequence<int, kSC>{});
            if constexpr (VARW) dpp_chunk<T, R, H>(bacc, qlo, qhi, xw, std::make_integer_sequence<int, kSC>{});
        } else {
            T ca[R], cq[R];
#pragma unroll
            for (int r = 0; r < R; ++r) ca[r] = cq[r] = (T)0;
            dpp_chunk<T, R, H>(ca, tlo, thi, x, std::make_integer_sequence<int, kSC>{});
            if constexpr (VARW) dpp_chunk<T, R, H>(cq, qlo, qhi, xw, std::make_integer_sequence<int, kSC>{});
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] += (double)ca[r];
                if constexpr (VARW) bacc[r] += (double)cq[r];
            }
        }
    };

    // Loader pieces: piece i of this lane belongs to run o = i OPI + a, whose
    // row o / 16 = i OPI / 16 is the same for every lane of the wave.
    const T* rbase[NP];
    const T* wbase[VARW ? NP : 1];
    uint32_t cb[NP], cend[NP];
    const void* frp = pick4(first, ri[0].rp, ri[1].rp, ri[2].rp, ri[3].rp);
    const void* fwp = pick4(first, ri[0].wp, ri[1].wp, ri[2].wp, ri[3].wp);
    const int64_t flimit = pick4(first, ri[0].limit, ri[1].limit, ri[2].limit, ri[3].limit);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int k = (i * OPI) >> 4;             // the same for every lane once unrolled
        const bool ka = ri[k].active;
        rbase[i] = (const T*)(ka ? ri[k].rp : frp);
        if constexpr (VARW) wbase[i] = (const T*)(ka ? ri[k].wp : fwp);
        const int lo = (i * OPI + a) & 15;        // owner's lane in its row
        const int64_t mrun = ka ? min(ri[k].m_lo + (int64_t)lo * R, ri[k].m_hi - 1) : 0;
        cb[i] = (uint32_t)((mrun * (ka ? ri[k].s : 0) + q * P) * (int64_t)sizeof(T));
        cend[i] = (uint32_t)((ka ? ri[k].limit : flimit) * (int64_t)sizeof(T));
    }
    auto xload = [&](bool w, int64_t c0, Piece<T> (&nx)[NP]) {
        const uint32_t co = (uint32_t)c0 * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < NP; ++i) nx[i] = load_at<Piece<T>>(w ? wbase[VARW ? i : 0] : rbase[i], min(cb[i] + co, cend[i]));
    };
    auto stage_put = [&](T* buf, const Piece<T> (&nx)[NP]) {
#pragma unroll
        for (int i = 0; i < NP; ++i) *reinterpret_cast<Piece<T>*>(buf + (i * OPI + a) * kStRow<T> + q * P) = nx[i];
    };
    auto restage = [&](Piece<T> (&nx)[NP], Piece<T> (&nw)[VARW ? NP : 1], T (&x)[kSC], T (&xw)[VARW ? kSC : 1]) {
        wave_sync();
        stage_put(stage, nx);
        if constexpr (VARW) stage_put(stage_w, nw);
        wave_sync();
        stage_get(srow, x);
        if constexpr (VARW) stage_get(srow_w, xw);
    };

    double acc[R], bacc[VARW ? R : 1];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
    for (int r = 0; r < (VARW ? R : 1); ++r) bacc[r] = 0.0;
    T x[2][kSC], xw[2][VARW ? kSC : 1];
    TPair tv[2][R];
    Piece<T> nx[NP], nw[VARW ? NP : 1];
    auto pieces = [&](int64_t j) {
        xload(false, j * kSC, nx);
        if constexpr (VARW) xload(true, j * kSC, nw);
    };
    pieces(0);
    tload(0, tv[0]);
    tload(2 * kSC, tv[1]);
    restage(nx, nw, x[0], xw[0]);
    pieces(1);
    auto pair = [&](auto slotc, int64_t j) {
        constexpr int sl = decltype(slotc)::value;
        restage(nx, nw, x[1], xw[1]);
        pieces(j + 2);
        products(std::integral_constant<int, 0>{}, acc, bacc, x[0], xw[0], tv[sl]);
        restage(nx, nw, x[0], xw[0]);
        pieces(j + 3);
        products(std::integral_constant<int, 1>{}, acc, bacc, x[1], xw[1], tv[sl]);
        tload((j + 4) * kSC, tv[sl]);
    };
    const int64_t npair = (nch + 1) / 2;
    int64_t c = 0;
    for (; c + 2 <= npair; c += 2) {
        pair(std::integral_constant<int, 0>{}, 2 * c);
        pair(std::integral_constant<int, 1>{}, 2 * c + 2);
    }
    if (c < npair) pair(std::integral_constant<int, 0>{}, 2 * c);
    if (act) {
        const void* pf = pick4(row, ri[0].pf, ri[1].pf, ri[2].pf, ri[3].pf);
        const double bconst = pick4(row, ri[0].bconst, ri[1].bconst, ri[2].bconst, ri[3].bconst);
        const double s1 = pick4(row, ri[0].s1, ri[1].s1, ri[2].s1, ri[3].s1);
        const int64_t ml = m_lo + (int64_t)lp * R;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t m = ml + r;
            if (m < m_hi) {
                const int64_t i = m * s;
                double dchi2, depth;
                fit<MEAN>(acc[r], VARW ? bacc[r] : bconst, window_deficit<T, MEAN>(pf, i, D), s1, dchi2, depth);
                consider(best, dchi2, depth, i);
                ++evals;
            }
        }
    }
}

// First-best over the 16 lanes of each row (largest dchi2, then smallest
// start), returned to every lane of the row.
__device__ __forceinline__ Best row_best(Best best) {
    for (int off = 8; off > 0; off >>= 1) {
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
    return best;
}

// Windows per lane for the cooperative strided slide (FP64, where the sums do
// not depend on it): R = 4 or 8, whichever needs fewer wave-chunks,
// waves(R) * chunks(R) = ceil(ceil(nw / R) / 64) * ceil((D + (R - 1) s) / 16);
// a chunk costs about the same whatever R is (its loads and LDS traffic do
// not depend on R), so a partly idle wave with more windows per lane can
// beat full waves with fewer.  (Allowing R = 1 or 2 as well saves under 5 %
// of the wave-chunks on the 3000-day grid but costs registers: every R is
// compiled into the one persistent kernel.)  Ties go to R = 4.
__host__ __device__ __forceinline__ int strided_r_cost(int64_t nw, int64_t s, int64_t d) {
    int best_r = 4;
    int64_t best = -1;
    for (int r = 4; r <= 8; r *= 2) {
        const int64_t lanes = (nw + r - 1) / r;
        const int64_t cost = ((lanes + 63) / 64) * ((d + (r - 1) * s + kSC - 1) / kSC);
        if (best < 0 || cost < best) {
            best = cost;
            best_r = r;
        }
    }
    return best_r;
}

// Wave tasks of a strided item: its window groups (64 R windows each) split
// into at most max_tasks contiguous runs.
struct StridedSplit {
    int R;
    int64_t nw, groups;
    int ntask;
};

__host__ __device__ __forceinline__ StridedSplit strided_split(int64_t n, int64_t d, int64_t s, int64_t fill,
                                                               int64_t max_tasks, int rmax, bool by_cost = false) {
    StridedSplit sp;
    sp.nw = (n + s - 1) / s;
    sp.R = by_cost ? (rmax >= 8 ? strided_r_cost(sp.nw, s, d) : 4) : strided_r(sp.nw, s, d, fill, rmax);
    const int64_t lanes = (sp.nw + sp.R - 1) / sp.R;
    sp.groups = (lanes + 63) / 64;
    sp.ntask = (int)min(sp.groups, max_tasks);
    return sp;
}

// Windows of task t of ntask.
__host__ __device__ __forceinline__ void strided_task_range(const StridedSplit& sp, int t, int64_t& m_lo,
                                                            int64_t& m_hi) {
    const int64_t g_lo = sp.groups * t / sp.ntask, g_hi = sp.groups * (t + 1) / sp.ntask;
    const int64_t per = 64 * (int64_t)sp.R;
    m_lo = min(sp.nw, g_lo * per);
    m_hi = min(sp.nw, g_hi * per);
}

template <typename T, bool MEAN>
__device__ __forceinline__ SlideItem make_item(const SlideArgs& a, const ItemInfo& it, bool varw) {
    SlideItem si;
    si.n = a.n;
    si.D = it.d;
    si.stride = it.stride;
    si.limit = a.n + it.d;
    si.dpad = rup32(it.d);
    si.rp = (const T*)a.rpad + (size_t)it.pl * a.pstride;
    si.wp = varw ? (const void*)((const T*)a.wpad + (size_t)it.pl * a.pstride) : nullptr;
    si.pf = MEAN ? (const void*)((const char*)a.pfx + (size_t)it.pl * (a.pstride + 1) *
                                 (sizeof(T) == 8 ? sizeof(__int128) : sizeof(float2)))
                 : nullptr;
    si.trow = (const T*)a.table + trow_off(it.d);
    si.bconst = varw ? 0.0 : a.bsum[it.d];
    si.s1 = MEAN ? a.s1sum[it.d] : 0.0;
    return si;
}

constexpr int kPlanThreads = 1024;
constexpr int kXcds = 8;                 // MI355X: workgroups go round-robin over 8 XCDs (L2 domains)

// Every-offset items: work unit u = (list entry u / ntiles, window tile
// u mod ntiles), taken in list order by a grid-stride loop, so a launch is
// sized by the work and not by the period x duration grid.
template <typename T, bool VARW, bool MEAN>
__global__ __launch_bounds__(kSlideThreads) void k_slide_unit(SlideArgs a) {
    __shared__ T x_sh[xpad<T>(kXs)];
    __shared__ T xw_sh[VARW ? xpad<T>(kXs) : 1];
    __shared__ Best red[kSlideThreads / 64];
    const int64_t units = (int64_t)a.queue[2 * kXcds + 1] * a.ntiles;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int32_t item = a.ulist[u / a.ntiles];
        ItemInfo it;
        it.pl = item / a.nd;
        it.j = item - it.pl * a.nd;
        it.tile = (int)(u % a.ntiles);
        it.period = a.periods[it.pl];
        it.valid = true;
        it.d = points_in(a.n, it.period, a.durations[it.j]);
        it.stride = 1;
        const SlideItem si = make_item<T, MEAN>(a, it, VARW);
        const int64_t i0 = (int64_t)it.tile * kTile;
        const Best b = block_best(slide_unit_tile<T, VARW, MEAN>(si, i0, x_sh, xw_sh), red);
        store_best(b, a, it, min((int64_t)kTile, a.n - i0), a.ntiles);
    }
}


// Strided items in queue order: periods are dealt to kXcds queues (pl mod
// kXcds), each queue lists its periods in order, and each period its
// durations longest first, so the waves of one XCD work on a few periods at
// a time and their padded curves stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_periods(int bp, int x) { return (bp - x + kXcds - 1) / kXcds; }

__device__ __forceinline__ int64_t queue_index(int bp, int nd, int pl, int j) {
    const int x = pl % kXcds;
    int64_t off = 0;
    for (int y = 0; y < x; ++y) off += xcd_periods(bp, y);
    return (off + pl / kXcds) * nd + (nd - 1 - j);
}

__device__ __forceinline__ void queue_item(int bp, int nd, int64_t idx, int& pl, int& j) {
    int64_t q = idx / nd;
    const int jrev = (int)(idx - q * nd);
    int x = 0;
    for (; x < kXcds - 1; ++x) {
        const int64_t c = xcd_periods(bp, x);
        if (q < c) break;
        q -= c;
    }
    pl = (int)(q * kXcds + x);
    j = nd - 1 - jrev;
}

// Planning of one launch.
//  - Every-offset items (T0 step 1) are listed for k_slide_unit.
//  - Strided items are cut into row tasks: rows of 16 lanes with R windows
//    per lane, at most kRowMax rows per item (a row then takes several
//    consecutive groups of 16 R windows).  Rows are packed four to a wave
//    task within a cell: one duration at kCellItems neighbouring periods of
//    one XCD's list, consecutive items with the same R sharing waves.  Cells
//    are queued per XCD (the XCD's periods in order, blocks of kCellItems,
//    durations longest first), so an XCD works on a few periods at a time.
// k_plan_count (items): every-offset flags.  k_rplan_count (cells): row
// slots and wave tasks per cell.  k_plan_scan (one workgroup): the
// every-offset list, the cell scans and the XCD queue bounds
// (queue[kXcds + x] first wave task of XCD x, queue[2 kXcds] total,
// queue[2 kXcds + 1] every-offset items, pop counters reset).
// k_rplan_fill (cells): toff, tcnt, rowmap and wfirst.

// FP64 windows per lane for row tasks: R = 4 or 8, whichever needs fewer
// row-chunks, rows(R) x chunks(R) = ceil(ceil(nw / R) / 16) x
// ceil((D + (R - 1) s) / 16); ties go to R = 4.
__host__ __device__ __forceinline__ int strided_r_rows(int64_t nw, int64_t s, int64_t d) {
    int best_r = 4;
    int64_t best = -1;
    for (int r = 4; r <= 8; r *= 2) {
        const int64_t lanes = (nw + r - 1) / r;
        const int64_t cost = ((lanes + kRowLanes - 1) / kRowLanes) * ((d + (r - 1) * s + kSC - 1) / kSC);
        if (best < 0 || cost < best) {
            best = cost;
            best_r = r;
        }
    }
    return best_r;
}

__device__ __forceinline__ int64_t xcd_blocks(int bp, int x) {
    return (xcd_periods(bp, x) + kCellItems - 1) / kCellItems;
}

__device__ __forceinline__ int64_t cell_first(int bp, int nd, int x) {
    int64_t c = 0;
    for (int y = 0; y < x; ++y) c += xcd_blocks(bp, y) * nd;
    return c;
}

__device__ __forceinline__ int64_t cell_count(int bp, int nd) { return cell_first(bp, nd, kXcds); }

struct CellItem {
    int32_t idx;             // queue index of the item, -1: no period here
    bool strided;
    int R, rows;
};

struct CellPlan {
    CellItem it[kCellItems];
    int nsub;
    int sub_k0[kCellItems], sub_k1[kCellItems];  // items [k0, k1) of each subgroup (strided ones count)
    int sub_rows[kCellItems], sub_waves[kCellItems];
    int slots, waves;
};

// Row tasks of a strided item: windows per lane, windows, groups of
// 16 R windows, rows.
__device__ __forceinline__ void item_rows(const SlideArgs& a, int64_t d, int64_t st, int& R, int64_t& nw,
                                          int64_t& groups, int& rows) {
    nw = (a.n + st - 1) / st;
    R = a.rcost ? strided_r_rows(nw, st, d) : strided_r(nw, st, d, 64, a.rmax);
    groups = ((nw + R - 1) / R + kRowLanes - 1) / kRowLanes;
    rows = (int)min(groups, (int64_t)kRowMax);
}

__device__ void plan_cell(const SlideArgs& a, int64_t c, CellPlan& cp) {
    int x = 0;
    int64_t cx = c;
    for (; x < kXcds - 1; ++x) {
        const int64_t cc = xcd_blocks(a.bp, x) * a.nd;
        if (cx < cc) break;
        cx -= cc;
    }
    const int64_t b = cx / a.nd;
    const int j = a.nd - 1 - (int)(cx - b * a.nd);
    const int64_t npx = xcd_periods(a.bp, x);
    for (int k = 0; k < kCellItems; ++k) {
        CellItem& it = cp.it[k];
        it.idx = -1;
        it.strided = false;
        it.R = 0;
        it.rows = 0;
        const int64_t i = b * kCellItems + k;
        if (i >= npx) continue;
        const int pl = (int)(x + kXcds * i);
        it.idx = (int32_t)queue_index(a.bp, a.nd, pl, j);
        const double period = a.periods[pl], dur = a.durations[j];
        if (!duration_valid(period, dur, a.prm)) continue;
        const int64_t d = points_in(a.n, period, dur);
        const int64_t st = t0_stride(d, a.prm.dt0);
        if (st < 2) continue;
        int64_t nw, groups;
        it.strided = true;
        item_rows(a, d, st, it.R, nw, groups, it.rows);
    }
    cp.nsub = 0;
    cp.slots = 0;
    cp.waves = 0;
    int prev_r = 0;
    for (int k = 0; k < kCellItems; ++k) {
        if (!cp.it[k].strided) continue;
        if (cp.it[k].R != prev_r) {
            cp.sub_k0[cp.nsub] = k;
            cp.sub_rows[cp.nsub] = 0;
            ++cp.nsub;
            prev_r = cp.it[k].R;
        }
        cp.sub_k1[cp.nsub - 1] = k + 1;
        cp.sub_rows[cp.nsub - 1] += cp.it[k].rows;
    }
    for (int g = 0; g < cp.nsub; ++g) {
        cp.sub_waves[g] = (cp.sub_rows[g] + 3) / 4;
        cp.slots += 4 * cp.sub_waves[g];
        cp.waves += cp.sub_waves[g];
    }
}

__global__ __launch_bounds__(256) void k_plan_count(SlideArgs a) {
    const int64_t items = (int64_t)a.bp * a.nd;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= items) return;
    int pl, j;
    queue_item(a.bp, a.nd, idx, pl, j);
    const double period = a.periods[pl], dur = a.durations[j];
    int unit = 0;
    if (duration_valid(period, dur, a.prm)) unit = t0_stride(points_in(a.n, period, dur), a.prm.dt0) < 2;
    a.ucnt[(int64_t)(a.nd - 1 - j) * a.bp + pl] = unit;
}

__global__ __launch_bounds__(256) void k_rplan_count(SlideArgs a) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cell_count(a.bp, a.nd)) return;
    CellPlan cp;
    plan_cell(a, c, cp);
    a.cell_s[c] = cp.slots;
    a.cell_w[c] = cp.waves;
}

// In-place exclusive scan of v[0 .. m) by one workgroup, v[m] = total.
__device__ void block_scan(int32_t* v, int64_t m, int32_t* part) {
    const int tid = threadIdx.x;
    const int64_t per = (m + kPlanThreads - 1) / kPlanThreads;
    const int64_t lo = min(m, (int64_t)tid * per), hi = min(m, lo + per);
    int32_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += v[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const int32_t o = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += o;
        __syncthreads();
    }
    int32_t run = part[tid] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        const int32_t c = v[i];
        v[i] = run;
        run += c;
    }
    if (tid == kPlanThreads - 1) v[m] = part[kPlanThreads - 1];
    __syncthreads();
}

__global__ __launch_bounds__(kPlanThreads) void k_plan_scan(SlideArgs a) {
    __shared__ int32_t part[kPlanThreads];
    const int tid = threadIdx.x;
    const int64_t items = (int64_t)a.bp * a.nd;
    // the every-offset list (list order jrev bp + pl -> item pl nd + j)
    {
        const int64_t per = (items + kPlanThreads - 1) / kPlanThreads;
        const int64_t lo = min(items, (int64_t)tid * per), hi = min(items, lo + per);
        int32_t usum = 0;
        for (int64_t i = lo; i < hi; ++i) usum += a.ucnt[i];
        part[tid] = usum;
        __syncthreads();
        for (int off = 1; off < kPlanThreads; off <<= 1) {
            const int32_t o = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += o;
            __syncthreads();
        }
        int32_t uo = part[tid] - usum;
        for (int64_t i = lo; i < hi; ++i)
            if (a.ucnt[i]) {
                const int32_t jrev = (int32_t)(i / a.bp), pl = (int32_t)(i - (int64_t)jrev * a.bp);
                a.ulist[uo++] = pl * a.nd + (a.nd - 1 - jrev);
            }
        if (tid == 0) a.queue[2 * kXcds + 1] = (uint32_t)part[kPlanThreads - 1];
        __syncthreads();
    }
    const int64_t cells = cell_count(a.bp, a.nd);
    block_scan(a.cell_s, cells, part);
    block_scan(a.cell_w, cells, part);
    if (tid < kXcds) {
        a.queue[tid] = 0u;
        a.queue[kXcds + tid] = (uint32_t)a.cell_w[cell_first(a.bp, a.nd, tid)];
    }
    if (tid == kXcds) a.queue[2 * kXcds] = (uint32_t)a.cell_w[cells];
}

__global__ __launch_bounds__(256) void k_rplan_fill(SlideArgs a) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cell_count(a.bp, a.nd)) return;
    CellPlan cp;
    plan_cell(a, c, cp);
    for (int k = 0; k < kCellItems; ++k)
        if (cp.it[k].idx >= 0 && !cp.it[k].strided) {
            a.toff[cp.it[k].idx] = 0;
            a.tcnt[cp.it[k].idx] = 0;
        }
    int32_t slot = a.cell_s[c], wave = a.cell_w[c];
    for (int g = 0; g < cp.nsub; ++g) {
        int32_t r = 0;
        for (int k = cp.sub_k0[g]; k < cp.sub_k1[g]; ++k) {
            const CellItem& it = cp.it[k];
            if (!it.strided) continue;
            a.toff[it.idx] = slot + r;
            a.tcnt[it.idx] = it.rows;
            for (int t = 0; t < it.rows; ++t) a.rowmap[slot + r + t] = it.idx;
            r += it.rows;
        }
        for (; r < 4 * cp.sub_waves[g]; ++r) a.rowmap[slot + r] = -1;
        for (int w = 0; w < cp.sub_waves[g]; ++w) a.wfirst[wave + w] = slot + 4 * w;
        slot += 4 * cp.sub_waves[g];
        wave += cp.sub_waves[g];
    }
}

template <typename T, bool VARW, bool MEAN>
__device__ __forceinline__ void strided_rows_r(int R, const RowItem (&ri)[4], Best& best, int64_t& evals, T* stage,
                                               T* stage_w) {
    if constexpr (sizeof(T) == 8) {
        if (R == 8) strided_rows<T, VARW, MEAN, 8>(ri, best, evals, stage, stage_w);
        else strided_rows<T, VARW, MEAN, 4>(ri, best, evals, stage, stage_w);
    } else {
        switch (R) {
            case 4: strided_rows<T, VARW, MEAN, 4>(ri, best, evals, stage, stage_w); break;
            case 2: strided_rows<T, VARW, MEAN, 2>(ri, best, evals, stage, stage_w); break;
            default: strided_rows<T, VARW, MEAN, 1>(ri, best, evals, stage, stage_w); break;
        }
    }
}

// Persistent: every wave pops wave tasks from its XCD's queue, then from the
// others, until all are exhausted.  A wave task is four row slots; each
// non-empty one is a row of an item (its rows split the item's groups of
// 16 R windows evenly).  Two waves per SIMD for constant weights; per-point
// weights double the staged operands and keep one.
template <typename T, bool VARW, bool MEAN>
__global__ __launch_bounds__(kSlideThreads, VARW ? 1 : 2) void k_slide_rows(SlideArgs a) {
    __shared__ __align__(16) T stages[(kSlideThreads / 64) * (VARW ? 2 : 1) * kStage<T>];
    const int lane = threadIdx.x & 63;
    const int row = lane >> 4;
    T* stage = stages + (threadIdx.x >> 6) * (VARW ? 2 : 1) * kStage<T>;
    T* stage_w = VARW ? stage + kStage<T> : nullptr;
    const size_t pfs = sizeof(T) == 8 ? sizeof(__int128) : sizeof(float2);
    const int x0 = (int)(blockIdx.x % kXcds);
    for (int xk = 0; xk < kXcds; ++xk) {
        const int x = (x0 + xk) % kXcds;
        const uint32_t qb = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.queue[kXcds + x]);
        const uint32_t qe = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.queue[kXcds + x + 1]);
        for (;;) {
            // Every lane takes part in the pop (lane 0 adds 1, the rest 0) so
            // no divergent branch feeds the broadcast of lane 0's ticket.
            const uint32_t ticket = atomicAdd(&a.queue[x], lane == 0 ? 1u : 0u);
            const uint32_t w = qb + (uint32_t)__builtin_amdgcn_readfirstlane((int)ticket);
            if (w >= qe) break;
            const int32_t fs = __builtin_amdgcn_readfirstlane(a.wfirst[w]);
            RowItem ri[4];
            int64_t g_lo[4], g_n[4], nw[4], dk[4];
            int R = 0;
            int64_t G = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int32_t idx = __builtin_amdgcn_readfirstlane(a.rowmap[fs + k]);
                g_n[k] = 0;
                g_lo[k] = 0;
                nw[k] = 1;
                dk[k] = 0;
                ri[k].active = false;
                ri[k].rp = ri[k].wp = ri[k].pf = ri[k].trow = nullptr;
                ri[k].D = ri[k].s = ri[k].limit = ri[k].m_lo = ri[k].m_hi = 0;
                ri[k].bconst = ri[k].s1 = 0.0;
                if (idx < 0) continue;
                int pl, j;
                queue_item(a.bp, a.nd, idx, pl, j);
                const double period = a.periods[pl];
                const int64_t d = points_in(a.n, period, a.durations[j]);
                const int64_t st = t0_stride(d, a.prm.dt0);
                int Rk, rows;
                int64_t groups;
                item_rows(a, d, st, Rk, nw[k], groups, rows);
                if (k == 0) R = Rk;                  // every row of a wave task has the same R
                const int64_t t = (fs + k) - __builtin_amdgcn_readfirstlane(a.toff[idx]);
                g_lo[k] = groups * t / rows;
                g_n[k] = groups * (t + 1) / rows - g_lo[k];
                G = max(G, g_n[k]);
                dk[k] = d;
                ri[k].rp = (const T*)a.rpad + (size_t)pl * a.pstride;
                ri[k].wp = VARW ? (const void*)((const T*)a.wpad + (size_t)pl * a.pstride) : nullptr;
                ri[k].pf = MEAN ? (const void*)((const char*)a.pfx + (size_t)pl * (a.pstride + 1) * pfs) : nullptr;
                ri[k].trow = (const T*)a.table + trow_off(d);
                ri[k].D = d;
                ri[k].s = st;
                ri[k].limit = a.n + d;
                ri[k].bconst = VARW ? 0.0 : a.bsum[d];
                ri[k].s1 = MEAN ? a.s1sum[d] : 0.0;
            }
            // An empty slot (only past the first row of a wave task, whose
            // slot 0 always holds a row) takes row 0's curve, template and
            // sizes, so every address its lanes form stays valid; it has no
            // windows and its results are not written.
#pragma unroll
            for (int k = 1; k < 4; ++k)
                if (ri[k].rp == nullptr) {
                    ri[k].rp = ri[0].rp;
                    ri[k].wp = ri[0].wp;
                    ri[k].pf = ri[0].pf;
                    ri[k].trow = ri[0].trow;
                    ri[k].D = ri[0].D;
                    ri[k].s = ri[0].s;
                    ri[k].limit = ri[0].limit;
                    ri[k].bconst = ri[0].bconst;
                    ri[k].s1 = ri[0].s1;
                }
            Best best{-INFINITY, 0.0, -1};
            int64_t evals = 0;
            for (int64_t g = 0; g < G; ++g) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    ri[k].active = g < g_n[k];
                    ri[k].m_lo = min(nw[k], (g_lo[k] + g) * kRowLanes * R);
                    ri[k].m_hi = min(nw[k], ri[k].m_lo + (int64_t)kRowLanes * R);
                }
                strided_rows_r<T, VARW, MEAN>(R, ri, best, evals, stage, stage_w);
            }
            best = row_best(best);
            for (int off = 8; off > 0; off >>= 1) evals += __shfl_xor(evals, off);
            const int32_t my_idx = pick4(row, a.rowmap[fs], a.rowmap[fs + 1], a.rowmap[fs + 2], a.rowmap[fs + 3]);
            if ((lane & 15) == 0 && my_idx >= 0) {
                ItemBest* o = a.sb + fs + row;
                o->dchi2 = best.dchi2;
                o->depth = best.depth;
                o->start = (int32_t)best.start;
                o->d = (int32_t)pick4(row, dk[0], dk[1], dk[2], dk[3]);
                o->evals = (int32_t)evals;
                o->ntiles = 0;
            }
        }
    }
}

// ------------------------------------------------------------------------
// Per-period reduction over durations and the T0 of the best window.

struct ReduceArgs {
    const double* t;
    int64_t n;
    const double* periods;   // batch-offset
    const double* durations;
    gtls_params prm;
    int32_t bp;
    int32_t nd;
    const ItemBest* items;
    int32_t ntiles;
    const int32_t* toff;     // strided items: first row slot
    const int32_t* tcnt;     // ... and row slots
    const ItemBest* sb;
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
        const double period = a.periods[pl];
        for (int j = 0; j < a.nd; ++j) {
            if (!duration_valid(period, a.durations[j], a.prm)) continue;
            const ItemBest* slots = a.items + ((size_t)pl * a.nd + j) * a.ntiles;
            int nt = a.ntiles;
            if (t0_stride(points_in(a.n, period, a.durations[j]), a.prm.dt0) >= 2) {
                const int64_t idx = queue_index(a.bp, a.nd, pl, j);
                slots = a.sb + a.toff[idx];
                nt = a.tcnt[idx];
            }
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
// Periodogram statistics.  The device functions work on one segment (one
// curve's periodogram) so single and batched searches share them.

// SR, the sequential mean and population standard deviation, SDE_raw; one
// 256-thread workgroup.
__device__ void sde_stats_seg(const double* __restrict__ chi2, int32_t n, double* __restrict__ sr,
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

__global__ __launch_bounds__(256) void k_sde_stats(const double* __restrict__ chi2, int32_t n, double* __restrict__ sr,
                                                   double* __restrict__ raw) {
    sde_stats_seg(chi2, n, sr, raw);
}

// The median of v[0..window) as the element of rank window/2 (ties by
// position), so it is an input element exactly.
__device__ __forceinline__ double rank_median(const double* v, int window) {
    const int half = window / 2;
    double med = v[0];
    for (int aidx = 0; aidx < window; ++aidx) {
        const double x = v[aidx];
        int lt = 0, le_before = 0;
        for (int b = 0; b < window; ++b) {
            const double y = v[b];
            lt += (y < x);
            le_before += (y == x) & (b < aidx);
        }
        if (lt + le_before == half) {
            med = x;
            break;
        }
    }
    return med;
}

// SDE = SDE_raw - running median over `window` points, ends replicated.
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
    sde[i] = raw[i] - rank_median(v + threadIdx.x, window);
}

// Batched: each thread finds its curve's segment and gathers its window.
__global__ __launch_bounds__(kMedThreads) void k_sde_median_batch(const int64_t* __restrict__ poff, int32_t nc,
                                                                  const double* __restrict__ raw, int32_t window,
                                                                  double* __restrict__ sde) {
    const int64_t total = poff[nc];
    const int64_t i = (int64_t)blockIdx.x * kMedThreads + threadIdx.x;
    if (i >= total) return;
    int lo = 0, hi = nc;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (poff[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int64_t s0 = poff[lo], s1 = poff[lo + 1] - 1;
    const int half = window / 2;
    double med = 0.0;
    for (int aidx = 0; aidx < window; ++aidx) {
        int64_t ia = i - half + aidx;
        ia = ia < s0 ? s0 : (ia > s1 ? s1 : ia);
        const double x = raw[ia];
        int lt = 0, le_before = 0;
        for (int b = 0; b < window; ++b) {
            int64_t ib = i - half + b;
            ib = ib < s0 ? s0 : (ib > s1 ? s1 : ib);
            const double y = raw[ib];
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

// First argmax of SDE over a segment (NT threads).
template <int NT>
__device__ void argmax_seg(const double* __restrict__ sde, int32_t n, double& best_v, int& best_i) {
    __shared__ double bv[NT];
    __shared__ int bi[NT];
    const int tid = threadIdx.x;
    double v = -INFINITY;
    int idx = -1;
    for (int i = tid; i < n; i += NT) {
        if (sde[i] > v) {
            v = sde[i];
            idx = i;
        }
    }
    bv[tid] = v;
    bi[tid] = idx;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
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
    best_v = bv[0];
    best_i = bi[0];
}

__global__ __launch_bounds__(1024) void k_sde_argmax(const double* __restrict__ sde, int32_t n, gtls_summary* summary,
                                                     const uint64_t* misc) {
    double v;
    int i;
    argmax_seg<1024>(sde, n, v, i);
    if (threadIdx.x == 0 && summary) {
        summary->best_period = i;
        summary->sde_max = v;
        if (misc) {
            summary->chi2_null = __longlong_as_double((long long)misc[kChi2Null]);
            summary->n_evals = (int64_t)misc[kEvals];
            summary->n_macs = (int64_t)misc[kMacs];
        }
    }
}

__global__ __launch_bounds__(256) void k_sde_stats_batch(const int64_t* __restrict__ poff,
                                                         const double* __restrict__ chi2, double* __restrict__ sr,
                                                         double* __restrict__ raw) {
    const int c = blockIdx.x;
    const int64_t o = poff[c];
    sde_stats_seg(chi2 + o, (int32_t)(poff[c + 1] - o), sr + o, raw + o);
}

__global__ __launch_bounds__(256) void k_sde_argmax_batch(const int64_t* __restrict__ poff,
                                                          const double* __restrict__ sde,
                                                          const uint64_t* __restrict__ cmisc,
                                                          const unsigned long long* __restrict__ cevals,
                                                          gtls_summary* summaries) {
    const int c = blockIdx.x;
    const int64_t o = poff[c];
    double v;
    int i;
    argmax_seg<256>(sde + o, (int32_t)(poff[c + 1] - o), v, i);
    if (threadIdx.x == 0) {
        gtls_summary& s = summaries[c];
        s.best_period = i;
        s.sde_max = v;
        s.chi2_null = __longlong_as_double((long long)cmisc[(size_t)c * kMiscSlots + kChi2Null]);
        s.n_evals = (int64_t)cevals[2 * c];
        s.n_macs = (int64_t)cevals[2 * c + 1];
        s.pad_ = 0;
    }
}

// ------------------------------------------------------------------------
// Batched survey: many light curves in one persistent launch.
//
// Points of all curves are stored back to back (CSR offsets); each curve has
// its own period grid (CSR offsets) and all share the duration grid and the
// template.  (curve, period) work items are enumerated in queue order:
// curves sorted by decreasing length, then period index; workgroups of the
// persistent kernel pop items from one atomic counter and run the whole
// per-period pipeline (fold, sort, padding, every duration's slide, first
// best) in workgroup-private scratch.

constexpr int kBatchThreads = 256;
constexpr int kBatchSortItems = 16;   // words per thread of a sort tile (4096-word tiles)
constexpr int kMaxBatchDurations = 64;

struct BatchArgs {
    const int64_t* offsets;      // [nc + 1] point offsets
    const double* t;
    int32_t nc;
    const int64_t* poffsets;     // [nc + 1] period offsets
    const double* periods;
    const double* durations;
    int32_t nd;
    gtls_params prm;
    const double* w;             // per point (global index)
    const double* r;
    const int64_t* u;
    const uint64_t* cmisc;       // [nc][kMiscSlots]
    const void* table;           // T template rows (shared)
    const double* tmpl;          // FP64 template samples
    int32_t nt;
    const double* s1sum;         // [D] template sums
    const int32_t* order;        // [nc] curves in queue order
    const int64_t* qoff;         // [nc + 1] first item of each queued curve
    int64_t total;               // items
    unsigned long long* queue;   // item counter
    uint64_t* scr_a;             // [grid][scr_n]
    uint64_t* scr_b;
    char* scr_r;                 // [grid][scr_pstride] T
    char* scr_w;
    char* scr_pf;                // [grid][scr_pstride + 1] prefix elements
    int64_t scr_n, scr_pstride;
    int64_t item_limit;          // stop after this many items (autotuning runs)
    double* chi2;                // [total periods] CSR outputs
    int32_t* best_dur;
    int32_t* best_start;
    double* depth;
    double* t0;
    unsigned long long* cevals;  // [nc][2] windows and template multiply-adds
};

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Per-curve preparation: weights, residuals, exact deficits, min/max weight,
// min time and the null chi2 (sequential Neumaier, input order).
__global__ __launch_bounds__(256) void k_prep_batch(const int64_t* __restrict__ offsets, const double* __restrict__ t,
                                                    const double* __restrict__ y, const double* __restrict__ dy,
                                                    double* __restrict__ w, double* __restrict__ r,
                                                    int64_t* __restrict__ u, uint64_t* __restrict__ cmisc) {
    constexpr int CH = 2048;
    __shared__ uint64_t red[3][256];
    __shared__ double xs[CH];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int64_t o0 = offsets[c], n = offsets[c + 1] - o0;
    uint64_t wmin = ~0ull, wmax = 0, tmin = ~0ull;
    for (int64_t k = tid; k < n; k += 256) {
        const int64_t i = o0 + k;
        const double wi = 1.0 / (dy[i] * dy[i]);
        w[i] = wi;
        r[i] = wi * (1.0 - y[i]);
        u[i] = (int64_t)((1.0 - y[i]) * kTwo53);
        const uint64_t wb = (uint64_t)__double_as_longlong(wi);
        wmin = min(wmin, wb);
        wmax = max(wmax, wb);
        tmin = min(tmin, ordered_bits(t[i]));
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
    double sum = 0.0, comp = 0.0;
    for (int64_t base = 0; base < n; base += CH) {
        for (int k = tid; k < CH; k += 256) {
            const int64_t i = base + k;
            if (i < n) {
                const double wi = 1.0 / (dy[o0 + i] * dy[o0 + i]);
                const double d = y[o0 + i] - 1.0;
                xs[k] = wi * (d * d);
            }
        }
        __syncthreads();
        if (tid == 0) {
            const int64_t m = min((int64_t)CH, n - base);
            for (int64_t k = 0; k < m; ++k) {
                const double x = xs[k];
                const double tt = sum + x;
                if (fabs(sum) >= fabs(x))
                    comp += (sum - tt) + x;
                else
                    comp += (x - tt) + sum;
                sum = tt;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        uint64_t* m = cmisc + (size_t)c * kMiscSlots;
        m[kChi2Null] = (uint64_t)__double_as_longlong(sum + comp);
        m[kTminOrd] = red[2][0];
        m[kWminBits] = red[0][0];
        m[kWmaxBits] = red[1][0];
    }
}

// Template sums s1 = sum_k s_k for every D (shared by all curves), over the
// table's values like k_tmpl_sums.
template <typename T>
__global__ __launch_bounds__(64) void k_tmpl_s1(const T* __restrict__ table, int64_t dmax, double* __restrict__ s1sum) {
    const int64_t d = (int64_t)blockIdx.x * 64 + threadIdx.x + 1;
    if (d > dmax) return;
    const T* row = table + trow_off(d);
    double s1 = 0.0;
    for (int64_t k = 0; k < d; ++k) s1 = s1 + (double)row[k];
    s1sum[d] = s1;
}

struct BatchShared {
    Best red[kBatchThreads / 64];
    double bconst[kMaxBatchDurations];
    int64_t item;
    int64_t dpad;
};

template <typename T, bool MEAN, bool ANYVARW>
__global__ __launch_bounds__(kBatchThreads, 2) void k_batch(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ BatchShared bs;
    SortShared<kBatchThreads, kBatchSortItems>& ssh =
        *reinterpret_cast<SortShared<kBatchThreads, kBatchSortItems>*>(dyn);
    const int tid = threadIdx.x;
    const size_t es = sizeof(T);
    const size_t ps = sizeof(T) == 8 ? sizeof(__int128) : sizeof(float2);
    uint64_t* A = a.scr_a + (size_t)blockIdx.x * a.scr_n;
    uint64_t* B = a.scr_b + (size_t)blockIdx.x * a.scr_n;
    void* rpad = a.scr_r + (size_t)blockIdx.x * a.scr_pstride * es;
    void* wpad = ANYVARW ? (void*)(a.scr_w + (size_t)blockIdx.x * a.scr_pstride * es) : nullptr;
    void* pfx = MEAN ? (void*)(a.scr_pf + (size_t)blockIdx.x * (a.scr_pstride + 1) * ps) : nullptr;
    const int64_t stop = min(a.total, a.item_limit);

    for (;;) {
        __syncthreads();
        if (tid == 0) bs.item = (int64_t)atomicAdd(a.queue, 1ull);
        __syncthreads();
        const int64_t item = ((int64_t)__builtin_amdgcn_readfirstlane((int)(bs.item >> 32)) << 32) |
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)bs.item);
        if (item >= stop) break;
        // queue position -> (curve, period)
        int lo = 0, hi = a.nc;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.qoff[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int c = a.order[lo];
        const int64_t pidx = a.poffsets[c] + (item - a.qoff[lo]);
        const int64_t o0 = a.offsets[c], n = a.offsets[c + 1] - o0;
        const double period = a.periods[pidx];
        const uint64_t* m = a.cmisc + (size_t)c * kMiscSlots;
        const bool varw = ANYVARW && (m[kWminBits] != m[kWmaxBits]);
        const double wc = __longlong_as_double((long long)m[kWminBits]);

        if (tid == 0) bs.dpad = max_points(n, period, a.durations, a.nd, a.prm);
        __syncthreads();
        const int64_t npad = n + bs.dpad;
        const PadOut po{a.r + o0, a.w + o0, rpad, varw ? wpad : nullptr, npad, sizeof(T) == 4};
        fold_sort_core<kBatchThreads, false, kBatchSortItems>(a.t + o0, n, period, A, B, po, ssh);
        pad_prefix<kBatchThreads, kBatchSortItems>(A, n, npad, a.u + o0, pfx, sizeof(T) == 4, ssh);
        for (int64_t k = npad + tid; k < npad + kOverRead; k += kBatchThreads) {
            ((T*)rpad)[k] = (T)0;
            if (varw) ((T*)wpad)[k] = (T)0;
        }
        // Constant-weight b per duration: one sequential chain per lane.
        if (!varw) {
            for (int j = tid; j < a.nd; j += kBatchThreads) {
                double b = 0.0;
                if (duration_valid(period, a.durations[j], a.prm)) {
                    const int64_t d = points_in(n, period, a.durations[j]);
                    const T* row = (const T*)a.table + trow_off(d);
                    for (int64_t k = 0; k < d; ++k) {
                        const double sv = (double)row[k];
                        b = fma(wc, sv * sv, b);
                    }
                }
                bs.bconst[j] = b;
            }
        }
        __syncthreads();

        Best pbest{-INFINITY, 0.0, -1};
        int bj = -1;
        int64_t bd = 0;
        uint64_t evals = 0, macs = 0;
        for (int j = 0; j < a.nd; ++j) {
            if (!duration_valid(period, a.durations[j], a.prm)) continue;
            SlideItem si;
            si.n = n;
            si.D = points_in(n, period, a.durations[j]);
            si.stride = t0_stride(si.D, a.prm.dt0);
            si.limit = n + si.D;
            si.dpad = rup32(si.D);
            si.rp = rpad;
            si.wp = varw ? wpad : nullptr;
            si.pf = pfx;
            si.trow = (const T*)a.table + trow_off(si.D);
            si.bconst = varw ? 0.0 : bs.bconst[j];
            si.s1 = MEAN ? a.s1sum[si.D] : 0.0;
            const int64_t nw = (n + si.stride - 1) / si.stride;
            evals += (uint64_t)nw;
            macs += (uint64_t)nw * (uint64_t)si.D;
            Best jb{-INFINITY, 0.0, -1};
            if (si.stride == 1) {
                T* xs = reinterpret_cast<T*>(dyn);
                T* xw = xs + xpad<T>(kXs);
                for (int64_t i0 = 0; i0 < n; i0 += kTile) {
                    Best lb;
                    if (ANYVARW && varw) lb = slide_unit_tile<T, ANYVARW, MEAN>(si, i0, xs, xw);
                    else lb = slide_unit_tile<T, false, MEAN>(si, i0, xs, xw);
                    const Best tb = block_best(lb, bs.red);
                    if (tb.dchi2 > jb.dchi2) jb = tb;
                }
            } else {
                // the item's window groups split into one contiguous run per wave, each computed by the
                // cooperative strided routine of the single-curve search with the same windows-per-lane
                // rule (FP32C flushes its float partial sums at chunk boundaries that depend on a window's
                // place in its lane, so both searches must choose the same R to give identical results)
                const int wave = tid >> 6;
                const StridedSplit sp = strided_split(n, si.D, si.stride, 64, kBatchThreads / 64, 4, sizeof(T) == 8);
                int64_t m_lo = 0, m_hi = 0;
                if (wave < sp.ntask) strided_task_range(sp, wave, m_lo, m_hi);
                Best lb;
                T* stage = reinterpret_cast<T*>(dyn) + wave * (ANYVARW ? 2 : 1) * kStage<T>;
                if (ANYVARW && varw)
                    lb = strided_windows_coop_r<T, ANYVARW, MEAN, 4>(sp.R, si, m_lo, m_hi, stage, stage + kStage<T>);
                else
                    lb = strided_windows_coop_r<T, false, MEAN, 4>(sp.R, si, m_lo, m_hi, stage, nullptr);
                jb = block_best(lb, bs.red);
            }
            if (jb.dchi2 > pbest.dchi2) {
                pbest = jb;
                bj = j;
                bd = si.D;
            }
        }
        if (tid == 0) {
            const double chi2_0 = __longlong_as_double((long long)m[kChi2Null]);
            if (bj < 0) {
                a.chi2[pidx] = chi2_0;
                a.best_dur[pidx] = -1;
                a.best_start[pidx] = -1;
                a.depth[pidx] = 0.0;
                a.t0[pidx] = NAN;
            } else {
                a.chi2[pidx] = chi2_0 - pbest.dchi2;
                a.best_dur[pidx] = bj;
                a.best_start[pidx] = (int32_t)pbest.start;
                a.depth[pidx] = pbest.depth;
                const int64_t mid = (pbest.start + bd / 2) % n;
                const uint32_t idx = (uint32_t)A[mid];
                const double phic = phase_of(a.t[o0 + idx], period);
                const double x = phic * period;
                const double tmin = from_ordered(m[kTminOrd]);
                a.t0[pidx] = x + period * ceil((tmin - x) / period);
            }
            atomicAdd(a.cevals + 2 * c, (unsigned long long)evals);
            atomicAdd(a.cevals + 2 * c + 1, (unsigned long long)macs);
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

const size_t kStaticScratchBytes = sizeof(scratch);

hipError_t static_scratch_address(int device, char** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static char* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (char*)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

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
    size_t off_a, off_b, off_r, off_w, off_pf, off_items, off_toff, off_tcnt, off_rowmap, off_wfirst, off_sb,
        off_cell_s, off_cell_w, off_queue, off_ulist, off_ucnt, per_batch;
};

// Cells of the row planner for bp periods and nd durations (the device's
// cell_count): the periods of each XCD's list in blocks of kCellItems.
static int64_t host_cells(int64_t bp, int64_t nd) {
    int64_t c = 0;
    for (int x = 0; x < kXcds; ++x) c += (((bp - x + kXcds - 1) / kXcds) + kCellItems - 1) / kCellItems * nd;
    return c;
}

Plan make_plan(int64_t n, int32_t n_periods, int32_t nd, const gtls_params& prm, bool varw, size_t budget) {
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
    p.pstride = ((n + dcap + kOverRead + 63) / 64) * 64;
    size_t per = 2 * sizeof(uint64_t) * (size_t)n + p.esize * (size_t)p.pstride +
                 (varw ? p.esize * (size_t)p.pstride : 0) + (p.mean ? p.psize * (size_t)(p.pstride + 1) : 0) +
                 sizeof(ItemBest) * (size_t)nd * (size_t)p.ntiles +
                 (sizeof(ItemBest) + 2 * sizeof(int32_t)) * (size_t)nd * kRowMax + 4 * sizeof(int32_t) * (size_t)nd +
                 1024;
    // Periods per launch: as many as the scratch budget holds, at most
    // 32768.  Fewer, larger launches leave fewer drained tails: on the
    // 3000-day grid, 19 launches instead of 55 (72 GiB against 24 GiB of
    // scratch) cut the sort by 9 % and the strided slide by 4 %.
    int64_t bp = (int64_t)(budget / per);
    bp = std::max<int64_t>(1, std::min<int64_t>(bp, 32768));
    bp = std::min<int64_t>(bp, n_periods);
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
    // Row slots: at most kRowMax per strided item, plus the padding of each
    // cell's subgroups to whole wave tasks (at most 3 per subgroup, at most
    // kCellItems subgroups per cell).
    const int64_t cells = host_cells(bp, nd);
    const size_t slots = (size_t)nd * kRowMax * bp + (size_t)3 * kCellItems * cells;
    p.off_toff = o;
    o = align256(o + sizeof(int32_t) * (size_t)nd * bp);
    p.off_tcnt = o;
    o = align256(o + sizeof(int32_t) * (size_t)nd * bp);
    p.off_rowmap = o;
    o = align256(o + sizeof(int32_t) * slots);
    p.off_wfirst = o;
    o = align256(o + sizeof(int32_t) * (slots / 4 + 1));
    p.off_sb = o;
    o = align256(o + sizeof(ItemBest) * slots);
    p.off_cell_s = o;
    o = align256(o + sizeof(int32_t) * (size_t)(cells + 1));
    p.off_cell_w = o;
    o = align256(o + sizeof(int32_t) * (size_t)(cells + 1));
    p.off_queue = o;
    o = align256(o + (2 * kXcds + 2) * sizeof(uint32_t));
    p.off_ulist = o;
    o = align256(o + sizeof(int32_t) * (size_t)nd * bp);
    p.off_ucnt = o;
    o = align256(o + sizeof(int32_t) * (size_t)nd * bp);
    p.per_batch = o;
    return p;
}

// Unit-stride tiles, then (strided T0 grids) the wave-task list and the
// persistent strided kernel, sized to fill every CU.
template <typename T, bool VARW, bool MEAN>
void launch_slides(gtls_ctx* ctx, const SlideArgs& la, int64_t units, bool strided, int num_cus, hipStream_t s) {
    {
        StageTimer tm(ctx, kStageSlide);
        const unsigned pgrid = (unsigned)(((int64_t)la.bp * la.nd + 255) / 256);
        const unsigned cgrid = (unsigned)((host_cells(la.bp, la.nd) + 255) / 256);
        k_plan_count<<<pgrid, 256, 0, s>>>(la);
        k_rplan_count<<<cgrid, 256, 0, s>>>(la);
        k_plan_scan<<<1, kPlanThreads, 0, s>>>(la);
        k_rplan_fill<<<cgrid, 256, 0, s>>>(la);
        // every-offset work units (list entries x window tiles) by a grid of
        // at most as many workgroups as are resident at once
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_slide_unit<T, VARW, MEAN>, kSlideThreads, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        const unsigned ugrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)per_cu * num_cus));
        k_slide_unit<T, VARW, MEAN><<<ugrid, kSlideThreads, 0, s>>>(la);
    }
    if (strided) {
        StageTimer tm(ctx, kStageStrided);
        // num_cus: compute units of the context's device, set at creation
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_slide_rows<T, VARW, MEAN>, kSlideThreads, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        k_slide_rows<T, VARW, MEAN><<<(unsigned)(per_cu * num_cus), kSlideThreads, 0, s>>>(la);
    }
}

template <typename T>
void launch_slides(gtls_ctx* ctx, const SlideArgs& la, int64_t units, bool strided, bool varw, bool mean,
                   int num_cus, hipStream_t s) {
    if (varw) {
        if (mean) launch_slides<T, true, true>(ctx, la, units, strided, num_cus, s);
        else launch_slides<T, true, false>(ctx, la, units, strided, num_cus, s);
    } else {
        if (mean) launch_slides<T, false, true>(ctx, la, units, strided, num_cus, s);
        else launch_slides<T, false, false>(ctx, la, units, strided, num_cus, s);
    }
}

}  // namespace

hipError_t run_search(gtls_ctx* ctx, const SearchArgs& a) {
    hipStream_t s = ctx->stream;
    const int64_t n = a.n;
    // Scratch regions: the context's grow-only buffers, or consecutive
    // pieces of the caller-provided fixed buffer (no allocation).
    size_t fixed_used = 0;
    auto region = [&](DeviceBuffer& b, size_t bytes, char** out) -> hipError_t {
        if (a.fixed) {
            if (fixed_used + align256(bytes) > a.fixed_bytes) return hipErrorOutOfMemory;
            *out = a.fixed + fixed_used;
            fixed_used += align256(bytes);
            return hipSuccess;
        }
        const hipError_t e = ensure(ctx, b, bytes);
        *out = (char*)b.ptr;
        return e;
    };
    // Per-curve arrays: misc | w | r | u
    const size_t off_w = 256, off_r = align256(off_w + 8 * (size_t)n), off_u = align256(off_r + 8 * (size_t)n);
    char* cb = nullptr;
    hipError_t e = region(ctx->curve, align256(off_u + 8 * (size_t)n), &cb);
    if (e != hipSuccess) return e;
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

    // Scratch budget: 72 GiB (a quarter of the HBM), at most half of what
    // the device has free beside the context's current period scratch; on
    // an allocation failure the budget halves and the plan is redone.
    size_t budget = (size_t)72 << 30;
    if (!a.fixed) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
            budget = std::min(budget, (free_b + ctx->batch.bytes) / 2);
    }
    Plan pl = make_plan(n, a.n_periods, a.n_durations, a.prm, varw, budget);
    // Template rows for every D in [1, dcap] and the per-D sums.
    const size_t tab_elems = (size_t)trow_off(pl.dcap + 1);
    const size_t off_bsum = align256(pl.esize * tab_elems), off_s1 = align256(off_bsum + 8 * (size_t)(pl.dcap + 1));
    char* tb = nullptr;
    e = region(ctx->table, align256(off_s1 + 8 * (size_t)(pl.dcap + 1)), &tb);
    if (e != hipSuccess) return e;
    void* table = tb;
    double* bsum = (double*)(tb + off_bsum);
    double* s1sum = (double*)(tb + off_s1);
    if (a.fixed) {
        // periods per launch: whatever the rest of the fixed buffer holds
        if (fixed_used >= a.fixed_bytes) return hipErrorOutOfMemory;
        pl = make_plan(n, a.n_periods, a.n_durations, a.prm, varw, a.fixed_bytes - fixed_used);
    }
    {
        StageTimer tm(ctx, kStagePrep);
        if (pl.f32) k_tmpl_table<float><<<(unsigned)pl.dcap, 256, 0, s>>>(a.tmpl, a.n_tmpl, pl.dcap, (float*)table);
        else k_tmpl_table<double><<<(unsigned)pl.dcap, 256, 0, s>>>(a.tmpl, a.n_tmpl, pl.dcap, (double*)table);
        if (pl.f32) k_tmpl_sums<float><<<(unsigned)((pl.dcap + 63) / 64), 64, 0, s>>>((const float*)table, pl.dcap, misc, bsum, s1sum);
        else k_tmpl_sums<double><<<(unsigned)((pl.dcap + 63) / 64), 64, 0, s>>>((const double*)table, pl.dcap, misc, bsum, s1sum);
    }
    char* bb = nullptr;
    e = region(ctx->batch, pl.per_batch, &bb);
    while (!a.fixed && e == hipErrorOutOfMemory && pl.bp > 1) {
        (void)hipGetLastError();
        budget /= 2;
        pl = make_plan(n, a.n_periods, a.n_durations, a.prm, varw, budget);
        e = region(ctx->batch, pl.per_batch, &bb);
    }
    if (e != hipSuccess) return e;
    uint64_t* keys_a = (uint64_t*)(bb + pl.off_a);
    uint64_t* keys_b = (uint64_t*)(bb + pl.off_b);
    void* rpad = bb + pl.off_r;
    void* wpad = varw ? (void*)(bb + pl.off_w) : nullptr;
    void* pfx = pl.mean ? (void*)(bb + pl.off_pf) : nullptr;
    ItemBest* items = (ItemBest*)(bb + pl.off_items);
    int32_t* toff = (int32_t*)(bb + pl.off_toff);
    int32_t* tcnt = (int32_t*)(bb + pl.off_tcnt);
    int32_t* rowmap = (int32_t*)(bb + pl.off_rowmap);
    int32_t* wfirst = (int32_t*)(bb + pl.off_wfirst);
    int32_t* cell_s = (int32_t*)(bb + pl.off_cell_s);
    int32_t* cell_w = (int32_t*)(bb + pl.off_cell_w);
    ItemBest* sb = (ItemBest*)(bb + pl.off_sb);
    uint32_t* queue = (uint32_t*)(bb + pl.off_queue);
    int32_t* ulist = (int32_t*)(bb + pl.off_ulist);
    int32_t* ucnt = (int32_t*)(bb + pl.off_ucnt);
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
                     misc, table, bsum, s1sum, items, pl.ntiles, toff, tcnt, rowmap, wfirst, cell_s, cell_w, sb,
                     queue, pl.f32 ? 4 : 8, pl.f32 ? 0 : 1, ulist, ucnt};
        const int64_t units = (int64_t)bp * a.n_durations * pl.ntiles;
        if (pl.f32) launch_slides<float>(ctx, la, units, strided, varw, pl.mean, ctx->num_cus, s);
        else launch_slides<double>(ctx, la, units, strided, varw, pl.mean, ctx->num_cus, s);
        ReduceArgs ra{a.t, n, a.periods + p0, a.durations, a.prm, bp, a.n_durations, items, pl.ntiles, toff, tcnt, sb,
                      keys_a, misc, misc,
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

// ------------------------------------------------------------------------
// Batched survey launcher.

namespace {

template <typename T, bool MEAN, bool ANYVARW>
size_t batch_lds_bytes() {
    const size_t es = sizeof(T), mult = ANYVARW ? 2 : 1;
    const size_t sort = sizeof(SortShared<kBatchThreads, kBatchSortItems>);
    const size_t unit = (size_t)xpad<T>(kXs) * es * mult;
    const size_t stage = (size_t)(kBatchThreads / 64) * mult * kStage<T> * es;
    return std::max(sort, std::max(unit, stage));
}

template <typename T, bool MEAN, bool ANYVARW>
hipError_t set_batch_attr_t() {
    return hipFuncSetAttribute((const void*)k_batch<T, MEAN, ANYVARW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)batch_lds_bytes<T, MEAN, ANYVARW>());
}

hipError_t set_batch_attr(bool f32, bool mean, bool anyvarw) {
    if (f32) {
        if (mean) return anyvarw ? set_batch_attr_t<float, true, true>() : set_batch_attr_t<float, true, false>();
        return anyvarw ? set_batch_attr_t<float, false, true>() : set_batch_attr_t<float, false, false>();
    }
    if (mean) return anyvarw ? set_batch_attr_t<double, true, true>() : set_batch_attr_t<double, true, false>();
    return anyvarw ? set_batch_attr_t<double, false, true>() : set_batch_attr_t<double, false, false>();
}

template <typename T, bool MEAN, bool ANYVARW>
hipError_t launch_batch_t(const BatchArgs& ba, int grid, hipStream_t s) {
    k_batch<T, MEAN, ANYVARW><<<grid, kBatchThreads, batch_lds_bytes<T, MEAN, ANYVARW>(), s>>>(ba);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& ba, int grid, bool f32, bool mean, bool anyvarw, hipStream_t s) {
    if (f32) {
        if (mean) return anyvarw ? launch_batch_t<float, true, true>(ba, grid, s) : launch_batch_t<float, true, false>(ba, grid, s);
        return anyvarw ? launch_batch_t<float, false, true>(ba, grid, s) : launch_batch_t<float, false, false>(ba, grid, s);
    }
    if (mean) return anyvarw ? launch_batch_t<double, true, true>(ba, grid, s) : launch_batch_t<double, true, false>(ba, grid, s);
    return anyvarw ? launch_batch_t<double, false, true>(ba, grid, s) : launch_batch_t<double, false, false>(ba, grid, s);
}

void fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
    k_fill_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

}  // namespace

static hipError_t run_search_batch_queued(gtls_ctx* ctx, const BatchArgsHost& h, std::vector<int32_t>& order,
                                          int64_t n_max, int64_t dcap);

hipError_t run_search_batch(gtls_ctx* ctx, const BatchArgsHost& h) {
    const int nc = h.nc;
    // Host planning: with batch_route_min > 0, curves of at least that many
    // points go through the single-curve pipeline (after the persistent
    // launch); the others are queued for it, longest first.
    int64_t n_max = 0, dcap = 1;
    std::vector<int32_t> order, routed;
    for (int c = 0; c < nc; ++c) {
        const int64_t n = h.offsets[c + 1] - h.offsets[c];
        if (h.prm.batch_route_min > 0 && n >= h.prm.batch_route_min) {
            routed.push_back(c);
            continue;
        }
        order.push_back(c);
        n_max = std::max(n_max, n);
        int64_t d = (int64_t)std::floor((double)n * h.prm.q_cap + 0.5);
        dcap = std::max(dcap, std::max<int64_t>(1, std::min(n, d)));
    }
    hipError_t e = order.empty() ? hipSuccess : run_search_batch_queued(ctx, h, order, n_max, dcap);
    for (const int32_t c : routed) {
        if (e != hipSuccess) break;
        const int64_t o = h.offsets[c], po = h.poffsets[c];
        const SearchArgs a{h.t + o, h.y + o, h.dy + o, h.offsets[c + 1] - o, h.periods + po,
                           (int32_t)(h.poffsets[c + 1] - po), h.durations, h.nd, h.tmpl, h.nt, h.prm,
                           h.chi2 + po, h.best_dur + po, h.best_start + po, h.depth + po, h.t0 + po, h.sr + po,
                           h.sde_raw + po, h.sde + po, h.summaries + c};
        e = run_search(ctx, a);
    }
    return e;
}

// The persistent launch over the queued curves.  The per-curve preparation and the periodogram kernels
// run over every curve of the batch; the routed curves' outputs are
// rewritten afterwards by their own searches.
static hipError_t run_search_batch_queued(gtls_ctx* ctx, const BatchArgsHost& h, std::vector<int32_t>& order,
                                          int64_t n_max, int64_t dcap) {
    hipStream_t s = ctx->stream;
    const int nc = h.nc, nq = (int)order.size();
    const bool f32 = h.prm.precision == GTLS_FP32C, mean = h.prm.depth_mode == GTLS_DEPTH_MEAN;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    const size_t ps = f32 ? sizeof(float2) : sizeof(__int128);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return h.offsets[a + 1] - h.offsets[a] > h.offsets[b + 1] - h.offsets[b];
    });
    std::vector<int64_t> qoff(nq + 1, 0);
    for (int q = 0; q < nq; ++q) qoff[q + 1] = qoff[q] + (h.poffsets[order[q] + 1] - h.poffsets[order[q]]);
    const int64_t total_points = h.offsets[nc], total_items = qoff[nq], total_periods = h.poffsets[nc];
    const int64_t pstride = ((n_max + dcap + kOverRead + 63) / 64) * 64;

    // Per-curve device arrays: offsets, poffsets, order, qoff, cmisc, cevals, queue, w, r, u, s1sum.
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t o_off = take(8 * (size_t)(nc + 1)), o_poff = take(8 * (size_t)(nc + 1)), o_ord = take(4 * (size_t)nc),
                 o_qoff = take(8 * (size_t)(nc + 1)), o_misc = take(8 * kMiscSlots * (size_t)nc),
                 o_ev = take(16 * (size_t)nc), o_q = take(8), o_w = take(8 * (size_t)total_points),
                 o_r = take(8 * (size_t)total_points), o_u = take(8 * (size_t)total_points),
                 o_s1 = take(8 * (size_t)(dcap + 1));
    hipError_t e = ensure(ctx, ctx->bcurve, o);
    if (e != hipSuccess) return e;
    char* cb = (char*)ctx->bcurve.ptr;
    const size_t tab_bytes = align256(es * (size_t)trow_off(dcap + 1));
    e = ensure(ctx, ctx->table, tab_bytes);
    if (e != hipSuccess) return e;
    int64_t* d_off = (int64_t*)(cb + o_off);
    int64_t* d_poff = (int64_t*)(cb + o_poff);
    int32_t* d_ord = (int32_t*)(cb + o_ord);
    int64_t* d_qoff = (int64_t*)(cb + o_qoff);
    uint64_t* cmisc = (uint64_t*)(cb + o_misc);
    unsigned long long* cevals = (unsigned long long*)(cb + o_ev);
    unsigned long long* queue = (unsigned long long*)(cb + o_q);
    double* w = (double*)(cb + o_w);
    double* r = (double*)(cb + o_r);
    int64_t* u = (int64_t*)(cb + o_u);
    double* s1sum = (double*)(cb + o_s1);
    if ((e = hipMemcpyAsync(d_off, h.offsets, 8 * (size_t)(nc + 1), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(d_poff, h.poffsets, 8 * (size_t)(nc + 1), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(d_ord, order.data(), 4 * (size_t)nq, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(d_qoff, qoff.data(), 8 * (size_t)(nq + 1), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    {
        StageTimer tm(ctx, kStagePrep);
        k_prep_batch<<<nc, 256, 0, s>>>(d_off, h.t, h.y, h.dy, w, r, u, cmisc);
        if (f32) k_tmpl_table<float><<<(unsigned)dcap, 256, 0, s>>>(h.tmpl, h.nt, dcap, (float*)ctx->table.ptr);
        else k_tmpl_table<double><<<(unsigned)dcap, 256, 0, s>>>(h.tmpl, h.nt, dcap, (double*)ctx->table.ptr);
        if (f32) k_tmpl_s1<float><<<(unsigned)((dcap + 63) / 64), 64, 0, s>>>((const float*)ctx->table.ptr, dcap, s1sum);
        else k_tmpl_s1<double><<<(unsigned)((dcap + 63) / 64), 64, 0, s>>>((const double*)ctx->table.ptr, dcap, s1sum);
    }
    std::vector<uint64_t> hm((size_t)nc * kMiscSlots);
    if ((e = hipMemcpyAsync(hm.data(), cmisc, 8 * hm.size(), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    bool anyvarw = false;
    for (int c = 0; c < nc; ++c)
        anyvarw |= hm[(size_t)c * kMiscSlots + kWminBits] != hm[(size_t)c * kMiscSlots + kWmaxBits];

    // Persistent grid: workgroups per CU from the autotuner (per shape).
    const int max_per_cu = 2;
    const int64_t grid_max = (int64_t)ctx->num_cus * max_per_cu;
    const size_t scr = align256(2 * 8 * (size_t)n_max) + align256(es * (size_t)pstride) * (anyvarw ? 2 : 1) +
                       (mean ? align256(ps * (size_t)(pstride + 1)) : 0);
    e = ensure(ctx, ctx->bscratch, scr * (size_t)grid_max + 4096);
    if (e != hipSuccess) return e;
    char* sb = (char*)ctx->bscratch.ptr;
    const size_t sz_ab = align256(8 * (size_t)n_max * grid_max);
    const size_t sz_r = align256(es * (size_t)pstride * grid_max);
    BatchArgs ba{d_off, h.t, nq, d_poff, h.periods, h.durations, h.nd, h.prm, w, r, u, cmisc, ctx->table.ptr,
                 h.tmpl, h.nt, s1sum, d_ord, d_qoff, total_items, queue,
                 (uint64_t*)sb, (uint64_t*)(sb + sz_ab), sb + 2 * sz_ab, anyvarw ? sb + 2 * sz_ab + sz_r : nullptr,
                 mean ? sb + 2 * sz_ab + sz_r * (anyvarw ? 2 : 1) : nullptr, n_max, pstride, INT64_MAX,
                 h.chi2, h.best_dur, h.best_start, h.depth, h.t0, cevals};

    int lg = 0;
    for (int64_t x = n_max; x > 1; x >>= 1) ++lg;
    uint64_t dt0_bits = 0;
    std::memcpy(&dt0_bits, &h.prm.dt0, sizeof(dt0_bits));
    const std::vector<uint64_t> shape{(uint64_t)lg, (uint64_t)f32, (uint64_t)mean, (uint64_t)anyvarw,
                                      (uint64_t)h.nd, dt0_bits};
    int per_cu = 0;
    for (auto& t : ctx->bcache.tuned)
        if (t.first == shape) per_cu = t.second;
    if ((e = set_batch_attr(f32, mean, anyvarw)) != hipSuccess) return e;
    if (per_cu == 0) {
        // Autotune: time each candidate on the first items of this batch.
        float best_ms = 0.f;
        hipEvent_t e0, e1;
        if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
        if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
        for (int cand = 1; cand <= max_per_cu; ++cand) {
            const int grid = ctx->num_cus * cand;
            BatchArgs tb = ba;
            tb.item_limit = std::min<int64_t>(total_items, (int64_t)grid_max * 2);
            fill_u64(queue, 1, 0ull, s);
            fill_u64(cevals, 2 * (int64_t)nc, 0ull, s);
            (void)hipEventRecord(e0, s);
            if ((e = launch_batch(tb, grid, f32, mean, anyvarw, s)) != hipSuccess) return e;
            (void)hipEventRecord(e1, s);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            // rate per item: both candidates process the same item prefix
            if (per_cu == 0 || ms < best_ms) {
                best_ms = ms;
                per_cu = cand;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->bcache.tuned.push_back({shape, per_cu});
    }
    const int grid = ctx->num_cus * per_cu;

    // The rest of the pipeline runs as one captured graph, replayed while
    // the arguments stay the same.
    // The key holds every value a captured launch reads from its arguments:
    // all parameters (their bytes), every device pointer of the kernels and
    // every size, so a call that changes any of them captures a new graph.
    std::vector<uint64_t> key = shape;
    {
        const gtls_params& pp = h.prm;
        for (const double v : {pp.dt0, pp.k_min, pp.k_max, pp.q_cap}) {
            uint64_t b = 0;
            std::memcpy(&b, &v, sizeof(b));
            key.push_back(b);
        }
        for (const int32_t v : {pp.envelope, pp.depth_mode, pp.precision, pp.median_window, pp.batch_route_min})
            key.push_back((uint64_t)(uint32_t)v);
    }
    for (const void* p : {(const void*)h.t, (const void*)h.y, (const void*)h.dy, (const void*)h.periods,
                          (const void*)h.durations, (const void*)h.tmpl, (const void*)h.chi2,
                          (const void*)h.best_dur, (const void*)h.best_start, (const void*)h.depth,
                          (const void*)h.t0, (const void*)h.sr, (const void*)h.sde_raw, (const void*)h.sde,
                          (const void*)h.summaries, (const void*)cb, (const void*)sb, (const void*)ctx->table.ptr,
                          (const void*)ba.w, (const void*)ba.r, (const void*)ba.u, (const void*)ba.cmisc,
                          (const void*)ba.s1sum, (const void*)ba.order, (const void*)ba.qoff, (const void*)ba.queue,
                          (const void*)ba.scr_a, (const void*)ba.scr_b, (const void*)ba.scr_r, (const void*)ba.scr_w,
                          (const void*)ba.scr_pf, (const void*)ba.cevals})
        key.push_back((uint64_t)(uintptr_t)p);
    for (const int64_t v : {(int64_t)nc, (int64_t)nq, (int64_t)h.nd, (int64_t)h.nt, total_items, total_periods,
                            (int64_t)grid, n_max, pstride, dcap, ba.scr_n, ba.scr_pstride, ba.item_limit})
        key.push_back((uint64_t)v);
    for (int c = 0; c <= nc; ++c) {
        key.push_back((uint64_t)h.offsets[c]);
        key.push_back((uint64_t)h.poffsets[c]);
    }
    if (!(ctx->bcache.exec && ctx->bcache.key == key)) {
        if (ctx->bcache.exec) {
            (void)hipGraphExecDestroy(ctx->bcache.exec);
            ctx->bcache.exec = nullptr;
        }
        if ((e = set_batch_attr(f32, mean, anyvarw)) != hipSuccess) return e;
        hipGraph_t g = nullptr;
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
        fill_u64(queue, 1, 0ull, s);
        fill_u64(cevals, 2 * (int64_t)nc, 0ull, s);
        hipError_t le = launch_batch(ba, grid, f32, mean, anyvarw, s);
        k_sde_stats_batch<<<nc, 256, 0, s>>>(d_poff, h.chi2, h.sr, h.sde_raw);
        k_sde_median_batch<<<(unsigned)((total_periods + kMedThreads - 1) / kMedThreads), kMedThreads, 0, s>>>(
            d_poff, nc, h.sde_raw, h.prm.median_window, h.sde);
        k_sde_argmax_batch<<<nc, 256, 0, s>>>(d_poff, h.sde, cmisc, cevals, h.summaries);
        e = hipStreamEndCapture(s, &g);
        if (le != hipSuccess) return le;
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&ctx->bcache.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ctx->bcache.exec = nullptr;
            return e;
        }
        ctx->bcache.key = key;
    }
    StageTimer tm(ctx, kStageSlide);
    return hipGraphLaunch(ctx->bcache.exec, s);
}


hipError_t run_fold_sort(gtls_ctx* ctx, const double* t, int64_t n, const double* periods, int32_t n_periods,
                         int32_t* perm) {
    hipStream_t s = ctx->stream;
    gtls_params prm;
    gtls_params_default(&prm);
    const Plan pl = make_plan(n, n_periods, 1, prm, false, (size_t)8 << 30);
    hipError_t e = ensure(ctx, ctx->batch, pl.per_batch);
    if (e != hipSuccess) return e;
    char* bb = (char*)ctx->batch.ptr;
    for (int32_t p0 = 0; p0 < n_periods; p0 += pl.bp) {
        const int32_t bp = std::min(pl.bp, n_periods - p0);
        // permutation only: no padded copies, no prefix sums
        SortArgs sa{t, nullptr, nullptr, nullptr, n, periods + p0, periods, 0, prm, (uint64_t*)(bb + pl.off_a),
                    (uint64_t*)(bb + pl.off_b), nullptr, nullptr, nullptr, pl.pstride, perm + (size_t)p0 * n, 0};
        k_fold_sort<<<bp, kSortThreads, 0, s>>>(sa);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {

// ------------------------------------------------------------------------
// Transit statistics at one window (SNR, per-transit and odd/even depths).
// Window point k (padded position p = start + k, sorted position p mod n,
// wrapped when p >= n) of input index idx belongs to the transit of epoch
// floor(t_idx / P) - wrapped.  Per epoch, over its points in ascending k,
// c = sum fma(r, s_k, .) and b = sum fma(w, s_k^2, .); odd, even and all
// epochs then pool c and b in ascending epoch order.  SNR = max(C, 0) /
// sqrt(B), the pooled depth over its standard error.

// Per window point: epoch, r, w, template value; the epoch range (epochs as
// order-preserving unsigned words: e XOR 2^63).
__global__ __launch_bounds__(256) void k_ts_points(const double* __restrict__ t, const double* __restrict__ y,
                                                   const double* __restrict__ dy, const int32_t* __restrict__ perm,
                                                   int64_t n, const double* __restrict__ period_p, int64_t d,
                                                   int64_t start, const double* __restrict__ tm, int32_t nt,
                                                   int64_t* __restrict__ ek, double* __restrict__ rk,
                                                   double* __restrict__ wk, double* __restrict__ sk,
                                                   unsigned long long* erange) {
    __shared__ unsigned long long lo[256], hi[256];
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * 256 + tid;
    const double period = *period_p;
    unsigned long long a = ~0ull, b = 0ull;
    if (k < d) {
        const int64_t p = start + k;
        const int wrapped = p >= n ? 1 : 0;
        const int32_t idx = perm[wrapped ? p - n : p];
        const double w = 1.0 / (dy[idx] * dy[idx]);
        const int64_t e = (int64_t)floor(t[idx] / period) - wrapped;
        ek[k] = e;
        rk[k] = w * (1.0 - y[idx]);
        wk[k] = w;
        sk[k] = resample(tm, nt, d, k);
        a = b = (unsigned long long)e ^ 0x8000000000000000ull;
    }
    lo[tid] = a;
    hi[tid] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            lo[tid] = min(lo[tid], lo[tid + s]);
            hi[tid] = max(hi[tid], hi[tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        atomicMin(&erange[0], lo[0]);
        atomicMax(&erange[1], hi[0]);
    }
}

// One thread per epoch: its points' sums in ascending k (every lane walks
// all window points, which it reads at the same address as the rest of its
// wave).
__global__ __launch_bounds__(256) void k_ts_epochs(const int64_t* __restrict__ ek, const double* __restrict__ rk,
                                                   const double* __restrict__ wk, const double* __restrict__ sk,
                                                   int64_t d, int64_t emin, int64_t nep, double* __restrict__ ce,
                                                   double* __restrict__ be, int64_t* __restrict__ ne) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t e = emin + j;
    double c = 0.0, b = 0.0;
    int64_t cnt = 0;
    for (int64_t k = 0; k < d; ++k) {
        if (ek[k] == e) {
            c = fma(rk[k], sk[k], c);
            const double s2 = sk[k] * sk[k];
            b = fma(wk[k], s2, b);
            ++cnt;
        }
    }
    if (j < nep) {
        ce[j] = c;
        be[j] = b;
        ne[j] = cnt;
    }
}

// Pools the epochs in ascending order and writes the statistics (one thread).
__global__ void k_ts_final(const double* __restrict__ ce, const double* __restrict__ be,
                           const int64_t* __restrict__ ne, int64_t emin, int64_t nep, const double* __restrict__ t,
                           const int32_t* __restrict__ perm, int64_t n, const double* __restrict__ period_p,
                           int64_t d, int64_t start, int64_t max_transits, gtls_transit_stats* __restrict__ st,
                           int64_t* __restrict__ epoch, double* __restrict__ t_mid, double* __restrict__ depth,
                           double* __restrict__ sigma, int64_t* __restrict__ count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double period = *period_p;
    const int64_t pm = start + d / 2;
    const double phase_mid = phase_of(t[perm[pm >= n ? pm - n : pm]], period) + (pm >= n ? 1.0 : 0.0);
    double c_all = 0.0, b_all = 0.0, c_odd = 0.0, b_odd = 0.0, c_even = 0.0, b_even = 0.0;
    int64_t nt = 0, first = 0;
    for (int64_t j = 0; j < nep; ++j) {
        if (ne[j] == 0) continue;
        const int64_t e = emin + j;
        if (nt == 0) first = e;
        if (nt < max_transits) {
            epoch[nt] = e;
            t_mid[nt] = ((double)e + phase_mid) * period;
            depth[nt] = ce[j] / be[j];
            sigma[nt] = 1.0 / sqrt(be[j]);
            count[nt] = ne[j];
        }
        ++nt;
        c_all += ce[j];
        b_all += be[j];
        if (((e % 2) + 2) % 2 == 1) {
            c_odd += ce[j];
            b_odd += be[j];
        } else {
            c_even += ce[j];
            b_even += be[j];
        }
    }
    const double d_odd = b_odd > 0.0 ? c_odd / b_odd : NAN, s_odd = b_odd > 0.0 ? 1.0 / sqrt(b_odd) : NAN;
    const double d_even = b_even > 0.0 ? c_even / b_even : NAN, s_even = b_even > 0.0 ? 1.0 / sqrt(b_even) : NAN;
    st->snr = (c_all > 0.0 ? c_all : 0.0) / sqrt(b_all);
    st->depth = c_all / b_all;
    st->depth_odd = d_odd;
    st->depth_even = d_even;
    st->sigma_odd = s_odd;
    st->sigma_even = s_even;
    st->odd_even_sigma =
        (b_odd > 0.0 && b_even > 0.0) ? fabs(d_odd - d_even) / sqrt(s_odd * s_odd + s_even * s_even) : NAN;
    st->phase_mid = phase_mid;
    st->n_in = d;
    st->n_transits = nt;
    st->first_epoch = first;
}

}  // namespace

// Statistics of the window of d points from sorted position `start` of the
// curve folded at *period_dev (device arrays; scratch from the context).
hipError_t run_transit_stats(gtls_ctx* ctx, const double* t, const double* y, const double* dy, int64_t n,
                             const double* period_dev, int64_t d, int64_t start, const double* tm, int32_t nt,
                             int64_t nep_max, int64_t max_transits, gtls_transit_stats* st_dev, int64_t* epoch,
                             double* t_mid, double* depth, double* sigma, int64_t* count) {
    hipStream_t s = ctx->stream;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t o_perm = take(4 * (size_t)n), o_ek = take(8 * (size_t)d), o_rk = take(8 * (size_t)d),
                 o_wk = take(8 * (size_t)d), o_sk = take(8 * (size_t)d), o_er = take(16),
                 o_ce = take(8 * (size_t)nep_max), o_be = take(8 * (size_t)nep_max), o_ne = take(8 * (size_t)nep_max);
    hipError_t e = ensure(ctx, ctx->sde_tmp, o);
    if (e != hipSuccess) return e;
    char* b = (char*)ctx->sde_tmp.ptr;
    int32_t* perm = (int32_t*)(b + o_perm);
    e = run_fold_sort(ctx, t, n, period_dev, 1, perm);
    if (e != hipSuccess) return e;
    unsigned long long* er = (unsigned long long*)(b + o_er);
    k_fill_u64<<<1, 256, 0, s>>>(er, 1, ~0ull);
    k_fill_u64<<<1, 256, 0, s>>>(er + 1, 1, 0ull);
    k_ts_points<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(t, y, dy, perm, n, period_dev, d, start, tm, nt,
                                                            (int64_t*)(b + o_ek), (double*)(b + o_rk),
                                                            (double*)(b + o_wk), (double*)(b + o_sk), er);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long range[2];
    e = hipMemcpyAsync(range, er, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const int64_t emin = (int64_t)(range[0] ^ 0x8000000000000000ull), emax = (int64_t)(range[1] ^ 0x8000000000000000ull);
    const int64_t nep = emax - emin + 1;
    if (nep < 1 || nep > nep_max) return hipErrorInvalidValue;   // cannot happen: epochs lie in the time span
    k_ts_epochs<<<(unsigned)((nep + 255) / 256), 256, 0, s>>>((const int64_t*)(b + o_ek), (const double*)(b + o_rk),
                                                              (const double*)(b + o_wk), (const double*)(b + o_sk),
                                                              d, emin, nep, (double*)(b + o_ce), (double*)(b + o_be),
                                                              (int64_t*)(b + o_ne));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ts_final<<<1, 64, 0, s>>>((const double*)(b + o_ce), (const double*)(b + o_be), (const int64_t*)(b + o_ne),
                                emin, nep, t, perm, n, period_dev, d, start, max_transits, st_dev, epoch, t_mid,
                                depth, sigma, count);
    return hipGetLastError();
}

}  // namespace gtls
