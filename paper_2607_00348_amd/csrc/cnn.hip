// Learned period proposal for gfx950: a small 1D CNN over a binned view of
// the light curve, trained and run with hand-written kernels.  Convolutions
// are implicit GEMMs on v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32
// accumulation); the head, loss and Adam update run on the vector ALUs in
// FP32 with FP32 master weights.
//
// Network: 5 x [conv1d k=7 pad 3, 32 channels, GELU(erf)] -> mean over the
// 4096 positions -> linear 32 -> 512 period bins -> softmax cross-entropy.
// Activations are channels-last ([sample][position][channel]); a 16-wide K
// slice of the implicit GEMM is one kernel tap and 16 consecutive channels,
// i.e. one contiguous 32-byte run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gtls.h"
#include "gtls_impl.hpp"

namespace gtls {
namespace cnn {

constexpr int L = 4096;
constexpr int C = 32;
constexpr int KW = 7;
constexpr int NB = 512;
constexpr int NL = 5;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

// Offsets of each tensor in the flat parameter vector (W_l: 32 x C_in x 7
// in (co, ci, k) order, then b_l; then Wf: 512 x 32, bf: 512).
__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 1 : C; }
__host__ __device__ constexpr int64_t w_off(int l) {
    int64_t o = 0;
    for (int q = 0; q < l; ++q) o += (int64_t)C * cin_of(q) * KW + C;
    return o;
}
__host__ __device__ constexpr int64_t b_off(int l) { return w_off(l) + (int64_t)C * cin_of(l) * KW; }
constexpr int64_t kWf = w_off(NL);
constexpr int64_t kBf = kWf + (int64_t)NB * C;
constexpr int64_t kNParams = kBf + NB;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------------------
// View: per curve, 4096 equal time bins; (bin median - 1) / (1.4826 MAD).

// k-th smallest (0-based) of f(i), i < n, by an 8-pass radix select on the
// order-preserving 64-bit image of the doubles.
template <typename F>
__device__ double select_kth(F f, int64_t n, int64_t k, uint32_t* hist) {
    uint64_t prefix = 0, mask = 0;
    for (int pass = 7; pass >= 0; --pass) {
        const int shift = 8 * pass;
        for (int d = threadIdx.x; d < 256; d += blockDim.x) hist[d] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            uint64_t b = (uint64_t)__double_as_longlong(f(i));
            b = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
            if ((b & mask) == prefix) atomicAdd(&hist[(b >> shift) & 255u], 1u);
        }
        __syncthreads();
        __shared__ int sh_digit;
        __shared__ int64_t sh_k;
        if (threadIdx.x == 0) {
            int64_t run = 0;
            int d = 0;
            for (; d < 256; ++d) {
                if (run + hist[d] > k) break;
                run += hist[d];
            }
            sh_digit = d;
            sh_k = k - run;
        }
        __syncthreads();
        prefix |= (uint64_t)sh_digit << shift;
        mask |= (uint64_t)255 << shift;
        k = sh_k;
        __syncthreads();
    }
    const uint64_t b = (prefix >> 63) ? (prefix & 0x7fffffffffffffffull) : ~prefix;
    return __longlong_as_double((long long)b);
}

template <typename F>
__device__ double median_of(F f, int64_t n, uint32_t* hist) {
    if (n % 2) return select_kth(f, n, n / 2, hist);
    const double a = select_kth(f, n, n / 2 - 1, hist);
    const double b = select_kth(f, n, n / 2, hist);
    return 0.5 * (a + b);
}

__device__ __forceinline__ int bin_of(double t, double t0, double span) {
    if (!(span > 0.0)) return 0;
    const double x = floor((t - t0) / span * (double)L);
    return x < 0.0 ? 0 : (x > (double)(L - 1) ? L - 1 : (int)x);
}

// One workgroup per curve; time must be non-decreasing within each curve.
__global__ __launch_bounds__(256) void k_view(const int64_t* __restrict__ offsets, const double* __restrict__ t,
                                              const double* __restrict__ y, float* __restrict__ views) {
    __shared__ uint32_t hist[256];
    __shared__ double sh_med, sh_scale;
    const int c = blockIdx.x;
    const int64_t o = offsets[c], n = offsets[c + 1] - o;
    const double* tc = t + o;
    const double* yc = y + o;
    const double t0 = tc[0], span = tc[n - 1] - tc[0];
    const double med = median_of([&](int64_t i) { return yc[i]; }, n, hist);
    if (threadIdx.x == 0) sh_med = med;
    __syncthreads();
    const double m0 = sh_med;
    const double mad = median_of([&](int64_t i) { return fabs(yc[i] - m0); }, n, hist);
    if (threadIdx.x == 0) sh_scale = 1.4826 * mad;
    __syncthreads();
    const double scale = sh_scale;
    float* v = views + (size_t)c * L;
    for (int b = threadIdx.x; b < L; b += 256) {
        // points of bin b: [lo, hi) found by binary search on the bin index
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (bin_of(tc[mid], t0, span) < b) lo = mid + 1;
            else hi = mid;
        }
        int64_t e = lo, h2 = n;
        while (e < h2) {
            const int64_t mid = (e + h2) >> 1;
            if (bin_of(tc[mid], t0, span) <= b) e = mid + 1;
            else h2 = mid;
        }
        const int64_t m = e - lo;
        double out = 0.0;
        if (m > 0 && scale > 0.0) {
            // ranks by counting (ties by position); median of an even count
            // is the mean of the two middle values
            double lo_v = 0.0, hi_v = 0.0;
            const int64_t r1 = (m - 1) / 2, r2 = m / 2;
            for (int64_t a = 0; a < m; ++a) {
                const double x = yc[lo + a];
                int64_t rank = 0;
                for (int64_t q = 0; q < m; ++q) {
                    const double z = yc[lo + q];
                    rank += (z < x) || (z == x && q < a);
                }
                if (rank == r1) lo_v = x;
                if (rank == r2) hi_v = x;
            }
            const double bm = (m % 2) ? lo_v : 0.5 * (lo_v + hi_v);
            out = (bm - 1.0) / scale;
        }
        v[b] = (float)out;
    }
}

// ------------------------------------------------------------------------
// Convolution as implicit GEMM on 32x32x16 BF16 MFMA tiles.
//
// One wave computes a 32 (positions) x 32 (output channels) tile.  Operand
// layout of v_mfma_f32_32x32x16_bf16: lane l supplies row (l % 32) of A and
// column (l % 32) of B, K elements 8 * (l / 32) .. +8 of the 16-wide slice;
// accumulator element r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.

struct ConvArgs {
    const __bf16* in;        // [B][L][cin] channels-last
    int cin;
    const __bf16* wt;        // [cout = 32][KW][cin]  (tap-major, channel-minor)
    const float* bias;       // [32] or null
    int B;
    float* z;                // [B][L][32] pre-activation (FP32), or null
    __bf16* act;             // [B][L][32] activation (bf16), or null
    const float* gz;         // backward-data: multiply by gelu'(gz[..]) (FP32) before storing, or null
    int gelu_out;            // 1: act = gelu(z)
};

__device__ __forceinline__ bf16x8 load8_in(const __bf16* base, int cin, int b, int pos, int ci0) {
    bf16x8 v;
    if (pos < 0 || pos >= L) {
        for (int q = 0; q < 8; ++q) v[q] = (__bf16)0.0f;
        return v;
    }
    const __bf16* p = base + ((size_t)b * L + pos) * cin + ci0;
    for (int q = 0; q < 8; ++q) v[q] = p[q];
    return v;
}

__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * 4 + wave;                 // 32-position tile over B * L
    const int tiles_per_sample = L / 32;
    if (tile >= a.B * tiles_per_sample) return;
    const int b = tile / tiles_per_sample;
    const int p0 = (tile - b * tiles_per_sample) * 32;
    const int row = lane & 31, half = lane >> 5;
    floatx16 acc;
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    if (a.cin == 1) {
        // K = 7 taps padded to 16
        bf16x8 av, bv;
        for (int q = 0; q < 8; ++q) {
            const int k = 8 * half + q;
            const int pos = p0 + row + k - 3;
            av[q] = (k < KW && pos >= 0 && pos < L) ? a.in[(size_t)b * L + pos] : (__bf16)0.0f;
            bv[q] = (k < KW) ? a.wt[(size_t)row * KW + k] : (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    } else {
        const int cblocks = a.cin / 16;
        for (int k = 0; k < KW; ++k) {
            for (int cb = 0; cb < cblocks; ++cb) {
                const int ci0 = cb * 16 + 8 * half;
                const bf16x8 av = load8_in(a.in, a.cin, b, p0 + row + k - 3, ci0);
                bf16x8 bv;
                const __bf16* wp = a.wt + ((size_t)row * KW + k) * a.cin + ci0;
                for (int q = 0; q < 8; ++q) bv[q] = wp[q];
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            }
        }
    }
    const int col = lane & 31;
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * half + (r & 3);
        const size_t idx = ((size_t)b * L + p0 + m) * C + col;
        float zv = acc[r] + (a.bias ? a.bias[col] : 0.0f);
        if (a.gz) zv *= gelu_grad(a.gz[idx]);
        if (a.z) a.z[idx] = zv;
        if (a.act) a.act[idx] = (__bf16)(a.gelu_out ? gelu(zv) : zv);
    }
}

// dW[co][k][ci] partials per sample (and the bias gradient's, dz summed per
// channel), reduced over the samples in a fixed order afterwards, so
// gradients are deterministic.
struct WGradArgs {
    const __bf16* dz;        // [B][L][32]
    const __bf16* in;        // [B][L][cin]
    int cin;
    int B;
    float* partial;          // [B][32][KW][cin]
    float* bpartial;         // [B][32]
};

constexpr int kWgWaves = 4;          // waves per sample, each over L / kWgWaves positions
constexpr int kWgChunk = 64;         // positions per LDS chunk of a wave
constexpr int kWgPad = C + 8;        // LDS row stride in bf16 (80 bytes: 16-byte rows, spread banks)
static_assert(L % (kWgWaves * kWgChunk) == 0 && kWgChunk % 16 == 0 && C % 8 == 0, "wgrad tiling");

// One workgroup per sample b.  Wave w sums the positions [w L/4, (w+1) L/4)
// for all KW taps at once (dW_k[co][ci] += dz[pos][co] in[pos + k - 3][ci]:
// one 32x32x16 MFMA per tap and 16 positions, the dz operand shared by the
// taps), from chunks staged in its own LDS rows with 16-byte loads.  The
// waves' sums are then added in wave order through LDS, and the bias
// gradient likewise, so the per-sample partials are deterministic.
__global__ __launch_bounds__(64 * kWgWaves) void k_conv_wgrad(WGradArgs a) {
    __shared__ __align__(16) __bf16 dzs[kWgWaves][kWgChunk][kWgPad];
    __shared__ __align__(16) __bf16 ins[kWgWaves][kWgChunk + KW - 1][kWgPad];
    __shared__ float red[C * KW * C];
    __shared__ float bred[kWgWaves][C];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int b = blockIdx.x;
    const int row = lane & 31, half = lane >> 5;
    const int cin = a.cin;
    floatx16 acc[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k)
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.0f;
    float bsum = 0.0f;
    const __bf16* dzb = a.dz + (size_t)b * L * C;
    const __bf16* inb = a.in + (size_t)b * L * cin;
    const int pbeg = w * (L / kWgWaves), pend = pbeg + L / kWgWaves;
    for (int p0 = pbeg; p0 < pend; p0 += kWgChunk) {
        // dz rows p0 .. p0 + kWgChunk - 1, eight channels per 16-byte piece
        for (int e = lane; e < kWgChunk * (C / 8); e += 64) {
            const int pp = e / (C / 8), c8 = (e % (C / 8)) * 8;
            *reinterpret_cast<uint4*>(&dzs[w][pp][c8]) =
                *reinterpret_cast<const uint4*>(dzb + (size_t)(p0 + pp) * C + c8);
        }
        // input rows p0 - 3 .. p0 + kWgChunk + 2 (zeros outside the curve)
        if (cin == C) {
            for (int e = lane; e < (kWgChunk + KW - 1) * (C / 8); e += 64) {
                const int pp = e / (C / 8), c8 = (e % (C / 8)) * 8;
                const int pos = p0 + pp - 3;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (pos >= 0 && pos < L) v = *reinterpret_cast<const uint4*>(inb + (size_t)pos * C + c8);
                *reinterpret_cast<uint4*>(&ins[w][pp][c8]) = v;
            }
        } else {
            for (int e = lane; e < (kWgChunk + KW - 1) * cin; e += 64) {
                const int pp = e / cin, cc = e - pp * cin;
                const int pos = p0 + pp - 3;
                ins[w][pp][cc] = (pos >= 0 && pos < L) ? inb[(size_t)pos * cin + cc] : (__bf16)0.0f;
            }
        }
        __syncthreads();
        for (int st = 0; st < kWgChunk / 16; ++st) {
            bf16x8 av;
#pragma unroll
            for (int q = 0; q < 8; ++q) av[q] = dzs[w][16 * st + 8 * half + q][row];         // A[co][pos]
#pragma unroll
            for (int k = 0; k < KW; ++k) {
                bf16x8 bv;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    bv[q] = (row < cin) ? ins[w][16 * st + 8 * half + q + k][row] : (__bf16)0.0f;   // B[pos][ci]
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[k], 0, 0, 0);
            }
        }
        if (lane < C)
            for (int pp = 0; pp < kWgChunk; ++pp) bsum += (float)dzs[w][pp][lane];
        __syncthreads();
    }
    // the waves' sums, added in wave order
    for (int ww = 0; ww < kWgWaves; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int k = 0; k < KW; ++k)
                for (int r = 0; r < 16; ++r) {
                    const int co = 8 * (r >> 2) + 4 * half + (r & 3);
                    const int i = (co * KW + k) * C + row;
                    red[i] = ww == 0 ? acc[k][r] : red[i] + acc[k][r];
                }
        }
        __syncthreads();
    }
    if (lane < C) bred[w][lane] = bsum;
    __syncthreads();
    float* out = a.partial + (size_t)b * C * KW * cin;
    for (int i = tid; i < C * KW * cin; i += 64 * kWgWaves) {
        const int co = i / (KW * cin), rem = i - co * KW * cin, k = rem / cin, ci = rem - k * cin;
        out[i] = red[(co * KW + k) * C + ci];
    }
    if (tid < C) {
        float s = bred[0][tid];
        for (int ww = 1; ww < kWgWaves; ++ww) s += bred[ww][tid];
        a.bpartial[(size_t)b * C + tid] = s;
    }
}

// Sum of the per-sample partials in sample order, written in the flat
// (co, ci, k) order, and the bias gradient likewise.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial,
                                                      const float* __restrict__ bpartial, int nparts, int cin,
                                                      float* __restrict__ grad_w, float* __restrict__ grad_b) {
    const int i = blockIdx.x * 256 + threadIdx.x;          // over (co, k, ci), then the 32 biases
    const int n = C * KW * cin;
    if (i < n) {
        float s = 0.0f;
        for (int p = 0; p < nparts; ++p) s += partial[(size_t)p * n + i];
        const int co = i / (KW * cin), rem = i - co * KW * cin, k = rem / cin, ci = rem - k * cin;
        grad_w[((size_t)co * cin + ci) * KW + k] = s;
    } else if (i < n + C) {
        const int co = i - n;
        float s = 0.0f;
        for (int p = 0; p < nparts; ++p) s += bpartial[(size_t)p * C + co];
        grad_b[co] = s;
    }
}

// ------------------------------------------------------------------------
// Pool, head, loss.

// g[b][c] = mean over positions of gelu(z5).
__global__ __launch_bounds__(256) void k_pool(const float* __restrict__ z, int B, float* __restrict__ g) {
    __shared__ float red[8][C];
    const int b = blockIdx.x;
    const int c = threadIdx.x & 31, part = threadIdx.x >> 5;
    float s = 0.0f;
    for (int p = part; p < L; p += 8) s += gelu(z[((size_t)b * L + p) * C + c]);
    red[part][c] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.0f;
        for (int q = 0; q < 8; ++q) t += red[q][threadIdx.x];
        g[(size_t)b * C + threadIdx.x] = t / (float)L;
    }
}

// logits, softmax cross-entropy, dlogits (mean over the batch).
__global__ __launch_bounds__(NB) void k_head(const float* __restrict__ params, const float* __restrict__ g, int B,
                                             const int32_t* __restrict__ labels, float* __restrict__ logits,
                                             float* __restrict__ dlogits, float* __restrict__ losses) {
    __shared__ float red[NB];
    const int b = blockIdx.x, j = threadIdx.x;
    const float* wf = params + kWf;
    float acc = params[kBf + j];
    for (int c = 0; c < C; ++c) acc += wf[j * C + c] * g[(size_t)b * C + c];
    logits[(size_t)b * NB + j] = acc;
    if (!labels) return;
    red[j] = acc;
    __syncthreads();
    for (int w = NB / 2; w > 0; w >>= 1) {
        if (j < w) red[j] = fmaxf(red[j], red[j + w]);
        __syncthreads();
    }
    const float mx = red[0];
    __syncthreads();
    const float e = expf(acc - mx);
    red[j] = e;
    __syncthreads();
    for (int w = NB / 2; w > 0; w >>= 1) {
        if (j < w) red[j] += red[j + w];
        __syncthreads();
    }
    const float se = red[0];
    const int lab = labels[b];
    dlogits[(size_t)b * NB + j] = (e / se - (j == lab ? 1.0f : 0.0f)) / (float)B;
    if (j == lab) losses[b] = (mx + logf(se)) - acc;
}

// dWf, dbf (one thread per head parameter) and dg.
__global__ __launch_bounds__(256) void k_head_bwd(const float* __restrict__ params, const float* __restrict__ g,
                                                  const float* __restrict__ dl, int B, float* __restrict__ grads,
                                                  float* __restrict__ dg) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < NB * C) {
        const int j = i / C, c = i - j * C;
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += dl[(size_t)b * NB + j] * g[(size_t)b * C + c];
        grads[kWf + i] = s;
    } else if (i < NB * C + NB) {
        const int j = i - NB * C;
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += dl[(size_t)b * NB + j];
        grads[kBf + j] = s;
    } else if (i < NB * C + NB + B * C) {
        const int q = i - NB * C - NB, b = q / C, c = q - b * C;
        float s = 0.0f;
        for (int j = 0; j < NB; ++j) s += dl[(size_t)b * NB + j] * params[kWf + j * C + c];
        dg[(size_t)b * C + c] = s;
    }
}

// dz5 = dg / L * gelu'(z5), stored bf16 for the MFMA backward passes.
__global__ __launch_bounds__(256) void k_pool_bwd(const float* __restrict__ dg, const float* __restrict__ z, int B,
                                                  __bf16* __restrict__ dz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)B * L * C) return;
    const int64_t b = i / ((int64_t)L * C);
    const int c = (int)(i % C);
    dz[i] = (__bf16)(dg[b * C + c] / (float)L * gelu_grad(z[i]));
}

// ------------------------------------------------------------------------
// Adam and the BF16 weight copies.

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Forward weights [co][k][ci] and flipped backward-data weights
// [ci][6 - k][co] for every layer.
__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ p, __bf16* __restrict__ wf_all,
                                                      __bf16* __restrict__ wb_all) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    int64_t off = 0;
    for (int l = 0; l < NL; ++l) {
        const int cin = cin_of(l), n = C * cin * KW;
        if (i < n) {
            const int co = i / (cin * KW), rem = i - co * cin * KW, ci = rem / KW, k = rem - ci * KW;
            const __bf16 w = (__bf16)p[w_off(l) + i];
            wf_all[off + ((size_t)co * KW + k) * cin + ci] = w;
            wb_all[off + ((size_t)ci * KW + (KW - 1 - k)) * C + co] = w;
        }
        off += n;
    }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ x, int64_t n, __bf16* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = (__bf16)x[i];
}

__global__ __launch_bounds__(256) void k_topk(const float* __restrict__ logits, int k, int32_t* __restrict__ bins) {
    // k largest of 512 logits per sample, largest first, ties to the lower index
    __shared__ float v[NB];
    const int b = blockIdx.x;
    for (int j = threadIdx.x; j < NB; j += 256) v[j] = logits[(size_t)b * NB + j];
    __syncthreads();
    for (int j = threadIdx.x; j < NB; j += 256) {
        int rank = 0;
        for (int q = 0; q < NB; ++q) rank += (v[q] > v[j]) || (v[q] == v[j] && q < j);
        if (rank < k) bins[(size_t)b * k + rank] = j;
    }
}

}  // namespace cnn
}  // namespace gtls

// ------------------------------------------------------------------------
// Network object and C ABI.

using namespace gtls::cnn;

struct gtls_cnn {
    gtls_ctx* ctx = nullptr;
    float* params = nullptr;     // FP32 master weights, flat
    float* grads = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    __bf16* wf = nullptr;        // packed forward weights
    __bf16* wb = nullptr;        // packed backward-data weights
    int64_t step = 0;
    // activations for the current batch capacity
    int cap = 0;
    __bf16* x = nullptr;         // [B][L] input view (bf16)
    float* z[NL] = {nullptr};    // [B][L][32]
    __bf16* h[NL] = {nullptr};   // [B][L][32]
    __bf16* dz = nullptr;        // [B][L][32]
    __bf16* dz2 = nullptr;
    float* g = nullptr;          // [B][32]
    float* dg = nullptr;
    float* logits = nullptr;     // [B][512]
    float* dlogits = nullptr;
    float* losses = nullptr;     // [B]
    int32_t* labels = nullptr;
    float* partial = nullptr;    // weight-gradient partials
    float* views = nullptr;      // [B][L] staging
    int32_t* bins = nullptr;
};

namespace {

int64_t packed_weights() {
    int64_t n = 0;
    for (int l = 0; l < NL; ++l) n += (int64_t)C * cin_of(l) * KW;
    return n;
}

hipError_t cnn_reserve(gtls_cnn* net, int B) {
    if (B <= net->cap) return hipSuccess;
    hipError_t e = hipStreamSynchronize(net->ctx->stream);
    if (e != hipSuccess) return e;
    void** bufs[] = {(void**)&net->x, (void**)&net->dz, (void**)&net->dz2, (void**)&net->g, (void**)&net->dg,
                     (void**)&net->logits, (void**)&net->dlogits, (void**)&net->losses, (void**)&net->labels,
                     (void**)&net->partial, (void**)&net->views, (void**)&net->bins};
    for (void** b : bufs)
        if (*b) {
            (void)hipFree(*b);
            *b = nullptr;
        }
    for (int l = 0; l < NL; ++l) {
        if (net->z[l]) (void)hipFree(net->z[l]);
        if (net->h[l]) (void)hipFree(net->h[l]);
        net->z[l] = nullptr;
        net->h[l] = nullptr;
    }
    net->cap = 0;
    const size_t act = (size_t)B * L * C;
    if ((e = hipMalloc(&net->x, 2 * (size_t)B * L)) != hipSuccess) return e;
    for (int l = 0; l < NL; ++l) {
        if ((e = hipMalloc(&net->z[l], 4 * act)) != hipSuccess) return e;
        if ((e = hipMalloc(&net->h[l], 2 * act)) != hipSuccess) return e;
    }
    if ((e = hipMalloc(&net->dz, 2 * act)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->dz2, 2 * act)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->g, 4 * (size_t)B * C)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->dg, 4 * (size_t)B * C)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->logits, 4 * (size_t)B * NB)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->dlogits, 4 * (size_t)B * NB)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->losses, 4 * (size_t)B)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->labels, 4 * (size_t)B)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->partial, 4 * (size_t)B * (C * KW * C + C))) != hipSuccess) return e;
    if ((e = hipMalloc(&net->views, 4 * (size_t)B * L)) != hipSuccess) return e;
    if ((e = hipMalloc(&net->bins, 4 * (size_t)B * NB)) != hipSuccess) return e;
    net->cap = B;
    return hipSuccess;
}

void cnn_forward(gtls_cnn* net, int B) {
    hipStream_t s = net->ctx->stream;
    k_to_bf16<<<(unsigned)(((int64_t)B * L + 255) / 256), 256, 0, s>>>(net->views, (int64_t)B * L, net->x);
    int64_t woff = 0;
    const __bf16* in = net->x;
    for (int l = 0; l < NL; ++l) {
        ConvArgs a{in, cin_of(l), net->wf + woff, net->params + b_off(l), B, net->z[l], net->h[l], nullptr, 1};
        k_conv<<<(unsigned)((B * (L / 32) + 3) / 4), 256, 0, s>>>(a);
        in = net->h[l];
        woff += (int64_t)C * cin_of(l) * KW;
    }
    k_pool<<<B, 256, 0, s>>>(net->z[NL - 1], B, net->g);
}

void cnn_backward(gtls_cnn* net, int B) {
    hipStream_t s = net->ctx->stream;
    k_head_bwd<<<(unsigned)((NB * C + NB + B * C + 255) / 256), 256, 0, s>>>(net->params, net->g, net->dlogits, B,
                                                                               net->grads, net->dg);
    k_pool_bwd<<<(unsigned)(((int64_t)B * L * C + 255) / 256), 256, 0, s>>>(net->dg, net->z[NL - 1], B, net->dz);
    int64_t woffs[NL];
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        woffs[l] = o;
        o += (int64_t)C * cin_of(l) * KW;
    }
    __bf16* dz = net->dz;
    __bf16* dzn = net->dz2;
    for (int l = NL - 1; l >= 0; --l) {
        const int cin = cin_of(l);
        const __bf16* in = l == 0 ? net->x : net->h[l - 1];
        float* bpart = net->partial + (size_t)B * C * KW * C;
        WGradArgs wa{dz, in, cin, B, net->partial, bpart};
        k_conv_wgrad<<<(unsigned)B, 64 * kWgWaves, 0, s>>>(wa);
        k_wgrad_reduce<<<(unsigned)((C * KW * cin + C + 255) / 256), 256, 0, s>>>(net->partial, bpart, B, cin,
                                                                                 net->grads + w_off(l),
                                                                                 net->grads + b_off(l));
        if (l > 0) {
            // dz_{l-1} = (W_l^T * dz_l) * gelu'(z_{l-1}): the forward kernel with flipped weights
            ConvArgs a{dz, C, net->wb + woffs[l], nullptr, B, nullptr, dzn, net->z[l - 1], 0};
            k_conv<<<(unsigned)((B * (L / 32) + 3) / 4), 256, 0, s>>>(a);
            __bf16* t = dz;
            dz = dzn;
            dzn = t;
        }
    }
}

gtls_status cnn_fail(gtls_cnn* net, hipError_t e, const char* where) {
    if (net && net->ctx) net->ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? GTLS_ENOMEM : GTLS_EDEVICE;
}

}  // namespace

extern "C" {

int64_t gtls_cnn_num_params(void) { return kNParams; }

gtls_status gtls_cnn_create(gtls_ctx* ctx, const float* init_params, gtls_cnn** out) {
    if (!ctx || !out || !init_params) return GTLS_EINVAL;
    *out = nullptr;
    gtls_cnn* net = new gtls_cnn();
    net->ctx = ctx;
    hipError_t e = hipSetDevice(ctx->device);
    const size_t pb = 4 * (size_t)kNParams;
    if (e == hipSuccess) e = hipMalloc(&net->params, pb);
    if (e == hipSuccess) e = hipMalloc(&net->grads, pb);
    if (e == hipSuccess) e = hipMalloc(&net->adam_m, pb);
    if (e == hipSuccess) e = hipMalloc(&net->adam_v, pb);
    if (e == hipSuccess) e = hipMalloc(&net->wf, 2 * (size_t)packed_weights());
    if (e == hipSuccess) e = hipMalloc(&net->wb, 2 * (size_t)packed_weights());
    if (e == hipSuccess) e = hipMemcpyAsync(net->params, init_params, pb, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(net->adam_m, 0, pb, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(net->adam_v, 0, pb, ctx->stream);
    if (e == hipSuccess) {
        k_pack_weights<<<(C * C * KW + 255) / 256, 256, 0, ctx->stream>>>(net->params, net->wf, net->wb);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        gtls_status st = cnn_fail(net, e, "cnn create");
        gtls_cnn_destroy(net);
        return st;
    }
    *out = net;
    return GTLS_OK;
}

void gtls_cnn_destroy(gtls_cnn* net) {
    if (!net) return;
    if (net->ctx) (void)hipStreamSynchronize(net->ctx->stream);
    void* bufs[] = {net->params, net->grads, net->adam_m, net->adam_v, net->wf, net->wb, net->x, net->dz, net->dz2,
                    net->g, net->dg, net->logits, net->dlogits, net->losses, net->labels, net->partial, net->views,
                    net->bins};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int l = 0; l < NL; ++l) {
        if (net->z[l]) (void)hipFree(net->z[l]);
        if (net->h[l]) (void)hipFree(net->h[l]);
    }
    delete net;
}

gtls_status gtls_cnn_view(gtls_ctx* ctx, const int64_t* offsets, const double* time, const double* flux,
                          int32_t n_curves, float* views) {
    if (!ctx || !offsets || !time || !flux || !views || n_curves < 1) return GTLS_EINVAL;
    const int64_t npts = offsets[n_curves];
    for (int32_t c = 0; c < n_curves; ++c) {
        if (offsets[c + 1] - offsets[c] < 1) {
            ctx->err = "each curve needs at least one point";
            return GTLS_EINVAL;
        }
        for (int64_t i = offsets[c] + 1; i < offsets[c + 1]; ++i)
            if (!(time[i] >= time[i - 1])) {
                ctx->err = "time must be non-decreasing within each curve for the view";
                return GTLS_EINVAL;
            }
    }
    for (int64_t i = 0; i < npts; ++i)
        if (!std::isfinite(time[i]) || !std::isfinite(flux[i])) {
            ctx->err = "non-finite time or flux";
            return GTLS_EINVAL;
        }
    hipError_t e = hipSetDevice(ctx->device);
    void *d_off = nullptr, *d_t = nullptr, *d_y = nullptr, *d_v = nullptr;
    hipStream_t s = ctx->stream;
    if (e == hipSuccess) e = hipMalloc(&d_off, 8 * (size_t)(n_curves + 1));
    if (e == hipSuccess) e = hipMalloc(&d_t, 8 * (size_t)npts);
    if (e == hipSuccess) e = hipMalloc(&d_y, 8 * (size_t)npts);
    if (e == hipSuccess) e = hipMalloc(&d_v, 4 * (size_t)n_curves * L);
    if (e == hipSuccess) e = hipMemcpyAsync(d_off, offsets, 8 * (size_t)(n_curves + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_t, time, 8 * (size_t)npts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_y, flux, 8 * (size_t)npts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_view<<<n_curves, 256, 0, s>>>((const int64_t*)d_off, (const double*)d_t, (const double*)d_y, (float*)d_v);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(views, d_v, 4 * (size_t)n_curves * L, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (void* p : {d_off, d_t, d_y, d_v})
        if (p) (void)hipFree(p);
    if (e != hipSuccess) {
        ctx->err = std::string("cnn view: ") + hipGetErrorString(e);
        return GTLS_EDEVICE;
    }
    return GTLS_OK;
}

gtls_status gtls_cnn_forward(gtls_cnn* net, const float* views, int32_t B, float* logits) {
    if (!net || !views || !logits || B < 1) return GTLS_EINVAL;
    hipStream_t s = net->ctx->stream;
    hipError_t e = cnn_reserve(net, B);
    if (e == hipSuccess) e = hipMemcpyAsync(net->views, views, 4 * (size_t)B * L, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return cnn_fail(net, e, "cnn forward");
    cnn_forward(net, B);
    k_head<<<B, NB, 0, s>>>(net->params, net->g, B, nullptr, net->logits, nullptr, nullptr);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(logits, net->logits, 4 * (size_t)B * NB, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GTLS_OK : cnn_fail(net, e, "cnn forward");
}

gtls_status gtls_cnn_gradients(gtls_cnn* net, const float* views, const int32_t* labels, int32_t B, float* loss,
                               float* grads) {
    if (!net || !views || !labels || B < 1) return GTLS_EINVAL;
    for (int32_t b = 0; b < B; ++b)
        if (labels[b] < 0 || labels[b] >= NB) return GTLS_EINVAL;
    hipStream_t s = net->ctx->stream;
    hipError_t e = cnn_reserve(net, B);
    if (e == hipSuccess) e = hipMemcpyAsync(net->views, views, 4 * (size_t)B * L, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(net->labels, labels, 4 * (size_t)B, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return cnn_fail(net, e, "cnn gradients");
    cnn_forward(net, B);
    k_head<<<B, NB, 0, s>>>(net->params, net->g, B, net->labels, net->logits, net->dlogits, net->losses);
    cnn_backward(net, B);
    e = hipGetLastError();
    std::vector<float> lb(B);
    if (e == hipSuccess) e = hipMemcpyAsync(lb.data(), net->losses, 4 * (size_t)B, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && grads)
        e = hipMemcpyAsync(grads, net->grads, 4 * (size_t)kNParams, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cnn_fail(net, e, "cnn gradients");
    if (loss) {
        double t = 0.0;
        for (float x : lb) t += x;
        *loss = (float)(t / B);
    }
    return GTLS_OK;
}

gtls_status gtls_cnn_train_step(gtls_cnn* net, const float* views, const int32_t* labels, int32_t B, float lr,
                                float* loss) {
    gtls_status st = gtls_cnn_gradients(net, views, labels, B, loss, nullptr);
    if (st != GTLS_OK) return st;
    hipStream_t s = net->ctx->stream;
    net->step += 1;
    const float c1 = 1.0f - std::pow(0.9f, (float)net->step), c2 = 1.0f - std::pow(0.999f, (float)net->step);
    k_adam<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(net->params, net->grads, net->adam_m, net->adam_v,
                                                              kNParams, lr, c1, c2);
    k_pack_weights<<<(C * C * KW + 255) / 256, 256, 0, s>>>(net->params, net->wf, net->wb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GTLS_OK : cnn_fail(net, e, "cnn train step");
}

gtls_status gtls_cnn_get_params(gtls_cnn* net, float* params) {
    if (!net || !params) return GTLS_EINVAL;
    hipError_t e = hipMemcpyAsync(params, net->params, 4 * (size_t)kNParams, hipMemcpyDeviceToHost, net->ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->ctx->stream);
    return e == hipSuccess ? GTLS_OK : cnn_fail(net, e, "cnn get params");
}

gtls_status gtls_cnn_topk(gtls_cnn* net, const float* views, int32_t B, int32_t k, int32_t* bins) {
    if (!net || !views || !bins || B < 1 || k < 1 || k > NB) return GTLS_EINVAL;
    hipStream_t s = net->ctx->stream;
    hipError_t e = cnn_reserve(net, B);
    if (e == hipSuccess) e = hipMemcpyAsync(net->views, views, 4 * (size_t)B * L, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return cnn_fail(net, e, "cnn topk");
    cnn_forward(net, B);
    k_head<<<B, NB, 0, s>>>(net->params, net->g, B, nullptr, net->logits, nullptr, nullptr);
    k_topk<<<B, 256, 0, s>>>(net->logits, k, net->bins);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(bins, net->bins, 4 * (size_t)B * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GTLS_OK : cnn_fail(net, e, "cnn topk");
}

// Checkpoint file: 8-byte magic "GTLSCNN1", int64 parameter count, int64
// Adam step, then the FP32 parameters, the Adam first and second moments
// (little-endian, parameter order).
static const char kCkptMagic[8] = {'G', 'T', 'L', 'S', 'C', 'N', 'N', '1'};

gtls_status gtls_cnn_save(gtls_cnn* net, const char* path) {
    if (!net || !path) return GTLS_EINVAL;
    std::vector<float> buf(3 * (size_t)kNParams);
    hipStream_t s = net->ctx->stream;
    hipError_t e = hipMemcpyAsync(buf.data(), net->params, 4 * (size_t)kNParams, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(buf.data() + kNParams, net->adam_m, 4 * (size_t)kNParams, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(buf.data() + 2 * kNParams, net->adam_v, 4 * (size_t)kNParams, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cnn_fail(net, e, "cnn save");
    FILE* f = std::fopen(path, "wb");
    if (!f) {
        net->ctx->err = std::string("cannot open ") + path + " for writing";
        return GTLS_EINVAL;
    }
    const int64_t hdr[2] = {kNParams, net->step};
    bool ok = std::fwrite(kCkptMagic, 1, 8, f) == 8 && std::fwrite(hdr, 8, 2, f) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        net->ctx->err = std::string("write to ") + path + " failed";
        return GTLS_EINVAL;
    }
    return GTLS_OK;
}

gtls_status gtls_cnn_load(gtls_cnn* net, const char* path) {
    if (!net || !path) return GTLS_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        net->ctx->err = std::string("cannot open ") + path;
        return GTLS_EINVAL;
    }
    char magic[8];
    int64_t hdr[2];
    std::vector<float> buf(3 * (size_t)kNParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kCkptMagic, 8) == 0 &&
              std::fread(hdr, 8, 2, f) == 2 && hdr[0] == kNParams && hdr[1] >= 0 &&
              std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!ok) {
        net->ctx->err = std::string(path) + " is not a checkpoint of this network";
        return GTLS_EINVAL;
    }
    hipStream_t s = net->ctx->stream;
    hipError_t e = hipMemcpyAsync(net->params, buf.data(), 4 * (size_t)kNParams, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(net->adam_m, buf.data() + kNParams, 4 * (size_t)kNParams, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(net->adam_v, buf.data() + 2 * kNParams, 4 * (size_t)kNParams, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_pack_weights<<<(C * C * KW + 255) / 256, 256, 0, s>>>(net->params, net->wf, net->wb);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cnn_fail(net, e, "cnn load");
    net->step = hdr[1];
    return GTLS_OK;
}

}  // extern "C"
