// Small MLP for the learned approximate mode: 8 -> 64 -> 64 -> 1 with ReLU,
// BF16 weights and activations into MFMA (V_MFMA_F32_16X16X32_BF16 for the
// 64-long contractions, V_MFMA_F32_16X16X16_BF16 for the 16-long ones),
// FP32 accumulation, FP32 biases, FP32 master weights and Adam (gfx950).
//
// It maps the 8 log-scaled cheap features of a vertex to its log-scaled
// h-degree.  The paper estimates updated h-degrees by sampling (Section
// IV-C); this estimator is trained on exact h-degrees the library itself
// computes, and the exact peeling stays the reference for its error.
//
// MFMA operand layouts (bf16 inputs), lane l of a wavefront, r = l % 16,
// q = l / 16, measured on the device:
//   16x16x16: A (16 x 16, M x K): a[i] = A[r][4q + i], i < 4
//             B (16 x 16, K x N): b[i] = B[4q + i][r]
//   16x16x32: A (16 x 32): a[i] = A[r][8q + i], i < 8; B (32 x 16): b[i] = B[8q + i][r]
//   both:     D (16 x 16, M x N): d[i] = D[4q + i][r]
// The contractions over the 64 hidden units (layers 2 and 3 forward, dH1
// backward) take two K = 32 steps; those over the 16 rows of a tile (dW1,
// dW2) and over the 8 features padded to 16 (layer 1) take one K = 16 step.
// A wavefront processes 16 rows (vertices) per tile.  Activations move
// between layers through LDS, where the D layout of one layer is re-read
// in the A layout of the next.
//
// Parameter vector (fp32, 4801 values): W1[64][8], b1[64], W2[64][64],
// b2[64], W3[64], b3.  BF16 copies: W1 padded to [64][16], W2 [64][64],
// W3 padded to [16][64] (row 0 real).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "khc_internal.h"

namespace khc {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 8, kHid = 64;
constexpr int oW1 = 0, ob1 = oW1 + kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid, oW3 = ob2 + kHid,
              ob3 = oW3 + kHid, kParams = ob3 + 1;
static_assert(kParams == 4801, "parameter count");
constexpr char kMlpMagic[8] = {'K', 'H', 'C', 'M', 'L', 'P', '0', '1'};
// bf16 copies (shorts): W1p [64][16], W2 [64][64], W3p [16][64]
constexpr int cW1 = 0, cW2 = cW1 + kHid * 16, cW3 = cW2 + kHid * kHid, kCopies = cW3 + 16 * kHid;

// fp32 -> bf16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (short)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(((uint32_t)(uint16_t)b) << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a), __builtin_bit_cast(bf16v8, b), c, 0,
                                                   0, 0);
}

// Forward pass of one 16-row tile (one wavefront).  X rows are given by
// ridx (null: consecutive from row0); rows >= n are zero and ignored.
// Leaves H1 and H2 (bf16, [16][64]) in the wave's LDS slices and returns
// y for lanes with r == 0 in out_y[i] (rows 4q + i).
struct TileLds {
    short h1[16][kHid + 4];
    short h2[16][kHid + 4];
    short x[16][16];
    float y[16];
    float dy[16];
};

__device__ void tile_forward(const float *X, const uint32_t *ridx, uint32_t row0, uint32_t n,
                             const float *params, const short *copies, TileLds &t) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    // X tile in bf16 ([16][16], features 8..15 zero)
    for (int e = lane; e < 256; e += 64) {
        const int rr = e >> 4, k = e & 15;
        const uint32_t row = row0 + rr;
        float v = 0.f;
        if (k < kIn && row < n) v = X[(size_t)(ridx ? ridx[row] : row) * kIn + k];
        t.x[rr][k] = f2bf(v);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    bf16x4 a;
    for (int i = 0; i < 4; ++i) a[i] = t.x[r][4 * q + i];
    const short *W1p = copies + cW1, *W2 = copies + cW2, *W3p = copies + cW3;
    for (int tn = 0; tn < 4; ++tn) {
        bf16x4 b;
        for (int i = 0; i < 4; ++i) b[i] = W1p[(16 * tn + r) * 16 + 4 * q + i];
        f32x4 acc = mfma(a, b, f32x4{0.f, 0.f, 0.f, 0.f});
        const float bias = params[ob1 + 16 * tn + r];
        for (int i = 0; i < 4; ++i) {
            const float hv = acc[i] + bias;
            t.h1[4 * q + i][16 * tn + r] = f2bf(hv > 0.f ? hv : 0.f);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    for (int tn = 0; tn < 4; ++tn) {
        f32x4 acc{0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < 2; ++s) {
            bf16x8 aa, b;
            for (int i = 0; i < 8; ++i) {
                aa[i] = t.h1[r][32 * s + 8 * q + i];
                b[i] = W2[(16 * tn + r) * kHid + 32 * s + 8 * q + i];
            }
            acc = mfma32(aa, b, acc);
        }
        const float bias = params[ob2 + 16 * tn + r];
        for (int i = 0; i < 4; ++i) {
            const float hv = acc[i] + bias;
            t.h2[4 * q + i][16 * tn + r] = f2bf(hv > 0.f ? hv : 0.f);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    f32x4 acc{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < 2; ++s) {
        bf16x8 aa, b;
        for (int i = 0; i < 8; ++i) {
            aa[i] = t.h2[r][32 * s + 8 * q + i];
            b[i] = W3p[r * kHid + 32 * s + 8 * q + i];
        }
        acc = mfma32(aa, b, acc);
    }
    if (r == 0)
        for (int i = 0; i < 4; ++i) t.y[4 * q + i] = acc[i] + params[ob3];
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
}

constexpr int kWaves = 4;

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *X, uint32_t n, const float *params,
                                                          const short *copies, float *y) {
    __shared__ TileLds lds[kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    TileLds &t = lds[wave];
    const uint32_t tiles = (n + 15) / 16;
    for (uint32_t tile = blockIdx.x * kWaves + wave; tile < tiles; tile += gridDim.x * kWaves) {
        tile_forward(X, nullptr, tile * 16, n, params, copies, t);
        if (lane < 16 && tile * 16 + lane < n) y[tile * 16 + lane] = t.y[lane];
        __builtin_amdgcn_wave_barrier();
    }
}

// Per-block partial gradient of L = sum over the batch rows of
// (y - target)^2 / batch, for rows ridx[first .. first+count).  Per-wave
// accumulators (MFMA fragments for dW2 and dW1) are summed over the block's
// waves in wave order in LDS and written to part[blockIdx.x][0 .. kParams)
// with the block's loss at index kParams; reduce_kernel sums the blocks in
// block order, so a training run is reproducible bit for bit.
constexpr int kPartStride = kParams + 1;
constexpr int kMaxGradBlocks = 256;

__global__ __launch_bounds__(256) void mlp_backward_kernel(const float *X, const float *target,
                                                           const uint32_t *ridx, uint32_t first,
                                                           uint32_t count, const float *params,
                                                           const short *copies, float *part) {
    __shared__ TileLds lds[kWaves];
    __shared__ short w2t[kHid][kHid + 4];  // W2 in bf16, [o][i]
    __shared__ float bsum[kPartStride];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    for (int e = threadIdx.x; e < kHid * kHid; e += blockDim.x) w2t[e / kHid][e % kHid] = copies[cW2 + e];
    __syncthreads();
    TileLds &t = lds[wave];
    f32x4 gW2[4][4], gW1[4];
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f, gb3 = 0.f, lsum = 0.f;
    const float inv_b = 1.f / (float)count;
    const uint32_t end = first + count;
    const uint32_t tiles = (count + 15) / 16;
    for (uint32_t tile = blockIdx.x * kWaves + wave; tile < tiles; tile += gridDim.x * kWaves) {
        const uint32_t row0 = first + tile * 16;
        tile_forward(X, ridx, row0, end, params, copies, t);
        // dL/dy
        if (lane < 16) {
            const uint32_t row = row0 + lane;
            float d = 0.f;
            if (row < end) {
                const float e = t.y[lane] - target[ridx ? ridx[row] : row];
                d = 2.f * e * inv_b;
                lsum += e * e * inv_b;
            }
            t.dy[lane] = d;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        // output layer: lane = hidden unit k of H2
        for (int rr = 0; rr < 16; ++rr) gW3 += t.dy[rr] * bf2f(t.h2[rr][lane]);
        if (lane == 0)
            for (int rr = 0; rr < 16; ++rr) gb3 += t.dy[rr];
        // dH2 = dy * W3 * relu'(H2), overwriting H2 after its use above
        const float w3 = params[oW3 + lane];
        __builtin_amdgcn_wave_barrier();
        short dh2col[16];
        for (int rr = 0; rr < 16; ++rr) {
            const float g = bf2f(t.h2[rr][lane]) > 0.f ? t.dy[rr] * w3 : 0.f;
            dh2col[rr] = f2bf(g);
            gb2 += g;
        }
        // dW2 += dH2^T H1 (M = output unit o, K = rows, N = input unit i)
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int rr = 0; rr < 16; ++rr) t.h2[rr][lane] = dh2col[rr];
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int tm = 0; tm < 4; ++tm) {
            bf16x4 a;
            for (int i = 0; i < 4; ++i) a[i] = t.h2[4 * q + i][16 * tm + r];  // A[o][row]
            for (int tn = 0; tn < 4; ++tn) {
                bf16x4 b;
                for (int i = 0; i < 4; ++i) b[i] = t.h1[4 * q + i][16 * tn + r];  // B[row][i]
                gW2[tm][tn] = mfma(a, b, gW2[tm][tn]);
            }
        }
        // dH1 = dH2 W2 * relu'(H1) (M = rows, K = o, N = i)
        short dh1v[4][4];
        for (int tn = 0; tn < 4; ++tn) {
            f32x4 acc{0.f, 0.f, 0.f, 0.f};
            for (int s = 0; s < 2; ++s) {
                bf16x8 a, b;
                for (int i = 0; i < 8; ++i) {
                    a[i] = t.h2[r][32 * s + 8 * q + i];        // A[row][o] = dH2
                    b[i] = w2t[32 * s + 8 * q + i][16 * tn + r];  // B[o][i] = W2[o][i]
                }
                acc = mfma32(a, b, acc);
            }
            for (int i = 0; i < 4; ++i) {
                const float h = bf2f(t.h1[4 * q + i][16 * tn + r]);
                dh1v[tn][i] = f2bf(h > 0.f ? acc[i] : 0.f);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int tn = 0; tn < 4; ++tn)
            for (int i = 0; i < 4; ++i) t.h1[4 * q + i][16 * tn + r] = dh1v[tn][i];  // h1 now holds dH1
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int rr = 0; rr < 16; ++rr) gb1 += bf2f(t.h1[rr][lane]);
        // dW1 += dH1^T X (M = hidden unit, K = rows, N = feature)
        bf16x4 bx;
        for (int i = 0; i < 4; ++i) bx[i] = t.x[4 * q + i][r];
        for (int tm = 0; tm < 4; ++tm) {
            bf16x4 a;
            for (int i = 0; i < 4; ++i) a[i] = t.h1[4 * q + i][16 * tm + r];
            gW1[tm] = mfma(a, bx, gW1[tm]);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    // block sum in wave order; D layout d[i] = G[16 tm + 4q + i][16 tn + r]
    for (int w = 0; w < kWaves; ++w) {
        __syncthreads();
        if (wave != w) continue;
        const bool set = w == 0;
        auto put = [&](int idx, float v) { bsum[idx] = set ? v : bsum[idx] + v; };
        for (int tm = 0; tm < 4; ++tm) {
            for (int tn = 0; tn < 4; ++tn)
                for (int i = 0; i < 4; ++i) put(oW2 + (16 * tm + 4 * q + i) * kHid + 16 * tn + r, gW2[tm][tn][i]);
            if (r < kIn)
                for (int i = 0; i < 4; ++i) put(oW1 + (16 * tm + 4 * q + i) * kIn + r, gW1[tm][i]);
        }
        put(ob1 + lane, gb1);
        put(ob2 + lane, gb2);
        put(oW3 + lane, gW3);
        if (lane == 0) {
            put(ob3, gb3);
            put(kParams, lsum);
        }
    }
    __syncthreads();
    float *out = part + (size_t)blockIdx.x * kPartStride;
    for (int i = threadIdx.x; i < kPartStride; i += blockDim.x) out[i] = bsum[i];
}

// grad[i] = sum over blocks b (in order) of part[b][i]; the loss entry is
// added to *loss when accumulate is set, else stored.
__global__ void reduce_kernel(const float *part, int nblocks, float *grad, float *loss, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kPartStride) return;
    float acc = 0.f;
    for (int b = 0; b < nblocks; ++b) acc += part[(size_t)b * kPartStride + i];
    if (i < kParams)
        grad[i] = acc;
    else
        *loss = accumulate ? *loss + acc : acc;
}

// Adam on the fp32 parameters, then refresh the bf16 copies and zero the
// gradient for the next step.
__global__ void adam_kernel(float *params, float *grad, float *m, float *v, short *copies, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) {
        const float g = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        grad[i] = 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCopies; e += blockDim.x) {
        float w = 0.f;
        if (e < cW2) {
            const int o = e / 16, k = e % 16;
            w = k < kIn ? params[oW1 + o * kIn + k] : 0.f;
        } else if (e < cW3) {
            w = params[oW2 + (e - cW2)];
        } else {
            const int rr = (e - cW3) / kHid, k = (e - cW3) % kHid;
            w = rr == 0 ? params[oW3 + k] : 0.f;
        }
        copies[e] = f2bf(w);
    }
}

__global__ void zero_f32_kernel(float *p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0.f;
}

}  // namespace
}  // namespace khc

struct khc_mlp {
    khc_ctx *ctx = nullptr;
    float *params = nullptr;  // fp32 [4801]
    float *grad = nullptr;
    float *m = nullptr, *v = nullptr;
    short *copies = nullptr;  // bf16
    float *loss = nullptr;
    float *part = nullptr;  // per-block partial gradients [kMaxGradBlocks][kPartStride]
    uint32_t *perm = nullptr;
    size_t perm_len = 0;
    uint64_t step = 0;
};

using namespace khc;

namespace {

int mlp_refresh_copies(khc_ctx *ctx, khc_mlp *m) {
    // an Adam step with lr 0 and zero gradient only rewrites the copies
    hipLaunchKernelGGL(zero_f32_kernel, dim3(1), dim3(256), 0, ctx->stream, m->grad, kParams);
    hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(256), 0, ctx->stream, m->params, m->grad, m->m, m->v,
                       m->copies, 0.f, 1.f, 1.f, 1.f, 1.f, 1.f);
    return check_hip(ctx, hipGetLastError(), "mlp copies");
}

}  // namespace

extern "C" {

int khc_mlp_create(khc_ctx *ctx, uint64_t seed, khc_mlp **out) {
    if (!ctx) return KHC_EINVAL;
    if (!out) return set_error(ctx, KHC_EINVAL, "out is null");
    (void)hipSetDevice(ctx->device);
    khc_mlp *m = new khc_mlp();
    m->ctx = ctx;
    const size_t fb = kParams * sizeof(float);
    if (hipMalloc(&m->params, fb) != hipSuccess || hipMalloc(&m->grad, fb) != hipSuccess ||
        hipMalloc(&m->m, fb) != hipSuccess || hipMalloc(&m->v, fb) != hipSuccess ||
        hipMalloc(&m->copies, kCopies * sizeof(short)) != hipSuccess || hipMalloc(&m->loss, 64) != hipSuccess ||
        hipMalloc(&m->part, (size_t)kMaxGradBlocks * kPartStride * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        khc_mlp_destroy(m);
        return set_error(ctx, KHC_ENOMEM, "mlp allocation failed");
    }
    // He-uniform initial weights (fan-in), zero biases, from the seed
    std::vector<float> p(kParams, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int count, int fan_in) {
        const float lim = std::sqrt(6.f / (float)fan_in);
        std::uniform_real_distribution<float> u(-lim, lim);
        for (int i = 0; i < count; ++i) p[off + i] = u(rng);
    };
    fill(oW1, kHid * kIn, kIn);
    fill(oW2, kHid * kHid, kHid);
    fill(oW3, kHid, kHid);
    int rc = khc_mlp_set_params(ctx, m, p.data());
    if (rc) {
        khc_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return KHC_OK;
}

int khc_mlp_destroy(khc_mlp *m) {
    if (!m) return KHC_EINVAL;
    if (m->ctx) (void)hipStreamSynchronize(m->ctx->stream);
    for (void *p : {(void *)m->params, (void *)m->grad, (void *)m->m, (void *)m->v, (void *)m->copies,
                    (void *)m->loss, (void *)m->part, (void *)m->perm})
        if (p) (void)hipFree(p);
    delete m;
    return KHC_OK;
}

int khc_mlp_set_params(khc_ctx *ctx, khc_mlp *m, const float *host_params) {
    if (!ctx) return KHC_EINVAL;
    if (!m || !host_params) return set_error(ctx, KHC_EINVAL, "null argument");
    hipStream_t st = ctx->stream;
    hipError_t e = hipMemcpyAsync(m->params, host_params, kParams * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, kParams * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, kParams * sizeof(float), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "mlp parameter upload");
    m->step = 0;
    return mlp_refresh_copies(ctx, m);
}

int khc_mlp_get_params(khc_ctx *ctx, const khc_mlp *m, float *host_params, float *host_grad) {
    if (!ctx) return KHC_EINVAL;
    if (!m) return set_error(ctx, KHC_EINVAL, "null argument");
    hipStream_t st = ctx->stream;
    hipError_t e = hipSuccess;
    if (host_params) e = hipMemcpyAsync(host_params, m->params, kParams * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && host_grad)
        e = hipMemcpyAsync(host_grad, m->grad, kParams * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "mlp parameter download");
    return KHC_OK;
}

int khc_mlp_get_moments(khc_ctx *ctx, const khc_mlp *m, float *host_m, float *host_v, uint64_t *host_step) {
    if (!ctx) return KHC_EINVAL;
    if (!m) return set_error(ctx, KHC_EINVAL, "null argument");
    hipStream_t st = ctx->stream;
    hipError_t e = hipSuccess;
    if (host_m) e = hipMemcpyAsync(host_m, m->m, kParams * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && host_v) e = hipMemcpyAsync(host_v, m->v, kParams * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "mlp moment download");
    if (host_step) *host_step = m->step;
    return KHC_OK;
}

int khc_mlp_save(khc_ctx *ctx, const khc_mlp *m, const char *path) {
    if (!ctx) return KHC_EINVAL;
    if (!m || !path) return set_error(ctx, KHC_EINVAL, "null argument");
    std::vector<float> p(kParams);
    int rc = khc_mlp_get_params(ctx, m, p.data(), nullptr);
    if (rc) return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_error(ctx, KHC_EINVAL, std::string("cannot open ") + path + " for writing");
    const uint32_t count = kParams;
    const bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(&count, 4, 1, f) == 1 &&
                    std::fwrite(p.data(), 4, kParams, f) == (size_t)kParams;
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) return set_error(ctx, KHC_EINVAL, std::string("write to ") + path + " failed");
    return KHC_OK;
}

int khc_mlp_load(khc_ctx *ctx, khc_mlp *m, const char *path) {
    if (!ctx) return KHC_EINVAL;
    if (!m || !path) return set_error(ctx, KHC_EINVAL, "null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_error(ctx, KHC_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    uint32_t count = 0;
    std::vector<float> p(kParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
              std::fread(&count, 4, 1, f) == 1 && count == (uint32_t)kParams &&
              std::fread(p.data(), 4, kParams, f) == (size_t)kParams;
    char extra;
    if (ok && std::fread(&extra, 1, 1, f) != 0) ok = false;  // trailing bytes
    std::fclose(f);
    if (!ok) return set_error(ctx, KHC_EINVAL, std::string(path) + " is not a saved network of this shape");
    return khc_mlp_set_params(ctx, m, p.data());
}

int khc_mlp_forward(khc_ctx *ctx, const khc_mlp *m, const float *X, uint32_t n, float *y) {
    if (!ctx) return KHC_EINVAL;
    if (!m || (n && (!X || !y))) return set_error(ctx, KHC_EINVAL, "null argument");
    if (!n) return KHC_OK;
    const uint32_t tiles = (n + 15) / 16;
    uint32_t grid = (tiles + kWaves - 1) / kWaves;
    if (grid > (uint32_t)ctx->num_cu * 8) grid = ctx->num_cu * 8;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, ctx->stream, X, n, m->params, m->copies, y);
    return check_hip(ctx, hipGetLastError(), "mlp forward");
}

int khc_mlp_gradient(khc_ctx *ctx, khc_mlp *m, const float *X, const float *target, uint32_t n,
                     float *host_loss) {
    if (!ctx) return KHC_EINVAL;
    if (!m || !n || !X || !target) return set_error(ctx, KHC_EINVAL, "null argument or empty batch");
    hipStream_t st = ctx->stream;
    const uint32_t tiles = (n + 15) / 16;
    uint32_t grid = (tiles + kWaves - 1) / kWaves;
    if (grid > (uint32_t)kMaxGradBlocks) grid = kMaxGradBlocks;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(grid), dim3(256), 0, st, X, target, (const uint32_t *)nullptr,
                       0u, n, m->params, m->copies, m->part);
    hipLaunchKernelGGL(reduce_kernel, dim3((kPartStride + 255) / 256), dim3(256), 0, st, (const float *)m->part,
                       (int)grid, m->grad, m->loss, 0);
    float l = 0.f;
    hipError_t e = hipMemcpyAsync(&l, m->loss, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "mlp gradient");
    if (host_loss) *host_loss = l;
    return KHC_OK;
}

int khc_mlp_train(khc_ctx *ctx, khc_mlp *m, const float *X, const float *target, uint32_t n, uint32_t epochs,
                  uint32_t batch, float lr, uint64_t seed, float *host_epoch_loss) {
    if (!ctx) return KHC_EINVAL;
    if (!m || !n || !X || !target || !batch || !epochs) return set_error(ctx, KHC_EINVAL, "bad training arguments");
    hipStream_t st = ctx->stream;
    if (m->perm_len < n) {
        if (m->perm) (void)hipFree(m->perm);
        m->perm = nullptr;
        if (hipMalloc(&m->perm, (size_t)n * 4) != hipSuccess) {
            (void)hipGetLastError();
            m->perm_len = 0;
            return set_error(ctx, KHC_ENOMEM, "mlp permutation allocation failed");
        }
        m->perm_len = n;
    }
    std::vector<uint32_t> perm(n);
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (uint32_t ep = 0; ep < epochs; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        hipError_t e = hipMemcpyAsync(m->perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // perm is reused next epoch
        if (e != hipSuccess) return check_hip(ctx, e, "permutation upload");
        hipLaunchKernelGGL(zero_f32_kernel, dim3(1), dim3(64), 0, st, m->loss, 1);
        uint32_t steps = 0;
        for (uint32_t first = 0; first < n; first += batch) {
            const uint32_t cnt = n - first < batch ? n - first : batch;
            const uint32_t tiles = (cnt + 15) / 16;
            uint32_t grid = (tiles + kWaves - 1) / kWaves;
            if (grid > 64) grid = 64;
            hipLaunchKernelGGL(mlp_backward_kernel, dim3(grid), dim3(256), 0, st, X, target,
                               (const uint32_t *)m->perm, first, cnt, m->params, m->copies, m->part);
            hipLaunchKernelGGL(reduce_kernel, dim3((kPartStride + 255) / 256), dim3(256), 0, st,
                               (const float *)m->part, (int)grid, m->grad, m->loss, 1);
            m->step++;
            const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
            hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(256), 0, st, m->params, m->grad, m->m, m->v, m->copies,
                               lr, b1, b2, eps, c1, c2);
            steps++;
        }
        float l = 0.f;
        e = hipMemcpyAsync(&l, m->loss, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "training epoch");
        if (host_epoch_loss) host_epoch_loss[ep] = l / (float)steps;
    }
    return check_hip(ctx, hipGetLastError(), "mlp training");
}

}  // extern "C"

namespace khc {
float *mlp_params(khc_mlp *m) { return m->params; }
const short *mlp_copies(const khc_mlp *m) { return m->copies; }
}  // namespace khc
