// rsv_mlp.hip -- the learned diagonal-mass network on gfx950 matrix cores.
//
// 27 -> 64 -> 64 -> 1 perceptron with GELU, bfloat16 operands and FP32
// accumulation (v_mfma_f32_16x16x32_bf16 for the layer products,
// v_mfma_f32_16x16x16_bf16 for the weight gradients, whose reduction
// dimension is a wavefront's 16 rows).  A 256-thread block takes 64 rows,
// 16 per wavefront.  Operand layouts (lane l, q = l/16, r = l%16):
//   16x16x32: A[r][8q+i], B[8q+i][r] (i < 8), D[4q+j][r] (j < 4);
//   16x16x16: A[r][4q+i], B[4q+i][r] (i < 4), D[4q+j][r].
// The D layout of one layer's output is the A layout of X^T-style products
// (weight gradients), so those need no transposition; the products that need
// a row-major A operand go through a per-wavefront LDS buffer.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rsv_internal.h"
#include "rsv_mlp.h"

namespace rsv {
namespace {

constexpr int kIn = RSV_MLP_INPUTS, kInPad = RSV_MLP_INPUTS_PAD, kHid = RSV_MLP_HIDDEN;
constexpr int kParams = RSV_MLP_PARAMS;
constexpr int oW1 = 0, oB1 = kInPad * kHid, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kHid;
static_assert(oB3 + 1 == kParams, "parameter layout");
constexpr int kRows = 64;            // rows per block (per chunk, for inference)
constexpr int64_t kForwardBlocks = 1024;  // inference grid: 4 blocks per compute unit
constexpr int kPartial = kParams + 1;  // gradient + loss per block
constexpr int kWindow = 5;
constexpr double kY2Floor = 1e-8;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ inline uint16_t to_bf16(float f) {  // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ inline float from_bf16(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

// erf in FP32 without branches: Hastings' rational approximation
// (Abramowitz and Stegun, Handbook of Mathematical Functions, 7.1.26),
// erf(z) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) e^{-z^2},
// t = 1 / (1 + p z) for z >= 0, odd in z; absolute error <= 1.5e-7, far
// below the bfloat16 rounding the activations receive.  A library erff
// branches on the argument's range, and the lanes of a wavefront take every
// branch.
__device__ inline float erf_fast(float x) {
    const float z = __builtin_fabsf(x);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, z, 1.0f));
    float q = 1.061405429f;
    q = __builtin_fmaf(q, t, -1.453152027f);
    q = __builtin_fmaf(q, t, 1.421413741f);
    q = __builtin_fmaf(q, t, -0.284496736f);
    q = __builtin_fmaf(q, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-z * z * 1.4426950408889634f);
    const float r = __builtin_fmaf(-q * t, e, 1.0f);
    return __builtin_copysignf(r, x);
}
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erf_fast(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
    return 0.5f * (1.0f + erf_fast(x * 0.70710678118654752f)) +
           x * __builtin_amdgcn_exp2f(-0.5f * x * x * 1.4426950408889634f) * 0.39894228040143268f;
}

__device__ inline bf16x8 load8(const uint16_t* p) {  // 16-byte aligned
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ inline s16x4 pack4(const uint16_t v[4]) {
    s16x4 r;
    r[0] = static_cast<short>(v[0]);
    r[1] = static_cast<short>(v[1]);
    r[2] = static_cast<short>(v[2]);
    r[3] = static_cast<short>(v[3]);
    return r;
}

struct MlpWeights {
    uint16_t w1t[kHid][kInPad];        // w1t[j][k] = W1[k][j]
    uint16_t w2t[kHid][kHid];          // w2t[j][k] = W2[k][j]
    uint16_t w2r[kHid][kHid];          // W2 row-major (back-propagation)
    float b1[kHid], b2[kHid], w3[kHid];
    float b3;
    uint16_t tb[4][16][kHid + 8];      // per-wavefront transposition buffer
};

__device__ void load_weights(MlpWeights& W, const float* P, bool need_rowmajor) {
    for (int i = threadIdx.x; i < kInPad * kHid; i += blockDim.x) {
        const int k = i / kHid, j = i % kHid;
        W.w1t[j][k] = to_bf16(P[oW1 + i]);
    }
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) {
        const int k = i / kHid, j = i % kHid;
        const uint16_t v = to_bf16(P[oW2 + i]);
        W.w2t[j][k] = v;
        if (need_rowmajor) W.w2r[k][j] = v;
    }
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        W.b1[i] = P[oB1 + i];
        W.b2[i] = P[oB2 + i];
        W.w3[i] = from_bf16(to_bf16(P[oW3 + i]));
    }
    if (threadIdx.x == 0) W.b3 = P[oB3];
}

// Forward (TRAIN = false: write outputs) or forward + backward (TRAIN:
// write this block's gradient and loss partial sums).
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp(int64_t n, const uint16_t* __restrict__ X,
                                             const float* __restrict__ target,
                                             const int32_t* __restrict__ rows,
                                             const float* __restrict__ P, float* out, int clip,
                                             float* partial) {
    __shared__ MlpWeights W;
    __shared__ float red[TRAIN ? 4 : 1][TRAIN ? kPartial : 1];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, q = l >> 4, r = l & 15;
    load_weights(W, P, TRAIN);
    __syncthreads();

    auto src_row = [&](int64_t i) -> int64_t { return rows ? static_cast<int64_t>(rows[i]) : i; };
    float pre1[4][4], pre2[4][4];
    uint16_t h1b[4][4];
    float h2f[4][4];
    float o[4];
    // the forward pass of the 16 rows from row0 of this wavefront (the block's
    // 64 rows from the chunk's first row)
    auto forward = [&](const int64_t row0) {
        // ---- layer 1: [16 x 32] x [32 x 64] ----
        bf16x8 a1;
        {
            const int64_t ri = row0 + r;
            if (ri < n) {
                a1 = load8(X + src_row(ri) * kInPad + 8 * q);
            } else {
                const uint4 z = {0u, 0u, 0u, 0u};
                a1 = __builtin_bit_cast(bf16x8, z);
            }
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a1, load8(&W.w1t[16 * nt + r][8 * q]), zero, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                pre1[nt][j] = d[j] + W.b1[16 * nt + r];
                h1b[nt][j] = to_bf16(gelu(pre1[nt][j]));
                W.tb[wv][4 * q + j][16 * nt + r] = h1b[nt][j];
            }
        }
        __syncthreads();

        // ---- layer 2: [16 x 64] x [64 x 64] ----
        const bf16x8 a2_0 = load8(&W.tb[wv][r][8 * q]);
        const bf16x8 a2_1 = load8(&W.tb[wv][r][32 + 8 * q]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a2_0, load8(&W.w2t[16 * nt + r][8 * q]), zero, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a2_1, load8(&W.w2t[16 * nt + r][32 + 8 * q]), d, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                pre2[nt][j] = d[j] + W.b2[16 * nt + r];
                h2f[nt][j] = from_bf16(to_bf16(gelu(pre2[nt][j])));
            }
        }

        // ---- layer 3: dot with w3 over the 64 columns (16 lanes x 4 tiles) ----
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float s = 0.f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) s += h2f[nt][j] * W.w3[16 * nt + r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
            o[j] = s + W.b3;
        }
    };
    if constexpr (!TRAIN) {
        // inference: each block stages the weights once and takes chunks of
        // kRows rows with a stride of the grid
        const int64_t n_chunks = (n + kRows - 1) / kRows;
        for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
            const int64_t row0 = chunk * kRows + wv * 16;
            forward(row0);
            if (r == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t ri = row0 + 4 * q + j;
                    // a non-finite output is passed on as it is, for the caller's fallback
                    if (ri < n)
                        out[ri] = clip && isfinite(o[j]) ? fminf(fmaxf(o[j], -5.0f), 5.0f) : o[j];
                }
            }
        }
        return;
    } else {
        const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows + wv * 16;
        forward(row0);
        // ---- d loss / d out for the four rows this lane's group holds ----
        const float inv_n = 1.0f / static_cast<float>(n);
        float dout[4], sq = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t ri = row0 + 4 * q + j;
            if (ri < n) {
                const float e = o[j] - target[src_row(ri)];
                dout[j] = 2.0f * e * inv_n;
                sq += e * e;
            } else {
                dout[j] = 0.f;
            }
        }
        // per-column sums over the wavefront's 16 rows: 4 rows in-lane, then
        // across the four row groups
        auto colsum = [&](float v) {
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            return v;
        };

        float dpre2[4][4];
        uint16_t dpre2b[4][4];
        float db2[4], dw3[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            float sb = 0.f, sw = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dpre2[nt][j] = dout[j] * W.w3[16 * nt + r] * gelu_grad(pre2[nt][j]);
                dpre2b[nt][j] = to_bf16(dpre2[nt][j]);
                sb += dpre2[nt][j];
                sw += dout[j] * h2f[nt][j];
            }
            db2[nt] = colsum(sb);
            dw3[nt] = colsum(sw);
        }
        float db3 = dout[0] + dout[1] + dout[2] + dout[3];
        db3 = colsum(db3);
        sq = colsum(sq);

        // dW2 = H1^T dPre2 over this wavefront's rows (K = 16)
        f32x4 gW2[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                gW2[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pack4(h1b[mt]),
                                                                        pack4(dpre2b[nt]), zero,
                                                                        0, 0, 0);
            }

        // dH1 = dPre2 W2^T: dPre2 to row-major through LDS
        __syncthreads();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) W.tb[wv][4 * q + j][16 * nt + r] = dpre2b[nt][j];
        __syncthreads();
        const bf16x8 a3_0 = load8(&W.tb[wv][r][8 * q]);
        const bf16x8 a3_1 = load8(&W.tb[wv][r][32 + 8 * q]);
        uint16_t dpre1b[4][4];
        float db1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a3_0, load8(&W.w2r[16 * nt + r][8 * q]), zero, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a3_1, load8(&W.w2r[16 * nt + r][32 + 8 * q]), d, 0, 0, 0);
            float sb = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float dp = d[j] * gelu_grad(pre1[nt][j]);
                dpre1b[nt][j] = to_bf16(dp);
                sb += dp;
            }
            db1[nt] = colsum(sb);
        }

        // dW1 = X^T dPre1 (K = 16 rows): A[i][k] = X[row 4q+k][16 mt + i]
        f32x4 gW1[2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            uint16_t xa[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t ri = row0 + 4 * q + j;
                xa[j] = ri < n ? X[src_row(ri) * kInPad + 16 * mt + r] : uint16_t(0);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                gW1[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pack4(xa), pack4(dpre1b[nt]),
                                                                        zero, 0, 0, 0);
            }
        }

        // ---- stage the wavefront's partials, then add the four in order ----
        float* R = red[wv];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    R[oW1 + (16 * mt + 4 * q + j) * kHid + 16 * nt + r] = gW1[mt][nt][j];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    R[oW2 + (16 * mt + 4 * q + j) * kHid + 16 * nt + r] = gW2[mt][nt][j];
        if (q == 0) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                R[oB1 + 16 * nt + r] = db1[nt];
                R[oB2 + 16 * nt + r] = db2[nt];
                R[oW3 + 16 * nt + r] = dw3[nt];
            }
        }
        if (l == 0) {
            R[oB3] = db3;
            R[kParams] = sq;
        }
        __syncthreads();
        float* dst = partial + static_cast<int64_t>(blockIdx.x) * kPartial;
        for (int i = tid; i < kPartial; i += blockDim.x)
            dst[i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
    }
}

// Sum of the block partials in block order; the loss slot divided by n.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* partial, int32_t n_blocks,
                                                    int64_t n, float* grad, double* loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kParams) return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += static_cast<double>(partial[static_cast<int64_t>(b) * kPartial + i]);
    if (i < kParams) grad[i] = static_cast<float>(s);
    else if (loss) *loss = s / static_cast<double>(n);
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* P, float* m, float* v, const float* g,
                                                  int32_t step, float lr, float b1, float b2,
                                                  float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, static_cast<float>(step)));
    const float vh = vi / (1.0f - powf(b2, static_cast<float>(step)));
    P[i] -= lr * mh / (sqrtf(vh) + eps);
}

// One thread per site: the 27 standardised inputs (FP64, rounded to FP32
// then to bfloat16) and five zero padding columns.
__global__ __launch_bounds__(256) void k_mlp_features(const int64_t* offsets, const double* y,
                                                      const double* log_rv,
                                                      const rsv_theta* theta, const double* mean,
                                                      const double* stdv, uint16_t* X) {
    const int s = blockIdx.y;
    const int64_t base = offsets[s];
    const int64_t T = offsets[s + 1] - base;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const rsv_theta th = theta[s];
    uint16_t v[kInPad];
#pragma unroll
    for (int d = -kWindow; d <= kWindow; ++d) {
        int64_t j = t + d;
        j = j < 0 ? 0 : (j > T - 1 ? T - 1 : j);
        const double yy = y[base + j];
        const int c = d + kWindow;
        v[c] = to_bf16(static_cast<float>((log(yy * yy + kY2Floor) - mean[c]) / stdv[c]));
        v[11 + c] = to_bf16(static_cast<float>((log_rv[base + j] - mean[11 + c]) / stdv[11 + c]));
    }
    const double tv[5] = {th.phi, th.mu, th.xi, th.sig2_eta, th.sig2_u};
#pragma unroll
    for (int i = 0; i < 5; ++i) v[22 + i] = to_bf16(static_cast<float>((tv[i] - mean[22 + i]) / stdv[22 + i]));
#pragma unroll
    for (int i = kIn; i < kInPad; ++i) v[i] = 0;
    uint4* dst = reinterpret_cast<uint4*>(X + (base + t) * kInPad);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint4 u;
        u.x = v[8 * w + 0] | (static_cast<uint32_t>(v[8 * w + 1]) << 16);
        u.y = v[8 * w + 2] | (static_cast<uint32_t>(v[8 * w + 3]) << 16);
        u.z = v[8 * w + 4] | (static_cast<uint32_t>(v[8 * w + 5]) << 16);
        u.w = v[8 * w + 6] | (static_cast<uint32_t>(v[8 * w + 7]) << 16);
        dst[w] = u;
    }
}

int64_t n_blocks(int64_t n) { return (n + kRows - 1) / kRows; }

#define MLP_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return set_error(RSV_EDEVICE, #call, hipGetErrorString(e_)); \
    } while (0)

}  // namespace
}  // namespace rsv

using namespace rsv;

extern "C" {

rsv_status rsv_mlp_features(int32_t n_series, const int64_t* offsets, const double* y,
                            const double* log_rv, const rsv_theta* theta, const double* mean,
                            const double* stdv, int64_t max_T, uint16_t* x, void* hip_stream) {
    if (n_series < 1 || n_series > 65535 || max_T < 1)
        return set_error(RSV_EINVAL, "rsv_mlp_features", "need 1 <= n_series <= 65535 and max_T >= 1");
    if (!offsets || !y || !log_rv || !theta || !mean || !stdv || !x)
        return set_error(RSV_EINVAL, "rsv_mlp_features", "NULL pointer");
    if (reinterpret_cast<uintptr_t>(x) % 16)
        return set_error(RSV_EINVAL, "rsv_mlp_features", "x must be 16-byte aligned");
    const dim3 g(static_cast<unsigned>((max_T + 255) / 256), n_series), b(256);
    hipLaunchKernelGGL(k_mlp_features, g, b, 0, static_cast<hipStream_t>(hip_stream), offsets, y,
                       log_rv, theta, mean, stdv, x);
    MLP_HIP(hipGetLastError());
    return RSV_OK;
}

rsv_status rsv_mlp_forward(int64_t n, const uint16_t* x, const float* params, float* out,
                           int32_t clip, void* hip_stream) {
    if (n < 1 || !x || !params || !out)
        return set_error(RSV_EINVAL, "rsv_mlp_forward", "need n >= 1 and non-NULL pointers");
    if (reinterpret_cast<uintptr_t>(x) % 16)
        return set_error(RSV_EINVAL, "rsv_mlp_forward", "x must be 16-byte aligned");
    // a few blocks per compute unit, each looping over its chunks of rows
    const int64_t grid = n_blocks(n) < kForwardBlocks ? n_blocks(n) : kForwardBlocks;
    hipLaunchKernelGGL(k_mlp<false>, dim3(static_cast<unsigned>(grid)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), n, x, nullptr, nullptr, params, out,
                       clip, nullptr);
    MLP_HIP(hipGetLastError());
    return RSV_OK;
}

size_t rsv_mlp_grad_workspace_bytes(int64_t n) {
    if (n < 1) return 0;
    return static_cast<size_t>(n_blocks(n)) * kPartial * sizeof(float);
}

rsv_status rsv_mlp_grad(int64_t n, const uint16_t* x, const float* target, const int32_t* rows,
                        const float* params, float* grad, double* loss, void* workspace,
                        size_t ws_bytes, void* hip_stream) {
    if (n < 1 || !x || !target || !params || !grad || !workspace)
        return set_error(RSV_EINVAL, "rsv_mlp_grad", "need n >= 1 and non-NULL pointers");
    if (n_blocks(n) > (int64_t(1) << 30))
        return set_error(RSV_EINVAL, "rsv_mlp_grad", "too many rows");
    if (ws_bytes < rsv_mlp_grad_workspace_bytes(n))
        return set_error(RSV_ENOMEM, "rsv_mlp_grad", "workspace too small");
    if (reinterpret_cast<uintptr_t>(x) % 16)
        return set_error(RSV_EINVAL, "rsv_mlp_grad", "x must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    float* partial = static_cast<float*>(workspace);
    const int64_t nb = n_blocks(n);
    hipLaunchKernelGGL(k_mlp<true>, dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, n, x,
                       target, rows, params, nullptr, 0, partial);
    MLP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartial + 255) / 256), dim3(256), 0, st, partial,
                       static_cast<int32_t>(nb), n, grad, loss);
    MLP_HIP(hipGetLastError());
    return RSV_OK;
}

rsv_status rsv_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                        float lr, float beta1, float beta2, float eps, void* hip_stream) {
    if (!params || !m || !v || !grad || step < 1)
        return set_error(RSV_EINVAL, "rsv_mlp_adam", "need non-NULL pointers and step >= 1");
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), params, m, v, grad, step, lr, beta1,
                       beta2, eps);
    MLP_HIP(hipGetLastError());
    return RSV_OK;
}

}  // extern "C"
