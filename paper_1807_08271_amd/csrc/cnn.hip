// Learned warm start: a small convolutional network that predicts the initial
// twist of an alignment from the 80 x 60 pyramid level of both frames.  It is
// an addition to the method (the paper starts from the identity or a
// constant-velocity guess, sec. 6.2 / 7.1); Gauss-Newton always runs after it.
//
// Network: 4 x [3x3 conv, stride 2, zero pad 1, bias, ReLU] with channels
// 4 -> 32 -> 64 -> 128 -> 128 on 60x80 -> 30x40 -> 15x20 -> 8x10 -> 4x5,
// global average pool, fully connected 128 -> 6.  Convolution and FC weights
// are used in bfloat16 (rounded from an FP32 master copy); activations,
// accumulation, gradients and the AdamW state are FP32.  Every reduction has
// a fixed order, so training is deterministic.
#include "rgbid_internal.h"

namespace rgbid {
namespace {

__device__ __forceinline__ float bf(const __hip_bfloat16 x) { return __bfloat162float(x); }

// ------------------------------------------------------------------ input

// x[n, 0..3, y, x] = (I_A / 255, W_A / 2, I_B / 255, W_B / 2) at the 80x60
// level of pair n (holes read as 0).
__global__ void __launch_bounds__(256) k_input(const CnnInput* __restrict__ in, int n, float* x)
{
    const int p = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || i >= kCnnH * kCnnW) return;
    const CnnInput& c = in[p];
    float2 a, b;
    if (c.f16) {
        a = __half22float2(static_cast<const __half2*>(c.A)[i]);
        b = __half22float2(static_cast<const __half2*>(c.B)[i]);
    } else {
        a = static_cast<const float2*>(c.A)[i];
        b = static_cast<const float2*>(c.B)[i];
    }
    float* xp = x + (size_t)p * 4 * kCnnH * kCnnW + i;
    xp[0] = a.x * (1.0f / 255.0f);
    xp[kCnnH * kCnnW] = a.y * 0.5f;
    xp[2 * kCnnH * kCnnW] = b.x * (1.0f / 255.0f);
    xp[3 * kCnnH * kCnnW] = b.y * 0.5f;
}

// ------------------------------------------------------------------ conv forward

// One thread per (n, co-group of CO_T channels, y, x); writes max(z, 0).
template <int CO_T>
__global__ void __launch_bounds__(256) k_conv_fwd(const float* __restrict__ x,
                                                  const __hip_bfloat16* __restrict__ w,
                                                  const float* __restrict__ b, float* __restrict__ a,
                                                  int N, int Ci, int Hi, int Wi, int Co, int Ho, int Wo)
{
    const int total = N * (Co / CO_T) * Ho * Wo;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int xo = t % Wo;
    const int yo = (t / Wo) % Ho;
    const int cg = (t / (Wo * Ho)) % (Co / CO_T);
    const int n = t / (Wo * Ho * (Co / CO_T));
    float acc[CO_T];
#pragma unroll
    for (int k = 0; k < CO_T; ++k) acc[k] = b[cg * CO_T + k];
    const float* xn = x + (size_t)n * Ci * Hi * Wi;
    for (int ci = 0; ci < Ci; ++ci) {
        const float* xc = xn + (size_t)ci * Hi * Wi;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int iy = 2 * yo - 1 + ky;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int ix = 2 * xo - 1 + kx;
                const bool in = iy >= 0 && iy < Hi && ix >= 0 && ix < Wi;
                const float v = in ? xc[iy * Wi + ix] : 0.0f;
#pragma unroll
                for (int k = 0; k < CO_T; ++k)
                    acc[k] = fmaf(bf(w[(((size_t)(cg * CO_T + k) * Ci + ci) * 3 + ky) * 3 + kx]), v,
                                  acc[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < CO_T; ++k)
        a[(((size_t)n * Co + cg * CO_T + k) * Ho + yo) * Wo + xo] = fmaxf(acc[k], 0.0f);
}

// ------------------------------------------------------------------ pool + FC

// out[n, k] = b[k] + sum_c W[k, c] mean_{y,x} a[n, c, y, x]; one block per n.
__global__ void __launch_bounds__(128) k_pool_fc(const float* __restrict__ a4,
                                                 const __hip_bfloat16* __restrict__ wfc,
                                                 const float* __restrict__ bfc, float* pooled,
                                                 float* out, int C, int HW)
{
    __shared__ float p[128];
    const int n = blockIdx.x, c = threadIdx.x;
    if (c < C) {
        const float* src = a4 + ((size_t)n * C + c) * HW;
        float s = 0.0f;
        for (int i = 0; i < HW; ++i) s += src[i];
        p[c] = s / (float)HW;
        pooled[(size_t)n * C + c] = p[c];
    }
    __syncthreads();
    if (c < 6) {
        float s = bfc[c];
        for (int j = 0; j < C; ++j) s = fmaf(bf(wfc[c * C + j]), p[j], s);
        out[(size_t)n * 6 + c] = s;
    }
}

// dout[n, k] = 2 (out - xi / SCALE) / N and the per-sample loss.
__global__ void k_loss(const float* __restrict__ out, const float* __restrict__ target, int N,
                       float* dout, float* loss_n)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float l = 0.0f;
    for (int k = 0; k < 6; ++k) {
        const float d = out[n * 6 + k] - target[n * 6 + k];
        dout[n * 6 + k] = 2.0f * d / (float)N;
        l = fmaf(d, d, l);
    }
    loss_n[n] = l;
}

// FC gradients: dW[k, c] = sum_n dout[n,k] pooled[n,c] and db[k] (fixed n
// order), then da4[n,c,y,x] = (sum_k dout[n,k] W[k,c]) / HW * (a4 > 0).
__global__ void __launch_bounds__(128) k_fc_bwd_w(const float* __restrict__ dout,
                                                  const float* __restrict__ pooled, int N, int C,
                                                  float* gW, float* gb)
{
    const int k = blockIdx.x, c = threadIdx.x;
    if (c < C) {
        float s = 0.0f;
        for (int n = 0; n < N; ++n) s = fmaf(dout[n * 6 + k], pooled[(size_t)n * C + c], s);
        gW[k * C + c] = s;
    }
    if (c == 0) {
        float s = 0.0f;
        for (int n = 0; n < N; ++n) s += dout[n * 6 + k];
        gb[k] = s;
    }
}

__global__ void __launch_bounds__(256) k_fc_bwd_x(const float* __restrict__ dout,
                                                  const __hip_bfloat16* __restrict__ wfc,
                                                  const float* __restrict__ a4, int N, int C, int HW,
                                                  float* dz4)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * C * HW) return;
    const int c = (t / HW) % C, n = t / (HW * C);
    float s = 0.0f;
    for (int k = 0; k < 6; ++k) s = fmaf(dout[n * 6 + k], bf(wfc[k * C + c]), s);
    dz4[t] = a4[t] > 0.0f ? s / (float)HW : 0.0f;
}

// ------------------------------------------------------------------ conv backward

// dz_prev[n,ci,iy,ix] = (sum_{co,ky,kx} dz[n,co,y,x] w[co,ci,ky,kx]) * (a_prev > 0)
// over the (y, x) with iy = 2y - 1 + ky, ix = 2x - 1 + kx.
__global__ void __launch_bounds__(256) k_conv_bwd_x(const float* __restrict__ dz,
                                                    const __hip_bfloat16* __restrict__ w,
                                                    const float* __restrict__ a_prev, float* dz_prev,
                                                    int N, int Ci, int Hi, int Wi, int Co, int Ho,
                                                    int Wo)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * Ci * Hi * Wi) return;
    if (!(a_prev[t] > 0.0f)) {
        dz_prev[t] = 0.0f;
        return;
    }
    const int ix = t % Wi;
    const int iy = (t / Wi) % Hi;
    const int ci = (t / (Wi * Hi)) % Ci;
    const int n = t / (Wi * Hi * Ci);
    float s = 0.0f;
    for (int co = 0; co < Co; ++co) {
        const float* d = dz + ((size_t)n * Co + co) * Ho * Wo;
        const __hip_bfloat16* wc = w + ((size_t)co * Ci + ci) * 9;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int yy = iy + 1 - ky;
            if (yy < 0 || (yy & 1) || (yy >> 1) >= Ho) continue;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int xx = ix + 1 - kx;
                if (xx < 0 || (xx & 1) || (xx >> 1) >= Wo) continue;
                s = fmaf(d[(yy >> 1) * Wo + (xx >> 1)], bf(wc[ky * 3 + kx]), s);
            }
        }
    }
    dz_prev[t] = s;
}

// dw[co,ci,ky,kx] = sum_{n,y,x} dz[n,co,y,x] x[n,ci,2y-1+ky,2x-1+kx]; one block
// per (co, ci); per-thread strided sums then a fixed LDS tree.  Block (co, 0)
// also writes db[co] = sum dz[n,co,:,:].
__global__ void __launch_bounds__(256) k_conv_bwd_w(const float* __restrict__ dz,
                                                    const float* __restrict__ x, int N, int Ci,
                                                    int Hi, int Wi, int Co, int Ho, int Wo, float* gw,
                                                    float* gb)
{
    __shared__ float red[256 * 10];
    const int co = blockIdx.x / Ci, ci = blockIdx.x % Ci;
    float acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.0f;
    const int P = N * Ho * Wo;
    for (int q = threadIdx.x; q < P; q += blockDim.x) {
        const int xo = q % Wo, yo = (q / Wo) % Ho, n = q / (Wo * Ho);
        const float d = dz[(((size_t)n * Co + co) * Ho + yo) * Wo + xo];
        const float* xc = x + ((size_t)n * Ci + ci) * Hi * Wi;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int iy = 2 * yo - 1 + ky;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int ix = 2 * xo - 1 + kx;
                const bool in = iy >= 0 && iy < Hi && ix >= 0 && ix < Wi;
                acc[ky * 3 + kx] = fmaf(d, in ? xc[iy * Wi + ix] : 0.0f, acc[ky * 3 + kx]);
            }
        }
        acc[9] += d;
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) red[k * 256 + threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 10; ++k) red[k * 256 + threadIdx.x] += red[k * 256 + threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9) gw[((size_t)co * Ci + ci) * 9 + threadIdx.x] = red[threadIdx.x * 256];
    if (threadIdx.x == 9 && ci == 0) gb[co] = red[9 * 256];
}

// ------------------------------------------------------------------ optimiser

// AdamW with decoupled weight decay on the weights (mask = 1) only; refreshes
// the bf16 copy of the weights.
__global__ void __launch_bounds__(256) k_adamw(float* w, float* m, float* v, const float* g,
                                               const float* decay, __hip_bfloat16* wb, int n,
                                               float lr, float b1, float b2, float eps, float wd,
                                               float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float wi = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * decay[i] * w[i]);
    w[i] = wi;
    wb[i] = __float2bfloat16(wi);
}

__global__ void __launch_bounds__(256) k_to_bf16(const float* w, __hip_bfloat16* wb, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = __float2bfloat16(w[i]);
}

inline unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t cnn_input(hipStream_t s, const CnnInput* in_dev, int n, float* x)
{
    dim3 grid(blocks(kCnnH * kCnnW, 256), n);
    hipLaunchKernelGGL(k_input, grid, dim3(256), 0, s, in_dev, n, x);
    return hipGetLastError();
}

hipError_t cnn_forward(hipStream_t s, const CnnBuffers& B, int N, const float* x)
{
    const float* in = x;
    for (int l = 0; l < 4; ++l) {
        const int Ci = kCnnCh[l], Co = kCnnCh[l + 1];
        const int Hi = kCnnHs[l], Wi = kCnnWs[l], Ho = kCnnHs[l + 1], Wo = kCnnWs[l + 1];
        const long long total = (long long)N * (Co / 8) * Ho * Wo;
        hipLaunchKernelGGL(k_conv_fwd<8>, dim3(blocks(total, 256)), dim3(256), 0, s, in,
                           B.wbf + kCnnOff[2 * l], B.w + kCnnOff[2 * l + 1], B.act[l], N, Ci, Hi,
                           Wi, Co, Ho, Wo);
        in = B.act[l];
    }
    hipLaunchKernelGGL(k_pool_fc, dim3(N), dim3(128), 0, s, B.act[3], B.wbf + kCnnOff[8],
                       B.w + kCnnOff[9], B.pooled, B.out, kCnnCh[4], kCnnHs[4] * kCnnWs[4]);
    return hipGetLastError();
}

hipError_t cnn_backward(hipStream_t s, const CnnBuffers& B, int N, const float* x,
                        const float* target)
{
    const int C4 = kCnnCh[4], HW4 = kCnnHs[4] * kCnnWs[4];
    hipLaunchKernelGGL(k_loss, dim3(blocks(N, 64)), dim3(64), 0, s, B.out, target, N, B.dout,
                       B.loss_n);
    hipLaunchKernelGGL(k_fc_bwd_w, dim3(6), dim3(128), 0, s, B.dout, B.pooled, N, C4,
                       B.grad + kCnnOff[8], B.grad + kCnnOff[9]);
    hipLaunchKernelGGL(k_fc_bwd_x, dim3(blocks((long long)N * C4 * HW4, 256)), dim3(256), 0, s,
                       B.dout, B.wbf + kCnnOff[8], B.act[3], N, C4, HW4, B.dz[3]);
    for (int l = 3; l >= 0; --l) {
        const int Ci = kCnnCh[l], Co = kCnnCh[l + 1];
        const int Hi = kCnnHs[l], Wi = kCnnWs[l], Ho = kCnnHs[l + 1], Wo = kCnnWs[l + 1];
        const float* xin = l == 0 ? x : B.act[l - 1];
        hipLaunchKernelGGL(k_conv_bwd_w, dim3(Co * Ci), dim3(256), 0, s, B.dz[l], xin, N, Ci, Hi,
                           Wi, Co, Ho, Wo, B.grad + kCnnOff[2 * l], B.grad + kCnnOff[2 * l + 1]);
        if (l > 0)
            hipLaunchKernelGGL(k_conv_bwd_x, dim3(blocks((long long)N * Ci * Hi * Wi, 256)),
                               dim3(256), 0, s, B.dz[l], B.wbf + kCnnOff[2 * l], B.act[l - 1],
                               B.dz[l - 1], N, Ci, Hi, Wi, Co, Ho, Wo);
    }
    return hipGetLastError();
}

hipError_t cnn_adamw(hipStream_t s, const CnnBuffers& B, float lr, float wd, int step)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adamw, dim3(blocks(kCnnParams, 256)), dim3(256), 0, s, B.w, B.m, B.v,
                       B.grad, B.decay, B.wbf, kCnnParams, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

hipError_t cnn_refresh_bf16(hipStream_t s, const CnnBuffers& B)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(kCnnParams, 256)), dim3(256), 0, s, B.w, B.wbf,
                       kCnnParams);
    return hipGetLastError();
}

}  // namespace rgbid
