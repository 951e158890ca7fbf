// Inference form of the warm-start network on the matrix cores: the forward
// pass of cnn.hip (same parameters, same result up to the order of FP32
// additions) as implicit GEMMs on v_mfma_f32_32x32x16_bf16.
//
// A 3x3 stride-2 convolution is out[co, p] = b[co] + sum_k W[co, k] x[k, p]
// with p an output pixel (n, y, x) and k = (ky, kx, ci) the taps of its
// receptive field: a GEMM of M = Co, N = pixels, K = 9 Ci.  The weights are
// bfloat16 already.  An FP32 activation a is carried as three bfloat16
// limbs h + m + l = a (exactly: h is a with its low 16 bits cleared, m
// likewise of a - h, and the remaining 8 significant bits fit l), so three
// bf16 products per weight, each exact in FP32, sum in the matrix core's
// FP32 accumulator to W a: the FP32 forward without rounding the
// activations.  Activations are stored as three NHWC planes of limbs, so
// the 8 consecutive k of a lane (8 channels of one tap) are one 16-byte
// load per limb.
//
// Lane layout of v_mfma_f32_32x32x16_bf16 (D = A B + C, A 32 x 16, B 16 x
// 32): lane l supplies A row l % 32 and B column l % 32, k = 8 (l / 32) ..
// 8 (l / 32) + 7; D element (i, j) sits in lane j + 32 ((i / 4) % 2),
// register 4 (i / 8) + i % 4.
#include "rgbid_internal.h"

namespace rgbid {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned short u4v __attribute__((ext_vector_type(4)));
typedef unsigned short u8v __attribute__((ext_vector_type(8)));

// The three limbs of a (their bit patterns).
__device__ __forceinline__ void split3(float a, unsigned short& h, unsigned short& m,
                                       unsigned short& l)
{
    const unsigned ua = __float_as_uint(a);
    const float r = a - __uint_as_float(ua & 0xffff0000u);
    const unsigned ur = __float_as_uint(r);
    const float r2 = r - __uint_as_float(ur & 0xffff0000u);
    h = (unsigned short)(ua >> 16);
    m = (unsigned short)(ur >> 16);
    l = (unsigned short)(__float_as_uint(r2) >> 16);
}

__device__ __forceinline__ float limb(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// Network input x[n, y, x, c] = (I_A / 255, W_A / 2, I_B / 255, W_B / 2) at
// the 80 x 60 level (the arithmetic of the FP32 input kernel), as limbs.
__global__ void __launch_bounds__(256) k_input_limbs(const CnnInput* __restrict__ in, int n,
                                                     unsigned short* __restrict__ x, size_t plane)
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
    const float v[4] = {a.x * (1.0f / 255.0f), a.y * 0.5f, b.x * (1.0f / 255.0f), b.y * 0.5f};
    u4v h, m, l;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        unsigned short hh, mm, ll;
        split3(v[k], hh, mm, ll);
        h[k] = hh;
        m[k] = mm;
        l[k] = ll;
    }
    const size_t o = ((size_t)p * kCnnH * kCnnW + i) * 4;
    *reinterpret_cast<u4v*>(x + o) = h;
    *reinterpret_cast<u4v*>(x + plane + o) = m;
    *reinterpret_cast<u4v*>(x + 2 * plane + o) = l;
}

// Weights of one layer in GEMM order: wg[co, k], k = (ky 3 + kx) Ci + ci,
// zero-padded to KP (a multiple of 16), from the bf16 copy laid out
// Co x Ci x 3 x 3.
__global__ void __launch_bounds__(256) k_gemm_weights(const __hip_bfloat16* __restrict__ wb,
                                                      unsigned short* __restrict__ wg, int Ci,
                                                      int Co, int KP)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Co * KP) return;
    const int co = t / KP, k = t % KP;
    unsigned short v = 0;
    if (k < 9 * Ci) {
        const int tap = k / Ci, ci = k % Ci;
        const __hip_bfloat16 w = wb[((size_t)co * Ci + ci) * 9 + tap];
        v = *reinterpret_cast<const unsigned short*>(&w);
    }
    wg[t] = v;
}

// The 8 limbs of one limb plane for k = k8 .. k8 + 7 of output pixel
// (n, yo, xo): 8 channels of one tap when CI >= 8, two taps of 4 channels
// when CI == 4 (taps past the ninth and pixels outside the input are zero).
template <int CI, int HI, int WI>
__device__ __forceinline__ u8v load_b(const unsigned short* __restrict__ x, int n, int yo, int xo,
                                      int k8)
{
    u8v r = u8v{0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (CI >= 8) {
        const int tap = k8 / CI, ci = k8 % CI;
        const int iy = 2 * yo - 1 + tap / 3, ix = 2 * xo - 1 + tap % 3;
        if (tap < 9 && (unsigned)iy < (unsigned)HI && (unsigned)ix < (unsigned)WI)
            r = *reinterpret_cast<const u8v*>(x + (((size_t)n * HI + iy) * WI + ix) * CI + ci);
    } else {
        static_assert(CI == 4, "channel groups of 4 or of at least 8");
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int tap = k8 / 4 + h;
            const int iy = 2 * yo - 1 + tap / 3, ix = 2 * xo - 1 + tap % 3;
            if (tap < 9 && (unsigned)iy < (unsigned)HI && (unsigned)ix < (unsigned)WI) {
                const u4v q =
                    *reinterpret_cast<const u4v*>(x + (((size_t)n * HI + iy) * WI + ix) * 4);
                r[4 * h + 0] = q[0];
                r[4 * h + 1] = q[1];
                r[4 * h + 2] = q[2];
                r[4 * h + 3] = q[3];
            }
        }
    }
    return r;
}

__device__ __forceinline__ bf8 as_bf8(u8v v)
{
    bf8 r;
    __builtin_memcpy(&r, &v, sizeof r);
    return r;
}

// One wave: 32 output channels x 32 output pixels of the flattened
// (n, yo, xo) range, K in steps of 16; bias, ReLU and the limbs of the
// result stored NHWC.  x and out hold three limb planes `xplane` /
// `oplane` elements apart.
template <int CI, int CO, int HI, int WI, int HO, int WO>
__global__ void __launch_bounds__(256) k_conv_mfma(const unsigned short* __restrict__ x,
                                                   size_t xplane,
                                                   const unsigned short* __restrict__ wg,
                                                   const float* __restrict__ bias,
                                                   unsigned short* __restrict__ out,
                                                   size_t oplane, int N)
{
    constexpr int KP = (9 * CI + 15) / 16 * 16;
    constexpr int NPIX = HO * WO, COT = CO / 32;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int total = N * NPIX;
    const int ct = wave % COT, pt = wave / COT;
    if (pt * 32 >= total) return;
    const int col = lane & 31, kg = lane >> 5;
    const int p = min(pt * 32 + col, total - 1);
    const int n = p / NPIX, rr = p % NPIX, yo = rr / WO, xo = rr % WO;
    const unsigned short* wrow = wg + (size_t)(ct * 32 + col) * KP + 8 * kg;
    f16v acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll 2
    for (int k0 = 0; k0 < KP; k0 += 16) {
        const bf8 a = as_bf8(*reinterpret_cast<const u8v*>(wrow + k0));
        const int k8 = k0 + 8 * kg;
        const bf8 bh = as_bf8(load_b<CI, HI, WI>(x, n, yo, xo, k8));
        const bf8 bm = as_bf8(load_b<CI, HI, WI>(x + xplane, n, yo, xo, k8));
        const bf8 bl = as_bf8(load_b<CI, HI, WI>(x + 2 * xplane, n, yo, xo, k8));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bm, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc, 0, 0, 0);
    }
    if (pt * 32 + col >= total) return;
    // lane holds pixel p, channels ct 32 + 8 g + 4 kg + j in register 4 g + j
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int c0 = ct * 32 + 8 * g + 4 * kg;
        u4v h, m, l;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            unsigned short hh, mm, ll;
            split3(fmaxf(acc[4 * g + j] + bias[c0 + j], 0.0f), hh, mm, ll);
            h[j] = hh;
            m[j] = mm;
            l[j] = ll;
        }
        const size_t o = (size_t)p * CO + c0;
        *reinterpret_cast<u4v*>(out + o) = h;
        *reinterpret_cast<u4v*>(out + oplane + o) = m;
        *reinterpret_cast<u4v*>(out + 2 * oplane + o) = l;
    }
}

// Global average pool of the last layer (limbs, NHWC, 4 x 5 pixels) and the
// fully connected layer: out[n, k] = b[k] + sum_c W[k, c] mean_p a[n, p, c];
// one block per sample, the pool in pixel order as in the FP32 kernel.
__global__ void __launch_bounds__(128) k_pool_fc_limbs(const unsigned short* __restrict__ a4,
                                                       size_t plane,
                                                       const __hip_bfloat16* __restrict__ wfc,
                                                       const float* __restrict__ bfc, float* out,
                                                       int C, int HW)
{
    __shared__ float pl[128];
    const int n = blockIdx.x, c = threadIdx.x;
    if (c < C) {
        float s = 0.0f;
        for (int i = 0; i < HW; ++i) {
            const size_t o = ((size_t)n * HW + i) * C + c;
            s += (limb(a4[o]) + limb(a4[plane + o])) + limb(a4[2 * plane + o]);
        }
        pl[c] = s / (float)HW;
    }
    __syncthreads();
    if (c < 6) {
        float s = bfc[c];
        for (int j = 0; j < C; ++j) s = fmaf(__bfloat162float(wfc[c * C + j]), pl[j], s);
        out[(size_t)n * 6 + c] = s;
    }
}

template <int CI, int CO, int HI, int WI, int HO, int WO>
hipError_t conv_layer(hipStream_t s, const unsigned short* x, size_t xplane,
                      const unsigned short* wg, const float* b, unsigned short* out,
                      size_t oplane, int N)
{
    const int tiles = (N * HO * WO + 31) / 32 * (CO / 32);
    hipLaunchKernelGGL((k_conv_mfma<CI, CO, HI, WI, HO, WO>), dim3((tiles + 3) / 4), dim3(256), 0,
                       s, x, xplane, wg, b, out, oplane, N);
    return hipGetLastError();
}

}  // namespace

size_t cnn_limb_bytes(int N)
{
    size_t total = 0;
    for (int l = 0; l < 5; ++l)
        total += (size_t)3 * N * kCnnCh[l] * kCnnHs[l] * kCnnWs[l] * sizeof(unsigned short) + 256;
    return total;
}

int cnn_gemm_k(int l) { return (9 * kCnnCh[l] + 15) / 16 * 16; }

hipError_t cnn_gemm_weights(hipStream_t s, const CnnBuffers& B, unsigned short* wg)
{
    size_t off = 0;
    for (int l = 0; l < 4; ++l) {
        const int Ci = kCnnCh[l], Co = kCnnCh[l + 1], KP = cnn_gemm_k(l);
        hipLaunchKernelGGL(k_gemm_weights, dim3((Co * KP + 255) / 256), dim3(256), 0, s,
                           B.wbf + kCnnOff[2 * l], wg + off, Ci, Co, KP);
        off += (size_t)Co * KP;
    }
    return hipGetLastError();
}

hipError_t cnn_forward_mfma(hipStream_t s, const CnnBuffers& B, const unsigned short* wg,
                            const CnnInput* in_dev, int N, unsigned short* limbs, float* out)
{
    // limb buffers of the input and the four layer outputs, back to back
    unsigned short* act[5];
    size_t plane[5];
    {
        char* p = reinterpret_cast<char*>(limbs);
        for (int l = 0; l < 5; ++l) {
            plane[l] = (size_t)N * kCnnCh[l] * kCnnHs[l] * kCnnWs[l];
            act[l] = reinterpret_cast<unsigned short*>(p);
            p += 3 * plane[l] * sizeof(unsigned short) + 256;
        }
    }
    hipLaunchKernelGGL(k_input_limbs, dim3((kCnnH * kCnnW + 255) / 256, N), dim3(256), 0, s, in_dev,
                       N, act[0], plane[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t wo = 0;
    const unsigned short* w1 = wg + wo;
    wo += (size_t)32 * cnn_gemm_k(0);
    const unsigned short* w2 = wg + wo;
    wo += (size_t)64 * cnn_gemm_k(1);
    const unsigned short* w3 = wg + wo;
    wo += (size_t)128 * cnn_gemm_k(2);
    const unsigned short* w4 = wg + wo;
    if ((e = conv_layer<4, 32, 60, 80, 30, 40>(s, act[0], plane[0], w1, B.w + kCnnOff[1], act[1],
                                                plane[1], N)) != hipSuccess)
        return e;
    if ((e = conv_layer<32, 64, 30, 40, 15, 20>(s, act[1], plane[1], w2, B.w + kCnnOff[3], act[2],
                                                 plane[2], N)) != hipSuccess)
        return e;
    if ((e = conv_layer<64, 128, 15, 20, 8, 10>(s, act[2], plane[2], w3, B.w + kCnnOff[5], act[3],
                                                 plane[3], N)) != hipSuccess)
        return e;
    if ((e = conv_layer<128, 128, 8, 10, 4, 5>(s, act[3], plane[3], w4, B.w + kCnnOff[7], act[4],
                                                plane[4], N)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_pool_fc_limbs, dim3(N), dim3(128), 0, s, act[4], plane[4],
                       B.wbf + kCnnOff[8], B.w + kCnnOff[9], out, 128, kCnnHs[4] * kCnnWs[4]);
    return hipGetLastError();
}

}  // namespace rgbid
