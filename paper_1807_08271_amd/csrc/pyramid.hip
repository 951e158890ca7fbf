// Image pyramid of {I, W} (sec. 6.2: the reference images are downsampled at
// every level).  Level 0 is the caller's FP32 image converted to the storage
// format; level l+1 is the 2x2 mean of level l, where the inverse-depth mean
// skips holes and is a hole when all four children are holes.
//
// Layout per level: an interleaved (I, W) array (float2 / __half2), used for
// bilinear gathers of the current frame and for stencils of the reference,
// plus a separate W plane (float / __half) for the full-resolution warp,
// which reads only W of the reference.
#include "rgbid_internal.h"

namespace rgbid {
namespace {

__device__ __forceinline__ bool w_valid(float w) { return w > 0.0f && w < INFINITY; }

template <bool F16>
__device__ __forceinline__ float2 load_iw(const void* p, int i)
{
    if constexpr (F16) return __half22float2(static_cast<const __half2*>(p)[i]);
    else return static_cast<const float2*>(p)[i];
}

template <bool F16>
__device__ __forceinline__ void store_level(void* iw, void* wp, int i, float I, float W)
{
    if constexpr (F16) {
        __half2 h = __floats2half2_rn(I, W);
        static_cast<__half2*>(iw)[i] = h;
        static_cast<__half*>(wp)[i] = __high2half(h);
    } else {
        static_cast<float2*>(iw)[i] = make_float2(I, W);
        static_cast<float*>(wp)[i] = W;
    }
}

template <bool F16>
__global__ void __launch_bounds__(256) k_level0(const PyrFrame* __restrict__ frames)
{
    const PyrFrame& f = frames[blockIdx.y];
    const int w = f.w[0], h = f.h[0];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w * h) return;
    const int v = i / w, u = i - v * w;
    const long long src = (long long)v * f.pitch + u;
    const float I = f.I[src];
    float W = f.W[src];
    if (!w_valid(W)) W = 0.0f;
    store_level<F16>(f.iw[0], f.wp[0], i, I, W);
}

// Level 0, four pixels of a row per thread (rows a multiple of 4 wide, the
// caller's rows 16-byte aligned): 16-byte loads of I and W, 16-byte stores of
// both planes; the values of k_level0.
template <bool F16>
__global__ void __launch_bounds__(256) k_level0_quad(const PyrFrame* __restrict__ frames)
{
    const PyrFrame& f = frames[blockIdx.y];
    const int w = f.w[0], h = f.h[0], qw = w >> 2;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= qw * h) return;
    const int v = q / qw, u0 = (q - v * qw) << 2;
    const long long src = (long long)v * f.pitch + u0;
    const float4 I = *reinterpret_cast<const float4*>(f.I + src);
    float4 W = *reinterpret_cast<const float4*>(f.W + src);
    W.x = w_valid(W.x) ? W.x : 0.0f;
    W.y = w_valid(W.y) ? W.y : 0.0f;
    W.z = w_valid(W.z) ? W.z : 0.0f;
    W.w = w_valid(W.w) ? W.w : 0.0f;
    const int i = v * w + u0;
    if constexpr (F16) {
        const __half2 h0 = __floats2half2_rn(I.x, W.x), h1 = __floats2half2_rn(I.y, W.y);
        const __half2 h2 = __floats2half2_rn(I.z, W.z), h3 = __floats2half2_rn(I.w, W.w);
        auto bits = [](__half2 x) { return *reinterpret_cast<const unsigned*>(&x); };
        *reinterpret_cast<uint4*>(static_cast<__half2*>(f.iw[0]) + i) =
            make_uint4(bits(h0), bits(h1), bits(h2), bits(h3));
        // the W halves are the high halves of the (I, W) pairs
        *reinterpret_cast<uint2*>(static_cast<__half*>(f.wp[0]) + i) =
            make_uint2((bits(h0) >> 16) | (bits(h1) & 0xffff0000u),
                       (bits(h2) >> 16) | (bits(h3) & 0xffff0000u));
    } else {
        float4* o = reinterpret_cast<float4*>(static_cast<float2*>(f.iw[0]) + i);
        o[0] = make_float4(I.x, W.x, I.y, W.y);
        o[1] = make_float4(I.z, W.z, I.w, W.w);
        *reinterpret_cast<float4*>(static_cast<float*>(f.wp[0]) + i) = W;
    }
}

// The value a stored W has: 0 for a hole, and in FP16 storage the rounded
// value (the flags and the next level are formed from what is stored).
template <bool F16>
__device__ __forceinline__ float stored_w(float W)
{
    W = w_valid(W) ? W : 0.0f;
    if constexpr (F16) return __half2float(__float2half_rn(W));
    else return W;
}

template <bool F16>
__device__ __forceinline__ float stored_i(float I)
{
    if constexpr (F16) return __half2float(__float2half_rn(I));
    else return I;
}

// Levels 0 and 1 and the flags of level 0 in one pass (even sizes, rows of
// the caller's images 8-byte aligned): a thread takes the 2x2 block of
// level-0 pixels under one level-1 pixel.  It stores the block (the values
// of k_level0), flags it (the rule of k_mask, the neighbours' W read from the
// caller's image at clamped positions and taken as stored) and stores the
// level-1 pixel (the mean of k_down over the stored block values), so level
// 0 is neither read back for the downsampling nor for the flags.
template <bool F16>
__global__ void __launch_bounds__(256) k_level01(const PyrFrame* __restrict__ frames)
{
    const PyrFrame& f = frames[blockIdx.y];
    const int w = f.w[0], h = f.h[0], bw = w >> 1;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bw * (h >> 1)) return;
    const int by = b / bw, bx = b - by * bw;
    const int u0 = 2 * bx, v0 = 2 * by;
    const long long p = f.pitch;
    const long long r0 = (long long)v0 * p + u0, r1 = r0 + p;
    // every load first: the block (I and W), then the W around it
    const float2 i0 = *reinterpret_cast<const float2*>(f.I + r0);
    const float2 i1 = *reinterpret_cast<const float2*>(f.I + r1);
    const float2 w0 = *reinterpret_cast<const float2*>(f.W + r0);
    const float2 w1 = *reinterpret_cast<const float2*>(f.W + r1);
    const long long ru = (long long)max(v0 - 1, 0) * p + u0, rd = (long long)min(v0 + 2, h - 1) * p + u0;
    const float2 wu = *reinterpret_cast<const float2*>(f.W + ru);
    const float2 wd = *reinterpret_cast<const float2*>(f.W + rd);
    const int ul = max(u0 - 1, 0), ur = min(u0 + 2, w - 1);
    const float wl0 = f.W[(long long)v0 * p + ul], wl1 = f.W[(long long)(v0 + 1) * p + ul];
    const float wr0 = f.W[(long long)v0 * p + ur], wr1 = f.W[(long long)(v0 + 1) * p + ur];
    // the block as stored, children in the order (0,0), (1,0), (0,1), (1,1)
    const float I00 = stored_i<F16>(i0.x), I10 = stored_i<F16>(i0.y);
    const float I01 = stored_i<F16>(i1.x), I11 = stored_i<F16>(i1.y);
    const float W00 = stored_w<F16>(w0.x), W10 = stored_w<F16>(w0.y);
    const float W01 = stored_w<F16>(w1.x), W11 = stored_w<F16>(w1.y);
    const int i = v0 * w + u0;
    store_level<F16>(f.iw[0], f.wp[0], i, I00, W00);
    store_level<F16>(f.iw[0], f.wp[0], i + 1, I10, W10);
    store_level<F16>(f.iw[0], f.wp[0], i + w, I01, W01);
    store_level<F16>(f.iw[0], f.wp[0], i + w + 1, I11, W11);
    // flags: bit 0 interior with a valid W, bit 1 also the four neighbours
    auto flag = [&](int u, int v, float c, float l, float r, float t, float d) -> unsigned {
        if (!(u >= 1 && v >= 1 && u <= w - 2 && v <= h - 2 && w_valid(c))) return 0u;
        return w_valid(l) && w_valid(r) && w_valid(t) && w_valid(d) ? 3u : 1u;
    };
    const float Wu0 = stored_w<F16>(wu.x), Wu1 = stored_w<F16>(wu.y);
    const float Wd0 = stored_w<F16>(wd.x), Wd1 = stored_w<F16>(wd.y);
    const float Wl0 = stored_w<F16>(wl0), Wl1 = stored_w<F16>(wl1);
    const float Wr0 = stored_w<F16>(wr0), Wr1 = stored_w<F16>(wr1);
    const unsigned m00 = flag(u0, v0, W00, Wl0, W10, Wu0, W01);
    const unsigned m10 = flag(u0 + 1, v0, W10, W00, Wr0, Wu1, W11);
    const unsigned m01 = flag(u0, v0 + 1, W01, Wl1, W11, W00, Wd0);
    const unsigned m11 = flag(u0 + 1, v0 + 1, W11, W01, Wr1, W10, Wd1);
    unsigned char* gm = static_cast<unsigned char*>(f.gm[0]);
    *reinterpret_cast<unsigned short*>(gm + i) = (unsigned short)(m00 | m10 << 8);
    *reinterpret_cast<unsigned short*>(gm + i + w) = (unsigned short)(m01 | m11 << 8);
    if (f.levels < 2) return;
    const float I = (((I00 + I10) + I01) + I11) * 0.25f;
    float sw = 0.0f;
    int n = 0;
    if (w_valid(W00)) { sw += W00; ++n; }
    if (w_valid(W10)) { sw += W10; ++n; }
    if (w_valid(W01)) { sw += W01; ++n; }
    if (w_valid(W11)) { sw += W11; ++n; }
    store_level<F16>(f.iw[1], f.wp[1], by * bw + bx, I, n ? sw / (float)n : 0.0f);
}

template <bool F16>
__global__ void __launch_bounds__(256) k_down(const PyrFrame* __restrict__ frames, int level)
{
    const PyrFrame& f = frames[blockIdx.y];
    if (level >= f.levels) return;
    const int w = f.w[level], h = f.h[level];
    const int ws = f.w[level - 1];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w * h) return;
    const int v = i / w, u = i - v * w;
    const void* src = f.iw[level - 1];
    const int r0 = (2 * v) * ws + 2 * u, r1 = r0 + ws;
    // children in the order (0,0), (1,0), (0,1), (1,1)
    const float2 c0 = load_iw<F16>(src, r0), c1 = load_iw<F16>(src, r0 + 1);
    const float2 c2 = load_iw<F16>(src, r1), c3 = load_iw<F16>(src, r1 + 1);
    const float I = (((c0.x + c1.x) + c2.x) + c3.x) * 0.25f;
    float sw = 0.0f;
    int n = 0;
    if (w_valid(c0.y)) { sw += c0.y; ++n; }
    if (w_valid(c1.y)) { sw += c1.y; ++n; }
    if (w_valid(c2.y)) { sw += c2.y; ++n; }
    if (w_valid(c3.y)) { sw += c3.y; ++n; }
    const float W = n ? sw / (float)n : 0.0f;
    store_level<F16>(f.iw[level], f.wp[level], i, I, W);
}

template <bool F16>
__device__ __forceinline__ float load_wp(const void* p, int i)
{
    if constexpr (F16) return __half2float(static_cast<const __half*>(p)[i]);
    else return static_cast<const float*>(p)[i];
}

// Four consecutive W values from element i (i a multiple of 4, the plane
// 16-byte aligned).
template <bool F16>
__device__ __forceinline__ void load_wp4(const void* p, int i, float* o)
{
    if constexpr (F16) {
        const uint2 b = *reinterpret_cast<const uint2*>(static_cast<const __half*>(p) + i);
        const __half2 lo = *reinterpret_cast<const __half2*>(&b.x);
        const __half2 hi = *reinterpret_cast<const __half2*>(&b.y);
        o[0] = __low2float(lo);
        o[1] = __high2float(lo);
        o[2] = __low2float(hi);
        o[3] = __high2float(hi);
    } else {
        const float4 f = *reinterpret_cast<const float4*>(static_cast<const float*>(p) + i);
        o[0] = f.x;
        o[1] = f.y;
        o[2] = f.z;
        o[3] = f.w;
    }
}

// Validity flags of a level used by the residuals (sec. 6.2): bit 0 = the
// pixel is interior (one pixel from every border) with a valid W, bit 1 =
// bit 0 and the four W neighbours valid, i.e. the central-difference gradient
// of W is defined.
// Workgroups are dealt to the 8 XCDs in turn, each with its own L2; this
// maps consecutive row ranges of an image to one XCD so that the stencil's
// neighbouring rows are found in that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

// A thread flags four consecutive pixels of a row.  Every W the four flags
// need (the row segment with one pixel on each side, and the segments of the
// rows above and below, all at clamped in-image positions) is loaded before
// any is tested, so a wave waits for one round of loads; one pixel per thread
// with the neighbours loaded after the centre test took two.
template <bool F16>
__global__ void __launch_bounds__(256) k_mask(const PyrFrame* __restrict__ frames, int level)
{
    const PyrFrame& f = frames[blockIdx.y];
    if (level >= f.levels) return;
    const int w = f.w[level], h = f.h[level];
    const int qw = (w + 3) >> 2;   // quads per row
    const int q = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (q >= qw * h) return;
    const int v = q / qw, u0 = (q - v * qw) * 4;
    const void* wp = f.wp[level];
    const int rc = v * w, ru = max(v - 1, 0) * w, rd = min(v + 1, h - 1) * w;
    float c[6], up[4], dn[4];
    c[0] = load_wp<F16>(wp, rc + max(u0 - 1, 0));
    c[5] = load_wp<F16>(wp, rc + min(u0 + 4, w - 1));
    if ((w & 3) == 0) {
        // whole, aligned quads: one 16-byte (8 with FP16) load per row
        load_wp4<F16>(wp, rc + u0, c + 1);
        load_wp4<F16>(wp, ru + u0, up);
        load_wp4<F16>(wp, rd + u0, dn);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int uk = min(u0 + k, w - 1);
            c[k + 1] = load_wp<F16>(wp, rc + uk);
            up[k] = load_wp<F16>(wp, ru + uk);
            dn[k] = load_wp<F16>(wp, rd + uk);
        }
    }
    unsigned char m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int u = u0 + k;
        m[k] = 0;
        if (u >= 1 && v >= 1 && u <= w - 2 && v <= h - 2 && w_valid(c[k + 1])) {
            m[k] = 1;
            if (w_valid(c[k]) && w_valid(c[k + 2]) && w_valid(up[k]) && w_valid(dn[k])) m[k] = 3;
        }
    }
    unsigned char* gm = static_cast<unsigned char*>(f.gm[level]) + rc + u0;
    if ((w & 3) == 0) {
        // the quad is whole and its first byte 4-aligned
        *reinterpret_cast<unsigned*>(gm) =
            m[0] | (unsigned)m[1] << 8 | (unsigned)m[2] << 16 | (unsigned)m[3] << 24;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (u0 + k < w) gm[k] = m[k];
    }
}

template <bool F16>
__global__ void __launch_bounds__(256) k_read(const void* __restrict__ iw, int n, float* I, float* W)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 p = load_iw<F16>(iw, i);
    if (I) I[i] = p.x;
    if (W) W[i] = p.y;
}

}  // namespace

hipError_t launch_pyramid(hipStream_t s, const PyrFrame* frames_dev, int nframes, int levels,
                          int f16, const int* max_w, const int* max_h, bool quad, bool pairs)
{
    if (nframes <= 0) return hipSuccess;
    if (pairs) {
        // levels 0 and 1 and the flags of level 0 in one pass
        const int n = (max_w[0] / 2) * (max_h[0] / 2);
        dim3 grid((n + 255) / 256, nframes);
        if (f16) hipLaunchKernelGGL(k_level01<true>, grid, dim3(256), 0, s, frames_dev);
        else hipLaunchKernelGGL(k_level01<false>, grid, dim3(256), 0, s, frames_dev);
    } else if (quad) {
        const int n = (max_w[0] / 4) * max_h[0];
        dim3 grid((n + 255) / 256, nframes);
        if (f16) hipLaunchKernelGGL(k_level0_quad<true>, grid, dim3(256), 0, s, frames_dev);
        else hipLaunchKernelGGL(k_level0_quad<false>, grid, dim3(256), 0, s, frames_dev);
    } else {
        const int n = max_w[0] * max_h[0];
        dim3 grid((n + 255) / 256, nframes);
        if (f16) hipLaunchKernelGGL(k_level0<true>, grid, dim3(256), 0, s, frames_dev);
        else hipLaunchKernelGGL(k_level0<false>, grid, dim3(256), 0, s, frames_dev);
    }
    for (int l = pairs ? 2 : 1; l < levels; ++l) {
        const int n = max_w[l] * max_h[l];
        if (n <= 0) break;
        dim3 grid((n + 255) / 256, nframes);
        if (f16) hipLaunchKernelGGL(k_down<true>, grid, dim3(256), 0, s, frames_dev, l);
        else hipLaunchKernelGGL(k_down<false>, grid, dim3(256), 0, s, frames_dev, l);
    }
    for (int l = pairs ? 1 : 0; l < levels; ++l) {
        const int n = ((max_w[l] + 3) / 4) * max_h[l];   // quads
        if (n <= 0) break;
        dim3 grid((n + 255) / 256, nframes);
        if (f16) hipLaunchKernelGGL(k_mask<true>, grid, dim3(256), 0, s, frames_dev, l);
        else hipLaunchKernelGGL(k_mask<false>, grid, dim3(256), 0, s, frames_dev, l);
    }
    return hipGetLastError();
}

hipError_t launch_level_read(hipStream_t s, const void* iw, int n, int f16, float* I, float* W)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((n + 255) / 256);
    if (f16) hipLaunchKernelGGL(k_read<true>, grid, dim3(256), 0, s, iw, n, I, W);
    else hipLaunchKernelGGL(k_read<false>, grid, dim3(256), 0, s, iw, n, I, W);
    return hipGetLastError();
}

}  // namespace rgbid
