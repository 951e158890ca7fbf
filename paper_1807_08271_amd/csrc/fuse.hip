// Keyframe inverse-depth fusion (sec. 7.2) by reverse warping (sec. 5.3).
// One thread per keyframe pixel; each keyframe pixel is read and written by
// exactly one thread, so no atomics touch the maps.  The covisibility check
// is the one of sec. 6.4: the transferred inverse depth 1/Y_z must agree with
// the frame's bilinear inverse depth within tol.
#include "rgbid_internal.h"

namespace rgbid {
namespace {

__device__ __forceinline__ bool w_valid(float w) { return w > 0.0f && w < INFINITY; }

// Transfer of pixel (u, v) with inverse depth wa into the other camera of
// the pose (D = R^T - I, Rtt = R^T t), in displacement form: with the ray x,
// W Y = R^T (x - W t) = x + d and d = D x - W Rtt, so Y_z W = 1 + d_z and
// the transferred position is p + (f_x (d_x - x_u d_z), f_y (d_y - x_v d_z)) /
// (1 + d_z).  The displacement is formed from small terms and keeps its
// relative precision, where an absolute position of hundreds of pixels would
// round to ~6e-5 px in FP32 (enough to move a bilinear sample across a depth
// edge).  Fills the bilinear taps of the other camera's W and returns whether
// the transfer is in front, inside [-0.5, w-0.5) x [-0.5, h-0.5) and has four
// valid taps.
struct Transfer {
    float wb;    // bilinear W at the transferred position
    float iz;    // 1 / (W Y_z)
    float az;    // (R^T x)_z
};

template <class LoadW>
__device__ __forceinline__ bool transfer(LoadW ld, int w, int h, float fx, float fy, float cx,
                                         float cy, const float* D, const float* Rtt, int u, int v,
                                         float wa, Transfer& o)
{
    const float rx = ((float)u - cx) / fx, ry = ((float)v - cy) / fy;
    const float dz0 = fmaf(D[6], rx, fmaf(D[7], ry, D[8]));
    const float dx = fmaf(D[0], rx, fmaf(D[1], ry, fmaf(-wa, Rtt[0], D[2])));
    const float dy = fmaf(D[3], rx, fmaf(D[4], ry, fmaf(-wa, Rtt[1], D[5])));
    const float dz = fmaf(-wa, Rtt[2], dz0);
    const float yz = 1.0f + dz;
    if (!(yz > 0.0f)) return false;
    const float iz = 1.0f / yz;
    const float du = fx * fmaf(-rx, dz, dx) * iz, dv = fy * fmaf(-ry, dz, dy) * iz;
    const float ub = (float)u + du, vb = (float)v + dv;
    if (!(ub >= -0.5f && ub < (float)w - 0.5f && vb >= -0.5f && vb < (float)h - 0.5f)) return false;
    // taps floor(p) = p + floor(displacement) (p integer) and the next ones,
    // clamped to the image; the weights are the displacement's fractions
    const float fu = floorf(du), fv = floorf(dv);
    const float al = du - fu, be = dv - fv;
    int x0 = u + (int)fu, y0 = v + (int)fv;
    const int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    x0 = max(x0, 0);
    y0 = max(y0, 0);
    const float p00 = ld(x0, y0), p10 = ld(x1, y0), p01 = ld(x0, y1), p11 = ld(x1, y1);
    if (!(w_valid(p00) && w_valid(p10) && w_valid(p01) && w_valid(p11))) return false;
    o.wb = (1.0f - al) * (1.0f - be) * p00 + al * (1.0f - be) * p10 + (1.0f - al) * be * p01 +
           al * be * p11;
    o.iz = iz;
    o.az = 1.0f + dz0;
    return true;
}

// One frame's fusion step at keyframe pixel (u, v) (sec. 7.2): the pixel
// with fused inverse depth wkf (valid) is transferred into frame k, W_k is
// sampled bilinearly, and if it passes the covisibility test the warped
// inverse depth W* = (R^T x)_z w_b / (1 + w_b (R^T t)_z) is merged into
// (wkf, ckf) with C_k = ((1 + w_b (R^T t)_z)^2 / (R^T x)_z)^2.  Returns
// whether the pixel fused.
__device__ __forceinline__ bool fuse_step(const float* __restrict__ Wk, long long pitch, int w,
                                          int h, float fx, float fy, float cx, float cy,
                                          const float* D, const float* Rtt, float tol, int u,
                                          int v, float& wkf, float& ckf)
{
    Transfer t;
    auto ld = [&](int x, int y) { return Wk[(long long)y * pitch + x]; };
    if (!transfer(ld, w, h, fx, fy, cx, cy, D, Rtt, u, v, wkf, t)) return false;
    // predicted inverse depth in frame k: 1 / Y_z = W_kf / (W_kf Y_z)
    const float wk = wkf * t.iz;
    if (!(fabsf(t.wb - wk) < tol)) return false;
    const float den = fmaf(t.wb, Rtt[2], 1.0f);
    const float ws = t.az * t.wb / den;
    const float q = den * den / t.az;
    const float ck = q * q;
    if (!(w_valid(ws) && ck > 0.0f && ck < INFINITY)) return false;
    wkf = (wkf * ckf + ck * ws) / (ckf + ck);
    ckf = ckf + ck;
    return true;
}

// Adds the workgroup's count of fused pixels (256 threads) to *count.
__device__ __forceinline__ void add_count(unsigned int* wave_counts, bool fused,
                                          unsigned long long* count)
{
    const unsigned long long bal = __ballot(fused);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wave_counts[wave] = (unsigned int)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int n = wave_counts[0] + wave_counts[1] + wave_counts[2] + wave_counts[3];
        if (n) atomicAdd(count, (unsigned long long)n);
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_fuse(FuseArgs a)
{
    __shared__ unsigned int wave_counts[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool fused = false;
    if (i < a.w * a.h) {
        const int v = i / a.w, u = i - v * a.w;
        float wkf = a.Wkf[i];
        if (w_valid(wkf)) {
            float ckf = a.Ckf[i];
            fused = fuse_step(a.Wk, a.pitch, a.w, a.h, a.fx, a.fy, a.cx, a.cy, a.D, a.Rtt, a.tol,
                              u, v, wkf, ckf);
            if (fused) {
                a.Wkf[i] = wkf;
                a.Ckf[i] = ckf;
            }
        }
    }
    if (a.count) add_count(wave_counts, fused, a.count);
}

// Frames 0 .. n-1 in order, each keyframe pixel read and written once: the
// same per-pixel steps as n launches of k_fuse.
__global__ void __launch_bounds__(256) k_fuse_batch(FuseBatchArgs a)
{
    __shared__ unsigned int wave_counts[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < a.w * a.h;
    int u = 0, v = 0;
    float wkf = 0.0f, ckf = 0.0f;
    if (in) {
        v = i / a.w;
        u = i - v * a.w;
        wkf = a.Wkf[i];
        ckf = a.Ckf[i];
    }
    bool any = false;
    for (int f = 0; f < a.n; ++f) {
        const FuseFrame& F = a.frames[f];
        bool fused = false;
        if (in && w_valid(wkf))
            fused = fuse_step(F.Wk, a.pitch, a.w, a.h, a.fx, a.fy, a.cx, a.cy, F.D, F.Rtt, a.tol, u,
                              v, wkf, ckf);
        any = any || fused;
        if (a.count) add_count(wave_counts, fused, a.count + f);
    }
    if (any) {
        a.Wkf[i] = wkf;
        a.Ckf[i] = ckf;
    }
}

}  // namespace

hipError_t launch_fuse(hipStream_t s, const FuseArgs& a)
{
    const int n = a.w * a.h;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fuse, dim3((n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fuse_batch(hipStream_t s, const FuseBatchArgs& a)
{
    const int n = a.w * a.h;
    if (n <= 0 || a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fuse_batch, dim3((n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace rgbid

namespace rgbid {
namespace {
__global__ void __launch_bounds__(256) k_fill(float* p, int n, float v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void __launch_bounds__(256) k_copy_valid(const float* src, long long pitch, int w, int h,
                                                   float* dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w * h) return;
    const int v = i / w, u = i - v * w;
    const float x = src[(long long)v * pitch + u];
    dst[i] = (x > 0.0f && x < INFINITY) ? x : 0.0f;
}
}  // namespace

hipError_t launch_fill(hipStream_t s, float* p, int n, float v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy_valid(hipStream_t s, const float* src, long long pitch, int w, int h,
                             float* dst)
{
    const int n = w * h;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_valid, dim3((n + 255) / 256), dim3(256), 0, s, src, pitch, w, h, dst);
    return hipGetLastError();
}

}  // namespace rgbid

namespace rgbid {
namespace {

template <bool F16>
__device__ __forceinline__ float load_wp(const void* p, long long i)
{
    if constexpr (F16) return __half2float(static_cast<const __half*>(p)[i]);
    else return static_cast<const float*>(p)[i];
}

// Dense covisibility (sec. 6.4), one direction: counts the pixels of A with a
// valid W_A (S_H) and those whose transfer into B is in bounds with four valid
// W_B taps and |W_B(p_B) - 1/Y_z| < tol (S_V).
template <bool F16>
__global__ void __launch_bounds__(256) k_covis(CovisArgs a)
{
    __shared__ unsigned int cnt[2][4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool inH = false, inV = false;
    if (i < a.w * a.h) {
        const int v = i / a.w, u = i - v * a.w;
        const float wa = load_wp<F16>(a.WA, i);
        if (w_valid(wa)) {
            inH = true;
            Transfer t;
            auto ld = [&](int x, int y) { return load_wp<F16>(a.WB, (long long)y * a.w + x); };
            if (transfer(ld, a.w, a.h, a.fx, a.fy, a.cx, a.cy, a.D, a.Rtt, u, v, wa, t))
                inV = fabsf(t.wb - wa * t.iz) < a.tol;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long bh = __ballot(inH), bv = __ballot(inV);
    if (lane == 0) {
        cnt[0][wave] = (unsigned int)__popcll(bh);
        cnt[1][wave] = (unsigned int)__popcll(bv);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const unsigned int n = cnt[threadIdx.x][0] + cnt[threadIdx.x][1] + cnt[threadIdx.x][2] +
                               cnt[threadIdx.x][3];
        if (n) atomicAdd(a.count + threadIdx.x, (unsigned long long)n);
    }
}

}  // namespace

hipError_t launch_covis(hipStream_t s, const CovisArgs& a)
{
    const int n = a.w * a.h;
    if (n <= 0) return hipSuccess;
    if (a.f16) hipLaunchKernelGGL(k_covis<true>, dim3((n + 255) / 256), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_covis<false>, dim3((n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace rgbid

namespace rgbid {
namespace {

// Bilateral filter of the reference (I, W) before the covariance iteration:
// spatial weight exp(-d^2 / (2 sigma_s^2)) over a (2r+1)^2 window, range
// weight exp(-dI^2 / (2 sigma_I^2)) for intensity and
// exp(-(dW / (rel_W W(p)))^2 / 2) for inverse depth; W holes neither
// contribute nor receive a value.  Output: dense FP32 images.
template <bool F16>
__global__ void __launch_bounds__(256) k_bilateral(const void* __restrict__ iw, int w, int h,
                                                   int radius, float inv2ss, float inv_sI,
                                                   float inv_relW, float* Io, float* Wo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w * h) return;
    const int v = i / w, u = i - v * w;
    auto ld = [&](int j) -> float2 {
        if constexpr (F16) return __half22float2(static_cast<const __half2*>(iw)[j]);
        else return static_cast<const float2*>(iw)[j];
    };
    const float2 c = ld(i);
    const bool wv = w_valid(c.y);
    const float iw0 = wv ? inv_relW / c.y : 0.0f;
    float si = 0.0f, swi = 0.0f, sw = 0.0f, sww = 0.0f;
    for (int dv = -radius; dv <= radius; ++dv) {
        const int y = v + dv;
        if (y < 0 || y >= h) continue;
        for (int du = -radius; du <= radius; ++du) {
            const int x = u + du;
            if (x < 0 || x >= w) continue;
            const float2 q = ld(y * w + x);
            const float gs = expf(-(float)(du * du + dv * dv) * inv2ss);
            const float di = (q.x - c.x) * inv_sI;
            const float gi = gs * expf(-0.5f * di * di);
            si = fmaf(gi, q.x, si);
            swi += gi;
            if (wv && w_valid(q.y)) {
                const float dw = (q.y - c.y) * iw0;
                const float gw = gs * expf(-0.5f * dw * dw);
                sw = fmaf(gw, q.y, sw);
                sww += gw;
            }
        }
    }
    Io[i] = si / swi;
    Wo[i] = wv ? sw / sww : 0.0f;
}

}  // namespace

hipError_t launch_bilateral(hipStream_t s, const void* iw, int f16, int w, int h, int radius,
                            float sigma_s, float sigma_I, float rel_W, float* Io, float* Wo)
{
    const int n = w * h;
    if (n <= 0) return hipSuccess;
    const float inv2ss = 1.0f / (2.0f * sigma_s * sigma_s);
    if (f16)
        hipLaunchKernelGGL(k_bilateral<true>, dim3((n + 255) / 256), dim3(256), 0, s, iw, w, h,
                           radius, inv2ss, 1.0f / sigma_I, 1.0f / rel_W, Io, Wo);
    else
        hipLaunchKernelGGL(k_bilateral<false>, dim3((n + 255) / 256), dim3(256), 0, s, iw, w, h,
                           radius, inv2ss, 1.0f / sigma_I, 1.0f / rel_W, Io, Wo);
    return hipGetLastError();
}

}  // namespace rgbid
