// Sensor input path (sec. 4.1, 4.2, 5.1, 5.2): depth correction of the raw
// depth, undistortion by inverse warping, and forward registration of the
// inverse depth into the colour camera (translation splat with an atomic
// maximum, then the rotation as a nearest-neighbour inverse warp).
//
//   k_undistort<DEPTH>     one image through the Brown model (sec. 5.1)
//   k_splat<RAW>           registration step 1 (eq:register_trans); RAW fuses
//                          the depth correction and the depth-lens
//                          undistortion into the source read, so the
//                          corrected and undistorted maps never reach memory
//   k_rotate<INTENSITY>    registration step 2; INTENSITY also undistorts the
//                          colour image on the same grid
//
// All arithmetic is FP32.  Memory-bound: per depth pixel about four raw taps
// (cached) and one or a few 4-byte atomics; per colour pixel one gathered
// B_t read, four intensity taps (cached) and two 4-byte writes.
#include <hip/hip_runtime.h>

#include "rgbid_internal.h"

namespace rgbid {
namespace {

__device__ __forceinline__ bool valid_wf(float w) { return w > 0.0f && w < 3.0e38f; }

// Pixel (u, v) of a lens through the distortion model: the sample position
// K h(K^-1 p) in the distorted image, formed as p + f (h(m) - m) so that a
// lens without distortion maps every pixel exactly onto itself.
__device__ __forceinline__ void distorted_position(const LensF& L, int u, int v, float& x, float& y)
{
    const float mx = ((float)u - L.cx) / L.fx, my = ((float)v - L.cy) / L.fy;
    const float r2 = mx * mx + my * my;
    const float rad = r2 * (L.k[0] + r2 * (L.k[1] + r2 * L.k[4]));
    const float xd = (1.0f + rad) * mx + 2.0f * L.k[2] * mx * my + L.k[3] * (r2 + 2.0f * mx * mx);
    const float yd = (1.0f + rad) * my + 2.0f * L.k[3] * mx * my + L.k[2] * (r2 + 2.0f * my * my);
    x = (float)u + L.fx * (xd - mx);
    y = (float)v + L.fy * (yd - my);
}

// Bilinear taps with the sampler's rules: bounds -0.5 <= x < w - 0.5 (same
// in y), taps clamped to the image.
struct Taps {
    int x0, x1, y0, y1;
    float a, b;
};

__device__ __forceinline__ bool taps_of(int w, int h, float x, float y, Taps& T)
{
    if (!(x >= -0.5f && x < (float)w - 0.5f && y >= -0.5f && y < (float)h - 0.5f)) return false;
    const float fx0 = floorf(x), fy0 = floorf(y);
    T.a = x - fx0;
    T.b = y - fy0;
    const int xf = (int)fx0, yf = (int)fy0;
    T.x0 = max(xf, 0);
    T.y0 = max(yf, 0);
    T.x1 = min(xf + 1, w - 1);
    T.y1 = min(yf + 1, h - 1);
    return true;
}

__device__ __forceinline__ float lerp4(const Taps& T, float v00, float v10, float v01, float v11)
{
    return (1.0f - T.a) * (1.0f - T.b) * v00 + T.a * (1.0f - T.b) * v10 +
           (1.0f - T.a) * T.b * v01 + T.a * T.b * v11;
}

// Nine-term polynomial of the spatial depth correction in m = K^-1 p.
__device__ __forceinline__ float depth_poly(const float q[9], float mx, float my)
{
    const float r2 = mx * mx + my * my;
    return q[0] + r2 * (q[1] + r2 * (q[2] + r2 * q[3])) + q[4] * mx + q[5] * my +
           mx * my * (q[6] + q[7] * mx + q[8] * my);
}

// Corrected inverse depth W_u at the integer pixel (x, y) of the raw grid:
// W_d = beta1 / Z_m(p - p0) + beta0, then W_u = D1 W_d + D0 (sec. 4.1).
__device__ __forceinline__ float corrected_w(const float* Z, long long pitch, const LensF& L,
                                             const DepthCorrF& D, int x, int y)
{
    const int xs = x - D.p0x, ys = y - D.p0y;
    if (xs < 0 || xs >= L.w || ys < 0 || ys >= L.h) return 0.0f;
    const float z = Z[(long long)ys * pitch + xs];
    if (!valid_wf(z)) return 0.0f;
    float W = D.beta1 * (1.0f / z) + D.beta0;
    if (D.spatial) {
        const float mx = ((float)x - L.cx) / L.fx, my = ((float)y - L.cy) / L.fy;
        W = depth_poly(D.q1, mx, my) * W + depth_poly(D.q0, mx, my);
    }
    return valid_wf(W) ? W : 0.0f;
}

template <bool DEPTH>
__global__ void __launch_bounds__(256) k_undistort(const float* src, long long pitch, LensF L,
                                                   float* dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.w * L.h) return;
    const int v = i / L.w, u = i - v * L.w;
    float x, y;
    distorted_position(L, u, v, x, y);
    Taps T;
    float out = 0.0f;
    if (taps_of(L.w, L.h, x, y, T)) {
        const float v00 = src[(long long)T.y0 * pitch + T.x0], v10 = src[(long long)T.y0 * pitch + T.x1];
        const float v01 = src[(long long)T.y1 * pitch + T.x0], v11 = src[(long long)T.y1 * pitch + T.x1];
        if (!DEPTH || (valid_wf(v00) && valid_wf(v10) && valid_wf(v01) && valid_wf(v11)))
            out = lerp4(T, v00, v10, v01, v11);
        if (DEPTH && !valid_wf(out)) out = 0.0f;
    }
    dst[i] = out;
}

// Registration step 1 from every source pixel (u, v) of camera A.  RAW: the
// source value is the corrected raw depth undistorted through the depth lens
// (four corrected taps, all valid); otherwise W_A itself.
template <bool RAW>
__global__ void __launch_bounds__(256) k_splat(const float* src, long long pitch, LensF A,
                                               DepthCorrF D, float tx, float ty, float tz,
                                               unsigned* Wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.w * A.h) return;
    const int v = i / A.w, u = i - v * A.w;
    float W = 0.0f;
    if constexpr (RAW) {
        float x, y;
        distorted_position(A, u, v, x, y);
        Taps T;
        if (taps_of(A.w, A.h, x, y, T)) {
            const float v00 = corrected_w(src, pitch, A, D, T.x0, T.y0);
            const float v10 = corrected_w(src, pitch, A, D, T.x1, T.y0);
            const float v01 = corrected_w(src, pitch, A, D, T.x0, T.y1);
            const float v11 = corrected_w(src, pitch, A, D, T.x1, T.y1);
            if (valid_wf(v00) && valid_wf(v10) && valid_wf(v01) && valid_wf(v11))
                W = lerp4(T, v00, v10, v01, v11);
        }
    } else {
        W = src[(long long)v * pitch + u];
    }
    if (!valid_wf(W)) return;
    const float den = 1.0f - W * tz;
    if (!(den > 0.0f)) return;
    const float wt = W / den;
    if (!valid_wf(wt)) return;
    const float x = ((float)u - W * tx) / den, y = ((float)v - W * ty) / den;
    const float half = 0.5f / den;
    // pixels whose centres lie in [x - half, x + half) x [y - half, y + half)
    const float fx0 = fmaxf(ceilf(x - half), 0.0f), fx1 = fminf(ceilf(x + half) - 1.0f, (float)(A.w - 1));
    const float fy0 = fmaxf(ceilf(y - half), 0.0f), fy1 = fminf(ceilf(y + half) - 1.0f, (float)(A.h - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    const int qx0 = (int)fx0, qx1 = (int)fx1, qy0 = (int)fy0, qy1 = (int)fy1;
    const unsigned bits = __float_as_uint(wt);   // positive floats order as their bits
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) atomicMax(&Wt[qy * A.w + qx], bits);
}

// Registration step 2 into camera B: d = R~_AB p, nearest B_t pixel,
// W_B = W_Bt d_z.  INTENSITY: also the undistorted colour image on B's grid.
template <bool INTENSITY>
__global__ void __launch_bounds__(256) k_rotate(const float* Wt, LensF A, LensF B, RotF R,
                                                const float* Iraw, long long pitchI, float* Wout,
                                                float* Iout)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B.w * B.h) return;
    const int v = i / B.w, u = i - v * B.w;
    const float mx = ((float)u - B.cx) / B.fx, my = ((float)v - B.cy) / B.fy;
    const float rx = R.m[0] * mx + R.m[1] * my + R.m[2];
    const float ry = R.m[3] * mx + R.m[4] * my + R.m[5];
    const float rz = R.m[6] * mx + R.m[7] * my + R.m[8];
    float out = 0.0f;
    if (rz > 0.0f) {
        const float x = (A.fx * rx + A.cx * rz) / rz, y = (A.fy * ry + A.cy * rz) / rz;
        const float qx = floorf(x + 0.5f), qy = floorf(y + 0.5f);
        if (qx >= 0.0f && qx <= (float)(A.w - 1) && qy >= 0.0f && qy <= (float)(A.h - 1)) {
            const float wt = Wt[(int)qy * A.w + (int)qx];
            if (valid_wf(wt)) out = wt * rz;
        }
    }
    Wout[i] = valid_wf(out) ? out : 0.0f;
    if constexpr (INTENSITY) {
        float x, y;
        distorted_position(B, u, v, x, y);
        Taps T;
        float o = 0.0f;
        if (taps_of(B.w, B.h, x, y, T))
            o = lerp4(T, Iraw[(long long)T.y0 * pitchI + T.x0], Iraw[(long long)T.y0 * pitchI + T.x1],
                      Iraw[(long long)T.y1 * pitchI + T.x0], Iraw[(long long)T.y1 * pitchI + T.x1]);
        Iout[i] = o;
    }
}

__global__ void __launch_bounds__(256) k_zero(unsigned* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

inline int blocks(int n) { return (n + 255) / 256; }

}  // namespace

hipError_t launch_undistort(hipStream_t s, const float* src, long long pitch, const LensF& L,
                            int is_depth, float* dst)
{
    const int n = L.w * L.h;
    if (is_depth)
        hipLaunchKernelGGL(k_undistort<true>, dim3(blocks(n)), dim3(256), 0, s, src, pitch, L, dst);
    else
        hipLaunchKernelGGL(k_undistort<false>, dim3(blocks(n)), dim3(256), 0, s, src, pitch, L, dst);
    return hipGetLastError();
}

hipError_t launch_register(hipStream_t s, const RegisterArgs& a)
{
    const int na = a.A.w * a.A.h, nb = a.B.w * a.B.h;
    hipLaunchKernelGGL(k_zero, dim3(blocks(na)), dim3(256), 0, s, a.Wt, na);
    if (a.raw)
        hipLaunchKernelGGL(k_splat<true>, dim3(blocks(na)), dim3(256), 0, s, a.src, a.pitch, a.A,
                           a.D, a.tx, a.ty, a.tz, a.Wt);
    else
        hipLaunchKernelGGL(k_splat<false>, dim3(blocks(na)), dim3(256), 0, s, a.src, a.pitch, a.A,
                           a.D, a.tx, a.ty, a.tz, a.Wt);
    const float* Wt = reinterpret_cast<const float*>(a.Wt);
    if (a.Iraw)
        hipLaunchKernelGGL(k_rotate<true>, dim3(blocks(nb)), dim3(256), 0, s, Wt, a.A, a.B, a.R,
                           a.Iraw, a.pitchI, a.Wout, a.Iout);
    else
        hipLaunchKernelGGL(k_rotate<false>, dim3(blocks(nb)), dim3(256), 0, s, Wt, a.A, a.B, a.R,
                           a.Iraw, a.pitchI, a.Wout, a.Iout);
    return hipGetLastError();
}

}  // namespace rgbid
