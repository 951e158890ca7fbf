// One Gauss-Newton / IRLS iteration of dense RGB-D alignment in inverse-depth
// parametrisation (sec. 6.2), for a batch of frame pairs at one pyramid level.
//
//   k_warp    inverse geometric warp of {I_B, W_B} towards A (sec. 5.3) and,
//             in FULLRES mode, the downsampling of the warped images to the
//             level (sec. 6.2); writes the residuals of the systematic sample
//             (sec. 6.3) and, in store mode, the warped level images.
//   k_scale   location / scale fixed point and the nu bisection of sec. 6.3
//             on the sample, one workgroup per (pair, channel).
//   k_reduce  residuals, Jacobians (eq:res_int, eq:res_depth, eq:DeltaX),
//             lambda_n and robust weights; reduction of the 21 + 6 normal-
//             equation terms (2eq:minimisationIRLS) into per-chunk compensated
//             FP32 partials.
//   k_solve   FP64 cross-chunk sum, 6x6 Cholesky and the update
//             T <- exp(xi)^-1 T with the decoupled exponential (sec. 3).
//
// Pixel work is organised in tiles of 64 consecutive pixels (raster order)
// of a level grid; a workgroup walks a chunk of tiles of one pair.  In FULLRES
// mode a level-l pixel has 4^l full-resolution children: the lanes of a
// wavefront split the children, reduce them with cross-lane shuffles, and in
// the end every lane owns one level-l pixel.
#include "rgbid_internal.h"
#include <type_traits>

namespace rgbid {
namespace {

__device__ __forceinline__ bool w_valid(float w) { return w > 0.0f && w < INFINITY; }

// Image and workspace pointers reach the kernels through tables in memory, so
// the compiler cannot tell they are global; these casts let it emit global
// (not flat) loads and stores, which do not hold up scalar loads.
#define RGBID_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const RGBID_GLOBAL T* gconst(const void* p)
{
    return (const RGBID_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ RGBID_GLOBAL T* gmut(void* p)
{
    return (RGBID_GLOBAL T*)p;
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

// Element i of a global array given a 32-bit element index: the byte offset
// is formed in 32 bits (every image is far below 4 GiB), so the load takes
// the uniform base from scalar registers and a 32-bit lane offset.
template <typename T>
__device__ __forceinline__ T ld_at(const void* base, unsigned i)
{
    const unsigned off = i * (unsigned)sizeof(T);
    return *(const RGBID_GLOBAL T*)((const RGBID_GLOBAL char*)base + off);
}

template <bool F16>
__device__ __forceinline__ float2 load_iw(const void* p, unsigned i)
{
    if constexpr (F16) {
        const h2v h = ld_at<h2v>(p, i);
        return make_float2((float)h.x, (float)h.y);
    } else {
        const f2v f = ld_at<f2v>(p, i);
        return make_float2(f.x, f.y);
    }
}

// (I, W) texel at byte offset off of an interleaved plane.
template <bool F16>
__device__ __forceinline__ float2 load_iw_at(const void* p, unsigned off)
{
    const RGBID_GLOBAL char* b = (const RGBID_GLOBAL char*)p + off;
    if constexpr (F16) {
        const h2v h = *(const RGBID_GLOBAL h2v*)b;
        return make_float2((float)h.x, (float)h.y);
    } else {
        const f2v f = *(const RGBID_GLOBAL f2v*)b;
        return make_float2(f.x, f.y);
    }
}

// Two consecutive (I, W) texels at byte offset off.
template <bool F16>
__device__ __forceinline__ void load_iw2_at(const void* p, unsigned off, float2& t0, float2& t1)
{
    const RGBID_GLOBAL char* b = (const RGBID_GLOBAL char*)p + off;
    if constexpr (F16) {
        typedef _Float16 h4v __attribute__((ext_vector_type(4)));
        const h4v h = *(const RGBID_GLOBAL h4v*)b;
        t0 = make_float2((float)h.x, (float)h.y);
        t1 = make_float2((float)h.z, (float)h.w);
    } else {
        typedef float f4v __attribute__((ext_vector_type(4)));
        const f4v f = *(const RGBID_GLOBAL f4v*)b;
        t0 = make_float2(f.x, f.y);
        t1 = make_float2(f.z, f.w);
    }
}

// floor(x) as an integer (v_cvt_flr_i32_f32) for |x| < 2^31.
__device__ __forceinline__ int floor_i(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

template <bool F16>
__device__ __forceinline__ float load_w(const void* p, unsigned i)
{
    if constexpr (F16) return (float)ld_at<_Float16>(p, i);
    else return ld_at<float>(p, i);
}

__device__ __forceinline__ float2 load_f2(const void* p, size_t i)
{
    const f2v f = gconst<f2v>(p)[i];
    return make_float2(f.x, f.y);
}

__device__ __forceinline__ void store_f2(void* p, size_t i, float a, float b)
{
    f2v v;
    v.x = a;
    v.y = b;
    gmut<f2v>(p)[i] = v;
}

// Row / column of raster index idx in a grid of width gw, with inv_gw =
// 1/gw and half_inv = 1/(2 gw): the row is floor((idx + 1/2) / gw) formed in
// FP32, whose fraction stays 1/(2 gw) away from an integer, more than the
// rounding error for idx < 2^22.
__device__ __forceinline__ void split_index(int idx, int gw, float inv_gw, float half_inv, int& gu,
                                            int& gv)
{
    const int v = (int)fmaf((float)idx, inv_gw, half_inv);
    gu = idx - (int)__umul24((unsigned)v, (unsigned)gw);
    gv = v;
}

__device__ __forceinline__ int chunk_of_block(int b, int n, int remap)
{
    if (!remap) return b;
    // Consecutive chunks on one XCD: XCD x = b % 8 runs a contiguous range.
    const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

// A value every lane holds alike, moved to a scalar register.
__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Reciprocal and reciprocal square root (v_rcp_f32 / v_rsq_f32, 1 ulp) for
// the per-pixel path.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Grid of a level for the pixel kernels: the full level grid, or the sample
// grid (every s-th pixel in both directions).
struct GridDim {
    int gw, n, gs;
    float inv_gw, half_inv;
};

__device__ __forceinline__ GridDim level_grid(const LevelView& A)
{
    GridDim d;
    d.gw = A.w;
    d.n = A.w * A.h;
    d.gs = 1;
    d.inv_gw = uniform_f(1.0f / (float)A.w);
    d.half_inv = uniform_f(0.5f * d.inv_gw);
    return d;
}

__device__ __forceinline__ GridDim sample_grid(const PairDesc& D, int l)
{
    GridDim d;
    d.gw = D.sw[l];
    d.n = D.sw[l] * D.sh[l];
    d.gs = D.stride[l];
    d.inv_gw = uniform_f(1.0f / (float)D.sw[l]);
    d.half_inv = uniform_f(0.5f * d.inv_gw);
    return d;
}

// Pixel rays of a level: x = K^-1 (u, v, 1) = (u/fx - cx/fx, v/fy - cy/fy, 1),
// and half the focal lengths for the central-difference gradients.
struct LevelRay {
    float ifx, ify, ncx, ncy, hfx, hfy;
};

__device__ __forceinline__ LevelRay level_ray(const LevelView& A)
{
    LevelRay R;
    R.ifx = uniform_f(1.0f / A.fx);
    R.ify = uniform_f(1.0f / A.fy);
    R.ncx = uniform_f(-A.cx * R.ifx);
    R.ncy = uniform_f(-A.cy * R.ify);
    R.hfx = 0.5f * A.fx;
    R.hfy = 0.5f * A.fy;
    return R;
}

__device__ __forceinline__ float ray_x(const LevelRay& R, int u) { return fmaf((float)u, R.ifx, R.ncx); }
__device__ __forceinline__ float ray_y(const LevelRay& R, int v) { return fmaf((float)v, R.ify, R.ncy); }

// Warp parameters of one pair at the warp level.  The first two rows of R^T
// are scaled by fx and fy: a ray x maps to a = (fx (R^T x)_x, fy (R^T x)_y,
// (R^T x)_z), and with q = (fx (R^T t)_x, fy (R^T t)_y, (R^T t)_z) the point
// W_A R^T (x / W_A - t) projects to (cx + (a_x - W_A q_x) / z,
// cy + (a_y - W_A q_y) / z), z = a_z - W_A q_z.  su, sv: the change of a per
// pixel step in u and in v.
struct Geom {
    float m[9];
    float q[3];
    float su[3], sv[3];
    float cx, cy, ulim, vlim;   // ulim = w - 1/2, vlim = h - 1/2
    LevelRay ray;
    int w, h;
    unsigned texb, rowb;        // bytes per texel and per row of B's (I, W) plane
    const void* WA;   // W plane of A at the warp level
    const void* Biw;  // interleaved (I, W) of B at the warp level
};

template <bool F16>
__device__ __forceinline__ Geom make_geom(const PairState& S, const LevelView& A, const LevelView& B)
{
    Geom G;
    G.ray = level_ray(A);
    const float sc[3] = {A.fx, A.fy, 1.0f};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) G.m[3 * r + c] = uniform_f(sc[r] * S.RT[3 * r + c]);
        G.q[r] = uniform_f(sc[r] * S.Rtt[r]);
        G.su[r] = uniform_f(G.m[3 * r] * G.ray.ifx);
        G.sv[r] = uniform_f(G.m[3 * r + 1] * G.ray.ify);
    }
    G.cx = A.cx;
    G.cy = A.cy;
    G.ulim = uniform_f((float)A.w - 0.5f);
    G.vlim = uniform_f((float)A.h - 0.5f);
    G.w = A.w;
    G.h = A.h;
    G.texb = F16 ? 4u : 8u;
    G.rowb = G.texb * (unsigned)A.w;
    G.WA = A.wp;
    G.Biw = B.iw;
    return G;
}

struct Ray3 {
    float x, y, z;
};

__device__ __forceinline__ Ray3 rotate_ray(const Geom& G, float xu, float xv)
{
    Ray3 a;
    a.x = fmaf(G.m[0], xu, fmaf(G.m[1], xv, G.m[2]));
    a.y = fmaf(G.m[3], xu, fmaf(G.m[4], xv, G.m[5]));
    a.z = fmaf(G.m[6], xu, fmaf(G.m[7], xv, G.m[8]));
    return a;
}

// Inverse geometric warp of one pixel of A (sec. 5.3) from its rotated ray a
// and w_a = W_A at the pixel.  I* is the bilinear I_B at the projection p_B
// and W* = (R^T x)_z w_b / (1 + w_b (R^T t)_z) with w_b the bilinear W_B.
// Valid iff w_a valid, in front, p_B in [-0.5, w-0.5) x [-0.5, h-0.5), four
// valid W taps and W* positive and finite; I* and W* are undefined otherwise.
// Branch-free: the four taps are always loaded (at in-bounds addresses).
// Split in two phases so that a lane can issue the tap loads of all its
// pixels before it consumes any of them.
//
// Taps at the image edge.  The taps are x0 = floor(u_B) and x0 + 1 (rows
// likewise), each clamped to the image; a clamped second tap is the first
// one, so the interpolation along that axis returns the first tap.  Instead
// of copying the first tap over the second, the second is loaded unclamped
// (one texel on, or one row on: the next row's first texel, or the zero
// guard row or texel after the plane) and the interpolation weight along that
// axis is set to 0: fma(0, t1 - t0, t0) = t0 exactly for finite texels
// (intensities are finite; W is stored finite in FP32, and in FP16 an unused
// second tap's W is replaced), and the second tap's validity is not asked
// for.
struct WarpTaps {
    float2 p00, p10, p01, p11;
    float a, b, az;
    bool ok, dx, dy;   // dx, dy: the second tap along u, v is one texel on
};

template <bool F16>
__device__ __forceinline__ void warp_fetch(const Geom& G, const Ray3& a, float wa, WarpTaps& T)
{
    const float yx = fmaf(-wa, G.q[0], a.x), yy = fmaf(-wa, G.q[1], a.y);
    const float yz = fmaf(-wa, G.q[2], a.z);
    const float iz = rcp(yz);
    float ub = fmaf(yx, iz, G.cx), vb = fmaf(yy, iz, G.cy);
    const bool ok = (int)w_valid(wa) & (yz > 0.0f) & (ub >= -0.5f) & (ub < G.ulim) &
                    (vb >= -0.5f) & (vb < G.vlim);
    ub = ok ? ub : 0.0f;
    vb = ok ? vb : 0.0f;
    // x0 = floor(u_B) >= -1 in bounds; the second tap is one texel on iff
    // 0 <= x0 < w - 1
    const int xf = floor_i(ub), yf = floor_i(vb);
    const unsigned x0 = (unsigned)max(xf, 0), y0 = (unsigned)max(yf, 0);
    T.dx = (unsigned)xf < (unsigned)(G.w - 1);
    T.dy = (unsigned)yf < (unsigned)(G.h - 1);
    T.a = T.dx ? __builtin_amdgcn_fractf(ub) : 0.0f;
    T.b = T.dy ? __builtin_amdgcn_fractf(vb) : 0.0f;
    T.az = a.z;
    T.ok = ok;
    // both taps of a row in one load, the second row from a base one row on
    // (the texel after the last row's last texel is still guard)
    const unsigned o00 = __umul24(y0, G.rowb) + x0 * G.texb;
    load_iw2_at<F16>(G.Biw, o00, T.p00, T.p10);
    load_iw2_at<F16>(static_cast<const char*>(G.Biw) + G.rowb, o00, T.p01, T.p11);
    if constexpr (F16) {
        // an inverse depth beyond the half range is stored as inf: the W of
        // an unused second tap is the first tap's, so no inf meets a weight 0
        T.p10.y = T.dx ? T.p10.y : T.p00.y;
        T.p11.y = T.dx ? T.p11.y : T.p01.y;
        T.p01.y = T.dy ? T.p01.y : T.p00.y;
        T.p11.y = T.dy ? T.p11.y : T.p10.y;
    }
}

__device__ __forceinline__ bool warp_finish(const Geom& G, const WarpTaps& T, float& Io, float& Wo)
{
    const bool ok = T.ok & (int)w_valid(T.p00.y) & ((int)w_valid(T.p10.y) | !T.dx) &
                    ((int)w_valid(T.p01.y) | !T.dy) & ((int)w_valid(T.p11.y) | !(T.dx & T.dy));
    // bilinear: along u on both rows, then along v
    const float i0 = fmaf(T.a, T.p10.x - T.p00.x, T.p00.x);
    const float i1 = fmaf(T.a, T.p11.x - T.p01.x, T.p01.x);
    const float w0 = fmaf(T.a, T.p10.y - T.p00.y, T.p00.y);
    const float w1 = fmaf(T.a, T.p11.y - T.p01.y, T.p01.y);
    const float wb = fmaf(T.b, w1 - w0, w0);
    Io = fmaf(T.b, i1 - i0, i0);
    Wo = T.az * wb * rcp(fmaf(wb, G.q[2], 1.0f));
    return ok & (int)w_valid(Wo);
}

// Sum over aligned groups of LPP lanes (a power of two), the same in every
// lane of the group, added in a fixed tree: pairs, quads (DPP quad_perm),
// eights (row_half_mirror), rows of 16 (row_mirror), then shuffles.
#define RGBID_DPP_MOV(v, ctrl) \
    __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xf, 0xf, true))

template <int LPP>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (LPP >= 2) v += RGBID_DPP_MOV(v, 0xb1);    // quad_perm [1,0,3,2]
    if constexpr (LPP >= 4) v += RGBID_DPP_MOV(v, 0x4e);    // quad_perm [2,3,0,1]
    if constexpr (LPP >= 8) v += RGBID_DPP_MOV(v, 0x141);   // row_half_mirror
    if constexpr (LPP >= 16) v += RGBID_DPP_MOV(v, 0x140);  // row_mirror
    if constexpr (LPP >= 32) v += __shfl_xor(v, 16);
    if constexpr (LPP >= 64) v += __shfl_xor(v, 32);
    return v;
}

// Lane layout of the children of level pixels: a level pixel has C = 4^LOG2B
// children at the warp level; each lane warps CPL of them (1, 2, 4 or 8 by
// level: independent load chains per lane), LPP = C / CPL lanes share one pixel and
// combine their sums across lanes, and GPP = 64 / LPP pixels are warped per
// pass.  Lane j of a group takes children c = j + LPP m (m < CPL), child c at
// offset (c % B, c / B) from the pixel's first child; du(m), dv(m) are the
// offsets of the lane's m-th child from its first.
template <int LOG2B>
struct ChildLayout {
    static constexpr int B = 1 << LOG2B;
    static constexpr int C = B * B;
    static constexpr int CPL = warp_children_per_lane(LOG2B);   // children per lane
    static constexpr int LPP = warp_lanes_per_pixel(LOG2B);     // lanes per pixel
    static constexpr int GPP = warp_pixels_per_pass(LOG2B);     // pixels per pass
    static_assert(CPL * LPP == C && LPP <= 64, "at most 64 lanes per level pixel");
    static_assert(LPP % B == 0 || B % LPP == 0, "children rows split evenly over lanes");
    static constexpr int du(int m)
    {
        if constexpr (LPP >= B) return 0;
        else return LPP * (m % (B / LPP));
    }
    static constexpr int dv(int m)
    {
        if constexpr (LPP >= B) return (LPP / B) * m;
        else return m / (B / LPP);
    }
};

// Grid position of the pixel of lane group g in the pass that starts at grid
// pixel `first`; past the grid end the position of the last pixel (so that
// every derived address stays in bounds).
struct PassPos {
    int idx, gu, gv;
};

__device__ __forceinline__ PassPos pass_pos(int first, int g, const GridDim& gd)
{
    PassPos p;
    p.idx = first + g;
    split_index(min(p.idx, gd.n - 1), gd.gw, gd.inv_gw, gd.half_inv, p.gu, p.gv);
    return p;
}

// The ray of the lane's first child and the W_A of all its children (loaded
// ahead so the next pass's loads overlap this pass's gathers).
template <int CPL>
struct PassChildren {
    float xu, xv;
    float wa[CPL];
};

template <bool F16, int LOG2B>
__device__ __forceinline__ PassChildren<ChildLayout<LOG2B>::CPL>
pass_children(const Geom& G, const PassPos& p, int gs, int lane, bool load_wa = true)
{
    using CL = ChildLayout<LOG2B>;
    PassChildren<CL::CPL> pc;
    const int j = lane % CL::LPP;
    const int u0 = (int)__umul24(p.gu, gs * CL::B) + j % CL::B;
    const int v0 = (int)__umul24(p.gv, gs * CL::B) + j / CL::B;
    pc.xu = ray_x(G.ray, u0);
    pc.xv = ray_y(G.ray, v0);
    const unsigned i0 = __umul24(v0, G.w) + u0;
#pragma unroll
    for (int m = 0; m < CL::CPL; ++m)
        pc.wa[m] = load_wa ? load_w<F16>(G.WA, i0 + CL::dv(m) * G.w + CL::du(m)) : 0.0f;
    return pc;
}

// One pass: every lane of group g returns the mean warped values of its pixel
// and whether the pixel is inside the grid (`in`) with all its children
// warp-valid (the strict downsampling rule).  The means are undefined for an
// invalid pixel.
template <bool F16, int LOG2B>
__device__ __forceinline__ void warp_pass(const Geom& G, const PassChildren<ChildLayout<LOG2B>::CPL>& pc,
                                          bool in, int lane, float& Io, float& Wo, bool& Vo)
{
    using CL = ChildLayout<LOG2B>;
    const Ray3 a0 = rotate_ray(G, pc.xu, pc.xv);
    // every child's tap loads first, then the arithmetic on them
    WarpTaps T[CL::CPL];
#pragma unroll
    for (int m = 0; m < CL::CPL; ++m) {
        Ray3 a = a0;
        if (CL::du(m) != 0) {
            const float d = (float)CL::du(m);
            a.x = fmaf(d, G.su[0], a.x);
            a.y = fmaf(d, G.su[1], a.y);
            a.z = fmaf(d, G.su[2], a.z);
        }
        if (CL::dv(m) != 0) {
            const float d = (float)CL::dv(m);
            a.x = fmaf(d, G.sv[0], a.x);
            a.y = fmaf(d, G.sv[1], a.y);
            a.z = fmaf(d, G.sv[2], a.z);
        }
        warp_fetch<F16>(G, a, pc.wa[m], T[m]);
    }
    bool ok = in;
    float sI, sW;
#pragma unroll
    for (int m = 0; m < CL::CPL; ++m) {
        float ci, cw;
        ok = ok & warp_finish(G, T[m], ci, cw);
        sI = m == 0 ? ci : sI + ci;
        sW = m == 0 ? cw : sW + cw;
    }
    sI = group_sum<CL::LPP>(sI);
    sW = group_sum<CL::LPP>(sW);
    bool gvalid = ok;
    if constexpr (CL::LPP > 1) {
        const int g = lane / CL::LPP;
        const unsigned long long bal = __ballot(ok);
        const unsigned long long full =
            CL::LPP == 64 ? ~0ull : ((1ull << CL::LPP) - 1ull) << (unsigned)(g * CL::LPP);
        gvalid = (bal & full) == full;
    }
    constexpr float invC = 1.0f / (float)CL::C;
    Io = sI * invC;
    Wo = sW * invC;
    Vo = gvalid;
}

// A tile of 64 consecutive grid pixels in LPP passes; afterwards lane L owns
// the tile pixel q = (L % LPP) * GPP + L / LPP, at level coordinates (uo, vo).
template <bool F16, int LOG2B>
__device__ __forceinline__ void warp_tile(const Geom& G, int tile_first, const GridDim& gd,
                                          int lane, float& Io, float& Wo, bool& Vo, int& uo,
                                          int& vo, int& idxo)
{
    using CL = ChildLayout<LOG2B>;
    const int j = lane % CL::LPP, g = lane / CL::LPP;
    float mI = 0.0f, mW = 0.0f;
    bool mV = false;
    PassPos own;
#pragma unroll 1
    for (int k = 0; k < CL::LPP; ++k) {
        const PassPos p = pass_pos(tile_first + k * CL::GPP, g, gd);
        const auto pc = pass_children<F16, LOG2B>(G, p, gd.gs, lane);
        float pI, pW;
        bool pV;
        warp_pass<F16, LOG2B>(G, pc, p.idx < gd.n, lane, pI, pW, pV);
        if (j == k) {
            mI = pI;
            mW = pW;
            mV = pV;
        }
        if constexpr (CL::LPP == 1) own = p;
    }
    if constexpr (CL::LPP > 1) own = pass_pos(tile_first + j * CL::GPP, g, gd);
    idxo = own.idx;
    uo = (int)__umul24(own.gu, gd.gs);
    vo = (int)__umul24(own.gv, gd.gs);
    Io = mI;
    Wo = mW;
    Vo = mV;
}

// Residuals of one level pixel (sec. 6.2) and whether they are defined: r_I
// needs an interior pixel, a valid W_A and warped values; r_W additionally
// the four W_A neighbours (central-difference gradient).
struct Terms {
    bool vI, vW;
    float rI, rW;
};

struct Nbrs {
    float2 l, r, t, b;
};

// The four neighbours of pixel i of A, read at the pixel's own byte offset
// from shifted bases.  Every (I, W) plane of a pyramid has a guard of one row
// and one texel (zeros) before and after it inside its allocation, so the
// reads of border pixels (which take no part: their flags say so) stay in
// bounds without clamping, and the four reads share the centre's address.
template <bool F16>
__device__ __forceinline__ Nbrs load_nbrs(const LevelView& A, unsigned i)
{
    constexpr unsigned tb = F16 ? 4u : 8u;
    const unsigned off = i * tb, rowb = tb * (unsigned)A.w;
    const char* base = static_cast<const char*>(A.iw);
    Nbrs n;
    n.l = load_iw_at<F16>(base - tb, off);
    n.r = load_iw_at<F16>(base + tb, off);
    n.t = load_iw_at<F16>(base - rowb, off);
    n.b = load_iw_at<F16>(base + rowb, off);
    return n;
}

__device__ __forceinline__ unsigned load_mask(const LevelView& A, unsigned i)
{
    return ld_at<unsigned char>(A.gm, i);
}

// Residuals of one level pixel (sec. 6.2): c = A's (I, W) at the pixel and m
// its validity flags (bit 0: interior with valid W, bit 1: also the W
// gradient defined): r_I needs the warp and bit 0, r_W the warp and bit 1.
__device__ __forceinline__ void residuals(float2 c, unsigned m, float Is, float Ws, bool wv,
                                          Terms& T)
{
    T.vI = wv & ((m & 1u) != 0u);
    T.vW = wv & ((m & 2u) != 0u);
    T.rI = Is - c.x;
    T.rW = Ws - c.y;
}

// Robust weighting of one iteration, folded for the per-pixel code.  With
// d = r - mu and x = d / sigma, the square-rooted weight over sigma is
//   Huber      sqrt(w) / sigma = min(1, sqrt(k / |x|)) / sigma
//                              = min(1 / sigma, a rsqrt|d|),   a = sqrt(k / sigma);
//   Student-t  sqrt(w) / sigma = sqrt((nu + 1) / (nu + x^2)) / sigma
//                              = a rsqrt(d^2 + c),  a = sqrt(nu + 1), c = nu sigma^2
// (sec. 6.3).  A channel with an empty sample takes no part.
struct RobustF {
    float muI, isI, aI, cI;
    float muW, isW, aW, cW;
    unsigned mI, mW;   // flag bit each channel needs (0: the channel takes no part)
};

__device__ __forceinline__ RobustF robust_f(const IterLaunch& L, const PairState& S)
{
    RobustF F;
    F.mI = S.ns[0] > 0 ? 1u : 0u;
    F.mW = S.ns[1] > 0 ? 2u : 0u;
    F.muI = S.mu[0];
    F.muW = S.mu[1];
    const float sgI = S.sigma[0], sgW = S.sigma[1];
    F.isI = 1.0f / sgI;
    F.isW = 1.0f / sgW;
    if (L.ip.weight == RGBID_W_HUBER) {
        F.aI = sqrtf(L.ip.huber_k * F.isI);
        F.aW = sqrtf(L.ip.huber_k * F.isW);
        F.cI = F.cW = 0.0f;
    } else {
        const float nuW = S.nu[1];
        const float nuI = L.ip.estimate_nu ? fmaxf(S.nu[0], nuW) : S.nu[0];
        F.aI = sqrtf(nuI + 1.0f);
        F.aW = sqrtf(nuW + 1.0f);
        F.cI = nuI * sgI * sgI;
        F.cW = nuW * sgW * sgW;
    }
    return F;
}

template <int KIND>
__device__ __forceinline__ float sqrt_weight(float d, float is, float a, float c)
{
    // Huber: min(is, a rsqrt|d|) as a median with 0 (both operands are >= 0;
    // fminf would re-canonicalise the loop-invariant is on every call)
    if constexpr (KIND == RGBID_W_HUBER) return __builtin_amdgcn_fmed3f(a * rsq(fabsf(d)), 0.0f, is);
    else return a * rsq(fmaf(d, d, c));
}

// The legacy multiply: 0 x anything (inf, NaN) = 0.
__device__ __forceinline__ float lmul(float a, float b)
{
    float r;
    asm("v_mul_legacy_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// The normal equations (2eq:minimisationIRLS) are the sums over pixels of
// w J J^T, w J r and w r^2: the upper blocks of the sum of the outer products
// of v = sqrt(w) (J_0 .. J_5, r, 0) with themselves, rows and columns 0-3
// (TL), rows 0-3 x columns 4-7 (TR) and rows and columns 4-7 (BR), a dense
// contraction over pixels that runs on the matrix cores.  Per tile a wave
// stages its 128 vectors (the I and W terms of 64 pixels) in LDS as two
// planes of float4, (v0, v4, v1, v5) and (v2, v6, v3, v7), each plane in
// vector order (a lane's stores are consecutive 16-byte words: no bank
// conflicts), and feeds them 16 at a time to v_mfma_f32_4x4x1_16b_f32: block
// b takes vector 16 q + b, lane 4 b + i supplying (v_i, v_4+i), and block b's
// 4x4 product accumulates in lanes 4 b + j, register i.
//
// Precision: the accumulators of a group of kNeGroupTiles tiles add at most
// 8 kNeGroupTiles terms per block in FP32; the group's 16 blocks are then
// added in order and the result joins a compensated (hi, lo) FP32 total
// (two-sum) per sum, in lanes 0..27; waves and chunks follow in (hi, lo)
// pairs and FP64.
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kStageFloat4PerWave = 256;   // 128 vectors x 8 floats
constexpr int kNeGroupTiles = 8;

// Where sum k of the 28 (H upper triangle row-major, g, cost) sits in the
// accumulators: entry (a, b), a <= b, of the 8 x 8 sum of v v^T (H is rows
// and columns 0-5, g column 6, the cost entry (6, 6)) is in register row
// 4 t + i (t = 0 TL, 1 TR, 2 BR; i = a mod 4) of lanes 4 b' + (b mod 4),
// coded 4 (4 t + i) + b mod 4.  Row a of H starts at k = a (13 - a) / 2.
// Formed from k (no table: a load in the loop would wait for every load in
// flight).
__device__ __forceinline__ unsigned ne_code(int k)
{
    int a, b;
    if (k < 21) {
        a = (k >= 6) + (k >= 11) + (k >= 15) + (k >= 18) + (k >= 20);
        b = k - a * (13 - a) / 2 + a;
    } else {
        a = min(k - 21, 6);
        b = 6;
    }
    const int t = b < 4 ? 0 : (a < 4 ? 1 : 2);
    return (unsigned)(4 * (4 * t + (a & 3)) + (b & 3));
}

struct NeAcc {
    v4f tl, tr, br;   // the current group's MFMA accumulators
    float hi, lo;     // lanes 0..27: compensated total of sum k = lane
    int tiles;        // tiles in the current group (uniform)
};

__device__ __forceinline__ void ne_init(NeAcc& na)
{
    na.tl = na.tr = na.br = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    na.hi = na.lo = 0.0f;
    na.tiles = 0;
}

// Knuth's two-sum: hi + lo + x = hi' + lo' with the rounding error of
// hi + x carried in lo.
__device__ __forceinline__ void two_sum_add(float& hi, float& lo, float x)
{
    const float s = hi + x;
    const float bp = s - hi;
    lo += (hi - (s - bp)) + (x - bp);
    hi = s;
}

// Ends a group: the 16 blocks of every sum are added in block order through
// the wave's staging area and the result joins (hi, lo); the accumulators
// restart from zero.
__device__ __forceinline__ void ne_flush(NeAcc& na, float4* st, int lane)
{
    float* sc = reinterpret_cast<float*>(st);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sc[(0 + r) * 64 + lane] = na.tl[r];
        sc[(4 + r) * 64 + lane] = na.tr[r];
        sc[(8 + r) * 64 + lane] = na.br[r];
    }
    if (lane < 28) {
        const unsigned c = ne_code(lane);
        const float* src = sc + (c >> 2) * 64 + (c & 3);
        float t = 0.0f;
#pragma unroll
        for (int b = 0; b < 16; ++b) t += src[4 * b];
        two_sum_add(na.hi, na.lo, t);
    }
    na.tl = na.tr = na.br = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    na.tiles = 0;
}

// The staged tile of the wave into the accumulators (the staging area is
// free again when this returns: LDS operations of a wave complete in order).
__device__ __forceinline__ void ne_feed(NeAcc& na, float4* st, int lane)
{
    // lane 4 b + i: plane i / 2, vector b (+ 16 q), half i % 2 of the float4
    const float2* rd = reinterpret_cast<const float2*>(st) + 256 * ((lane & 3) >> 1) +
                       2 * (lane >> 2) + (lane & 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float2 e = rd[32 * q];
        na.tl = __builtin_amdgcn_mfma_f32_4x4x1f32(e.x, e.x, na.tl, 0, 0, 0);
        na.tr = __builtin_amdgcn_mfma_f32_4x4x1f32(e.x, e.y, na.tr, 0, 0, 0);
        na.br = __builtin_amdgcn_mfma_f32_4x4x1f32(e.y, e.y, na.br, 0, 0, 0);
    }
    na.tiles = __builtin_amdgcn_readfirstlane(na.tiles + 1);
    if (na.tiles == kNeGroupTiles) ne_flush(na, st, lane);
}

// The wave's compensated totals of the 28 sums and the two counts into
// out[0 .. 29] (LDS, as (hi, lo) pairs); cI, cW are the lane's counts.
__device__ __forceinline__ void ne_wave_totals(NeAcc& na, float4* st, int lane, unsigned cI,
                                               unsigned cW, float2* out)
{
    if (na.tiles > 0) ne_flush(na, st, lane);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        cI += __shfl_xor(cI, o);
        cW += __shfl_xor(cW, o);
    }
    if (lane < 28) out[lane] = make_float2(na.hi, na.lo);
    else if (lane == 28) out[28] = make_float2((float)cI, 0.0f);
    else if (lane == 29) out[29] = make_float2((float)cW, 0.0f);
}

// The two staged vectors of one level pixel (sec. 6.2): v_I = sqrt(w_I)
// (J_I, r_I, 0) and v_W = sqrt(w_W) (J_W, r_W, 0), in the staging slots of
// lane `lane`.  The Jacobians of eq:res_int / eq:res_depth are formed in the
// ray x = (xu, xv, 1): with X = x / W_A, J = (a, X x a) = (a, x x (a / W_A)),
//   a_I = W_A (g_u, g_v, g_3),  g_3 = -(xu g_u + xv g_v),
//   a_W = W_A (k_u, k_v, k_3 + W*),  k_3 = -(xu k_u + xv k_v),
// where (g_u, g_v) and (k_u, k_v) are the central differences of I_A and
// W_A times (f_x / 2, f_y / 2) (the third entries are g (c - p) written in
// the ray).  The square-rooted weights multiply the gradients before the
// Jacobians are formed.  w_W carries lambda_n = 1 / (|n~| |x|) (sec. 6.2):
// n~ = Z (k_u, k_v, k_3) + e_z with Z = 1 / W_A, so |n~| W_A = sqrt(q),
// q = k_u^2 + k_v^2 + (k_3 + W_A)^2, and lambda_n = W_A / sqrt(q |x|^2).
// A term that takes no part (invalid pixel, or its channel without a sample)
// stages zeros: its weight is 0 and the legacy multiply gives 0 x anything
// = 0.  The lane's counts of contributing terms are cI, cW.
// fI, fW: the pixel's flag bits 0 and 1 (sec. 6.2 residual definitions)
// with the channel's enable.
template <int KIND>
__device__ __forceinline__ void pixel_vectors(const LevelRay& R, float xu, float xv, float2 c,
                                              const Nbrs& n, bool fI, bool fW, float Is,
                                              float Ws, bool wv, const RobustF& F, float4* st,
                                              int lane, unsigned& cI, unsigned& cW)
{
    const bool tI = wv & fI;
    const bool tW = wv & fW;
    cI += tI ? 1u : 0u;
    cW += tW ? 1u : 0u;
    const float wa = c.y;
    const float rI = Is - c.x, rW = Ws - wa;
    float sI = sqrt_weight<KIND>(rI - F.muI, F.isI, F.aI, F.cI);
    sI = tI ? sI : 0.0f;
    const float k0 = (n.r.y - n.l.y) * R.hfx, k1 = (n.b.y - n.t.y) * R.hfy;
    const float k3 = -fmaf(xu, k0, xv * k1);
    const float e = k3 + wa;
    const float q = fmaf(k0, k0, fmaf(k1, k1, e * e));
    const float xx = fmaf(xu, xu, fmaf(xv, xv, 1.0f));
    const float sl = __builtin_amdgcn_sqrtf(wa * rsq(q * xx));   // sqrt(lambda_n)
    float sW = sqrt_weight<KIND>(rW - F.muW, F.isW, F.aW, F.cW) * sl;
    sW = tW ? sW : 0.0f;
    // intensity term
    const float g0 = lmul(sI * R.hfx, n.r.x - n.l.x), g1 = lmul(sI * R.hfy, n.b.x - n.t.x);
    const float g3 = -fmaf(xu, g0, xv * g1);
    st[lane] = make_float4(wa * g0, fmaf(-xu, g3, g0), wa * g1, fmaf(xu, g1, -(xv * g0)));
    st[128 + lane] = make_float4(wa * g3, lmul(sI, rI), fmaf(xv, g3, -g1), 0.0f);
    // inverse-depth term
    const float K0 = lmul(sW, k0), K1 = lmul(sW, k1);
    const float KW = lmul(sW, k3) + lmul(sW, Ws);
    st[64 + lane] = make_float4(wa * K0, fmaf(-xu, KW, K0), wa * K1, fmaf(xu, K1, -(xv * K0)));
    st[192 + lane] = make_float4(wa * KW, lmul(sW, rW), fmaf(xv, KW, -K1), 0.0f);
}

// ------------------------------------------------------------------ k_warp

// Membership of the systematic sample of stride s: x = s q exactly, with the
// quotient q = floor((x + 1/2) / s) formed in FP32 (exact for x < 2^20, s <=
// 64: the fraction stays at least 1/(2s) away from an integer).
struct SampleDiv {
    int s;
    float inv, half_inv;
};

__device__ __forceinline__ SampleDiv sample_div(int s)
{
    SampleDiv d;
    d.s = s;
    d.inv = uniform_f(1.0f / (float)s);
    d.half_inv = uniform_f(0.5f * d.inv);
    return d;
}

__device__ __forceinline__ int sample_quot(const SampleDiv& d, int x)
{
    return (int)fmaf((float)x, d.inv, d.half_inv);
}

// Reference values a pass's group leader needs for its pixel's sample
// residuals: A's (I, W) and validity flags at the pixel, and its ray.
// Loaded one pass ahead, together with that pass's children, so the residual
// step has no dependent load.
struct SampleRef {
    int sidx;           // sample index (-1: not a sample pixel)
    float xu, xv;
    float2 c;
    unsigned m;
};

template <bool F16, int LOG2B>
__device__ __forceinline__ SampleRef sample_ref(const LevelView& A, const LevelRay& R,
                                                const PassPos& p, const GridDim& gd, int lane,
                                                bool fused, const SampleDiv& sd, int sw)
{
    using CL = ChildLayout<LOG2B>;
    SampleRef r;
    r.sidx = -1;
    r.xu = r.xv = 0.0f;
    r.c = make_float2(0.0f, 0.0f);
    r.m = 0;
    if ((lane % CL::LPP) != 0 || p.idx >= gd.n) return r;
    const int u = (int)__umul24(p.gu, gd.gs), v = (int)__umul24(p.gv, gd.gs);
    if (fused) {
        r.sidx = p.idx;
    } else {
        const int qu = sample_quot(sd, u), qv = sample_quot(sd, v);
        if (u == (int)__umul24(qu, sd.s) && v == (int)__umul24(qv, sd.s))
            r.sidx = (int)__umul24(qv, sw) + qu;
    }
    if (r.sidx >= 0) {
        const unsigned i = __umul24(v, A.w) + u;
        r.c = load_iw<F16>(A.iw, i);
        r.m = load_mask(A, i);
        r.xu = ray_x(R, u);
        r.xv = ray_y(R, v);
    }
    return r;
}

// Tiles of this kernel are single passes of GPP grid pixels.  The group
// leader of each pixel stores the warped values (store mode; zeros for an
// invalid pixel) and, for sample pixels, the two residuals (NaN = not
// defined).
template <bool F16, int LOG2B>
__global__ void __launch_bounds__(512) k_warp(IterLaunch L)
{
    using CL = ChildLayout<LOG2B>;
    const int ci = chunk_of_block(blockIdx.x, L.n_warp_chunks, L.tune.xcd_remap);
    const Chunk ch = L.warp_chunks[ci];
    const PairState& S = L.states[ch.pair];
    if (!S.active || S.level_stop) return;
    const PairDesc& D = L.pairs[ch.pair];
    const int l = L.level;
    const int wl = L.ip.warp_mode == RGBID_WARP_FULLRES ? 0 : l;
    const Geom G = make_geom<F16>(S, D.A[wl], D.B[wl]);
    const LevelView A = D.A[l];
    const LevelRay R = level_ray(A);
    const bool fused = L.tune.fused;
    const GridDim gd = fused ? sample_grid(D, l) : level_grid(A);
    const SampleDiv sd = sample_div(D.stride[l]);
    const int sw = D.sw[l];
    void* const warped = D.warped;
    void* const sample = D.sample;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / CL::LPP;
    const int waves = blockDim.x >> 6;
    const int end = ch.first + ch.count;
    int tile = ch.first + wave;
    // sample-only pass at level 0: the pixel is its own child, so W_A comes
    // with the reference values and the W plane is not read
    const bool own = LOG2B == 0 && fused;
    PassPos pp = pass_pos(tile * CL::GPP, g, gd);
    SampleRef sr = sample_ref<F16, LOG2B>(A, R, pp, gd, lane, fused, sd, sw);
    auto pc = pass_children<F16, LOG2B>(G, pp, gd.gs, lane, !own);
    if (own) pc.wa[0] = sr.c.y;
    for (; tile < end; tile += waves) {
        float Is, Ws;
        bool wv;
        const int idx = pp.idx;
        warp_pass<F16, LOG2B>(G, pc, idx < gd.n, lane, Is, Ws, wv);
        // the next tile's children and reference values: their loads overlap
        // this tile's tail
        const int ntile = tile + waves < end ? tile + waves : tile;
        const SampleRef cur = sr;
        pp = pass_pos(ntile * CL::GPP, g, gd);
        sr = sample_ref<F16, LOG2B>(A, R, pp, gd, lane, fused, sd, sw);
        pc = pass_children<F16, LOG2B>(G, pp, gd.gs, lane, !own);
        if (own) pc.wa[0] = sr.c.y;
        if ((lane % CL::LPP) != 0 || idx >= gd.n) continue;
        if (!fused) store_f2(warped, idx, wv ? Is : 0.0f, wv ? Ws : 0.0f);
        if (cur.sidx < 0) continue;
        Terms T;
        residuals(cur.c, cur.m, Is, Ws, wv, T);
        store_f2(sample, cur.sidx, T.vI ? T.rI : __int_as_float(0x7fc00000),
                 T.vW ? T.rW : __int_as_float(0x7fc00000));
    }
}

// ------------------------------------------------------------------ k_scale

// The asymptotic series of psi without its ln x term, -1/(2x) - sum_k B_2k /
// (2k x^2k) (Abramowitz & Stegun 6.3.18), for x >= 12, from ix = 1/x.
__device__ __forceinline__ double psi_tail(double ix)
{
    const double z = ix * ix;
    return -0.5 * ix -
           z * (1.0 / 12 + z * (-1.0 / 120 + z * (1.0 / 252 + z * (-1.0 / 240 + z * (1.0 / 132)))));
}

// One step of a DPP sum over the lanes of a wave (row mask `rows`).
#define RGBID_DPP_ADD(v, ctrl, rows)                                                            \
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, rows, 0xf, true))

// Block totals of NV <= 4 per-thread FP32 values, in FP64 and valid in every
// lane of wave 0: every wave reduces its values (lane 63 stores them to LDS);
// after a barrier, row k of wave 0 (lanes 16 k .. 16 k + 15) takes value k of
// waves 0 .. 15 (zero past the last wave), one FP64 scan across the rows of
// 16 lanes leaves total k in lane 16 k + 15, and the totals are read from
// there.  A fixed order.  The scale kernel's update runs in wave 0 and
// reaches the other waves through LDS after a second barrier.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

constexpr int kTotalsLane = 15;

template <int NV>
__device__ __forceinline__ void block_totals(const float (&x)[NV], float* part, double (&tot)[NV])
{
    static_assert(NV >= 1 && NV <= 4, "one row of wave 0 per value");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // Sum of each value over the 64 lanes of the wave, left in lane 63: a
    // scan inside each row of 16 lanes (row_shr 1, 2, 4, 8, zero fill), then
    // the totals of rows 0 and 2 added into rows 1 and 3 (row_bcast:15), then
    // the total of rows 0-1 into rows 2-3 (row_bcast:31); the NV values step
    // by step, so that their DPP steps interleave.
    float w[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) w[k] = x[k];
#pragma unroll
    for (int k = 0; k < NV; ++k) RGBID_DPP_ADD(w[k], 0x111, 0xf);
#pragma unroll
    for (int k = 0; k < NV; ++k) RGBID_DPP_ADD(w[k], 0x112, 0xf);
#pragma unroll
    for (int k = 0; k < NV; ++k) RGBID_DPP_ADD(w[k], 0x114, 0xf);
#pragma unroll
    for (int k = 0; k < NV; ++k) RGBID_DPP_ADD(w[k], 0x118, 0xf);
#pragma unroll
    for (int k = 0; k < NV; ++k) RGBID_DPP_ADD(w[k], 0x142, 0xa);
#pragma unroll
    for (int k = 0; k < NV; ++k) RGBID_DPP_ADD(w[k], 0x143, 0xc);
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[wave * NV + k] = w[k];
    }
    __syncthreads();
    if (wave == 0) {
        const int k = lane >> 4, j = lane & 15;
        double t = k < NV && j < nw ? (double)part[j * NV + k] : 0.0;
        t += dpp_d<0x111>(t);   // row_shr:1
        t += dpp_d<0x112>(t);   // row_shr:2
        t += dpp_d<0x114>(t);   // row_shr:4
        t += dpp_d<0x118>(t);   // row_shr:8
#pragma unroll
        for (int q = 0; q < NV; ++q) tot[q] = readlane_d(t, 16 * q + 15);
    }
}

// n f_c(nu), f_c(nu) = psi(b) - psi(a) - ln(b/a) with a = nu/2, b = a + 1/2:
// the data-free part of the left side of the nu equation of sec. 6.3
// (eq:robustnessValue); the data part is sum_i (1 + ln w_i - w_i).  Both
// digammas move up the same k steps (psi(x) = psi(x + 1) - 1/x) until
// a + k >= 12, where the series holds; with 1/(a+j) - 1/(b+j) =
// 1/(2 (a+j)(b+j)) and T the series without ln x,
//   f_c = sum_{j<k} 1/(2 (a+j)(b+j)) + ln(a (b+k) / (b (a+k))) + T(b+k) - T(a+k),
// the k terms summed as one fraction p/q: four divisions and one logarithm.
__device__ double nu_equation_const(double n, double nud)
{
    const double a = 0.5 * nud, b = a + 0.5;
    double p = 0.0, q = 1.0, x = a;
    while (x < 12.0) {
        const double d = 2.0 * x * (x + 0.5);
        p = fma(p, d, q);
        q *= d;
        x += 1.0;
    }
    const double fc = p / q + log(a * (x + 0.5) / (b * x)) + psi_tail(1.0 / (x + 0.5)) -
                      psi_tail(1.0 / x);
    return n * fc;
}

// Entries of the sample that take no part (undefined residuals) are dropped
// before the fixed point: the block compacts the n defined residuals through
// LDS into F = n / 1024 full slots and a remainder of n mod 1024 entries in
// the last slot (PER - 1), so the steps run without a per-entry validity
// test.  Dead slots hold kNoSample.
constexpr float kNoSample = __builtin_inff();

// Which slots of a thread hold sample entries after the compaction.
struct LiveSlots {
    int full;     // slots 0 .. full-1 (full < PER) are live in every thread (uniform)
    bool tail;    // slot PER - 1 is live in this thread
    int n;        // entries in the sample (uniform)
};

// f(q) for the slots q = Q .. N-1 in order, up to the first q >= n (n
// uniform); expanded at compile time, so that every slot stays in its
// register and a dead slot costs one scalar branch.
template <int Q, int N, class Fn>
__device__ __forceinline__ void for_live(int n, Fn&& f)
{
    if constexpr (Q < N) {
        if (Q >= n) return;
        f(std::integral_constant<int, Q>{});
        for_live<Q + 1, N>(n, f);
    }
}

// Inclusive scan of an integer over the 64 lanes of a wave, in DPP steps:
// row_shr 1, 2, 4, 8 inside every row of 16 lanes (zero fill), then the
// totals of rows 0 and 2 into rows 1 and 3, then the total of rows 0-1
// into rows 2-3.
__device__ __forceinline__ int wave_scan_i(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return v;
}

// Moves the defined entries of r (those below kNoSample) to the front of
// the block's sample, in thread order and, inside a thread, slot order, then
// reloads them: with F = n / 1024, entry j < 1024 F goes to thread j mod
// 1024, slot j / 1024, and entry 1024 F + t to thread t, slot PER - 1.
// cmp holds 1024 PER floats; wcnt 16 ints.  Returns the live slots.
template <int PER>
__device__ __forceinline__ LiveSlots compact_sample(float (&r)[PER], float* cmp, int* wcnt)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int nw = kScaleThreads / 64;
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) cnt += r[q] < kNoSample ? 1 : 0;
    const int incl = wave_scan_i(cnt);
    if (lane == 63) wcnt[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < nw; ++w) {
        const int c = wcnt[w];
        before += w < wave ? c : 0;
        total += c;
    }
    int off = before + incl - cnt;
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (r[q] < kNoSample) cmp[off++] = r[q];
    __syncthreads();
    const int F = __builtin_amdgcn_readfirstlane(total / kScaleThreads);
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER - 1; ++q) r[q] = q < F ? cmp[t + q * kScaleThreads] : kNoSample;
    LiveSlots ls;
    ls.full = min(F, PER - 1);
    ls.tail = F == PER || t < total % kScaleThreads;
    ls.n = total;
    r[PER - 1] = ls.tail ? cmp[t + ls.full * kScaleThreads] : kNoSample;
    return ls;
}

// The location / scale fixed point with nu = 5 (Student-t) or the Huber
// threshold k: every step sums w, w d and w d^2 (d = r - mu, weights from
// the previous estimate) over the block and moves mu by S1/S0, sigma^2 to
// (S2 - S1^2/S0)/n.  At most `iters` steps; the step that moves mu and sigma
// by at most tol sigma' is the last (tol = 0: a step that changes nothing,
// which every further step would repeat).  The per-entry terms are written so that a constant
// factor of the weight is applied to the block totals instead:
//   Huber      w = hk min(1/hk, 1/|d|), w d = clamp(d, -hk, hk),
//              w d^2 = clamp(d, -hk, hk) d               (hk = k sigma)
//   Student-t  w = 6 sigma^2 w' with w' = 1 / (d^2 + 5 sigma^2).
// Sums in FP32 per lane (two partial sums in a fixed order), FP64 across
// the block; mu is kept in FP64, S1/S0 and sigma are formed in FP32 from
// the FP64 sums.  bcd / bcf broadcast mu and sigma.
template <int KIND, int PER>
__device__ __forceinline__ void scale_fixed_point(const float (&r)[PER], LiveSlots ls, float inv_n,
                                                  float floor_s, float k, int iters, float tol,
                                                  float* part, double* bcd, float* bcf,
                                                  double& mu, float& sigma)
{
    float fmu = (float)mu, sg = sigma;
    for (int it = 0; it < iters; ++it) {
        const float hk = k * sg, ihk = rcp(hk), tB = 5.0f * sg * sg;
        float s0[2] = {0.0f, 0.0f}, s1[2] = {0.0f, 0.0f}, s2[2] = {0.0f, 0.0f};
        auto term = [&](float x, int h) {
            const float d = x - fmu;
            if constexpr (KIND == RGBID_W_HUBER) {
                s0[h] += fminf(ihk, rcp(fabsf(d)));
                const float c = __builtin_amdgcn_fmed3f(d, -hk, hk);
                s1[h] += c;
                s2[h] = fmaf(c, d, s2[h]);
            } else {
                const float w = rcp(fmaf(d, d, tB));
                const float t = w * d;
                s0[h] += w;
                s1[h] += t;
                s2[h] = fmaf(t, d, s2[h]);
            }
        };
        for_live<0, PER - 1>(ls.full, [&](auto qc) {
            constexpr int q = decltype(qc)::value;
            term(r[q], q & 1);
        });
        if (ls.tail) term(r[PER - 1], (PER - 1) & 1);
        const float acc[3] = {s0[0] + s0[1], s1[0] + s1[1], s2[0] + s2[1]};
        double tot[3];
        block_totals<3>(acc, part, tot);
        if (threadIdx.x == kTotalsLane) {
            double S0 = tot[0], S1 = tot[1], S2 = tot[2];
            if constexpr (KIND == RGBID_W_HUBER) {
                S0 *= (double)hk;
            } else {
                const double f = (double)(6.0f * sg * sg);
                S0 *= f;
                S1 *= f;
                S2 *= f;
            }
            // mu' = mu + S1/S0; sum w (r - mu')^2 = S2 - S1^2 / S0
            const float dm = (float)S1 * rcp((float)S0);
            const double ss = S2 - S1 * (double)dm;
            const float var = fmaxf((float)ss * inv_n, 0.0f);
            const float sn = fmaxf(__builtin_amdgcn_sqrtf(var), floor_s);
            bcd[0] = mu + (double)dm;
            bcf[0] = sn;
            bcf[1] = fabsf(dm) <= tol * sn && fabsf(sn - sg) <= tol * sn ? 1.0f : 0.0f;
        }
        __syncthreads();
        mu = bcd[0];
        sg = bcf[0];
        fmu = (float)mu;
        if (bcf[1] != 0.0f) break;
    }
    sigma = sg;
}

// One workgroup per (pair, channel): location mu and scale sigma of the
// channel's sample residuals by the fixed point of the two stationarity
// equations of sec. 6.3 (weights from the previous estimate), with nu = 5
// for Student-t, starting at mu = 0, sigma^2 = mean r^2 or (scale_warm, after
// the first iteration at a level whose sample for the channel was not empty)
// at the previous iteration's mu, sigma, with the convergence stop at
// 2^-16 sigma; then (Student-t with
// estimation) nu by bisection of the nu equation on [2, 10] with the
// normalised residuals frozen: f(10) > 0 gives 10, f(2) < 0 gives 2, else 30
// halvings of [2, 10] and the midpoint.  Thread t loads entries t + 1024 q,
// q < PER, of the sample (PER * 1024 at least the largest sample of the
// launch); the defined ones are then compacted.
template <int PER>
__global__ void __launch_bounds__(kScaleThreads) k_scale(IterLaunch L)
{
    __shared__ float cmp[kScaleThreads * PER];
    __shared__ float part[16 * 3];
    __shared__ int wcnt[16];
    __shared__ double bcd[2];
    __shared__ float bcf[2];
    const int p = blockIdx.x, ch = blockIdx.y;
    PairState& S = L.states[p];
    if (!S.active || S.level_stop) return;
    const PairDesc& D = L.pairs[p];
    const int n_all = D.sw[L.level] * D.sh[L.level];
    const float floor_s = ch == 0 ? 1e-3f : 1e-6f;
    // the previous estimate (read before thread 0 replaces it at the end)
    const bool warm = L.ip.scale_warm && S.ns[ch] > 0;
    const float mu_prev = S.mu[ch], sg_prev = S.sigma[ch];
    const float tol = L.ip.scale_warm ? 1.52587890625e-5f : 0.0f;   // 2^-16
    float r[PER];
    float cs[2] = {0.0f, 0.0f};
    // every load is issued (past the end at the last entry, which the buffer
    // holds) before any is used: a load under a condition would wait for the
    // one before it
    const int last = max(n_all - 1, 0);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x + k * kScaleThreads;
        const float y = ld_at<float>(D.sample, 2u * (unsigned)min(i, last) + (unsigned)ch);
        const float x = i < n_all && y == y ? y : kNoSample;   // NaN: residual not defined
        r[k] = x;
        const bool ok = x < kNoSample;
        cs[0] += ok ? 1.0f : 0.0f;
        cs[1] = ok ? fmaf(x, x, cs[1]) : cs[1];
    }
    // a cold start takes the root mean square as its first sigma; a warm one
    // only needs the count, which the compaction gives
    double mu = warm ? (double)mu_prev : 0.0;
    float sigma = sg_prev;
    if (!warm) {
        double t[2];
        block_totals<2>(cs, part, t);
        if (threadIdx.x == kTotalsLane)
            bcf[0] = t[0] > 0.0 ? (float)fmax(sqrt(t[1] / t[0]), (double)floor_s) : floor_s;
        __syncthreads();
        sigma = bcf[0];
    }
    const LiveSlots ls = compact_sample<PER>(r, cmp, wcnt);
    const double n = (double)ls.n;
    float nu = 5.0f;
    if (n > 0.0) {
        const float inv_n = (float)(1.0 / n);
        if (L.ip.weight == RGBID_W_HUBER)
            scale_fixed_point<RGBID_W_HUBER, PER>(r, ls, inv_n, floor_s, L.ip.huber_k,
                                                  L.ip.scale_iters, tol, part, bcd, bcf, mu,
                                                  sigma);
        else
            scale_fixed_point<RGBID_W_STUDENT_T, PER>(r, ls, inv_n, floor_s, L.ip.huber_k,
                                                      L.ip.scale_iters, tol, part, bcd, bcf, mu,
                                                      sigma);
        if (L.ip.weight == RGBID_W_STUDENT_T && L.ip.estimate_nu) {
            const float fmu = (float)mu, isg = 1.0f / sigma;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const float x = (r[q] - fmu) * isg;
                r[q] = x * x;     // r now holds x^2
            }
            // evaluations f(10), f(2), then up to 30 bisection steps; the
            // bracket lives in the totals lane, the next nu and the stop flag
            // reach every wave through LDS
            double lo = 2.0, hi = 10.0, nud = 10.0;
            for (int ev = 0;; ++ev) {
                // the data-free part for this nu, formed in wave 0 (whose
                // lane kTotalsLane needs it) while the other waves sum
                double fcn = 0.0;
                if (threadIdx.x < 64) fcn = nu_equation_const(n, nud);
                const float nf = (float)nud, nf1 = nf + 1.0f;
                float e2[2] = {0.0f, 0.0f};
                // 1 + ln w - w with w = (nu + 1) / (nu + x^2) in (0, 1.5]: a
                // hardware reciprocal and base-2 logarithm (1 ulp each; w is
                // never denormal since x^2 is finite), ln w = ln 2 log2 w
                auto term = [&](float x2, int h) {
                    const float w = nf1 * rcp(nf + x2);
                    e2[h] += fmaf(0.693147180559945f, __builtin_amdgcn_logf(w), 1.0f - w);
                };
                for_live<0, PER - 1>(ls.full, [&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    term(r[q], q & 1);
                });
                if (ls.tail) term(r[PER - 1], (PER - 1) & 1);
                const float acc[1] = {e2[0] + e2[1]};
                double tot[1];
                block_totals<1>(acc, part, tot);
                if (threadIdx.x == kTotalsLane) {
                    const double f = fcn + tot[0];
                    double next = nud;
                    bool stop = false;
                    if (ev == 0) {
                        stop = f > 0.0;           // nu = 10
                        next = stop ? 10.0 : 2.0;
                    } else if (ev == 1) {
                        stop = f < 0.0;           // nu = 2
                        next = stop ? 2.0 : 0.5 * (lo + hi);
                    } else {
                        if (f > 0.0) lo = nud;
                        else hi = nud;
                        next = 0.5 * (lo + hi);
                        stop = ev == 31;
                    }
                    bcd[1] = next;
                    bcf[1] = stop ? 1.0f : 0.0f;
                }
                __syncthreads();
                nud = bcd[1];
                if (bcf[1] != 0.0f) break;
            }
            nu = (float)nud;
        }
    }
    if (threadIdx.x == 0) {
        S.mu[ch] = (float)mu;
        S.sigma[ch] = sigma;
        S.nu[ch] = nu;
        S.ns[ch] = (int)n;
    }
}

// ------------------------------------------------------------------ k_reduce

// A level pixel of A with everything its terms need: whether it is a pixel
// of the level, ray, (I, W), validity flags and the four neighbours.
struct RefPx {
    bool in;
    float xu, xv;
    float2 c;
    unsigned m;
    Nbrs nb;
};

// Position (u, v), raster index idx; in: a pixel of the level (otherwise
// pixel 0 is read in its place).
template <bool F16>
__device__ __forceinline__ void load_ref(const LevelView& A, const LevelRay& R, bool in, int idx,
                                         int u, int v, RefPx& r)
{
    const unsigned ic = in ? (unsigned)idx : 0u;
    r.in = in;
    r.xu = ray_x(R, u);
    r.xv = ray_y(R, v);
    r.c = load_iw<F16>(A.iw, ic);
    r.m = load_mask(A, ic);
    r.nb = load_nbrs<F16>(A, ic);
}

// Raster position `step` pixels further on (step = sv rows + su columns,
// su < gw).
__device__ __forceinline__ void advance(int& idx, int& u, int& v, int step, int su, int sv, int gw)
{
    idx += step;
    u += su;
    v += sv;
    if (u >= gw) {
        u -= gw;
        ++v;
    }
}

// The level-0 path of the fused reduction (the level pixel is its own warp
// child) works on blocks of kBlockW x kBlockH pixels, a lane per pixel.  The
// four neighbours of the central differences come from a per-wave tile in
// LDS: the block's own (I, W), which the lanes load anyway, and its halo (the
// rows above and below, the columns left and right), which lanes 0..39 load
// with one instruction.  The tile has kBlockH + 2 rows of kBlockW + 2 texels;
// the corners are not used.
constexpr int kTileW = kBlockW + 2, kTileTexels = kTileW * (kBlockH + 2);
static_assert(2 * kBlockW + 2 * kBlockH <= 64, "one halo texel per lane");

// The halo texel lane `lane` brings: its offset (du, dv) from the block's
// first pixel and its place in the tile.  Lanes 40..63 bring none; they load
// the block's first pixel and store it in the unused corner slot 0, so that
// every lane issues the same loads and stores.
struct HaloLane {
    int du, dv, slot;
};

__device__ __forceinline__ HaloLane halo_lane(int lane)
{
    HaloLane h{0, 0, 0};
    if (lane < kBlockW) {                            // row above
        h.du = lane, h.dv = -1, h.slot = lane + 1;
    } else if (lane < 2 * kBlockW) {                 // row below
        h.du = lane - kBlockW, h.dv = kBlockH, h.slot = (kBlockH + 1) * kTileW + h.du + 1;
    } else if (lane < 2 * kBlockW + kBlockH) {       // column left
        h.du = -1, h.dv = lane - 2 * kBlockW, h.slot = (h.dv + 1) * kTileW;
    } else if (lane < 2 * kBlockW + 2 * kBlockH) {   // column right
        h.du = kBlockW, h.dv = lane - 2 * kBlockW - kBlockH, h.slot = (h.dv + 1) * kTileW + kBlockW + 1;
    }
    return h;
}

// A level-0 pixel of a block tile: whether it is a pixel of the level and an
// interior one (1 <= u <= w - 2, 1 <= v <= h - 2), the block's first pixel
// (u0, v0) (uniform), the pixel's (I, W) and the halo texel of the lane.
struct RefL0 {
    bool in, inner;
    int u0, v0;
    float2 c, h;
};

// What a level-0 pixel carries from l0_fetch to l0_finish: its ray and taps.
struct L0Taps {
    float xu, xv;
    WarpTaps T;
};

// Warp, residuals and weighted Jacobians of a level-0 pixel into the
// accumulators, in two steps: l0_fetch issues the pixel's tap loads (the
// caller then issues the next tile's loads, so that waiting for the taps does
// not wait for those), l0_finish does the rest.  tl: the wave's neighbour
// tile; cslot: the pixel's place in it, nslot: the place of its upper-left
// diagonal neighbour, hslot: the place of the lane's halo texel.  The
// validity flags are those the pyramid stores (bit 0: interior with valid W;
// bit 1: also the four W neighbours valid), formed here from the values at
// hand.
template <bool F16>
__device__ __forceinline__ void l0_fetch(const Geom& G, const LevelRay& R, const RefL0& r, int lu,
                                         int lv, L0Taps& t)
{
    t.xu = ray_x(R, r.u0 + lu);
    t.xv = ray_y(R, r.v0 + lv);
    warp_fetch<F16>(G, rotate_ray(G, t.xu, t.xv), r.c.y, t.T);
}

template <int KIND>
__device__ __forceinline__ void l0_finish(const Geom& G, const LevelRay& R, const RefL0& r,
                                          const L0Taps& t, float2* tl, int cslot, int nslot,
                                          int hslot, const RobustF& F, NeAcc& na, float4* st,
                                          int lane, unsigned& cI, unsigned& cW)
{
    // the block and its halo into the tile (the wave's earlier reads of it
    // are done: LDS operations of a wave complete in order), then the four
    // neighbours
    tl[cslot] = r.c;
    tl[hslot] = r.h;
    Nbrs n;
    n.t = tl[nslot + 1];
    n.l = tl[nslot + kTileW];
    n.r = tl[nslot + kTileW + 2];
    n.b = tl[nslot + 2 * kTileW + 1];
    float Is, Ws;
    const bool wv = warp_finish(G, t.T, Is, Ws) & r.in;
    const bool f0 = r.inner & (int)w_valid(r.c.y);
    const bool f1 = f0 & (int)w_valid(n.l.y) & (int)w_valid(n.r.y) & (int)w_valid(n.t.y) &
                    (int)w_valid(n.b.y);
    pixel_vectors<KIND>(R, t.xu, t.xv, r.c, n, f0 & (F.mI != 0u), f1 & (F.mW != 0u), Is, Ws, wv,
                        F, st, lane, cI, cW);
    ne_feed(na, st, lane);
}

// Level pixel whose warped values come from the store: residuals, weighted
// Jacobians into the accumulators.
template <int KIND>
__device__ __forceinline__ void stored_pixel(const LevelRay& R, const RefPx& r, float2 e,
                                             const RobustF& F, NeAcc& na, float4* st, int lane,
                                             unsigned& cI, unsigned& cW)
{
    const bool wv = (e.y > 0.0f) & r.in;
    pixel_vectors<KIND>(R, r.xu, r.xv, r.c, r.nb, (r.m & F.mI) != 0u, (r.m & F.mW) != 0u, e.x,
                        e.y, wv, F, st, lane, cI, cW);
    ne_feed(na, st, lane);
}

// Dynamic LDS: kStageFloat4PerWave float4 per wave (the normal-equation
// staging area).
template <bool F16, int LOG2B, bool FUSED, int KIND>
__global__ void __launch_bounds__(512) k_reduce(IterLaunch L)
{
    __shared__ float2 lds[8 * kNSum];
    extern __shared__ float4 ne_stage[];
    const int ci = chunk_of_block(blockIdx.x, L.n_red_chunks, L.tune.xcd_remap);
    const Chunk ch = L.red_chunks[ci];
    const PairState& S = L.states[ch.pair];
    if (!S.active || S.level_stop) return;
    const PairDesc& D = L.pairs[ch.pair];
    const int l = L.level;
    const LevelView A = D.A[l];
    const LevelRay R = level_ray(A);
    const GridDim gd = level_grid(A);
    const void* const warped = D.warped;
    const RobustF F = robust_f(L, S);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    NeAcc na;
    ne_init(na);
    unsigned cI = 0, cW = 0;

    float4* const st = ne_stage + wave * kStageFloat4PerWave;
    const int waves = blockDim.x >> 6;
    const int end = ch.first + ch.count;
    const int wl = L.ip.warp_mode == RGBID_WARP_FULLRES ? 0 : l;
    Geom G = make_geom<F16>(S, D.A[wl], D.B[wl]);
    if constexpr (FUSED && LOG2B == 0) {
        // the rotation's constant column in vector registers for the whole
        // loop (an FMA takes one scalar operand)
        asm volatile("" : "+v"(G.m[2]), "+v"(G.m[5]), "+v"(G.m[8]));
        // The level pixel is its own warp child, so W_A comes with A's (I, W).
        // A tile is a kBlockW x kBlockH block of the level (lane l at column
        // l mod kBlockW, row l / kBlockW of it; pixels past the level's edge
        // take no part), blocks in raster order: the centre and tap lines of
        // a tile are mostly the same lines, so they are fetched once.  A's
        // loads for the next tile are issued while this tile's gathers from B
        // are in flight.
        __shared__ float2 nb_tiles[8 * kTileTexels];
        float2* const tl = nb_tiles + wave * kTileTexels;
        const int bxn = (gd.gw + kBlockW - 1) / kBlockW, gh = A.h;
        const int lu = lane % kBlockW, lv = lane / kBlockW;
        const int cslot = (lv + 1) * kTileW + lu + 1, nslot = lv * kTileW + lu;
        const HaloLane hl = halo_lane(lane);
        // lane offsets from the block's first pixel, kept in registers (not
        // re-derived per tile as v * w + u)
        int loff = lv * gd.gw + lu, hoff = hl.dv * gd.gw + hl.du;
        asm volatile("" : "+v"(loff), "+v"(hoff));
        // halo texels are read from a base one row and one texel before the
        // plane (inside its zero guard), their index clamped to the guard
        // after it: only pixels that are not interior see clamped values
        const unsigned texb = F16 ? 4u : 8u;
        const char* const hbase = static_cast<const char*>(A.iw) - (gd.gw + 1) * (int)texb;
        const int hmax = gd.n + 2 * gd.gw + 1;
        const unsigned uin = (unsigned)max(gd.gw - 2, 0), vin = (unsigned)max(gh - 2, 0);
        auto load = [&](int t, RefL0& r) {
            // the block's first pixel (uniform) plus the lane's place in it
            const int by = t / bxn, bx = t - by * bxn, u0 = bx * kBlockW, v0 = by * kBlockH;
            const int corner = v0 * gd.gw + u0;
            const int u = u0 + lu, v = v0 + lv;
            r.in = (u < gd.gw) & (v < gh);
            r.inner = ((unsigned)(u - 1) < uin) & ((unsigned)(v - 1) < vin);
            r.u0 = u0;
            r.v0 = v0;
            unsigned co = (r.in ? (unsigned)(corner + loff) : 0u) * texb;
            asm volatile("" : "+v"(co));   // a 32-bit offset from the plane's base
            r.c = load_iw_at<F16>(A.iw, co);
            r.h = load_iw_at<F16>(hbase, (unsigned)min(corner + hoff + gd.gw + 1, hmax) * texb);
        };
        int tile = __builtin_amdgcn_readfirstlane(ch.first + wave);
        // two tiles per trip, the prefetch alternating between ra and rb, so
        // the reference values are never copied from one to the other; per
        // tile: its taps, then the next tile's loads, then its arithmetic
        RefL0 ra, rb;
        L0Taps T;
        load(tile, ra);
        while (tile < end) {
            l0_fetch<F16>(G, R, ra, lu, lv, T);
            __builtin_amdgcn_sched_barrier(0);
            load(tile + waves, rb);
            __builtin_amdgcn_sched_barrier(0);
            l0_finish<KIND>(G, R, ra, T, tl, cslot, nslot, hl.slot, F, na, st, lane, cI, cW);
            tile += waves;
            if (tile >= end) break;
            l0_fetch<F16>(G, R, rb, lu, lv, T);
            __builtin_amdgcn_sched_barrier(0);
            load(tile + waves, ra);
            __builtin_amdgcn_sched_barrier(0);
            l0_finish<KIND>(G, R, rb, T, tl, cslot, nslot, hl.slot, F, na, st, lane, cI, cW);
            tile += waves;
        }
    } else if constexpr (!FUSED) {
        // The warped values come from the store.  Two tiles per trip as
        // above; the next tile's loads (warped pair, reference values) are
        // issued before this tile's arithmetic, which has no gathers to wait
        // for, so a wave waits for a tile's loads only when it arrives at it.
        const int step = waves * 64, su = step % gd.gw, sv = step / gd.gw;
        int tile = ch.first + wave;
        int idx = tile * 64 + lane, u, v;
        split_index(idx, gd.gw, gd.inv_gw, gd.half_inv, u, v);
        RefPx ra, rb;
        load_ref<F16>(A, R, idx < gd.n, idx, u, v, ra);
        float2 ea = load_f2(warped, min(idx, gd.n - 1)), eb;
        while (tile < end) {
            advance(idx, u, v, step, su, sv, gd.gw);
            load_ref<F16>(A, R, idx < gd.n, idx, u, v, rb);
            eb = load_f2(warped, min(idx, gd.n - 1));
            __builtin_amdgcn_sched_barrier(0);
            stored_pixel<KIND>(R, ra, ea, F, na, st, lane, cI, cW);
            tile += waves;
            if (tile >= end) break;
            advance(idx, u, v, step, su, sv, gd.gw);
            load_ref<F16>(A, R, idx < gd.n, idx, u, v, ra);
            ea = load_f2(warped, min(idx, gd.n - 1));
            __builtin_amdgcn_sched_barrier(0);
            stored_pixel<KIND>(R, rb, eb, F, na, st, lane, cI, cW);
            tile += waves;
        }
    } else {
        for (int tile = ch.first + wave; tile < end; tile += waves) {
            float Is = 0.0f, Ws = 0.0f;
            bool wv = false;
            int u = 0, v = 0, idx;
            warp_tile<F16, LOG2B>(G, tile * 64, gd, lane, Is, Ws, wv, u, v, idx);
            const unsigned i = __umul24(v, A.w) + u;
            const unsigned m = load_mask(A, i);
            pixel_vectors<KIND>(R, ray_x(R, u), ray_y(R, v), load_iw<F16>(A.iw, i),
                                load_nbrs<F16>(A, i), (m & F.mI) != 0u, (m & F.mW) != 0u, Is,
                                Ws, wv, F, st, lane, cI, cW);
            ne_feed(na, st, lane);
        }
    }
    ne_wave_totals(na, st, lane, cI, cW, lds + wave * kNSum);
    __syncthreads();
    if (threadIdx.x < kNSum) {
        // the waves' (hi, lo) totals in wave order: two-sum of the high parts,
        // the low parts added
        float hi = 0.0f, lo = 0.0f;
        for (int w = 0; w < waves; ++w) {
            const float2 x = lds[w * kNSum + threadIdx.x];
            two_sum_add(hi, lo, x.x);
            lo += x.y;
        }
        store_f2(L.partials, (size_t)ci * kNSum + threadIdx.x, hi, lo);
    }
}

// ------------------------------------------------------------------ k_solve

// Rotation of the axis-angle vector th: cos|th| I + sin|th| [k]x +
// (1 - cos|th|) k k^T with k = th/|th| (identity + [th]x + [th]x^2/2 for
// |th| < 1e-8).
__device__ void rot_of(const double th[3], double E[9])
{
    const double n = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    if (n < 1e-8) {
        const double S[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s2 = 0;
                for (int k = 0; k < 3; ++k) s2 += S[3 * i + k] * S[3 * k + j];
                E[3 * i + j] = (i == j) + S[3 * i + j] + 0.5 * s2;
            }
        return;
    }
    const double k[3] = {th[0] / n, th[1] / n, th[2] / n};
    double s, c;
    sincos(n, &s, &c);
    const double oc = 1.0 - c;
    E[0] = c + oc * k[0] * k[0];
    E[1] = oc * k[0] * k[1] - s * k[2];
    E[2] = oc * k[0] * k[2] + s * k[1];
    E[3] = oc * k[1] * k[0] + s * k[2];
    E[4] = c + oc * k[1] * k[1];
    E[5] = oc * k[1] * k[2] - s * k[0];
    E[6] = oc * k[2] * k[0] - s * k[1];
    E[7] = oc * k[2] * k[1] + s * k[0];
    E[8] = c + oc * k[2] * k[2];
}

// One wave per pair: the FP64 sums over the pair's chunks (term k < kNSum of
// chunk beg + j goes to lane k for even j and to lane 32 + k for odd j; each
// lane adds its chunks in order into two sums, alternately, 16 loads in
// flight at a time; then each lane adds its two sums and lane k adds lane
// 32 + k), the normal equations into the state, the 6x6 Cholesky and the
// update.
__global__ void __launch_bounds__(64) k_solve(IterLaunch L)
{
    const int p = blockIdx.x;
    PairState& S = L.states[p];
    if (!S.active || S.level_stop) return;
    const int lane = threadIdx.x;
    const int beg = L.pair_red_begin[p], end = L.pair_red_begin[p + 1];
    const int term = lane & 31;
    double t2[2] = {0.0, 0.0};
    if (term < kNSum) {
        // the loads of a batch are issued at clamped (valid) chunks before
        // any is used; chunks past the end count zero
        constexpr int kBatch = 16;
        for (int c = beg + (lane >> 5); c < end; c += 2 * kBatch) {
            float2 q[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                q[j] = load_f2(L.partials, (size_t)min(c + 2 * j, end - 1) * kNSum + term);
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (c + 2 * j < end) t2[j & 1] += (double)q[j].x + (double)q[j].y;
        }
    }
    double t = t2[0] + t2[1];
    t += __shfl_down(t, 32);
    double s[kNSum];
#pragma unroll
    for (int q = 0; q < kNSum; ++q) s[q] = readlane_d(t, q);
    if (lane != 0) return;

    for (int k = 0; k < 21; ++k) S.H[k] = s[k];
    for (int k = 0; k < 6; ++k) S.g[k] = s[21 + k];
    S.cost = s[27];
    S.nI = (long long)(s[28] + 0.5);
    S.nW = (long long)(s[29] + 0.5);
    if (L.ip.weight == RGBID_W_STUDENT_T && L.ip.estimate_nu) S.nu[0] = fmaxf(S.nu[0], S.nu[1]);
    if (!L.update) return;

    // 6x6 Cholesky of H (upper triangle, row-major) and xi = -H^-1 g; a pivot
    // <= 1e-12 max(diag H) or fewer than 6 valid residuals is degenerate.
    double A[6][6];
    {
        int k = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = a; b < 6; ++b) {
                A[a][b] = A[b][a] = s[k];
                ++k;
            }
    }
    double dmax = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) dmax = fmax(dmax, A[a][a]);
    bool ok = (S.nI + S.nW >= 6) && dmax > 0.0;
    double Lm[6][6], inv[6];   // inv[j] = 1 / L_jj
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
        ok = ok && d > 1e-12 * dmax;
        Lm[j][j] = sqrt(ok ? d : 1.0);
        inv[j] = 1.0 / Lm[j][j];
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double e = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) e -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = e * inv[j];
        }
    }
    if (!ok) {
        S.status = RGBID_E_DEGENERATE;
        S.active = 0;
        return;
    }
    double y[6], xi[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double e = -s[21 + i];
#pragma unroll
        for (int k = 0; k < i; ++k) e -= Lm[i][k] * y[k];
        y[i] = e * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double e = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) e -= Lm[k][i] * xi[k];
        xi[i] = e * inv[i];
    }
    // T <- exp(xi)^-1 T = (E^T R, E^T (t - v))
    double E[9];
    rot_of(xi + 3, E);
    double Rn[9], tn[3];
    const double d[3] = {S.t[0] - xi[0], S.t[1] - xi[1], S.t[2] - xi[2]};
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            Rn[3 * i + j] = E[i] * S.R[j] + E[3 + i] * S.R[3 + j] + E[6 + i] * S.R[6 + j];
        tn[i] = E[i] * d[0] + E[3 + i] * d[1] + E[6 + i] * d[2];
    }
    for (int k = 0; k < 9; ++k) S.R[k] = Rn[k];
    for (int k = 0; k < 3; ++k) S.t[k] = tn[k];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) S.RT[3 * i + j] = (float)Rn[3 * j + i];
        S.Rtt[i] = (float)(Rn[i] * tn[0] + Rn[3 + i] * tn[1] + Rn[6 + i] * tn[2]);
    }
    S.iters_done[L.level] += 1;
    if (L.ip.stop_eps_t > 0.0 || L.ip.stop_eps_r > 0.0) {
        const double nv = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        const double nr = sqrt(xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5]);
        if (nv < L.ip.stop_eps_t && nr < L.ip.stop_eps_r) S.level_stop = 1;
    }
}

__global__ void k_level_start(PairState* states, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        states[i].level_stop = 0;
        // no scale estimate at this level yet: the first fixed point starts cold
        states[i].ns[0] = states[i].ns[1] = 0;
    }
}

template <bool F16, int LOG2B>
hipError_t launch_iteration_t(hipStream_t s, const IterLaunch& L, hipEvent_t const* ev)
{
    const dim3 blk(64 * L.tune.waves);
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if ((L.kernels & 1) && L.n_warp_chunks > 0)
        hipLaunchKernelGGL((k_warp<F16, LOG2B>), dim3(L.n_warp_chunks), blk, 0, s, L);
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (L.kernels & 2) {
        const dim3 sg(L.npairs, 2), sb(kScaleThreads);
        if (L.scale_per <= 5) hipLaunchKernelGGL(k_scale<5>, sg, sb, 0, s, L);
        else if (L.scale_per <= 10) hipLaunchKernelGGL(k_scale<10>, sg, sb, 0, s, L);
        else if (L.scale_per <= 15) hipLaunchKernelGGL(k_scale<15>, sg, sb, 0, s, L);
        else if (L.scale_per <= 19) hipLaunchKernelGGL(k_scale<19>, sg, sb, 0, s, L);
        else hipLaunchKernelGGL(k_scale<kScalePerThread>, sg, sb, 0, s, L);
    }
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    if ((L.kernels & 4) && L.n_red_chunks > 0) {
        const size_t lds_bytes = sizeof(float4) * kStageFloat4PerWave * L.tune.waves;
        const dim3 g(L.n_red_chunks);
        constexpr int HU = RGBID_W_HUBER, ST = RGBID_W_STUDENT_T;
        if (L.ip.weight == HU) {
            if (L.tune.fused) hipLaunchKernelGGL((k_reduce<F16, LOG2B, true, HU>), g, blk, lds_bytes, s, L);
            else hipLaunchKernelGGL((k_reduce<F16, LOG2B, false, HU>), g, blk, lds_bytes, s, L);
        } else {
            if (L.tune.fused) hipLaunchKernelGGL((k_reduce<F16, LOG2B, true, ST>), g, blk, lds_bytes, s, L);
            else hipLaunchKernelGGL((k_reduce<F16, LOG2B, false, ST>), g, blk, lds_bytes, s, L);
        }
    }
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    if (L.kernels & 8) hipLaunchKernelGGL(k_solve, dim3(L.npairs), dim3(64), 0, s, L);
    if (ev && (e = hipEventRecord(ev[4], s)) != hipSuccess) return e;
    return hipGetLastError();
}

template <bool F16>
hipError_t launch_iteration_f(hipStream_t s, const IterLaunch& L, hipEvent_t const* ev)
{
    switch (L.block_log2) {
    case 0: return launch_iteration_t<F16, 0>(s, L, ev);
    case 1: return launch_iteration_t<F16, 1>(s, L, ev);
    case 2: return launch_iteration_t<F16, 2>(s, L, ev);
    case 3: return launch_iteration_t<F16, 3>(s, L, ev);
    case 4: return launch_iteration_t<F16, 4>(s, L, ev);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_iteration(hipStream_t s, const IterLaunch& L, hipEvent_t const* ev)
{
    if (L.tune.waves < 1 || L.tune.waves > 8) return hipErrorInvalidValue;
    return L.f16 ? launch_iteration_f<true>(s, L, ev) : launch_iteration_f<false>(s, L, ev);
}

namespace {

// Per-pair results in the public layouts, written to device memory (the
// asynchronous batch call): the pose and the statistics of the last
// linearisation, field by field as the synchronous call fills them on the host.
__global__ void __launch_bounds__(64) k_export(const PairState* __restrict__ states, int n,
                                               rgbid_pose* out, rgbid_align_stats* stats)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PairState& s = states[i];
    if (out) {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[i].R[k] = s.R[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) out[i].t[k] = s.t[k];
    }
    if (stats) {
        rgbid_align_stats& o = stats[i];
#pragma unroll
        for (int k = 0; k < 21; ++k) o.H[k] = s.H[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) o.g[k] = s.g[k];
        o.mu_I = s.mu[0];
        o.sigma_I = s.sigma[0];
        o.nu_I = s.nu[0];
        o.mu_W = s.mu[1];
        o.sigma_W = s.sigma[1];
        o.nu_W = s.nu[1];
        o.cost = s.cost;
        o.n_valid_I = s.nI;
        o.n_valid_W = s.nW;
#pragma unroll
        for (int l = 0; l < 8; ++l) o.iters_done[l] = l < kMaxLevels ? s.iters_done[l] : 0;
        o.status = s.status;
    }
}

}  // namespace

hipError_t launch_export(hipStream_t s, const PairState* states, int n, rgbid_pose* out,
                         rgbid_align_stats* stats)
{
    if (n <= 0 || (!out && !stats)) return hipSuccess;
    hipLaunchKernelGGL(k_export, dim3((n + 63) / 64), dim3(64), 0, s, states, n, out, stats);
    return hipGetLastError();
}

namespace {

// One thread per chunk of the tables; thread 0 also writes the descriptor,
// the state and the per-level chunk ranges.
__global__ void __launch_bounds__(256) k_noalloc_setup(NoAllocSetup a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *a.desc_dev = a.desc;
        *a.state_dev = a.state;
        for (int l = 0; l < a.levels; ++l) {
            a.begins[2 * l] = 0;
            a.begins[2 * l + 1] = a.n_red[l];
        }
    }
    if (i >= a.seg_first[a.nseg]) return;
    int k = 0;
    while (i >= a.seg_first[k + 1]) ++k;
    const int t = (i - a.seg_first[k]) * a.seg_per[k];
    a.chunks[i] = Chunk{0, t, min(a.seg_per[k], a.seg_tiles[k] - t)};
}

}  // namespace

hipError_t launch_noalloc_setup(hipStream_t s, const NoAllocSetup& a)
{
    const int n = a.seg_first[a.nseg];
    hipLaunchKernelGGL(k_noalloc_setup, dim3(((n > 0 ? n : 1) + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

namespace {

struct Scale6 {
    double s[6];
};

// R = I + a [th]x + b [th]x^2, a = sin|th| / |th|, b = (1 - cos|th|) / |th|^2
// (a = 1, b = 1/2 below |th| = 1e-8), t = v.
__global__ void __launch_bounds__(64) k_init_from_twist(PairState* __restrict__ states, int n,
                                                        const float* __restrict__ o, Scale6 sc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xi[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) xi[k] = (double)o[6 * i + k] * sc.s[k];
    const double* th = xi + 3;
    const double nn = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    const double S[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
    const double a = nn < 1e-8 ? 1.0 : sin(nn) / nn;
    const double b = nn < 1e-8 ? 0.5 : (1.0 - cos(nn)) / (nn * nn);
    PairState& st = states[i];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s2 = 0.0;
            for (int k = 0; k < 3; ++k) s2 += S[3 * r + k] * S[3 * k + c];
            st.R[3 * r + c] = (r == c ? 1.0 : 0.0) + a * S[3 * r + c] + b * s2;
        }
    for (int k = 0; k < 3; ++k) st.t[k] = xi[k];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) st.RT[3 * r + c] = (float)st.R[3 * c + r];
        st.Rtt[r] = (float)(st.R[r] * st.t[0] + st.R[3 + r] * st.t[1] + st.R[6 + r] * st.t[2]);
    }
}

}  // namespace

hipError_t launch_init_from_twist(hipStream_t s, PairState* states, int n, const float* o,
                                  const double scale[6])
{
    Scale6 sc;
    for (int k = 0; k < 6; ++k) sc.s[k] = scale[k];
    hipLaunchKernelGGL(k_init_from_twist, dim3((n + 63) / 64), dim3(64), 0, s, states, n, o, sc);
    return hipGetLastError();
}

hipError_t launch_level_start(hipStream_t s, PairState* states, int npairs)
{
    hipLaunchKernelGGL(k_level_start, dim3((npairs + 63) / 64), dim3(64), 0, s, states, npairs);
    return hipGetLastError();
}

}  // namespace rgbid
