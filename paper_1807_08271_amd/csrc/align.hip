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

// Row / column of raster index idx in a grid of width gw (idx < 2^24).
__device__ __forceinline__ void split_index(int idx, int gw, float inv_gw, int& gu, int& gv)
{
    int v = (int)((float)idx * inv_gw);
    int u = idx - (int)__umul24((unsigned)v, (unsigned)gw);
    if (u < 0) { u += gw; --v; }
    else if (u >= gw) { u -= gw; ++v; }
    gu = u;
    gv = v;
}

__device__ __forceinline__ int chunk_of_block(int b, int n, int remap)
{
    if (!remap) return b;
    // Consecutive chunks on one XCD: XCD x = b % 8 runs a contiguous range.
    const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

// Warp parameters of one pair at the warp level.
struct Geom {
    float m[9];       // R^T
    float q[3];       // R^T t
    float fx, fy, cx, cy, ifx, ify;
    int w, h;
    const void* WA;   // W plane of A at the warp level
    const void* Biw;  // interleaved (I, W) of B at the warp level
};

__device__ __forceinline__ Geom make_geom(const PairState& S, const LevelView& A, const LevelView& B)
{
    Geom G;
#pragma unroll
    for (int k = 0; k < 9; ++k) G.m[k] = S.RT[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) G.q[k] = S.Rtt[k];
    G.fx = A.fx;
    G.fy = A.fy;
    G.cx = A.cx;
    G.cy = A.cy;
    G.ifx = 1.0f / A.fx;
    G.ify = 1.0f / A.fy;
    G.w = A.w;
    G.h = A.h;
    G.WA = A.wp;
    G.Biw = B.iw;
    return G;
}

// Reciprocal and reciprocal square root (v_rcp_f32 / v_rsq_f32, 1 ulp) for
// the per-pixel path.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Inverse geometric warp of one pixel (u, v) of A (sec. 5.3) with w_a =
// W_A(u, v) already loaded.  With x = K^-1 p,
// W_A(p) * R^T (x / w_a - t) = R^T x - w_a R^T t locates p_B; I* is the
// bilinear I_B(p_B) and W* = (R^T x)_z w_b / (1 + w_b (R^T t)_z) with w_b the
// bilinear W_B(p_B).  Valid iff w_a valid, in front, p_B in
// [-0.5, w-0.5) x [-0.5, h-0.5), four valid W taps and W* positive and
// finite.  Branch-free: the four taps are always loaded (at clamped, in-bounds
// addresses).  Split in two phases so that a lane can issue the tap loads of
// all its pixels before it consumes any of them.
struct WarpTaps {
    float2 p00, p10, p01, p11;
    float a, b, az;
    bool ok;
};

template <bool F16>
__device__ __forceinline__ void warp_fetch(const Geom& G, int u, int v, float wa, WarpTaps& T)
{
    bool ok = w_valid(wa);
    const float rx = ((float)u - G.cx) * G.ifx, ry = ((float)v - G.cy) * G.ify;
    const float ax = fmaf(G.m[0], rx, fmaf(G.m[1], ry, G.m[2]));
    const float ay = fmaf(G.m[3], rx, fmaf(G.m[4], ry, G.m[5]));
    const float az = fmaf(G.m[6], rx, fmaf(G.m[7], ry, G.m[8]));
    const float yx = fmaf(-wa, G.q[0], ax), yy = fmaf(-wa, G.q[1], ay), yz = fmaf(-wa, G.q[2], az);
    ok = ok && yz > 0.0f;
    const float iz = rcp(yz);
    float ub = fmaf(G.fx * yx, iz, G.cx), vb = fmaf(G.fy * yy, iz, G.cy);
    ok = ok && ub >= -0.5f && ub < (float)G.w - 0.5f && vb >= -0.5f && vb < (float)G.h - 0.5f;
    ub = ok ? ub : 0.0f;
    vb = ok ? vb : 0.0f;
    const float fu = floorf(ub), fv = floorf(vb);
    T.a = ub - fu;
    T.b = vb - fv;
    T.az = az;
    T.ok = ok;
    // taps: x0 = floor(u_B) (>= -1 in bounds), clamped to the image
    const int xf = (int)fu, yf = (int)fv;
    const unsigned x0 = (unsigned)max(xf, 0), y0 = (unsigned)max(yf, 0);
    const unsigned dx = xf + 1 <= G.w - 1 && xf >= 0 ? 1u : 0u;
    const unsigned dy = yf + 1 <= G.h - 1 && yf >= 0 ? (unsigned)G.w : 0u;
    const unsigned i00 = __umul24(y0, (unsigned)G.w) + x0;
    T.p00 = load_iw<F16>(G.Biw, i00);
    T.p10 = load_iw<F16>(G.Biw, i00 + dx);
    T.p01 = load_iw<F16>(G.Biw, i00 + dy);
    T.p11 = load_iw<F16>(G.Biw, i00 + dy + dx);
}

__device__ __forceinline__ bool warp_finish(const Geom& G, const WarpTaps& T, float& Io, float& Wo)
{
    bool ok = T.ok && w_valid(T.p00.y) && w_valid(T.p10.y) && w_valid(T.p01.y) &&
              w_valid(T.p11.y);
    const float a = T.a, b = T.b;
    const float c00 = (1.0f - a) * (1.0f - b), c10 = a * (1.0f - b);
    const float c01 = (1.0f - a) * b, c11 = a * b;
    const float ib = c00 * T.p00.x + c10 * T.p10.x + c01 * T.p01.x + c11 * T.p11.x;
    const float wb = c00 * T.p00.y + c10 * T.p10.y + c01 * T.p01.y + c11 * T.p11.y;
    const float ws = T.az * wb * rcp(fmaf(wb, G.q[2], 1.0f));
    ok = ok && w_valid(ws);
    Io = ok ? ib : 0.0f;
    Wo = ok ? ws : 0.0f;
    return ok;
}

template <bool F16>
__device__ __forceinline__ bool warp_core(const Geom& G, int u, int v, float wa, float& Io,
                                          float& Wo)
{
    WarpTaps T;
    warp_fetch<F16>(G, u, v, wa, T);
    return warp_finish(G, T, Io, Wo);
}

// Warp-level coordinates of the children this lane handles in one pass, and
// their W_A (loaded ahead so the next pass's loads overlap this pass's
// gathers).
template <bool F16, int CPL>
struct PassChildren {
    int u[CPL], v[CPL];
    float wa[CPL];
};

// Lane layout of the children of level pixels: a level pixel has C = 4^LOG2B
// children at the warp level; each lane warps CPL = min(C, 4) of them (four
// independent load chains per lane), LPP = C / CPL lanes share one pixel and
// combine their sums with cross-lane shuffles, and GPP = 64 / LPP pixels are
// warped per pass.
template <int LOG2B>
struct ChildLayout {
    static constexpr int B = 1 << LOG2B;
    static constexpr int C = B * B;
    static constexpr int CPL = warp_children_per_lane(LOG2B);   // children per lane
    static constexpr int LPP = warp_lanes_per_pixel(LOG2B);     // lanes per pixel
    static constexpr int GPP = warp_pixels_per_pass(LOG2B);     // pixels per pass
    static_assert(CPL * LPP == C && LPP <= 64, "at most 64 lanes per level pixel");
};

// Children of the pixel of lane group g in the pass starting at grid pixel
// `first` (grid of width gw, grid stride gs in level pixels), with their W_A.
template <bool F16, int LOG2B>
__device__ __forceinline__ PassChildren<F16, ChildLayout<LOG2B>::CPL>
pass_children(const Geom& G, int first, int gw, float inv_gw, int ngrid, int gs, int lane,
              bool load_wa = true)
{
    using CL = ChildLayout<LOG2B>;
    PassChildren<F16, CL::CPL> pc;
    const int j = lane % CL::LPP, g = lane / CL::LPP;
    const int idx = first + g;
    int gu = 0, gv = 0;
    if (idx < ngrid) split_index(idx, gw, inv_gw, gu, gv);
#pragma unroll
    for (int m = 0; m < CL::CPL; ++m) {
        const int c = j + CL::LPP * m;
        pc.u[m] = __umul24(gu, gs * CL::B) + (c % CL::B);
        pc.v[m] = __umul24(gv, gs * CL::B) + (c / CL::B);
        pc.wa[m] = load_wa ? load_w<F16>(G.WA, __umul24(pc.v[m], G.w) + pc.u[m]) : 0.0f;
    }
    return pc;
}

// One pass: the GPP consecutive grid pixels first .. first+GPP-1.  Every lane
// of group g = lane / LPP returns the mean warped values of pixel first + g
// and whether all its children are warp-valid (the strict downsampling rule).
template <bool F16, int LOG2B>
__device__ __forceinline__ void warp_pass_pc(const Geom& G, const PassChildren<F16, ChildLayout<LOG2B>::CPL>& pc,
                                             int first, int ngrid, int lane, float& Io,
                                             float& Wo, bool& Vo, int& idxo)
{
    using CL = ChildLayout<LOG2B>;
    const int g = lane / CL::LPP;
    const int idx = first + g;
    bool ok = idx < ngrid;
    float sI = 0.0f, sW = 0.0f;
    // every child's tap loads first, then the arithmetic on them
    WarpTaps T[CL::CPL];
#pragma unroll
    for (int m = 0; m < CL::CPL; ++m) warp_fetch<F16>(G, pc.u[m], pc.v[m], pc.wa[m], T[m]);
#pragma unroll
    for (int m = 0; m < CL::CPL; ++m) {
        float ci, cw;
        const bool okc = warp_finish(G, T[m], ci, cw);
        ok = ok && okc;
        sI += ci;
        sW += cw;
    }
#pragma unroll
    for (int off = 1; off < CL::LPP; off <<= 1) {
        sI += __shfl_xor(sI, off);
        sW += __shfl_xor(sW, off);
    }
    bool gvalid = ok;
    if constexpr (CL::LPP > 1) {
        const unsigned long long bal = __ballot(ok);
        const unsigned long long full =
            CL::LPP == 64 ? ~0ull : ((1ull << CL::LPP) - 1ull) << (unsigned)(g * CL::LPP);
        gvalid = (bal & full) == full;
    }
    constexpr float invC = 1.0f / (float)CL::C;
    Io = sI * invC;
    Wo = sW * invC;
    Vo = gvalid;
    idxo = idx;
}

template <bool F16, int LOG2B>
__device__ __forceinline__ void warp_pass(const Geom& G, int first, int gw, float inv_gw, int ngrid,
                                          int gs, int lane, float& Io, float& Wo, bool& Vo,
                                          int& idxo)
{
    const auto pc = pass_children<F16, LOG2B>(G, first, gw, inv_gw, ngrid, gs, lane);
    warp_pass_pc<F16, LOG2B>(G, pc, first, ngrid, lane, Io, Wo, Vo, idxo);
}

// A tile of 64 consecutive grid pixels in LPP passes; afterwards lane L owns
// the tile pixel q = (L % LPP) * GPP + L / LPP.
template <bool F16, int LOG2B>
__device__ __forceinline__ void warp_tile(const Geom& G, int tile_first, int gw, float inv_gw,
                                          int ngrid, int gs, int lane, float& Io, float& Wo,
                                          bool& Vo, int& uo, int& vo, int& idxo)
{
    using CL = ChildLayout<LOG2B>;
    const int j = lane % CL::LPP, g = lane / CL::LPP;
    float mI = 0.0f, mW = 0.0f;
    bool mV = false;
#pragma unroll 1
    for (int k = 0; k < CL::LPP; ++k) {
        float pI, pW;
        bool pV;
        int pidx;
        warp_pass<F16, LOG2B>(G, tile_first + k * CL::GPP, gw, inv_gw, ngrid, gs, lane, pI, pW,
                              pV, pidx);
        if (j == k) {
            mI = pI;
            mW = pW;
            mV = pV;
        }
    }
    idxo = tile_first + j * CL::GPP + g;
    const bool in = idxo < ngrid;
    int gu = 0, gv = 0;
    if (in) split_index(idxo, gw, inv_gw, gu, gv);
    uo = gu * gs;
    vo = gv * gs;
    Io = mI;
    Wo = mW;
    Vo = in && mV;
}

// Residuals (and Jacobians) of one level pixel (sec. 6.2).  r_I needs an
// interior pixel, a valid W_A and warped values; r_W additionally the four
// W_A neighbours (central-difference gradient).  c is A's (I, W) at the
// pixel; the four neighbours are loaded at clamped (in-bounds) positions.
struct Terms {
    bool vI, vW;
    float rI, rW, lam;
    float JI[6], JW[6];
};

struct Nbrs {
    float2 l, r, t, b;
};

template <bool F16>
__device__ __forceinline__ Nbrs load_nbrs(const LevelView& A, int u, int v)
{
    const int i = (int)__umul24(v, A.w) + u;
    Nbrs n;
    n.l = load_iw<F16>(A.iw, u > 0 ? i - 1 : i);
    n.r = load_iw<F16>(A.iw, u < A.w - 1 ? i + 1 : i);
    n.t = load_iw<F16>(A.iw, v > 0 ? i - A.w : i);
    n.b = load_iw<F16>(A.iw, v < A.h - 1 ? i + A.w : i);
    return n;
}

__device__ __forceinline__ unsigned load_mask(const LevelView& A, unsigned i)
{
    return ld_at<unsigned char>(A.gm, i);
}

// Residuals of one level pixel (sec. 6.2) with c = A's (I, W) at the pixel
// and m its validity flags (bit 0: interior with valid W, bit 1: also the W
// gradient defined): r_I needs the warp and bit 0, r_W the warp and bit 1.
// JAC: also the Jacobians J = (a, X x a) of eq:res_int / eq:res_depth from
// the central differences of the neighbours n, and lambda_n.
template <bool JAC>
__device__ __forceinline__ void terms_core(const LevelView& A, float ifx, float ify, int u, int v,
                                           float2 c, const Nbrs& n, unsigned m, float Is, float Ws,
                                           bool wv, Terms& T)
{
    T.vI = wv && (m & 1u);
    T.vW = wv && (m & 2u);
    T.rI = Is - c.x;
    T.rW = Ws - c.y;
    if constexpr (JAC) {
        const float wa = c.y, Z = rcp(wa);
        const float du = A.cx - (float)u, dv = A.cy - (float)v;
        const float xu = -du * ifx, xv = -dv * ify;
        const float X0 = Z * xu, X1 = Z * xv, X2 = Z;
        const float gu = 0.5f * (n.r.x - n.l.x), gv = 0.5f * (n.b.x - n.t.x);
        const float a0 = wa * gu * A.fx, a1 = wa * gv * A.fy, a2 = wa * fmaf(gu, du, gv * dv);
        T.JI[0] = a0;
        T.JI[1] = a1;
        T.JI[2] = a2;
        T.JI[3] = X1 * a2 - X2 * a1;
        T.JI[4] = X2 * a0 - X0 * a2;
        T.JI[5] = X0 * a1 - X1 * a0;
        const float wu = 0.5f * (n.r.y - n.l.y), wv2 = 0.5f * (n.b.y - n.t.y);
        const float k0 = wu * A.fx, k1 = wv2 * A.fy, k2 = fmaf(wu, du, wv2 * dv);
        const float b0 = wa * k0, b1 = wa * k1, b2 = wa * (k2 + Ws);
        T.JW[0] = b0;
        T.JW[1] = b1;
        T.JW[2] = b2;
        T.JW[3] = X1 * b2 - X2 * b1;
        T.JW[4] = X2 * b0 - X0 * b2;
        T.JW[5] = X0 * b1 - X1 * b0;
        // n~ = Z grad W (K - p e_z^T) + e_z, n~ . x = 1, lambda = 1/(|n~||x|)
        const float n0 = Z * k0, n1 = Z * k1, n2 = fmaf(Z, k2, 1.0f);
        const float nn = fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
        const float xx = fmaf(xu, xu, fmaf(xv, xv, 1.0f));
        T.lam = rsq(nn * xx);
    }
}

template <bool F16, bool JAC>
__device__ __forceinline__ void pixel_terms(const LevelView& A, float ifx, float ify, int u, int v,
                                            float Is, float Ws, bool wv, Terms& T)
{
    const unsigned i = __umul24(v, A.w) + u;
    const float2 c = load_iw<F16>(A.iw, i);
    const unsigned m = load_mask(A, i);
    Nbrs n;
    if constexpr (JAC) n = load_nbrs<F16>(A, u, v);
    else n.l = n.r = n.t = n.b = c;
    terms_core<JAC>(A, ifx, ify, u, v, c, n, m, Is, Ws, wv, T);
}

// Robust weight of a normalised residual x: Huber min(1, k/|x|) or Student-t
// (nu + 1)/(nu + x^2) (sec. 6.3).  Both branches of the Huber rule are
// evaluated and selected, so the weight costs no divergent branch.
template <int KIND>
__device__ __forceinline__ float omega_k(float x, float nu, float k)
{
    if constexpr (KIND == RGBID_W_HUBER) {
        const float ax = fabsf(x);
        const float h = k * rcp(ax);
        return ax <= k ? 1.0f : h;
    } else {
        return (nu + 1.0f) * rcp(fmaf(x, x, nu));
    }
}

__device__ __forceinline__ float omega(int kind, float x, float nu, float k)
{
    return kind == RGBID_W_HUBER ? omega_k<RGBID_W_HUBER>(x, nu, k)
                                 : omega_k<RGBID_W_STUDENT_T>(x, nu, k);
}

__device__ __forceinline__ void accum(float* acc, const float* J, float w, float r)
{
    float s[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) s[a] = w * J[a];
    int k = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b) {
            acc[k] = fmaf(s[a], J[b], acc[k]);
            ++k;
        }
#pragma unroll
    for (int a = 0; a < 6; ++a) acc[21 + a] = fmaf(s[a], r, acc[21 + a]);
    acc[27] = fmaf(w * r, r, acc[27]);
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Grid of a level for the pixel kernels: the full level grid, or the sample
// grid (every s-th pixel in both directions).
struct GridDim {
    int gw, n, gs;
    float inv_gw;
};

__device__ __forceinline__ GridDim level_grid(const LevelView& A)
{
    GridDim d;
    d.gw = A.w;
    d.n = A.w * A.h;
    d.gs = 1;
    d.inv_gw = 1.0f / (float)A.w;
    return d;
}

__device__ __forceinline__ GridDim sample_grid(const PairDesc& D, int l)
{
    GridDim d;
    d.gw = D.sw[l];
    d.n = D.sw[l] * D.sh[l];
    d.gs = D.stride[l];
    d.inv_gw = 1.0f / (float)D.sw[l];
    return d;
}

// ------------------------------------------------------------------ k_warp

// Reference values a pass's group leader needs for its pixel's sample
// residuals: A's (I, W) at the pixel and its four neighbours (for the
// validity of the inverse-depth gradient).  Loaded one pass ahead, together
// with that pass's children, so the residual step has no dependent load.
struct SampleRef {
    int idx, sidx;      // grid index, sample index (-1: not a sample pixel)
    int u, v;           // level coordinates
    float2 c;
    unsigned m;
};

template <bool F16, int LOG2B>
__device__ __forceinline__ SampleRef sample_ref(const LevelView& A, const GridDim& gd, int first,
                                                int lane, bool fused, int s, int sw)
{
    using CL = ChildLayout<LOG2B>;
    SampleRef r;
    r.idx = first + lane / CL::LPP;
    r.sidx = -1;
    r.u = r.v = 0;
    r.c = make_float2(0.0f, 0.0f);
    r.m = 0;
    if ((lane % CL::LPP) != 0 || r.idx >= gd.n) return r;
    int gu, gv;
    split_index(r.idx, gd.gw, gd.inv_gw, gu, gv);
    r.u = gu * gd.gs;
    r.v = gv * gd.gs;
    if (fused) r.sidx = r.idx;
    else if ((r.u % s) == 0 && (r.v % s) == 0) r.sidx = (r.v / s) * sw + r.u / s;
    if (r.sidx >= 0) {
        const unsigned i = __umul24(r.v, A.w) + r.u;
        r.c = load_iw<F16>(A.iw, i);
        r.m = load_mask(A, i);
    }
    return r;
}

// Tiles of this kernel are single passes of GPP grid pixels.  The group
// leader of each pixel stores the warped values (store mode) and, for sample
// pixels, the two residuals (NaN = not defined).
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
    const Geom G = make_geom(S, D.A[wl], D.B[wl]);
    const LevelView A = D.A[l];
    const float ifx = 1.0f / A.fx, ify = 1.0f / A.fy;
    const bool fused = L.tune.fused;
    const GridDim gd = fused ? sample_grid(D, l) : level_grid(A);
    const int s = D.stride[l], sw = D.sw[l];
    void* const warped = D.warped;
    void* const sample = D.sample;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int end = ch.first + ch.count;
    int tile = ch.first + wave;
    // sample-only pass at level 0: the pixel is its own child, so W_A comes
    // with the reference values and the W plane is not read
    const bool own = LOG2B == 0 && fused;
    SampleRef sr = sample_ref<F16, LOG2B>(A, gd, tile * CL::GPP, lane, fused, s, sw);
    auto pc = pass_children<F16, LOG2B>(G, tile * CL::GPP, gd.gw, gd.inv_gw, gd.n, gd.gs, lane,
                                        !own);
    if (own) pc.wa[0] = sr.c.y;
    for (; tile < end; tile += waves) {
        float Is, Ws;
        bool wv;
        int idx;
        warp_pass_pc<F16, LOG2B>(G, pc, tile * CL::GPP, gd.n, lane, Is, Ws, wv, idx);
        // the next tile's children and reference values: their loads overlap
        // this tile's tail
        const int ntile = tile + waves < end ? tile + waves : tile;
        const SampleRef cur = sr;
        sr = sample_ref<F16, LOG2B>(A, gd, ntile * CL::GPP, lane, fused, s, sw);
        pc = pass_children<F16, LOG2B>(G, ntile * CL::GPP, gd.gw, gd.inv_gw, gd.n, gd.gs, lane,
                                       !own);
        if (own) pc.wa[0] = sr.c.y;
        if ((lane % CL::LPP) != 0 || idx >= gd.n) continue;
        if (!fused) store_f2(warped, idx, Is, wv ? Ws : 0.0f);
        if (cur.sidx < 0) continue;
        Terms T;
        Nbrs none;
        none.l = none.r = none.t = none.b = cur.c;
        terms_core<false>(A, ifx, ify, cur.u, cur.v, cur.c, none, cur.m, Is, Ws, wv, T);
        store_f2(sample, cur.sidx, T.vI ? T.rI : __int_as_float(0x7fc00000),
                 T.vW ? T.rW : __int_as_float(0x7fc00000));
    }
}

// ------------------------------------------------------------------ k_scale

// psi(x), x > 0: upward recurrence to x >= 12 then the Stirling-type series
// psi(x) ~ ln x - 1/(2x) - sum_k B_2k / (2k x^2k) (Abramowitz & Stegun 6.3.18).
__device__ double digamma_d(double x)
{
    double r = 0.0;
    while (x < 12.0) {
        r -= 1.0 / x;
        x += 1.0;
    }
    const double z = 1.0 / (x * x);
    const double series =
        z * (1.0 / 12 + z * (-1.0 / 120 + z * (1.0 / 252 + z * (-1.0 / 240 + z * (1.0 / 132)))));
    return r + log(x) - 0.5 / x - series;
}

// Sum of v over the 64 lanes of a wave, left in lane 63, with DPP: a scan
// inside each row of 16 lanes (row_shr 1, 2, 4, 8, zero fill), then the
// totals of rows 0 and 2 added into rows 1 and 3 (row_bcast:15), then the
// total of rows 0-1 into rows 2-3 (row_bcast:31).  A fixed order.
#define RGBID_DPP_ADD(v, ctrl, rows)                                                            \
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, rows, 0xf, true))

__device__ __forceinline__ float wave_sum_to_last(float v)
{
    RGBID_DPP_ADD(v, 0x111, 0xf);   // row_shr:1
    RGBID_DPP_ADD(v, 0x112, 0xf);   // row_shr:2
    RGBID_DPP_ADD(v, 0x114, 0xf);   // row_shr:4
    RGBID_DPP_ADD(v, 0x118, 0xf);   // row_shr:8
    RGBID_DPP_ADD(v, 0x142, 0xa);   // row_bcast:15 into rows 1 and 3
    RGBID_DPP_ADD(v, 0x143, 0xc);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Block totals of NV per-thread FP32 values, in FP64 and valid in wave 0
// only: every wave reduces its values (lane 63 stores them to LDS), then
// after a barrier wave 0 adds the per-wave values in wave order.  The scale
// kernel's FP64 step runs once per block (in wave 0) and its result reaches
// the other waves through LDS after a second barrier.
template <int NV>
__device__ __forceinline__ void block_totals(const float (&x)[NV], float* part, double (&tot)[NV])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const float w = wave_sum_to_last(x[k]);
        if (lane == 63) part[wave * NV + k] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
    if (wave == 0)
        for (int w = 0; w < nw; ++w)
#pragma unroll
            for (int k = 0; k < NV; ++k) tot[k] += (double)part[w * NV + k];
}

// n f_c(nu) with f_c(nu) = -psi(nu/2) + ln(nu/2) + psi((nu+1)/2) - ln((nu+1)/2):
// the data-free part of the left side of the nu equation of sec. 6.3
// (eq:robustnessValue); the data part is sum_i (1 + ln w_i - w_i).
__device__ __forceinline__ double nu_equation_const(double n, double nud)
{
    return n * (-digamma_d(0.5 * nud) + log(0.5 * nud) + digamma_d(0.5 * (nud + 1.0)) -
                log(0.5 * (nud + 1.0)));
}

// The location / scale fixed point with nu = 5 (Student-t) or the Huber
// threshold k: every step sums w, w d and w d^2 (d = r - mu, weights from
// the previous estimate) over the block and moves mu by S1/S0, sigma^2 to
// (S2 - S1^2/S0)/n.  Branch-free per element (padding entries get w = 0;
// entries past `per` are padding in every thread and skipped); two partial
// sums per lane in a fixed order.  bc[0..2] broadcast mu, sigma and 1/sigma.
template <int KIND>
__device__ __forceinline__ void scale_fixed_point(const float (&r)[kScalePerThread], int per,
                                                  double n, float floor_s, float k, int iters,
                                                  float* part, double* bc, double& mu,
                                                  double& sigma)
{
    const int wave = threadIdx.x >> 6;
    float fmu = (float)mu, isg = (float)(1.0 / sigma);
    for (int it = 0; it < iters; ++it) {
        // the weight of x = d / sigma written in d: Huber min(1, k sigma / |d|),
        // Student-t (nu + 1) sigma^2 / (nu sigma^2 + d^2) with nu = 5
        const float sg = 1.0f / isg;
        const float hk = k * sg, tA = 6.0f * sg * sg, tB = 5.0f * sg * sg;
        float s0[2] = {0.0f, 0.0f}, s1[2] = {0.0f, 0.0f}, s2[2] = {0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < kScalePerThread; ++q) {
            if (q < per) {
                const bool ok = r[q] == r[q];
                const float d = r[q] - fmu;
                float w;
                if constexpr (KIND == RGBID_W_HUBER) w = fminf(1.0f, hk * rcp(fabsf(d)));
                else w = tA * rcp(fmaf(d, d, tB));
                w = ok ? w : 0.0f;
                const float dd = ok ? d : 0.0f;
                s0[q & 1] += w;
                s1[q & 1] = fmaf(w, dd, s1[q & 1]);
                s2[q & 1] = fmaf(w * dd, dd, s2[q & 1]);
            }
        }
        const float acc[3] = {s0[0] + s0[1], s1[0] + s1[1], s2[0] + s2[1]};
        double tot[3];
        block_totals<3>(acc, part, tot);
        if (wave == 0) {
            // mu' = mu + S1/S0; sum w (r - mu')^2 = S2 - S1^2 / S0
            const double dm = tot[1] / tot[0];
            const double var = fmax((tot[2] - tot[1] * dm) / n, 0.0);
            const double sg = fmax(sqrt(var), (double)floor_s);
            if (threadIdx.x == 0) {
                bc[0] = mu + dm;
                bc[1] = sg;
                bc[2] = 1.0 / sg;
            }
        }
        __syncthreads();
        mu = bc[0];
        sigma = bc[1];
        fmu = (float)mu;
        isg = (float)bc[2];
    }
}

// One workgroup per (pair, channel): location mu and scale sigma of the
// channel's sample residuals by the fixed point of the two stationarity
// equations of sec. 6.3 (weights from the previous estimate), starting at
// mu = 0, sigma^2 = mean r^2, with nu = 5 for Student-t; then (Student-t with
// estimation) nu by bisection of the nu equation on [2, 10] with the
// normalised residuals frozen: f(10) > 0 gives 10, f(2) < 0 gives 2, else 30
// halvings of [2, 10] and the midpoint.
__global__ void __launch_bounds__(kScaleThreads) k_scale(IterLaunch L)
{
    __shared__ float part[16 * 3];
    __shared__ double bc[4];
    const int p = blockIdx.x, ch = blockIdx.y;
    PairState& S = L.states[p];
    if (!S.active || S.level_stop) return;
    const PairDesc& D = L.pairs[p];
    const int n_all = D.sw[L.level] * D.sh[L.level];
    const int per = (n_all + kScaleThreads - 1) / kScaleThreads;
    const int wave = threadIdx.x >> 6;
    const float floor_s = ch == 0 ? 1e-3f : 1e-6f;
    float r[kScalePerThread];
    float cs[2] = {0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kScalePerThread; ++k) {
        const int i = threadIdx.x + k * kScaleThreads;
        float x = __int_as_float(0x7fc00000);
        if (i < n_all) {
            const float2 e = load_f2(D.sample, i);
            x = ch == 0 ? e.x : e.y;
        }
        r[k] = x;
        const bool ok = x == x;
        cs[0] += ok ? 1.0f : 0.0f;
        cs[1] = ok ? fmaf(x, x, cs[1]) : cs[1];
    }
    {
        double t[2];
        block_totals<2>(cs, part, t);
        if (threadIdx.x == 0) {
            bc[0] = t[0];
            bc[1] = t[0] > 0.0 ? fmax(sqrt(t[1] / t[0]), (double)floor_s) : (double)floor_s;
        }
        __syncthreads();
    }
    const double n = bc[0];
    double mu = 0.0, sigma = bc[1];
    float nu = 5.0f;
    if (n > 0.0) {
        if (L.ip.weight == RGBID_W_HUBER)
            scale_fixed_point<RGBID_W_HUBER>(r, per, n, floor_s, L.ip.huber_k, L.ip.scale_iters,
                                             part, bc, mu, sigma);
        else
            scale_fixed_point<RGBID_W_STUDENT_T>(r, per, n, floor_s, L.ip.huber_k,
                                                 L.ip.scale_iters, part, bc, mu, sigma);
        if (L.ip.weight == RGBID_W_STUDENT_T && L.ip.estimate_nu) {
            const float fmu = (float)mu, isg = (float)(1.0 / sigma);
#pragma unroll
            for (int q = 0; q < kScalePerThread; ++q) {
                const float x = (r[q] - fmu) * isg;
                r[q] = x * x;     // r now holds x^2 (NaN stays NaN)
            }
            // evaluations f(10), f(2), then up to 30 bisection steps; the
            // bracket lives in wave 0, the next nu and the stop flag reach
            // every wave through LDS
            double lo = 2.0, hi = 10.0, nud = 10.0;
            for (int ev = 0;; ++ev) {
                const float nf = (float)nud;
                float e2[2] = {0.0f, 0.0f};
#pragma unroll
                for (int q = 0; q < kScalePerThread; ++q) {
                    if (q < per) {
                        // a padding entry (NaN) takes w = 1, whose term 1 + ln 1 - 1 is 0
                        const float w = r[q] == r[q] ? (nf + 1.0f) / (nf + r[q]) : 1.0f;
                        e2[q & 1] += 1.0f + logf(w) - w;
                    }
                }
                const float acc[1] = {e2[0] + e2[1]};
                double tot[1];
                block_totals<1>(acc, part, tot);
                if (wave == 0) {
                    const double f = nu_equation_const(n, nud) + tot[0];
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
                    if (threadIdx.x == 0) {
                        bc[2] = next;
                        bc[3] = stop ? 1.0 : 0.0;
                    }
                }
                __syncthreads();
                nud = bc[2];
                if (bc[3] != 0.0) break;
            }
            nu = (float)nud;
        }
    }
    if (threadIdx.x == 0) {
        S.mu[ch] = (float)mu;
        S.sigma[ch] = (float)sigma;
        S.nu[ch] = nu;
        S.ns[ch] = (int)n;
    }
}

// ------------------------------------------------------------------ k_reduce

template <bool F16, int LOG2B, bool FUSED>
__global__ void __launch_bounds__(512) k_reduce(IterLaunch L)
{
    __shared__ float lds[8 * kNSum];
    const int ci = chunk_of_block(blockIdx.x, L.n_red_chunks, L.tune.xcd_remap);
    const Chunk ch = L.red_chunks[ci];
    const PairState& S = L.states[ch.pair];
    if (!S.active || S.level_stop) return;
    const PairDesc& D = L.pairs[ch.pair];
    const int l = L.level;
    const LevelView A = D.A[l];
    const float ifx = 1.0f / A.fx, ify = 1.0f / A.fy;
    const GridDim gd = level_grid(A);
    const void* const warped = D.warped;

    const int kind = L.ip.weight;
    const float kh = L.ip.huber_k;
    const bool enI = S.ns[0] > 0, enW = S.ns[1] > 0;
    const float muI = S.mu[0], isI = 1.0f / S.sigma[0], muW = S.mu[1], isW = 1.0f / S.sigma[1];
    const float nuW = S.nu[1];
    const float nuI = (kind == RGBID_W_STUDENT_T && L.ip.estimate_nu) ? fmaxf(S.nu[0], nuW) : S.nu[0];
    const float wI0 = isI * isI, wW0 = isW * isW;

    float acc[kNSum];
#pragma unroll
    for (int k = 0; k < kNSum; ++k) acc[k] = 0.0f;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int end = ch.first + ch.count;
    const int wl = L.ip.warp_mode == RGBID_WARP_FULLRES ? 0 : l;
    const Geom G = make_geom(S, D.A[wl], D.B[wl]);
    if constexpr (FUSED && LOG2B == 0) {
        // The level pixel is its own warp child, so W_A comes with A's (I, W).
        // A's loads for the next tile are issued while this tile's gathers
        // from B are in flight.
        int tile = ch.first + wave;
        int idx = tile * 64 + lane;
        int ic = idx < gd.n ? idx : 0;
        int u, v;
        split_index(ic, gd.gw, gd.inv_gw, u, v);
        float2 c = load_iw<F16>(A.iw, ic);
        unsigned m = load_mask(A, ic);
        Nbrs nb = load_nbrs<F16>(A, u, v);
        for (; tile < end; tile += waves) {
            float Is, Ws;
            const bool wv = warp_core<F16>(G, u, v, c.y, Is, Ws) && idx < gd.n;
            const int ntile = tile + waves;
            const int nidx = ntile * 64 + lane;
            const int nic = (ntile < end && nidx < gd.n) ? nidx : ic;
            int nu, nv;
            split_index(nic, gd.gw, gd.inv_gw, nu, nv);
            const float2 nc = load_iw<F16>(A.iw, nic);
            const unsigned nm = load_mask(A, nic);
            const Nbrs nnb = load_nbrs<F16>(A, nu, nv);
            Terms T;
            terms_core<true>(A, ifx, ify, u, v, c, nb, m, Is, Ws, wv, T);
            if (T.vI && enI) {
                const float w = omega(kind, (T.rI - muI) * isI, nuI, kh) * wI0;
                accum(acc, T.JI, w, T.rI);
                acc[28] += 1.0f;
            }
            if (T.vW && enW) {
                const float w = T.lam * omega(kind, (T.rW - muW) * isW, nuW, kh) * wW0;
                accum(acc, T.JW, w, T.rW);
                acc[29] += 1.0f;
            }
            idx = nidx;
            ic = nic;
            u = nu;
            v = nv;
            c = nc;
            m = nm;
            nb = nnb;
        }
    } else {
        for (int tile = ch.first + wave; tile < end; tile += waves) {
            float Is = 0.0f, Ws = 0.0f;
            bool wv = false;
            int u = 0, v = 0, idx;
            if constexpr (FUSED) {
                warp_tile<F16, LOG2B>(G, tile * 64, gd.gw, gd.inv_gw, gd.n, 1, lane, Is, Ws, wv, u,
                                      v, idx);
            } else {
                idx = tile * 64 + lane;
                const int ic = idx < gd.n ? idx : 0;
                const float2 e = load_f2(warped, ic);
                Is = e.x;
                Ws = e.y;
                wv = Ws > 0.0f && idx < gd.n;
                split_index(ic, gd.gw, gd.inv_gw, u, v);
            }
            Terms T;
            pixel_terms<F16, true>(A, ifx, ify, u, v, Is, Ws, wv, T);
            if (T.vI && enI) {
                const float w = omega(kind, (T.rI - muI) * isI, nuI, kh) * wI0;
                accum(acc, T.JI, w, T.rI);
                acc[28] += 1.0f;
            }
            if (T.vW && enW) {
                const float w = T.lam * omega(kind, (T.rW - muW) * isW, nuW, kh) * wW0;
                accum(acc, T.JW, w, T.rW);
                acc[29] += 1.0f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kNSum; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kNSum; ++k) lds[wave * kNSum + k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x < kNSum) {
        // compensated (two-sum) FP32 sum over the waves of the workgroup
        float hi = 0.0f, lo = 0.0f;
        for (int w = 0; w < waves; ++w) {
            const float x = lds[w * kNSum + threadIdx.x];
            const float s = hi + x;
            const float bp = s - hi;
            lo += (hi - (s - bp)) + (x - bp);
            hi = s;
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
    const double c = cos(n), s = sin(n), oc = 1.0 - c;
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

__global__ void __launch_bounds__(64) k_solve(IterLaunch L)
{
    const int p = blockIdx.x;
    PairState& S = L.states[p];
    if (!S.active || S.level_stop) return;
    const int lane = threadIdx.x;
    const int beg = L.pair_red_begin[p], end = L.pair_red_begin[p + 1];
    double s[kNSum];
#pragma unroll
    for (int k = 0; k < kNSum; ++k) s[k] = 0.0;
    for (int c = beg + lane; c < end; c += 64) {
#pragma unroll
        for (int k = 0; k < kNSum; ++k) {
            const float2 q = load_f2(L.partials, (size_t)c * kNSum + k);
            s[k] += (double)q.x + (double)q.y;
        }
    }
#pragma unroll
    for (int k = 0; k < kNSum; ++k) s[k] = wave_sum_d(s[k]);
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
    double Lm[6][6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
        ok = ok && d > 1e-12 * dmax;
        Lm[j][j] = sqrt(ok ? d : 1.0);
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double e = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) e -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = e / Lm[j][j];
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
        y[i] = e / Lm[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double e = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) e -= Lm[k][i] * xi[k];
        xi[i] = e / Lm[i][i];
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
    if (i < n) states[i].level_stop = 0;
}

template <bool F16, int LOG2B>
hipError_t launch_iteration_t(hipStream_t s, const IterLaunch& L, hipEvent_t const* ev)
{
    const dim3 blk(64 * L.tune.waves);
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if (L.n_warp_chunks > 0)
        hipLaunchKernelGGL((k_warp<F16, LOG2B>), dim3(L.n_warp_chunks), blk, 0, s, L);
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scale, dim3(L.npairs, 2), dim3(kScaleThreads), 0, s, L);
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    if (L.n_red_chunks > 0) {
        if (L.tune.fused)
            hipLaunchKernelGGL((k_reduce<F16, LOG2B, true>), dim3(L.n_red_chunks), blk, 0, s, L);
        else
            hipLaunchKernelGGL((k_reduce<F16, LOG2B, false>), dim3(L.n_red_chunks), blk, 0, s, L);
    }
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_solve, dim3(L.npairs), dim3(64), 0, s, L);
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

hipError_t launch_level_start(hipStream_t s, PairState* states, int npairs)
{
    hipLaunchKernelGGL(k_level_start, dim3((npairs + 63) / 64), dim3(64), 0, s, states, npairs);
    return hipGetLastError();
}

}  // namespace rgbid
