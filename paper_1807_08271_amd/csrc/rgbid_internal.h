// Internal declarations of the gfx950 RGB-D alignment library: device-side
// tables, per-pair state and the host launchers of each kernel family.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rgbid.h"

namespace rgbid {

constexpr int kMaxLevels = 8;
constexpr int kWave = 64;
// 21 unique entries of H, 6 of g, cost, and the two valid-pixel counts.
constexpr int kNSum = 30;
constexpr int kScaleThreads = 1024;
constexpr int kScalePerThread = 24;   // sample_max <= 24576
constexpr int kMaxSample = kScaleThreads * kScalePerThread;

// Lane layout of the full-resolution warp for level pixels with
// C = 4^log2b children: each lane warps 1 child at log2b = 0, 2 at 1, 4 at 2
// and 8 from 3 on (independent load chains per lane: 8 measured slower at
// level 2 for the lower occupancy, faster at level 3, where a level pixel has
// 64 children; at level 1, 2 beat 4 and 1), C / that many lanes share a level
// pixel, and a 64-lane pass
// covers 64 / that pixels.  Host launch tables and kernels both use these.
constexpr int warp_children_per_lane(int log2b)
{
    return log2b == 0 ? 1 : log2b == 1 ? 2 : log2b == 2 ? 4 : 8;
}
// Tiles of the reduction at a level: 64 consecutive pixels in raster order,
// or, where the reduction warps its own pixels one to one (fused, one child
// per pixel), blocks of kBlockW x kBlockH pixels (a lane per pixel, row by
// row), so that a tile's neighbours and bilinear taps mostly fall inside the
// lines the tile itself reads.
constexpr int kBlockW = 16, kBlockH = 4;
inline long long reduce_tiles(int w, int h, bool blocks)
{
    return blocks ? (long long)((w + kBlockW - 1) / kBlockW) * ((h + kBlockH - 1) / kBlockH)
                  : ((long long)w * h + 63) / 64;
}
constexpr int warp_lanes_per_pixel(int log2b) { return (1 << (2 * log2b)) / warp_children_per_lane(log2b); }
constexpr int warp_pixels_per_pass(int log2b) { return 64 / warp_lanes_per_pixel(log2b); }

// One pyramid level as the kernels see it.
struct LevelView {
    const void* iw;   // interleaved (I, W): float2 or __half2, w*h, dense rows
    const void* wp;   // W plane: float or __half, w*h
    const unsigned char* gm;   // per pixel: bit 0 interior with valid W, bit 1 also
                               // the four W neighbours valid (gradient defined)
    int w, h;
    float fx, fy, cx, cy;
};

// Everything a kernel needs to know about one pair; uploaded per call.
struct PairDesc {
    LevelView A[kMaxLevels];
    LevelView B[kMaxLevels];
    float2* warped;                 // store mode: warped (I*, W*) of the level grid
    float2* sample;                 // sample residuals (r_I, r_W), NaN = invalid
    int stride[kMaxLevels];         // systematic-sample stride per level
    int sw[kMaxLevels], sh[kMaxLevels];
};

// Per-pair iteration state, resident in device memory for a whole alignment.
struct PairState {
    double R[9], t[3];              // current estimate of T_A^B
    double H[21], g[6], cost;       // last linearisation
    long long nI, nW;
    float RT[9];                    // R^T, row-major (FP32 copy for the warp)
    float Rtt[3];                   // R^T t
    float mu[2], sigma[2], nu[2];   // channel 0 = intensity, 1 = inverse depth
    int ns[2];                      // valid sample sizes
    int iters_done[kMaxLevels];
    int status;                     // rgbid_status
    int active;                     // 1 while the pair iterates
    int level_stop;                 // early stop reached at the current level
    int pad;
};

// A contiguous range of 64-pixel tiles of one pair's grid.
struct Chunk {
    int pair;
    int first;
    int count;
};

// Kernel-visible constants of one alignment call.
struct IterParams {
    int weight;          // rgbid_weight
    float huber_k;
    int estimate_nu;
    int scale_iters;
    int warp_mode;       // rgbid_warp_mode
    int scale_warm;      // warm-started scale fixed point with the convergence stop
    double stop_eps_t, stop_eps_r;
};

// Launch shape of one level (picked by the autotuner or the defaults).
struct LevelTune {
    int fused;           // 1: reduce kernel warps itself; 0: warped images stored
    int waves;           // waves per workgroup of the pixel kernels
    int tiles_per_wave;  // tiles each wave of the reduction walks
    int xcd_remap;       // map consecutive chunks onto one XCD
    int warp_passes;     // passes each wave of the warp kernel walks
};

// ---------------------------------------------------------------- launchers

// One frame of a (batched) pyramid build.  Level 0 is read from the caller's
// FP32 images; level l+1 is built from level l.
struct PyrFrame {
    const float* I;
    const float* W;
    long long pitch;                // elements
    void* iw[kMaxLevels];
    void* wp[kMaxLevels];
    void* gm[kMaxLevels];
    int w[kMaxLevels], h[kMaxLevels];
    int levels;
    int pad;
};
// quad: every frame is a multiple of 4 wide, its pitch a multiple of 4 and its
// I and W 16-byte aligned (level 0 then moves four pixels per thread); pairs:
// quad and every frame an even number of rows high (levels 0 and 1 and the
// level-0 flags are then formed in one pass)
hipError_t launch_pyramid(hipStream_t s, const PyrFrame* frames_dev, int nframes, int levels,
                          int f16, const int* max_w, const int* max_h, bool quad, bool pairs);
hipError_t launch_level_read(hipStream_t s, const void* iw, int n, int f16, float* I, float* W);

// One Gauss-Newton iteration (or one linearisation without update) for all
// pairs of a batch at `level`.
struct IterLaunch {
    const PairDesc* pairs;
    PairState* states;
    int npairs;
    int level;
    IterParams ip;
    LevelTune tune;
    int f16;
    int block_log2;          // FULLRES: level (2^level children per side); PER_LEVEL: 0
    const Chunk* warp_chunks;
    int n_warp_chunks;
    const Chunk* red_chunks;
    int n_red_chunks;
    const int* pair_red_begin;   // npairs + 1
    float2* partials;            // n_red_chunks * kNSum
    int update;                  // 0: normal equations only
    int scale_per;               // sample entries per scale thread: ceil(max sample / kScaleThreads)
    int kernels;                 // kernels to launch: 1 warp, 2 scale, 4 reduce, 8 solve
};
// ev: NULL, or 5 events recorded before the warp kernel and after each of
// the four kernels (for per-kernel timing).
hipError_t launch_iteration(hipStream_t s, const IterLaunch& L, hipEvent_t const* ev);
hipError_t launch_level_start(hipStream_t s, PairState* states, int npairs);
// Initial poses of n pairs from normalised twists o (n x 6, device): xi =
// o * scale, T = (exp(theta), v), written into the states (pose, its FP32
// copies); the rest of each state is left as uploaded.
hipError_t launch_init_from_twist(hipStream_t s, PairState* states, int n, const float* o,
                                  const double scale[6]);
hipError_t launch_export(hipStream_t s, const PairState* states, int n, rgbid_pose* out,
                         rgbid_align_stats* stats);

// Device-side set-up of the allocation-free single-pair alignment: the pair
// descriptor, its initial state and the chunk tables are written from the
// kernel arguments into device memory the caller provides (no host-to-device
// copy, no staging buffer).  The chunk tables are nseg segments back to back:
// segment k covers seg_tiles[k] tiles in chunks of seg_per[k] tiles, chunks
// seg_first[k] .. seg_first[k + 1] - 1 (seg_first[nseg] = all chunks).
constexpr int kNoAllocSegs = 2 * kMaxLevels;
struct NoAllocSetup {
    PairDesc desc;
    PairState state;
    PairDesc* desc_dev;
    PairState* state_dev;
    Chunk* chunks;
    int* begins;                         // per level: {0, reduction chunks}
    int levels;
    int nseg;
    int seg_first[kNoAllocSegs + 1];
    int seg_tiles[kNoAllocSegs];
    int seg_per[kNoAllocSegs];
    int n_red[kMaxLevels];
};
hipError_t launch_noalloc_setup(hipStream_t s, const NoAllocSetup& a);

struct FuseArgs {
    float* Wkf;
    float* Ckf;
    const float* Wk;
    long long pitch;
    int w, h;
    float fx, fy, cx, cy;
    float D[9];           // R^T - I for the pose of frame k in the keyframe (formed in FP64)
    float Rtt[3];         // R^T t
    float tol;
    unsigned long long* count;
};
hipError_t launch_fuse(hipStream_t s, const FuseArgs& a);

// A frame of a batched fusion (device-side table).
struct FuseFrame {
    const float* Wk;
    float D[9];     // R^T - I (formed in FP64)
    float Rtt[3];   // R^T t
};
constexpr int kMaxFuseBatch = 256;
struct FuseBatchArgs {
    float* Wkf;
    float* Ckf;
    const FuseFrame* frames;      // n entries in device memory
    int n;
    long long pitch;              // of every W_k
    int w, h;
    float fx, fy, cx, cy;
    float tol;
    unsigned long long* count;    // n counters, or NULL
};
hipError_t launch_fuse_batch(hipStream_t s, const FuseBatchArgs& a);
hipError_t launch_fill(hipStream_t s, float* p, int n, float v);

struct CovisArgs {
    const void* WA;       // W planes of one pyramid level (float or __half)
    const void* WB;
    int f16;
    int w, h;
    float fx, fy, cx, cy;
    float D[9];           // R^T - I for the pose of B in A (formed in FP64)
    float Rtt[3];         // R^T t
    float tol;
    unsigned long long* count;   // [0] += |S_H|, [1] += |S_V|
};
hipError_t launch_covis(hipStream_t s, const CovisArgs& a);
hipError_t launch_bilateral(hipStream_t s, const void* iw, int f16, int w, int h, int radius,
                            float sigma_s, float sigma_I, float rel_W, float* Io, float* Wo);
// Dense copy of a pitched inverse-depth map with holes normalised to 0.
hipError_t launch_copy_valid(hipStream_t s, const float* src, long long pitch, int w, int h,
                             float* dst);

// ---------------------------------------------------------------- sensor input path

// A lens on the device: pinhole part and Brown distortion k1..k5.
struct LensF {
    int w, h;
    float fx, fy, cx, cy;
    float k[5];
};

// Depth correction: beta0, beta1, the correlation-window shift and the two
// nine-term polynomials (q0: offset D0, q1: factor D1).
struct DepthCorrF {
    float beta0, beta1;
    int p0x, p0y;
    int spatial;
    float q0[9], q1[9];
};

struct RotF {
    float m[9];
};

// Forward registration of camera A's inverse depth into camera B with
// T_A^B; raw = 1 reads raw depth and applies the correction and A's lens.
struct RegisterArgs {
    const float* src;
    long long pitch;
    int raw;
    LensF A, B;
    DepthCorrF D;
    float tx, ty, tz;       // K_A t
    RotF R;                 // R_A^B
    unsigned* Wt;           // intermediate frame B_t (A's grid), as float bits
    float* Wout;            // B's grid, dense
    const float* Iraw;      // optional colour image to undistort on B's grid
    long long pitchI;
    float* Iout;
};

hipError_t launch_undistort(hipStream_t s, const float* src, long long pitch, const LensF& L,
                            int is_depth, float* dst);
hipError_t launch_register(hipStream_t s, const RegisterArgs& a);

// ---------------------------------------------------------------- warm start

constexpr int kCnnH = 60, kCnnW = 80;
constexpr int kCnnCh[5] = {4, 32, 64, 128, 128};
constexpr int kCnnHs[5] = {60, 30, 15, 8, 4};
constexpr int kCnnWs[5] = {80, 40, 20, 10, 5};
// parameter layout: w1 b1 w2 b2 w3 b3 w4 b4 wfc bfc (conv weights Co x Ci x 3 x 3)
constexpr int kCnnOff[11] = {0,      1152,   1184,   19616,  19680, 93408,
                             93536,  240992, 241120, 241888, 241894};
constexpr int kCnnParams = 241894;

// The 80x60 level of one pair's pyramids.
struct CnnInput {
    const void* A;     // interleaved (I, W) of A at the 80x60 level
    const void* B;
    int f16;
    int pad;
};

struct CnnBuffers {
    float* w;              // FP32 master parameters
    float* m;              // AdamW moments
    float* v;
    float* grad;
    float* decay;          // 1 for weights, 0 for biases
    __hip_bfloat16* wbf;   // bf16 copy used by forward / backward
    float* act[4];         // post-ReLU activations of the conv layers
    float* dz[4];          // gradients w.r.t. the pre-activations
    float* pooled;         // N x 128
    float* out;            // N x 6 (normalised twist)
    float* dout;
    float* loss_n;
    float* target;         // N x 6
};

hipError_t cnn_input(hipStream_t s, const CnnInput* in_dev, int n, float* x);
hipError_t cnn_forward(hipStream_t s, const CnnBuffers& B, int N, const float* x);
hipError_t cnn_backward(hipStream_t s, const CnnBuffers& B, int N, const float* x,
                        const float* target);
hipError_t cnn_adamw(hipStream_t s, const CnnBuffers& B, float lr, float wd, int step);
hipError_t cnn_refresh_bf16(hipStream_t s, const CnnBuffers& B);

// Inference forward on the matrix cores (cnn_mfma.hip): the input assembled
// from the pyramids' 80x60 level and the four convolutions as implicit GEMMs
// of bf16 weights and three-limb bf16 activations with FP32 accumulation;
// writes the normalised output (N x 6) to `out`.  wg holds the weights in
// GEMM order (cnn_gemm_weights, sum over layers of Co x cnn_gemm_k(l)
// elements); limbs holds cnn_limb_bytes(N) bytes.
int cnn_gemm_k(int layer);
size_t cnn_limb_bytes(int N);
hipError_t cnn_gemm_weights(hipStream_t s, const CnnBuffers& B, unsigned short* wg);
hipError_t cnn_forward_mfma(hipStream_t s, const CnnBuffers& B, const unsigned short* wg,
                            const CnnInput* in_dev, int N, unsigned short* limbs, float* out);

}  // namespace rgbid
