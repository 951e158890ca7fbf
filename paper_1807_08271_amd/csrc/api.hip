// C ABI of the library (include/rgbid.h): contexts, pyramids, the batched
// coarse-to-fine alignment driver with HIP-graph replay, normal equations and
// keyframe fusion.  All device work of the method runs in the kernels of
// pyramid.hip, align.hip and fuse.hip; this file validates arguments, lays
// out device tables and enqueues launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "rgbid_internal.h"

using namespace rgbid;

struct rgbid_pyr {
    int device;
    rgbid_camera cam;
    int levels;
    int f16;
    int w[kMaxLevels], h[kMaxLevels];
    double fx[kMaxLevels], fy[kMaxLevels], cx[kMaxLevels], cy[kMaxLevels];
    void* base;
    void* iw[kMaxLevels];
    void* wp[kMaxLevels];
    void* gm[kMaxLevels];
};

struct rgbid_kf {
    int device;
    rgbid_camera cam;
    float* W;
    float* C;
    unsigned long long* count;
    void* base;
};

struct rgbid_net {
    int device;
    rgbid::CnnBuffers buf;
    void* base;           // parameters, moments, gradient, bf16 copy
    void* act_base;       // activations for `cap` samples
    int cap;
    int step;
    void* inf_base;       // matrix-core inference: GEMM-order weights, limb activations, output
    int inf_cap;
    int wg_step;          // training step the GEMM-order weights were made at (-1: none)
};

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Launch tables of one batch shape, laid out in one device buffer.
struct LevelTables {
    size_t warp_off, red_off, begin_off;   // byte offsets into the table buffer
    int n_warp, n_red;
};

}  // namespace

struct rgbid_ctx {
    int device = 0;
    hipStream_t stream = nullptr;    // work stream (the caller's)
    hipStream_t cap = nullptr;       // private stream for graph capture
    std::string err;
    DevBuf pairs, states, tables, partials, warped, sample, frames, covis, cov_img, reg, fuse;
    rgbid_pyr* cov_pyr = nullptr;    // filtered reference of the covariance iteration
    void* h_stage = nullptr;         // pinned upload staging
    size_t h_stage_bytes = 0;
    hipEvent_t stage_done = nullptr; // last upload from h_stage finished
    void* h_down = nullptr;          // pinned download buffer
    size_t h_down_bytes = 0;
    int generation = 0;              // bumps when a workspace buffer moves
    bool use_graphs = true;
    std::map<std::string, std::vector<hipGraphExec_t>> graphs;   // one graph per chain
    std::map<std::string, LevelTune> tunes;   // per (level shape) launch shape
    hipEvent_t tev[2] = {nullptr, nullptr};   // launch-region timing (autotuner)
    int chains = 4;                           // parallel branches of a batch graph
    std::vector<hipStream_t> chain_streams;   // capture streams of branches 1..
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    bool profiling = false;
    void* scratch_dev = nullptr;     // this device's copy of `scratch` (allocation-free call)
    std::vector<hipEvent_t> events;  // timing events, grown on demand
    double prof_ms[kMaxLevels * 4] = {};
    long long prof_n[kMaxLevels * 4] = {};
};

// Device memory of the allocation-free alignment (rgbid_align_noalloc):
// descriptor, state, chunk tables, partial sums, sample residuals and the
// stored warped level images of one pair.  Each device holds its own copy
// for the life of the process; kernels reach it only through the address
// hipGetSymbolAddress returns on that device (the array's name in host code
// is a host-side stand-in).
constexpr size_t kScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

rgbid_status set_err(rgbid_ctx* c, rgbid_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return set_err((ctx), e_ == hipErrorOutOfMemory ? RGBID_E_NOMEM : RGBID_E_DEVICE,   \
                           "%s failed: %s", #expr, hipGetErrorString(e_));                     \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

rgbid_status ensure(rgbid_ctx* c, DevBuf& b, size_t bytes)
{
    if (b.bytes >= bytes) return RGBID_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (b.p) HIPCHK(c, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    const size_t nb = align_up(bytes + bytes / 4, 4096);
    HIPCHK(c, hipMalloc(&b.p, nb));
    b.bytes = nb;
    c->generation++;
    return RGBID_OK;
}

// Host staging for uploads: one region per call; the next call waits for the
// previous upload to have left the pinned buffer.
rgbid_status stage_begin(rgbid_ctx* c, size_t bytes, char** out)
{
    HIPCHK(c, hipEventSynchronize(c->stage_done));
    if (c->h_stage_bytes < bytes) {
        if (c->h_stage) HIPCHK(c, hipHostFree(c->h_stage));
        c->h_stage = nullptr;
        c->h_stage_bytes = 0;
        const size_t nb = align_up(bytes + bytes / 4, 4096);
        HIPCHK(c, hipHostMalloc(&c->h_stage, nb, hipHostMallocDefault));
        c->h_stage_bytes = nb;
    }
    *out = static_cast<char*>(c->h_stage);
    return RGBID_OK;
}

rgbid_status stage_end(rgbid_ctx* c)
{
    HIPCHK(c, hipEventRecord(c->stage_done, c->stream));
    return RGBID_OK;
}

rgbid_status ensure_down(rgbid_ctx* c, size_t bytes)
{
    if (c->h_down_bytes >= bytes) return RGBID_OK;
    if (c->h_down) HIPCHK(c, hipHostFree(c->h_down));
    c->h_down = nullptr;
    c->h_down_bytes = 0;
    const size_t nb = align_up(bytes + bytes / 4, 4096);
    HIPCHK(c, hipHostMalloc(&c->h_down, nb, hipHostMallocDefault));
    c->h_down_bytes = nb;
    return RGBID_OK;
}

// Scale of the warm-start network's normalised output: (0.15 m) x 3, (0.1745 rad) x 3.
const double kXiScale[6] = {0.15, 0.15, 0.15, 0.1745, 0.1745, 0.1745};

// Smallest stride s >= 1 whose sample grid ceil(w/s) x ceil(h/s) has at most
// nmax pixels (systematic sample of maximum size N, sec. 6.3).
int sample_stride(int w, int h, int nmax)
{
    int s = 1;
    while ((long long)((w + s - 1) / s) * ((h + s - 1) / s) > nmax) ++s;
    return s;
}

void level_camera(const rgbid_camera& c0, int l, double& fx, double& fy, double& cx, double& cy)
{
    const double s = std::ldexp(1.0, -l);
    fx = c0.fx * s;
    fy = c0.fy * s;
    cx = (c0.cx + 0.5) * s - 0.5;
    cy = (c0.cy + 0.5) * s - 0.5;
}

LevelTune default_tune(int block_log2)
{
    LevelTune t;
    if (block_log2 == 0) {
        t.fused = 1;
        t.waves = 4;
        t.tiles_per_wave = 8;
        t.warp_passes = 1;
    } else {
        t.fused = 0;
        t.waves = 4;
        t.tiles_per_wave = 2;
        t.warp_passes = 4;
    }
    t.xcd_remap = 1;
    return t;
}

void pose_floats(const double R[9], const double t[3], float RT[9], float Rtt[3])
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) RT[3 * i + j] = (float)R[3 * j + i];
        Rtt[i] = (float)(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
    }
}

// The pose for the displacement form of a transfer: D = R^T - I, formed in
// FP64 before rounding (its entries are small for small motions and keep
// their relative precision), and R^T t.
void pose_flow_floats(const double R[9], const double t[3], float D[9], float Rtt[3])
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) D[3 * i + j] = (float)(R[3 * j + i] - (i == j ? 1.0 : 0.0));
        Rtt[i] = (float)(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
    }
}

// NULL if the parameters are usable, else a static description.
const char* params_problem(const rgbid_align_params* p)
{
    if (!p) return "params is NULL";
    if (p->levels < 1 || p->levels > kMaxLevels) return "levels outside 1..8";
    for (int l = 0; l < p->levels; ++l)
        if (p->iters[l] < 0 || p->iters[l] > 10000) return "iters outside 0..10000";
    if (p->weight != RGBID_W_STUDENT_T && p->weight != RGBID_W_HUBER) return "unknown weight";
    if (!(p->huber_k > 0.0)) return "huber_k must be > 0";
    if (p->sample_max < 1 || p->sample_max > kMaxSample) return "sample_max outside 1..24576";
    if (p->scale_iters < 0 || p->scale_iters > 1000) return "scale_iters outside 0..1000";
    if (p->warp != RGBID_WARP_FULLRES && p->warp != RGBID_WARP_PER_LEVEL) return "unknown warp mode";
    if (p->warp == RGBID_WARP_FULLRES && p->levels > 5) return "FULLRES warp supports at most 5 levels";
    if (p->stop_eps_t < 0 || p->stop_eps_r < 0) return "negative stop epsilon";
    if (p->scale_warm != 0 && p->scale_warm != 1) return "scale_warm must be 0 or 1";
    return nullptr;
}

bool params_ok(const rgbid_align_params* p, std::string& why)
{
    const char* e = params_problem(p);
    if (e) why = e;
    return !e;
}

struct Step {
    int level;
    int iters;
};

// Launch shapes are tuned per batch shape: level, warp mode, storage format
// and the run-length encoded list of pair sizes.
std::string tune_key(int n, const rgbid_pyr* const* A, int level, int warp, int f16)
{
    char buf[64];
    snprintf(buf, sizeof buf, "l%d_m%d_f%d", level, warp, f16);
    std::string k = buf;
    int i = 0;
    while (i < n) {
        int j = i;
        while (j < n && A[j]->w[0] == A[i]->w[0] && A[j]->h[0] == A[i]->h[0]) ++j;
        snprintf(buf, sizeof buf, "_%dx%dx%d", A[i]->w[0], A[i]->h[0], j - i);
        k += buf;
        i = j;
    }
    return k;
}

void clear_graphs(rgbid_ctx* c)
{
    // an asynchronous call may still run a graph: let every stream drain first
    if (!c->graphs.empty()) {
        (void)hipStreamSynchronize(c->stream);
        for (hipStream_t s : c->chain_streams) (void)hipStreamSynchronize(s);
    }
    for (auto& kv : c->graphs)
        for (hipGraphExec_t g : kv.second) (void)hipGraphExecDestroy(g);
    c->graphs.clear();
}

// Streams (default priority) and fork / join events for the chains of a
// batch; chain 0 runs on the context's stream.
rgbid_status ensure_chain_streams(rgbid_ctx* c, int nch)
{
    if (!c->fork) HIPCHK(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    while ((int)c->chain_streams.size() < nch - 1) {
        hipStream_t s;
        HIPCHK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c->chain_streams.push_back(s);
        hipEvent_t e;
        HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->joins.push_back(e);
    }
    return RGBID_OK;
}

// The batched driver: n pairs, a schedule of (level, iterations), update on
// or off.  Writes poses and stats (host) and returns OK unless an argument or
// the device failed.
rgbid_status run_batch(rgbid_ctx* c, int n, const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                       const rgbid_pose* init, const rgbid_align_params* P,
                       const std::vector<Step>& sched, int update, rgbid_pose* out,
                       rgbid_align_stats* stats, float* launch_ms = nullptr,
                       bool device_out = false, const float* init_twist_dev = nullptr)
{
    if (!c) return RGBID_E_ARG;
    if (n < 1 || !A || !B) return set_err(c, RGBID_E_ARG, "need n >= 1 and pyramid arrays");
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    const int f16 = A[0] ? A[0]->f16 : 0;
    for (int i = 0; i < n; ++i) {
        if (!A[i] || !B[i]) return set_err(c, RGBID_E_ARG, "pyramid %d is NULL", i);
        if (A[i]->device != c->device || B[i]->device != c->device)
            return set_err(c, RGBID_E_ARG, "pyramid %d lives on another device", i);
        if (A[i]->w[0] != B[i]->w[0] || A[i]->h[0] != B[i]->h[0] || A[i]->f16 != B[i]->f16)
            return set_err(c, RGBID_E_SHAPE, "pair %d: A and B differ in size or format", i);
        if (A[i]->cam.fx != B[i]->cam.fx || A[i]->cam.fy != B[i]->cam.fy ||
            A[i]->cam.cx != B[i]->cam.cx || A[i]->cam.cy != B[i]->cam.cy)
            return set_err(c, RGBID_E_SHAPE, "pair %d: A and B have different cameras", i);
        if (A[i]->levels < P->levels || B[i]->levels < P->levels)
            return set_err(c, RGBID_E_SHAPE, "pair %d: pyramid has fewer levels than params", i);
        if (A[i]->f16 != f16)
            return set_err(c, RGBID_E_SHAPE, "all pyramids of a batch need one storage format");
    }
    const int L = P->levels;
    const bool fullres = P->warp == RGBID_WARP_FULLRES;

    // ---- chains: with graphs, the batch is split into independent groups of
    // pairs captured as parallel branches, so one group's latency-bound
    // kernels (scale, solve) overlap another group's pixel kernels.
    const bool graphed = c->use_graphs && !c->profiling;
    const int nch = graphed ? std::max(1, std::min(c->chains, n)) : 1;
    std::vector<int> cfirst(nch + 1, n);
    {
        long long tot = 0, cum = 0;
        for (int i = 0; i < n; ++i) tot += (long long)A[i]->w[0] * A[i]->h[0];
        cfirst[0] = 0;
        int k = 1;
        for (int i = 0; i < n && k < nch; ++i) {
            cum += (long long)A[i]->w[0] * A[i]->h[0];
            if (cum * nch >= tot * k && i + 1 < n) cfirst[k++] = i + 1;
        }
        for (; k < nch; ++k) cfirst[k] = n;
        cfirst[nch] = n;
    }

    // ---- launch shapes and tables
    LevelTune tune[kMaxLevels];
    std::vector<int> stride(n * L), sw(n * L), sh(n * L);
    // [chain][level]
    std::vector<std::vector<std::vector<Chunk>>> wch(nch, std::vector<std::vector<Chunk>>(L)),
        rch(nch, std::vector<std::vector<Chunk>>(L));
    std::vector<std::vector<std::vector<int>>> rbeg(nch, std::vector<std::vector<int>>(L));
    std::vector<std::vector<int>> scale_per(nch, std::vector<int>(L, 1));
    std::vector<size_t> max_red(nch, 0);
    size_t warped_per_pair_total = 0;
    std::vector<size_t> warped_off(n, 0);
    for (int l = 0; l < L; ++l) {
        const int b = fullres ? l : 0;
        const std::string key = tune_key(n, A, l, P->warp, f16);
        auto it = c->tunes.find(key);
        tune[l] = it != c->tunes.end() ? it->second : default_tune(b);
        const int gpp = warp_pixels_per_pass(b);
        const int rtiles_per_chunk = tune[l].waves * tune[l].tiles_per_wave;
        const int wtiles_per_chunk = tune[l].waves * tune[l].warp_passes;
        for (int k = 0; k < nch; ++k) {
            rbeg[k][l].push_back(0);
            for (int i = cfirst[k]; i < cfirst[k + 1]; ++i) {
                const int li = i - cfirst[k];
                const int w = A[i]->w[l], h = A[i]->h[l];
                const int s = sample_stride(w, h, P->sample_max);
                stride[i * L + l] = s;
                sw[i * L + l] = (w + s - 1) / s;
                sh[i * L + l] = (h + s - 1) / s;
                const int per = (sw[i * L + l] * sh[i * L + l] + kScaleThreads - 1) / kScaleThreads;
                scale_per[k][l] = std::max(scale_per[k][l], per);
                const long long ngrid = tune[l].fused ? (long long)sw[i * L + l] * sh[i * L + l]
                                                      : (long long)w * h;
                const long long wt = (ngrid + gpp - 1) / gpp;
                for (long long t = 0; t < wt; t += wtiles_per_chunk)
                    wch[k][l].push_back(
                        Chunk{li, (int)t, (int)std::min<long long>(wtiles_per_chunk, wt - t)});
                const long long rt = reduce_tiles(w, h, tune[l].fused && b == 0);
                for (long long t = 0; t < rt; t += rtiles_per_chunk)
                    rch[k][l].push_back(
                        Chunk{li, (int)t, (int)std::min<long long>(rtiles_per_chunk, rt - t)});
                rbeg[k][l].push_back((int)rch[k][l].size());
            }
            max_red[k] = std::max(max_red[k], rch[k][l].size());
        }
    }
    std::vector<size_t> poff(nch + 1, 0);
    for (int k = 0; k < nch; ++k) poff[k + 1] = poff[k] + max_red[k];
    for (int i = 0; i < n; ++i) {
        size_t need = 0;
        for (int l = 0; l < L; ++l)
            if (!tune[l].fused) need = std::max(need, (size_t)A[i]->w[l] * A[i]->h[l]);
        warped_off[i] = warped_per_pair_total;
        warped_per_pair_total += align_up(need, 64);
    }

    // ---- workspace
    rgbid_status st;
    size_t tbytes = 0;
    std::vector<std::vector<LevelTables>> lt(nch, std::vector<LevelTables>(L));
    for (int k = 0; k < nch; ++k)
        for (int l = 0; l < L; ++l) {
            lt[k][l].warp_off = tbytes;
            tbytes = align_up(tbytes + wch[k][l].size() * sizeof(Chunk), 256);
            lt[k][l].red_off = tbytes;
            tbytes = align_up(tbytes + rch[k][l].size() * sizeof(Chunk), 256);
            lt[k][l].begin_off = tbytes;
            tbytes = align_up(tbytes + rbeg[k][l].size() * sizeof(int), 256);
            lt[k][l].n_warp = (int)wch[k][l].size();
            lt[k][l].n_red = (int)rch[k][l].size();
        }
    if ((st = ensure(c, c->pairs, n * sizeof(PairDesc))) != RGBID_OK) return st;
    if ((st = ensure(c, c->states, n * sizeof(PairState))) != RGBID_OK) return st;
    if ((st = ensure(c, c->tables, tbytes)) != RGBID_OK) return st;
    if ((st = ensure(c, c->partials, std::max<size_t>(1, poff[nch]) * kNSum * sizeof(float2))) != RGBID_OK) return st;
    if ((st = ensure(c, c->warped, std::max<size_t>(1, warped_per_pair_total) * sizeof(float2))) != RGBID_OK) return st;
    if ((st = ensure(c, c->sample, (size_t)n * P->sample_max * sizeof(float2))) != RGBID_OK) return st;

    // ---- host tables
    const size_t pairs_bytes = n * sizeof(PairDesc), states_bytes = n * sizeof(PairState);
    char* stage;
    if ((st = stage_begin(c, pairs_bytes + states_bytes + tbytes, &stage)) != RGBID_OK) return st;
    PairDesc* pd = reinterpret_cast<PairDesc*>(stage);
    PairState* ps = reinterpret_cast<PairState*>(stage + pairs_bytes);
    char* tb = stage + pairs_bytes + states_bytes;
    std::memset(stage, 0, pairs_bytes + states_bytes + tbytes);
    for (int i = 0; i < n; ++i) {
        PairDesc& d = pd[i];
        for (int l = 0; l < L; ++l) {
            const rgbid_pyr* Pa = A[i];
            const rgbid_pyr* Pb = B[i];
            d.A[l] = LevelView{Pa->iw[l], Pa->wp[l], static_cast<const unsigned char*>(Pa->gm[l]),
                               Pa->w[l], Pa->h[l], (float)Pa->fx[l], (float)Pa->fy[l],
                               (float)Pa->cx[l], (float)Pa->cy[l]};
            d.B[l] = LevelView{Pb->iw[l], Pb->wp[l], static_cast<const unsigned char*>(Pb->gm[l]),
                               Pb->w[l], Pb->h[l], (float)Pb->fx[l], (float)Pb->fy[l],
                               (float)Pb->cx[l], (float)Pb->cy[l]};
            d.stride[l] = stride[i * L + l];
            d.sw[l] = sw[i * L + l];
            d.sh[l] = sh[i * L + l];
        }
        d.warped = static_cast<float2*>(c->warped.p) + warped_off[i];
        d.sample = static_cast<float2*>(c->sample.p) + (size_t)i * P->sample_max;
        PairState& s = ps[i];
        if (init) {
            std::memcpy(s.R, init[i].R, sizeof s.R);
            std::memcpy(s.t, init[i].t, sizeof s.t);
        } else {
            s.R[0] = s.R[4] = s.R[8] = 1.0;
        }
        pose_floats(s.R, s.t, s.RT, s.Rtt);
        s.status = RGBID_OK;
        s.active = 1;
        s.sigma[0] = s.sigma[1] = 1.0f;
        s.nu[0] = s.nu[1] = 5.0f;
    }
    for (int k = 0; k < nch; ++k)
        for (int l = 0; l < L; ++l) {
            std::memcpy(tb + lt[k][l].warp_off, wch[k][l].data(), wch[k][l].size() * sizeof(Chunk));
            std::memcpy(tb + lt[k][l].red_off, rch[k][l].data(), rch[k][l].size() * sizeof(Chunk));
            std::memcpy(tb + lt[k][l].begin_off, rbeg[k][l].data(), rbeg[k][l].size() * sizeof(int));
        }
    HIPCHK(c, hipMemcpyAsync(c->pairs.p, pd, pairs_bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->states.p, ps, states_bytes, hipMemcpyHostToDevice, c->stream));
    if (init_twist_dev)
        HIPCHK(c, launch_init_from_twist(c->stream, static_cast<PairState*>(c->states.p), n,
                                         init_twist_dev, kXiScale));
    HIPCHK(c, hipMemcpyAsync(c->tables.p, tb, tbytes, hipMemcpyHostToDevice, c->stream));
    if ((st = stage_end(c)) != RGBID_OK) return st;

    // ---- enqueue (directly or through a cached graph)
    // zeroed first: the struct's padding bytes are part of the graph-cache key
    IterParams ip;
    std::memset(&ip, 0, sizeof ip);
    ip.weight = P->weight;
    ip.huber_k = (float)P->huber_k;
    ip.estimate_nu = P->estimate_nu;
    ip.scale_iters = P->scale_iters;
    ip.scale_warm = P->scale_warm;
    ip.warp_mode = P->warp;
    ip.stop_eps_t = P->stop_eps_t;
    ip.stop_eps_r = P->stop_eps_r;
    int total_iters = 0;
    for (const Step& stp : sched) total_iters += stp.iters;
    if (c->profiling) {
        while ((int)c->events.size() < 5 * total_iters) {
            hipEvent_t ev;
            HIPCHK(c, hipEventCreate(&ev));
            c->events.push_back(ev);
        }
    }
    // the whole schedule of chain k on stream s
    // part 0: everything; part 1: the first level start and the warp kernel
    // of the first iteration; part 2: the rest
    auto enqueue = [&](hipStream_t s, int k, int part) -> hipError_t {
        hipError_t e = hipSuccess;
        int ev_base = 0;
        const int p0 = cfirst[k], np = cfirst[k + 1] - cfirst[k];
        if (np <= 0) return e;
        PairState* states = static_cast<PairState*>(c->states.p) + p0;
        bool first = true;
        for (const Step& stp : sched) {
            const int l = stp.level;
            if (stp.iters <= 0) continue;
            if (part != 2 || !first)
                if ((e = launch_level_start(s, states, np)) != hipSuccess) return e;
            IterLaunch il;
            il.pairs = static_cast<const PairDesc*>(c->pairs.p) + p0;
            il.states = states;
            il.npairs = np;
            il.level = l;
            il.ip = ip;
            il.tune = tune[l];
            il.f16 = f16;
            il.block_log2 = fullres ? l : 0;
            char* tbase = static_cast<char*>(c->tables.p);
            il.warp_chunks = reinterpret_cast<const Chunk*>(tbase + lt[k][l].warp_off);
            il.n_warp_chunks = lt[k][l].n_warp;
            il.red_chunks = reinterpret_cast<const Chunk*>(tbase + lt[k][l].red_off);
            il.n_red_chunks = lt[k][l].n_red;
            il.pair_red_begin = reinterpret_cast<const int*>(tbase + lt[k][l].begin_off);
            il.partials = static_cast<float2*>(c->partials.p) + poff[k] * kNSum;
            il.update = update;
            il.scale_per = scale_per[k][l];
            for (int it = 0; it < stp.iters; ++it) {
                const hipEvent_t* ev = c->profiling ? &c->events[5 * (ev_base + it)] : nullptr;
                il.kernels = 15;
                if (first && it == 0) il.kernels = part == 1 ? 1 : part == 2 ? 14 : 15;
                else if (part == 1) break;
                if ((e = launch_iteration(s, il, ev)) != hipSuccess) return e;
            }
            ev_base += stp.iters;
            first = false;
            if (part == 1) break;
        }
        return e;
    };
    // Timing events inside a captured graph cannot be read back, so a profiled
    // call launches directly.
    if (graphed) {
        std::string key;
        {
            char buf[160];
            snprintf(buf, sizeof buf, "n%d f%d u%d L%d g%d c%d|", n, f16, update, L, c->generation,
                     nch);
            key = buf;
            for (int i = 0; i < n; ++i) {
                snprintf(buf, sizeof buf, "%dx%d,", A[i]->w[0], A[i]->h[0]);
                key += buf;
            }
            key += "|";
            for (const Step& stp : sched) {
                snprintf(buf, sizeof buf, "%d:%d,", stp.level, stp.iters);
                key += buf;
            }
            key.append(reinterpret_cast<const char*>(&ip), sizeof ip);
            key.append(reinterpret_cast<const char*>(tune), sizeof(LevelTune) * L);
            // everything else a captured launch holds: the sample length per
            // thread and the table layout (both follow sample_max as well as
            // the sizes) and the partials offset of every chain
            snprintf(buf, sizeof buf, "|s%d|", P->sample_max);
            key += buf;
            for (int k = 0; k < nch; ++k) {
                for (int l = 0; l < L; ++l) {
                    const LevelTables& t = lt[k][l];
                    snprintf(buf, sizeof buf, "%d,%zu,%zu,%zu,%d,%d;", scale_per[k][l], t.warp_off,
                             t.red_off, t.begin_off, t.n_warp, t.n_red);
                    key += buf;
                }
                snprintf(buf, sizeof buf, "p%zu|", poff[k]);
                key += buf;
            }
        }
        if ((st = ensure_chain_streams(c, nch)) != RGBID_OK) return st;
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            // with several chains, chain 0 is captured in two parts (graphs 0
            // and nch) so the other chains start one kernel later
            std::vector<hipGraphExec_t> execs;
            for (int gi = 0; gi < nch + (nch > 1 ? 1 : 0); ++gi) {
                const int k = gi < nch ? gi : 0;
                const int part = nch == 1 ? 0 : gi == 0 ? 1 : gi == nch ? 2 : 0;
                hipGraph_t g = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
                hipError_t e = enqueue(c->cap, k, part);
                hipError_t e2 = hipStreamEndCapture(c->cap, &g);
                hipGraphExec_t ex = nullptr;
                if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                if (g) (void)hipGraphDestroy(g);
                if (e != hipSuccess || e2 != hipSuccess) {
                    for (hipGraphExec_t x : execs) (void)hipGraphExecDestroy(x);
                    return set_err(c, RGBID_E_DEVICE, "graph capture failed: %s",
                                   hipGetErrorString(e != hipSuccess ? e : e2));
                }
                execs.push_back(ex);
            }
            if (c->graphs.size() > 64) clear_graphs(c);
            it = c->graphs.emplace(key, std::move(execs)).first;
        }
        // chains run concurrently on their own streams, forked from and joined
        // back into the context's stream
        if (launch_ms) HIPCHK(c, hipEventRecord(c->tev[0], c->stream));
        HIPCHK(c, hipGraphLaunch(it->second[0], c->stream));
        if (nch > 1) {
            HIPCHK(c, hipEventRecord(c->fork, c->stream));
            for (int k = 1; k < nch; ++k)
                HIPCHK(c, hipStreamWaitEvent(c->chain_streams[k - 1], c->fork, 0));
            for (int k = 1; k < nch; ++k)
                HIPCHK(c, hipGraphLaunch(it->second[k], c->chain_streams[k - 1]));
            HIPCHK(c, hipGraphLaunch(it->second[nch], c->stream));
        }
        for (int k = 1; k < nch; ++k) {
            HIPCHK(c, hipEventRecord(c->joins[k - 1], c->chain_streams[k - 1]));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->joins[k - 1], 0));
        }
        if (launch_ms) HIPCHK(c, hipEventRecord(c->tev[1], c->stream));
    } else {
        if (launch_ms) HIPCHK(c, hipEventRecord(c->tev[0], c->stream));
        HIPCHK(c, enqueue(c->stream, 0, 0));
        if (launch_ms) HIPCHK(c, hipEventRecord(c->tev[1], c->stream));
    }

    // ---- results
    if (device_out && !c->profiling && !launch_ms) {
        // asynchronous form: results stay in device memory, nothing waits
        HIPCHK(c, launch_export(c->stream, static_cast<const PairState*>(c->states.p), n, out, stats));
        return RGBID_OK;
    }
    if (device_out) HIPCHK(c, launch_export(c->stream, static_cast<const PairState*>(c->states.p), n,
                                            out, stats));
    if ((st = ensure_down(c, states_bytes)) != RGBID_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->h_down, c->states.p, states_bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->profiling) {
        int j = 0;
        for (const Step& stp : sched)
            for (int it = 0; it < stp.iters; ++it, ++j)
                for (int k = 0; k < 4; ++k) {
                    float ms = 0.0f;
                    HIPCHK(c, hipEventElapsedTime(&ms, c->events[5 * j + k], c->events[5 * j + k + 1]));
                    c->prof_ms[stp.level * 4 + k] += ms;
                    c->prof_n[stp.level * 4 + k] += 1;
                }
    }
    if (launch_ms) HIPCHK(c, hipEventElapsedTime(launch_ms, c->tev[0], c->tev[1]));
    if (device_out) return RGBID_OK;
    const PairState* res = static_cast<const PairState*>(c->h_down);
    for (int i = 0; i < n; ++i) {
        const PairState& s = res[i];
        if (out) {
            std::memcpy(out[i].R, s.R, sizeof s.R);
            std::memcpy(out[i].t, s.t, sizeof s.t);
        }
        if (stats) {
            rgbid_align_stats& o = stats[i];
            std::memcpy(o.H, s.H, sizeof o.H);
            std::memcpy(o.g, s.g, sizeof o.g);
            o.mu_I = s.mu[0];
            o.sigma_I = s.sigma[0];
            o.nu_I = s.nu[0];
            o.mu_W = s.mu[1];
            o.sigma_W = s.sigma[1];
            o.nu_W = s.nu[1];
            o.cost = s.cost;
            o.n_valid_I = s.nI;
            o.n_valid_W = s.nW;
            for (int l = 0; l < 8; ++l) o.iters_done[l] = l < kMaxLevels ? s.iters_done[l] : 0;
            o.status = s.status;
        }
    }
    return RGBID_OK;
}

rgbid_status build_pyramids(rgbid_ctx* c, int n, rgbid_pyr* const* pyrs, const float* const* I,
                            const float* const* W, const size_t* pitch)
{
    rgbid_status st;
    if ((st = ensure(c, c->frames, n * sizeof(PyrFrame))) != RGBID_OK) return st;
    char* stage;
    if ((st = stage_begin(c, n * sizeof(PyrFrame), &stage)) != RGBID_OK) return st;
    PyrFrame* fr = reinterpret_cast<PyrFrame*>(stage);
    int levels = 0, mw[kMaxLevels] = {0}, mh[kMaxLevels] = {0};
    bool quad = true, even_h = true;
    for (int i = 0; i < n; ++i) {
        const rgbid_pyr* p = pyrs[i];
        quad = quad && p->w[0] % 4 == 0 && pitch[i] % 4 == 0 &&
               reinterpret_cast<uintptr_t>(I[i]) % 16 == 0 &&
               reinterpret_cast<uintptr_t>(W[i]) % 16 == 0;
        even_h = even_h && p->h[0] % 2 == 0;
        PyrFrame& f = fr[i];
        std::memset(&f, 0, sizeof f);
        f.I = I[i];
        f.W = W[i];
        f.pitch = (long long)pitch[i];
        f.levels = p->levels;
        for (int l = 0; l < p->levels; ++l) {
            f.iw[l] = p->iw[l];
            f.wp[l] = p->wp[l];
            f.gm[l] = p->gm[l];
            f.w[l] = p->w[l];
            f.h[l] = p->h[l];
            mw[l] = std::max(mw[l], p->w[l]);
            mh[l] = std::max(mh[l], p->h[l]);
        }
        levels = std::max(levels, p->levels);
    }
    HIPCHK(c, hipMemcpyAsync(c->frames.p, fr, n * sizeof(PyrFrame), hipMemcpyHostToDevice, c->stream));
    if ((st = stage_end(c)) != RGBID_OK) return st;
    HIPCHK(c, launch_pyramid(c->stream, static_cast<const PyrFrame*>(c->frames.p), n, levels,
                             pyrs[0]->f16, mw, mh, quad, quad && even_h));
    return RGBID_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

void rgbid_default_params(rgbid_align_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->levels = 4;
    for (int l = 0; l < 8; ++l) p->iters[l] = 10;
    p->weight = RGBID_W_HUBER;
    p->huber_k = 1.345;
    p->estimate_nu = 1;
    p->sample_max = 19200;
    p->scale_iters = 20;
    p->warp = RGBID_WARP_FULLRES;
    p->scale_warm = 1;
}

rgbid_status rgbid_create(rgbid_ctx** ctx, int device, void* hip_stream)
{
    if (!ctx) return RGBID_E_ARG;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RGBID_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return RGBID_E_DEVICE;
    rgbid_ctx* c = new (std::nothrow) rgbid_ctx();
    if (!c) return RGBID_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&c->tev[0]) != hipSuccess || hipEventCreate(&c->tev[1]) != hipSuccess) {
        delete c;
        return RGBID_E_DEVICE;
    }
    // this device's copy of the allocation-free call's scratch array
    if (hipGetSymbolAddress(&c->scratch_dev, HIP_SYMBOL(scratch)) != hipSuccess || !c->scratch_dev) {
        (void)hipStreamDestroy(c->cap);
        (void)hipEventDestroy(c->stage_done);
        (void)hipEventDestroy(c->tev[0]);
        (void)hipEventDestroy(c->tev[1]);
        delete c;
        return RGBID_E_DEVICE;
    }
    c->err.reserve(512);   // error texts never reallocate (allocation-free call)
    const char* g = std::getenv("RGBID_NO_GRAPH");
    c->use_graphs = !(g && g[0] == '1');
    if (const char* ch = std::getenv("RGBID_CHAINS")) c->chains = std::max(1, std::min(8, std::atoi(ch)));
    *ctx = c;
    return RGBID_OK;
}

void rgbid_destroy(rgbid_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    clear_graphs(c);
    if (c->cov_pyr) rgbid_pyramid_free(c->cov_pyr);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (DevBuf* b : {&c->pairs, &c->states, &c->tables, &c->partials, &c->warped, &c->sample,
                      &c->frames, &c->covis, &c->cov_img, &c->reg, &c->fuse})
        if (b->p) (void)hipFree(b->p);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    if (c->h_down) (void)hipHostFree(c->h_down);
    if (c->stage_done) (void)hipEventDestroy(c->stage_done);
    for (hipEvent_t e : c->tev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t cs : c->chain_streams) (void)hipStreamDestroy(cs);
    for (hipEvent_t e : c->joins) (void)hipEventDestroy(e);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

const char* rgbid_last_error(const rgbid_ctx* c) { return c ? c->err.c_str() : "no context"; }

rgbid_status rgbid_pyramid(rgbid_ctx* c, const rgbid_camera* cam, int levels, rgbid_format storage,
                           const float* I_dev, const float* W_dev, size_t pitch_elems,
                           rgbid_pyr** out)
{
    if (!c) return RGBID_E_ARG;
    if (!out) return set_err(c, RGBID_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cam || !I_dev || !W_dev) return set_err(c, RGBID_E_ARG, "NULL camera or image");
    if (levels < 1 || levels > kMaxLevels) return set_err(c, RGBID_E_ARG, "levels outside 1..8");
    if (storage != RGBID_F32 && storage != RGBID_F16) return set_err(c, RGBID_E_ARG, "unknown storage");
    if (cam->width < 1 || cam->height < 1 || pitch_elems < (size_t)cam->width)
        return set_err(c, RGBID_E_ARG, "bad image size or pitch");
    if ((long long)cam->width * cam->height >= (1ll << 22))
        return set_err(c, RGBID_E_ARG, "images of 2^22 pixels or more are not supported");
    if (!(cam->fx > 0 && cam->fy > 0)) return set_err(c, RGBID_E_ARG, "focal lengths must be > 0");
    if ((cam->width >> (levels - 1)) < 1 || (cam->height >> (levels - 1)) < 1)
        return set_err(c, RGBID_E_ARG, "level %d would be empty", levels - 1);
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_pyr* p = new (std::nothrow) rgbid_pyr();
    if (!p) return set_err(c, RGBID_E_NOMEM, "host allocation failed");
    p->device = c->device;
    p->cam = *cam;
    p->levels = levels;
    p->f16 = storage == RGBID_F16;
    const size_t e_iw = p->f16 ? 4 : 8, e_wp = p->f16 ? 2 : 4;
    size_t off[3 * kMaxLevels], total = 0;
    for (int l = 0; l < levels; ++l) {
        p->w[l] = cam->width >> l;
        p->h[l] = cam->height >> l;
        level_camera(*cam, l, p->fx[l], p->fy[l], p->cx[l], p->cy[l]);
        const size_t np = (size_t)p->w[l] * p->h[l];
        // the (I, W) plane between guards of at least one row and one texel
        // (zeros): the alignment kernels read the neighbours of border pixels
        // unclamped, and a bilinear tap pair may read one texel past the end
        const size_t guard = align_up(((size_t)p->w[l] + 1) * e_iw, 256);
        off[3 * l] = total + guard;
        total = align_up(off[3 * l] + np * e_iw, 256) + guard;
        off[3 * l + 1] = total;
        total = align_up(total + np * e_wp, 256);
        off[3 * l + 2] = total;
        total = align_up(total + np, 256);
    }
    hipError_t e = hipMalloc(&p->base, total);
    if (e != hipSuccess) {
        delete p;
        return set_err(c, RGBID_E_NOMEM, "hipMalloc(%zu) failed: %s", total, hipGetErrorString(e));
    }
    for (int l = 0; l < levels; ++l) {
        p->iw[l] = static_cast<char*>(p->base) + off[3 * l];
        p->wp[l] = static_cast<char*>(p->base) + off[3 * l + 1];
        p->gm[l] = static_cast<char*>(p->base) + off[3 * l + 2];
    }
    e = hipMemsetAsync(p->base, 0, total, c->stream);
    if (e != hipSuccess) {
        (void)hipFree(p->base);
        delete p;
        return set_err(c, RGBID_E_DEVICE, "hipMemsetAsync failed: %s", hipGetErrorString(e));
    }
    rgbid_pyr* const arr[1] = {p};
    const float* const Is[1] = {I_dev};
    const float* const Ws[1] = {W_dev};
    const size_t pt[1] = {pitch_elems};
    rgbid_status st = build_pyramids(c, 1, arr, Is, Ws, pt);
    if (st != RGBID_OK) {
        (void)hipFree(p->base);
        delete p;
        return st;
    }
    *out = p;
    return RGBID_OK;
}

rgbid_status rgbid_pyramid_update(rgbid_ctx* c, rgbid_pyr* pyr, const float* I_dev,
                                  const float* W_dev, size_t pitch_elems)
{
    rgbid_pyr* const arr[1] = {pyr};
    const float* const Is[1] = {I_dev};
    const float* const Ws[1] = {W_dev};
    const size_t pt[1] = {pitch_elems};
    return rgbid_pyramid_update_batch(c, 1, arr, Is, Ws, pt);
}

rgbid_status rgbid_pyramid_update_batch(rgbid_ctx* c, int n, rgbid_pyr* const* pyrs,
                                        const float* const* I_dev, const float* const* W_dev,
                                        const size_t* pitch_elems)
{
    if (!c) return RGBID_E_ARG;
    if (n < 1 || !pyrs || !I_dev || !W_dev || !pitch_elems)
        return set_err(c, RGBID_E_ARG, "need n >= 1 and non-NULL arrays");
    for (int i = 0; i < n; ++i) {
        if (!pyrs[i] || !I_dev[i] || !W_dev[i]) return set_err(c, RGBID_E_ARG, "NULL entry %d", i);
        if (pyrs[i]->device != c->device) return set_err(c, RGBID_E_ARG, "pyramid on another device");
        if (pitch_elems[i] < (size_t)pyrs[i]->w[0]) return set_err(c, RGBID_E_ARG, "pitch < width");
        if (pyrs[i]->f16 != pyrs[0]->f16) return set_err(c, RGBID_E_SHAPE, "mixed storage formats");
    }
    HIPCHK(c, hipSetDevice(c->device));
    return build_pyramids(c, n, pyrs, I_dev, W_dev, pitch_elems);
}

rgbid_status rgbid_pyramid_read(rgbid_ctx* c, const rgbid_pyr* p, int level, float* I_out,
                                float* W_out)
{
    if (!c) return RGBID_E_ARG;
    if (!p || level < 0 || level >= p->levels) return set_err(c, RGBID_E_ARG, "bad pyramid or level");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_level_read(c->stream, p->iw[level], p->w[level] * p->h[level], p->f16, I_out, W_out));
    return RGBID_OK;
}

rgbid_status rgbid_pyramid_level_size(const rgbid_pyr* p, int level, int* w, int* h)
{
    if (!p || level < 0 || level >= p->levels) return RGBID_E_ARG;
    if (w) *w = p->w[level];
    if (h) *h = p->h[level];
    return RGBID_OK;
}

void rgbid_pyramid_free(rgbid_pyr* p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->base);
    delete p;
}

rgbid_status rgbid_align_batch(rgbid_ctx* c, int n, const rgbid_pyr* const* A,
                               const rgbid_pyr* const* B, const rgbid_pose* init,
                               const rgbid_align_params* P, rgbid_pose* out,
                               rgbid_align_stats* stats)
{
    if (!c) return RGBID_E_ARG;
    if (!out) return set_err(c, RGBID_E_ARG, "out is NULL");
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<Step> sched;
    for (int l = P->levels - 1; l >= 0; --l)
        if (P->iters[l] > 0) sched.push_back(Step{l, P->iters[l]});
    return run_batch(c, n, A, B, init, P, sched, 1, out, stats);
}

rgbid_status rgbid_align_batch_async(rgbid_ctx* c, int n, const rgbid_pyr* const* A,
                                     const rgbid_pyr* const* B, const rgbid_pose* init,
                                     const rgbid_align_params* P, rgbid_pose* out_dev,
                                     rgbid_align_stats* stats_dev)
{
    if (!c) return RGBID_E_ARG;
    if (!out_dev) return set_err(c, RGBID_E_ARG, "out_dev is NULL");
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<Step> sched;
    for (int l = P->levels - 1; l >= 0; --l)
        if (P->iters[l] > 0) sched.push_back(Step{l, P->iters[l]});
    return run_batch(c, n, A, B, init, P, sched, 1, out_dev, stats_dev, nullptr, true);
}

rgbid_status rgbid_align(rgbid_ctx* c, const rgbid_pyr* A, const rgbid_pyr* B,
                         const rgbid_pose* init, const rgbid_align_params* P, rgbid_pose* out,
                         rgbid_align_stats* stats)
{
    if (!c) return RGBID_E_ARG;
    rgbid_align_stats s;
    const rgbid_pyr* const a[1] = {A};
    const rgbid_pyr* const b[1] = {B};
    rgbid_status st = rgbid_align_batch(c, 1, a, b, init, P, out, &s);
    if (st != RGBID_OK) return st;
    if (stats) *stats = s;
    if (s.status != RGBID_OK)
        return set_err(c, (rgbid_status)s.status, "alignment stopped: degenerate normal equations");
    return RGBID_OK;
}

// The single-pair alignment of rgbid_align with every device buffer carved
// from this device's `scratch` array and the tables written by a set-up
// kernel: no device or host allocation, no graph, default launch shapes
// (the ones rgbid_align uses for a pair it has not tuned).
rgbid_status rgbid_align_noalloc(rgbid_ctx* c, const rgbid_pyr* A, const rgbid_pyr* B,
                                 const rgbid_pose* init, const rgbid_align_params* P,
                                 rgbid_pose* out, rgbid_align_stats* stats)
{
    if (!c) return RGBID_E_ARG;
    if (!out || !A || !B) return set_err(c, RGBID_E_ARG, "NULL pyramid or output");
    if (const char* e = params_problem(P)) return set_err(c, RGBID_E_ARG, "%s", e);
    if (A->device != c->device || B->device != c->device)
        return set_err(c, RGBID_E_ARG, "pyramid lives on another device");
    if (A->w[0] != B->w[0] || A->h[0] != B->h[0] || A->f16 != B->f16)
        return set_err(c, RGBID_E_SHAPE, "A and B differ in size or format");
    if (A->cam.fx != B->cam.fx || A->cam.fy != B->cam.fy || A->cam.cx != B->cam.cx ||
        A->cam.cy != B->cam.cy)
        return set_err(c, RGBID_E_SHAPE, "A and B have different cameras");
    if (A->levels < P->levels || B->levels < P->levels)
        return set_err(c, RGBID_E_SHAPE, "pyramid has fewer levels than params");
    HIPCHK(c, hipSetDevice(c->device));
    const int L = P->levels;
    const bool fullres = P->warp == RGBID_WARP_FULLRES;

    // ---- launch shapes, chunk segments and the scratch layout
    NoAllocSetup su;
    std::memset(&su, 0, sizeof su);
    LevelTune tune[kMaxLevels];
    int nwarp[kMaxLevels], scale_per[kMaxLevels];
    size_t warped_px = 0;
    int nch = 0;
    for (int l = 0; l < L; ++l) {
        const int b = fullres ? l : 0;
        tune[l] = default_tune(b);
        const int w = A->w[l], h = A->h[l];
        const int s = sample_stride(w, h, P->sample_max);
        su.desc.stride[l] = s;
        su.desc.sw[l] = (w + s - 1) / s;
        su.desc.sh[l] = (h + s - 1) / s;
        scale_per[l] = (su.desc.sw[l] * su.desc.sh[l] + kScaleThreads - 1) / kScaleThreads;
        const long long ngrid =
            tune[l].fused ? (long long)su.desc.sw[l] * su.desc.sh[l] : (long long)w * h;
        const int gpp = warp_pixels_per_pass(b);
        const int wper = tune[l].waves * tune[l].warp_passes;
        const int rper = tune[l].waves * tune[l].tiles_per_wave;
        const int wt = (int)((ngrid + gpp - 1) / gpp);
        const int rt = (int)reduce_tiles(w, h, tune[l].fused && b == 0);
        nwarp[l] = (wt + wper - 1) / wper;
        su.n_red[l] = (rt + rper - 1) / rper;
        su.seg_first[2 * l] = nch;
        su.seg_tiles[2 * l] = wt;
        su.seg_per[2 * l] = wper;
        nch += nwarp[l];
        su.seg_first[2 * l + 1] = nch;
        su.seg_tiles[2 * l + 1] = rt;
        su.seg_per[2 * l + 1] = rper;
        nch += su.n_red[l];
        if (!tune[l].fused) warped_px = std::max(warped_px, (size_t)w * h);
    }
    su.levels = L;
    su.nseg = 2 * L;
    su.seg_first[2 * L] = nch;
    int max_red = 0;
    for (int l = 0; l < L; ++l) max_red = std::max(max_red, su.n_red[l]);
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_desc = carve(sizeof(PairDesc)), o_state = carve(sizeof(PairState));
    const size_t o_chunks = carve((size_t)nch * sizeof(Chunk));
    const size_t o_begins = carve((size_t)2 * L * sizeof(int));
    const size_t o_part = carve((size_t)std::max(max_red, 1) * kNSum * sizeof(float2));
    const size_t o_sample = carve((size_t)P->sample_max * sizeof(float2));
    const size_t o_warped = carve(std::max<size_t>(warped_px, 1) * sizeof(float2));
    if (off > kScratchBytes)
        return set_err(c, RGBID_E_ARG,
                       "pair needs %zu bytes of scratch, the allocation-free call has %zu", off,
                       kScratchBytes);
    char* base = static_cast<char*>(c->scratch_dev);

    // ---- descriptor, initial state, tables: written on the device
    for (int l = 0; l < L; ++l) {
        su.desc.A[l] = LevelView{A->iw[l], A->wp[l], static_cast<const unsigned char*>(A->gm[l]),
                                 A->w[l], A->h[l], (float)A->fx[l], (float)A->fy[l],
                                 (float)A->cx[l], (float)A->cy[l]};
        su.desc.B[l] = LevelView{B->iw[l], B->wp[l], static_cast<const unsigned char*>(B->gm[l]),
                                 B->w[l], B->h[l], (float)B->fx[l], (float)B->fy[l],
                                 (float)B->cx[l], (float)B->cy[l]};
    }
    su.desc.warped = reinterpret_cast<float2*>(base + o_warped);
    su.desc.sample = reinterpret_cast<float2*>(base + o_sample);
    PairState& s0 = su.state;
    if (init) {
        std::memcpy(s0.R, init->R, sizeof s0.R);
        std::memcpy(s0.t, init->t, sizeof s0.t);
    } else {
        s0.R[0] = s0.R[4] = s0.R[8] = 1.0;
    }
    pose_floats(s0.R, s0.t, s0.RT, s0.Rtt);
    s0.status = RGBID_OK;
    s0.active = 1;
    s0.sigma[0] = s0.sigma[1] = 1.0f;
    s0.nu[0] = s0.nu[1] = 5.0f;
    su.desc_dev = reinterpret_cast<PairDesc*>(base + o_desc);
    su.state_dev = reinterpret_cast<PairState*>(base + o_state);
    su.chunks = reinterpret_cast<Chunk*>(base + o_chunks);
    su.begins = reinterpret_cast<int*>(base + o_begins);
    HIPCHK(c, launch_noalloc_setup(c->stream, su));

    // ---- the schedule: levels L-1 .. 0, plain launches
    IterParams ip;
    std::memset(&ip, 0, sizeof ip);
    ip.weight = P->weight;
    ip.huber_k = (float)P->huber_k;
    ip.estimate_nu = P->estimate_nu;
    ip.scale_iters = P->scale_iters;
    ip.scale_warm = P->scale_warm;
    ip.warp_mode = P->warp;
    ip.stop_eps_t = P->stop_eps_t;
    ip.stop_eps_r = P->stop_eps_r;
    for (int l = L - 1; l >= 0; --l) {
        if (P->iters[l] <= 0) continue;
        HIPCHK(c, launch_level_start(c->stream, su.state_dev, 1));
        IterLaunch il;
        std::memset(&il, 0, sizeof il);
        il.pairs = su.desc_dev;
        il.states = su.state_dev;
        il.npairs = 1;
        il.level = l;
        il.ip = ip;
        il.tune = tune[l];
        il.f16 = A->f16;
        il.block_log2 = fullres ? l : 0;
        il.warp_chunks = su.chunks + su.seg_first[2 * l];
        il.n_warp_chunks = nwarp[l];
        il.red_chunks = su.chunks + su.seg_first[2 * l + 1];
        il.n_red_chunks = su.n_red[l];
        il.pair_red_begin = su.begins + 2 * l;
        il.partials = reinterpret_cast<float2*>(base + o_part);
        il.update = 1;
        il.scale_per = scale_per[l];
        il.kernels = 15;
        for (int it = 0; it < P->iters[l]; ++it) HIPCHK(c, launch_iteration(c->stream, il, nullptr));
    }

    // ---- results: the state into host memory the call owns on its stack
    PairState r;
    HIPCHK(c, hipMemcpyAsync(&r, su.state_dev, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(out->R, r.R, sizeof r.R);
    std::memcpy(out->t, r.t, sizeof r.t);
    if (stats) {
        std::memcpy(stats->H, r.H, sizeof r.H);
        std::memcpy(stats->g, r.g, sizeof r.g);
        stats->mu_I = r.mu[0];
        stats->sigma_I = r.sigma[0];
        stats->nu_I = r.nu[0];
        stats->mu_W = r.mu[1];
        stats->sigma_W = r.sigma[1];
        stats->nu_W = r.nu[1];
        stats->cost = r.cost;
        stats->n_valid_I = r.nI;
        stats->n_valid_W = r.nW;
        for (int l = 0; l < 8; ++l) stats->iters_done[l] = l < kMaxLevels ? r.iters_done[l] : 0;
        stats->status = r.status;
    }
    if (r.status != RGBID_OK)
        return set_err(c, (rgbid_status)r.status, "alignment stopped: degenerate normal equations");
    return RGBID_OK;
}

rgbid_status rgbid_normal_equations(rgbid_ctx* c, const rgbid_pyr* A, const rgbid_pyr* B, int level,
                                    const rgbid_pose* T, const rgbid_align_params* P,
                                    rgbid_align_stats* out)
{
    if (!c) return RGBID_E_ARG;
    if (!out || !T) return set_err(c, RGBID_E_ARG, "NULL pose or output");
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    if (level < 0 || level >= P->levels) return set_err(c, RGBID_E_ARG, "level outside 0..levels-1");
    HIPCHK(c, hipSetDevice(c->device));
    const rgbid_pyr* const a[1] = {A};
    const rgbid_pyr* const b[1] = {B};
    std::vector<Step> sched{Step{level, 1}};
    rgbid_pose o;
    return run_batch(c, 1, a, b, T, P, sched, 0, &o, out);
}

rgbid_status rgbid_autotune(rgbid_ctx* c, int n, const rgbid_pyr* const* A,
                            const rgbid_pyr* const* B, const rgbid_align_params* P, int reps,
                            double* best_ms)
{
    if (!c) return RGBID_E_ARG;
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    if (n < 1 || !A || !B || reps < 1) return set_err(c, RGBID_E_ARG, "bad arguments");
    for (int i = 0; i < n; ++i)
        if (!A[i] || !B[i]) return set_err(c, RGBID_E_ARG, "NULL pyramid %d", i);
    HIPCHK(c, hipSetDevice(c->device));
    const int f16 = A[0]->f16;
    const bool saved_prof = c->profiling;
    c->profiling = false;
    std::vector<rgbid_pose> o(n);
    // per level, the picks of the per-level round in order (best first)
    std::vector<std::vector<LevelTune>> top(P->levels);
    for (int l = 0; l < P->levels; ++l) {
        const std::string key = tune_key(n, A, l, P->warp, f16);
        const int b = P->warp == RGBID_WARP_FULLRES ? l : 0;
        // every candidate is timed twice (the faster counts); the four best
        // are timed four more times and the lowest median of their six
        // timings wins
        struct Cand {
            LevelTune t;
            std::vector<float> ms;
        };
        std::vector<Cand> cands;
        for (int fused = 0; fused < 2; ++fused)
            for (int waves : {2, 4, 8})
                for (int tpw : {1, 2, 4, 8, 16, 32})
                    for (int remap = 0; remap < 2; ++remap) {
                        LevelTune t;
                        t.fused = fused;
                        t.waves = waves;
                        t.tiles_per_wave = tpw;
                        t.xcd_remap = remap;
                        // when the reduction warps its own pixels, the warp
                        // kernel only forms the systematic sample: few passes
                        // per pair, so one per wave
                        t.warp_passes = fused ? 1 : tpw;
                        cands.push_back(Cand{t, {}});
                    }
        auto time_cand = [&](Cand& cd, int times) -> rgbid_status {
            c->tunes[key] = cd.t;
            std::vector<Step> sched{Step{l, reps}};
            // the first call captures the graph (when not yet cached)
            rgbid_status st = run_batch(c, n, A, B, nullptr, P, sched, 0, o.data(), nullptr);
            for (int r = 0; r < times && st == RGBID_OK; ++r) {
                float ms = 0.0f;
                st = run_batch(c, n, A, B, nullptr, P, sched, 0, o.data(), nullptr, &ms);
                cd.ms.push_back(ms);
            }
            return st;
        };
        auto fail = [&](rgbid_status st) {
            c->profiling = saved_prof;
            c->tunes[key] = default_tune(b);
            return st;
        };
        for (Cand& cd : cands)
            if (rgbid_status st = time_cand(cd, 2); st != RGBID_OK) return fail(st);
        auto lowest = [](const Cand& x) { return *std::min_element(x.ms.begin(), x.ms.end()); };
        std::sort(cands.begin(), cands.end(),
                  [&](const Cand& x, const Cand& y) { return lowest(x) < lowest(y); });
        const size_t nfin = std::min<size_t>(4, cands.size());
        for (size_t i = 0; i < nfin; ++i)
            if (rgbid_status st = time_cand(cands[i], 4); st != RGBID_OK) return fail(st);
        auto median = [](std::vector<float> v) {
            std::sort(v.begin(), v.end());
            return 0.5f * (v[(v.size() - 1) / 2] + v[v.size() / 2]);
        };
        LevelTune best = cands[0].t;
        float best_t = median(cands[0].ms);
        for (size_t i = 1; i < nfin; ++i)
            if (median(cands[i].ms) < best_t) {
                best_t = median(cands[i].ms);
                best = cands[i].t;
            }
        // then the warp kernel's passes per wave, the rest fixed
        {
            std::vector<Cand> wc;
            for (int wp : {1, 2, 4, 8, 16})
                if (wp != best.warp_passes) {
                    LevelTune t = best;
                    t.warp_passes = wp;
                    wc.push_back(Cand{t, {}});
                }
            for (Cand& cd : wc) {
                if (rgbid_status st = time_cand(cd, 4); st != RGBID_OK) return fail(st);
                if (median(cd.ms) < best_t) {
                    best_t = median(cd.ms);
                    best = cd.t;
                }
            }
        }
        c->tunes[key] = best;
        if (best_ms) best_ms[l] = best_t / reps;
        top[l].push_back(best);
        std::vector<std::pair<float, LevelTune>> rest;
        for (size_t i = 0; i < nfin; ++i) rest.push_back({median(cands[i].ms), cands[i].t});
        std::sort(rest.begin(), rest.end(),
                  [](const auto& x, const auto& y) { return x.first < y.first; });
        for (const auto& r : rest) {
            if (top[l].size() >= 3) break;
            const LevelTune& t = r.second;
            bool dup = false;
            for (const LevelTune& u : top[l])
                dup = dup || std::memcmp(&t, &u, sizeof t) == 0;
            if (!dup) top[l].push_back(t);
        }
    }
    // Each level was timed alone; in the caller's whole schedule, on the
    // default chains, the launch shapes also decide how one chain's kernels
    // overlap another's.  So, level by level, the runners-up of the level and
    // the other warp passes per wave are tried in the whole schedule against
    // the current choice, the two timed in turn five times each (the fastest
    // run of each counts), and a candidate is kept when it is 0.5% faster.
    {
        std::vector<Step> full;
        for (int l = P->levels - 1; l >= 0; --l)
            if (P->iters[l] > 0) full.push_back(Step{l, P->iters[l]});
        auto run_full = [&](float* ms) {
            return run_batch(c, n, A, B, nullptr, P, full, 0, o.data(), nullptr, ms);
        };
        rgbid_status st = RGBID_OK;
        for (int l = 0; l < P->levels && st == RGBID_OK && !full.empty(); ++l) {
            const std::string key = tune_key(n, A, l, P->warp, f16);
            std::vector<LevelTune> tries(top[l].begin() + 1, top[l].end());
            for (int wp : {1, 2, 4, 8}) {
                LevelTune t = top[l][0];
                t.warp_passes = wp;
                if (wp != top[l][0].warp_passes) tries.push_back(t);
            }
            for (const LevelTune& cand : tries) {
                const LevelTune keep = c->tunes[key];
                if (std::memcmp(&cand, &keep, sizeof cand) == 0) continue;
                float t_keep = 1e30f, t_cand = 1e30f, ms = 0.0f;
                // first runs capture the graphs of both choices
                if ((st = run_full(nullptr)) != RGBID_OK) break;
                c->tunes[key] = cand;
                if ((st = run_full(nullptr)) != RGBID_OK) break;
                for (int r = 0; r < 5 && st == RGBID_OK; ++r) {
                    c->tunes[key] = keep;
                    if ((st = run_full(&ms)) != RGBID_OK) break;
                    t_keep = std::min(t_keep, ms);
                    c->tunes[key] = cand;
                    if ((st = run_full(&ms)) != RGBID_OK) break;
                    t_cand = std::min(t_cand, ms);
                }
                c->tunes[key] = st == RGBID_OK && t_cand < 0.995f * t_keep ? cand : keep;
            }
        }
        if (st != RGBID_OK) {
            c->profiling = saved_prof;
            return st;
        }
    }
    // drop the candidate graphs
    clear_graphs(c);
    c->profiling = saved_prof;
    return RGBID_OK;
}

rgbid_status rgbid_tune_save(const rgbid_ctx* c, const char* path)
{
    if (!c || !path) return RGBID_E_ARG;
    FILE* f = std::fopen(path, "w");
    if (!f) return RGBID_E_ARG;
    for (const auto& kv : c->tunes)
        std::fprintf(f, "%s %d %d %d %d %d\n", kv.first.c_str(), kv.second.fused, kv.second.waves,
                     kv.second.tiles_per_wave, kv.second.xcd_remap, kv.second.warp_passes);
    std::fclose(f);
    return RGBID_OK;
}

rgbid_status rgbid_tune_load(rgbid_ctx* c, const char* path)
{
    if (!c || !path) return RGBID_E_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return set_err(c, RGBID_E_ARG, "cannot open %s", path);
    char key[512];
    LevelTune t;
    int nread = 0;
    while (std::fscanf(f, "%511s %d %d %d %d %d", key, &t.fused, &t.waves, &t.tiles_per_wave,
                       &t.xcd_remap, &t.warp_passes) == 6) {
        if (t.waves < 1 || t.waves > 8 || t.tiles_per_wave < 1 || t.tiles_per_wave > 64 ||
            t.warp_passes < 1 || t.warp_passes > 64)
            continue;
        c->tunes[key] = t;
        ++nread;
    }
    std::fclose(f);
    clear_graphs(c);
    return nread > 0 ? RGBID_OK : set_err(c, RGBID_E_ARG, "no tune entries in %s", path);
}

rgbid_status rgbid_keyframe_init(rgbid_ctx* c, const rgbid_camera* cam, const float* W_dev,
                                 size_t pitch_elems, rgbid_kf** out)
{
    if (!c) return RGBID_E_ARG;
    if (!out) return set_err(c, RGBID_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cam || !W_dev) return set_err(c, RGBID_E_ARG, "NULL camera or image");
    if (cam->width < 1 || cam->height < 1 || pitch_elems < (size_t)cam->width)
        return set_err(c, RGBID_E_ARG, "bad image size or pitch");
    if (!(cam->fx > 0 && cam->fy > 0)) return set_err(c, RGBID_E_ARG, "focal lengths must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_kf* k = new (std::nothrow) rgbid_kf();
    if (!k) return set_err(c, RGBID_E_NOMEM, "host allocation failed");
    k->device = c->device;
    k->cam = *cam;
    const size_t np = (size_t)cam->width * cam->height;
    const size_t bytes = align_up(np * 4, 256) * 2 + 256;
    hipError_t e = hipMalloc(&k->base, bytes);
    if (e != hipSuccess) {
        delete k;
        return set_err(c, RGBID_E_NOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    }
    k->W = static_cast<float*>(k->base);
    k->C = reinterpret_cast<float*>(static_cast<char*>(k->base) + align_up(np * 4, 256));
    k->count = reinterpret_cast<unsigned long long*>(static_cast<char*>(k->base) +
                                                     2 * align_up(np * 4, 256));
    e = launch_copy_valid(c->stream, W_dev, (long long)pitch_elems, cam->width, cam->height, k->W);
    if (e == hipSuccess) e = launch_fill(c->stream, k->C, (int)np, 1.0f);
    if (e != hipSuccess) {
        (void)hipFree(k->base);
        delete k;
        return set_err(c, RGBID_E_DEVICE, "keyframe init failed: %s", hipGetErrorString(e));
    }
    *out = k;
    return RGBID_OK;
}

rgbid_status rgbid_fuse(rgbid_ctx* c, rgbid_kf* kf, const float* Wk_dev, size_t pitch_elems,
                        const rgbid_pose* T, double tol, long long* n_fused)
{
    if (!c) return RGBID_E_ARG;
    if (!kf || !Wk_dev || !T) return set_err(c, RGBID_E_ARG, "NULL keyframe, image or pose");
    if (kf->device != c->device) return set_err(c, RGBID_E_ARG, "keyframe on another device");
    if (pitch_elems < (size_t)kf->cam.width) return set_err(c, RGBID_E_ARG, "pitch < width");
    if (!(tol > 0.0)) return set_err(c, RGBID_E_ARG, "tol must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    FuseArgs a;
    a.Wkf = kf->W;
    a.Ckf = kf->C;
    a.Wk = Wk_dev;
    a.pitch = (long long)pitch_elems;
    a.w = kf->cam.width;
    a.h = kf->cam.height;
    a.fx = (float)kf->cam.fx;
    a.fy = (float)kf->cam.fy;
    a.cx = (float)kf->cam.cx;
    a.cy = (float)kf->cam.cy;
    pose_flow_floats(T->R, T->t, a.D, a.Rtt);
    a.tol = (float)tol;
    a.count = n_fused ? kf->count : nullptr;
    if (n_fused) HIPCHK(c, hipMemsetAsync(kf->count, 0, sizeof(unsigned long long), c->stream));
    HIPCHK(c, launch_fuse(c->stream, a));
    if (n_fused) {
        rgbid_status st;
        if ((st = ensure_down(c, sizeof(unsigned long long))) != RGBID_OK) return st;
        HIPCHK(c, hipMemcpyAsync(c->h_down, kf->count, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *n_fused = (long long)*static_cast<unsigned long long*>(c->h_down);
    }
    return RGBID_OK;
}

rgbid_status rgbid_fuse_batch(rgbid_ctx* c, rgbid_kf* kf, int n, const float* const* Wk_dev,
                              size_t pitch_elems, const rgbid_pose* T, double tol,
                              long long* n_fused)
{
    if (!c) return RGBID_E_ARG;
    if (!kf || !Wk_dev || !T) return set_err(c, RGBID_E_ARG, "NULL keyframe, images or poses");
    if (n < 1 || n > kMaxFuseBatch) return set_err(c, RGBID_E_ARG, "n outside 1..%d", kMaxFuseBatch);
    for (int i = 0; i < n; ++i)
        if (!Wk_dev[i]) return set_err(c, RGBID_E_ARG, "NULL image %d", i);
    if (kf->device != c->device) return set_err(c, RGBID_E_ARG, "keyframe on another device");
    if (pitch_elems < (size_t)kf->cam.width) return set_err(c, RGBID_E_ARG, "pitch < width");
    if (!(tol > 0.0)) return set_err(c, RGBID_E_ARG, "tol must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    // device workspace: the frame table, then n counters
    const size_t tab = align_up((size_t)n * sizeof(FuseFrame), 256);
    if ((st = ensure(c, c->fuse, tab + (size_t)n * sizeof(unsigned long long))) != RGBID_OK)
        return st;
    char* stage = nullptr;
    if ((st = stage_begin(c, (size_t)n * sizeof(FuseFrame), &stage)) != RGBID_OK) return st;
    FuseFrame* fr = reinterpret_cast<FuseFrame*>(stage);
    for (int i = 0; i < n; ++i) {
        fr[i].Wk = Wk_dev[i];
        pose_flow_floats(T[i].R, T[i].t, fr[i].D, fr[i].Rtt);
    }
    HIPCHK(c, hipMemcpyAsync(c->fuse.p, stage, (size_t)n * sizeof(FuseFrame), hipMemcpyHostToDevice,
                             c->stream));
    if ((st = stage_end(c)) != RGBID_OK) return st;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(static_cast<char*>(c->fuse.p) + tab);
    FuseBatchArgs a;
    a.Wkf = kf->W;
    a.Ckf = kf->C;
    a.frames = static_cast<const FuseFrame*>(c->fuse.p);
    a.n = n;
    a.pitch = (long long)pitch_elems;
    a.w = kf->cam.width;
    a.h = kf->cam.height;
    a.fx = (float)kf->cam.fx;
    a.fy = (float)kf->cam.fy;
    a.cx = (float)kf->cam.cx;
    a.cy = (float)kf->cam.cy;
    a.tol = (float)tol;
    a.count = n_fused ? cnt : nullptr;
    if (n_fused) HIPCHK(c, hipMemsetAsync(cnt, 0, (size_t)n * sizeof(unsigned long long), c->stream));
    HIPCHK(c, launch_fuse_batch(c->stream, a));
    if (n_fused) {
        if ((st = ensure_down(c, (size_t)n * sizeof(unsigned long long))) != RGBID_OK) return st;
        HIPCHK(c, hipMemcpyAsync(c->h_down, cnt, (size_t)n * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < n; ++i) n_fused[i] = (long long)static_cast<unsigned long long*>(c->h_down)[i];
    }
    return RGBID_OK;
}

rgbid_status rgbid_keyframe_read(rgbid_ctx* c, const rgbid_kf* kf, float* W_out, float* C_out)
{
    if (!c) return RGBID_E_ARG;
    if (!kf) return set_err(c, RGBID_E_ARG, "NULL keyframe");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t bytes = (size_t)kf->cam.width * kf->cam.height * sizeof(float);
    if (W_out) HIPCHK(c, hipMemcpyAsync(W_out, kf->W, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (C_out) HIPCHK(c, hipMemcpyAsync(C_out, kf->C, bytes, hipMemcpyDeviceToDevice, c->stream));
    return RGBID_OK;
}

rgbid_status rgbid_covisibility(rgbid_ctx* c, const rgbid_pyr* A, const rgbid_pyr* B, int level,
                                const rgbid_pose* T, double tol, double* ratio, long long* counts)
{
    if (!c) return RGBID_E_ARG;
    if (!A || !B || !T || !ratio) return set_err(c, RGBID_E_ARG, "NULL argument");
    if (level < 0 || level >= A->levels || level >= B->levels)
        return set_err(c, RGBID_E_ARG, "level outside the pyramids");
    if (A->w[level] != B->w[level] || A->h[level] != B->h[level] || A->f16 != B->f16)
        return set_err(c, RGBID_E_SHAPE, "A and B differ in size or format");
    if (!(tol > 0.0)) return set_err(c, RGBID_E_ARG, "tol must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    if ((st = ensure(c, c->covis, 4 * sizeof(unsigned long long))) != RGBID_OK) return st;
    unsigned long long* cnt = static_cast<unsigned long long*>(c->covis.p);
    HIPCHK(c, hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), c->stream));
    // A -> B with T, then B -> A with T^-1 = (R^T, -R^T t)
    double Ri[9], ti[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Ri[3 * i + j] = T->R[3 * j + i];
        ti[i] = -(Ri[3 * i] * T->t[0] + Ri[3 * i + 1] * T->t[1] + Ri[3 * i + 2] * T->t[2]);
    }
    for (int dir = 0; dir < 2; ++dir) {
        CovisArgs a;
        a.WA = dir == 0 ? A->wp[level] : B->wp[level];
        a.WB = dir == 0 ? B->wp[level] : A->wp[level];
        a.f16 = A->f16;
        a.w = A->w[level];
        a.h = A->h[level];
        a.fx = (float)A->fx[level];
        a.fy = (float)A->fy[level];
        a.cx = (float)A->cx[level];
        a.cy = (float)A->cy[level];
        if (dir == 0) pose_flow_floats(T->R, T->t, a.D, a.Rtt);
        else pose_flow_floats(Ri, ti, a.D, a.Rtt);
        a.tol = (float)tol;
        a.count = cnt + 2 * dir;
        HIPCHK(c, launch_covis(c->stream, a));
    }
    if ((st = ensure_down(c, 4 * sizeof(unsigned long long))) != RGBID_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->h_down, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const unsigned long long* h = static_cast<const unsigned long long*>(c->h_down);
    const double ra = h[0] ? (double)h[1] / (double)h[0] : 0.0;
    const double rb = h[2] ? (double)h[3] / (double)h[2] : 0.0;
    *ratio = std::min(ra, rb);
    if (counts)
        for (int i = 0; i < 4; ++i) counts[i] = (long long)h[i];
    return RGBID_OK;
}

rgbid_status rgbid_covariance(rgbid_ctx* c, const rgbid_pyr* A, const rgbid_pyr* B,
                              const rgbid_pose* T, const rgbid_align_params* P,
                              const rgbid_bilateral* bf, double Sigma[36], rgbid_align_stats* stats)
{
    if (!c) return RGBID_E_ARG;
    if (!A || !B || !T || !Sigma) return set_err(c, RGBID_E_ARG, "NULL argument");
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    rgbid_bilateral b{2, 1.5, 10.0, 0.05};
    if (bf) b = *bf;
    if (b.radius < 0 || b.radius > 7 || !(b.sigma_s > 0) || !(b.sigma_I > 0) || !(b.rel_W > 0))
        return set_err(c, RGBID_E_ARG, "bilateral parameters out of range");
    HIPCHK(c, hipSetDevice(c->device));
    // filtered copy of A: level 0 filtered, then its pyramid (cached per size)
    rgbid_pyr*& F = c->cov_pyr;
    if (F && (F->w[0] != A->w[0] || F->h[0] != A->h[0] || F->levels != A->levels || F->f16 != A->f16 ||
              F->cam.fx != A->cam.fx || F->cam.fy != A->cam.fy || F->cam.cx != A->cam.cx ||
              F->cam.cy != A->cam.cy)) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        rgbid_pyramid_free(F);
        F = nullptr;
    }
    const size_t n0 = (size_t)A->w[0] * A->h[0];
    rgbid_status st;
    if ((st = ensure(c, c->cov_img, 2 * n0 * sizeof(float))) != RGBID_OK) return st;
    float* If = static_cast<float*>(c->cov_img.p);
    float* Wf = If + n0;
    HIPCHK(c, launch_bilateral(c->stream, A->iw[0], A->f16, A->w[0], A->h[0], b.radius,
                               (float)b.sigma_s, (float)b.sigma_I, (float)b.rel_W, If, Wf));
    if (!F) {
        if ((st = rgbid_pyramid(c, &A->cam, A->levels, A->f16 ? RGBID_F16 : RGBID_F32, If, Wf,
                                (size_t)A->w[0], &F)) != RGBID_OK)
            return st;
    } else if ((st = rgbid_pyramid_update(c, F, If, Wf, (size_t)A->w[0])) != RGBID_OK) {
        return st;
    }
    rgbid_align_stats s;
    if ((st = rgbid_normal_equations(c, F, B, 0, T, P, &s)) != RGBID_OK) return st;
    if (stats) *stats = s;
    // Sigma = H^-1 by FP64 Cholesky on the host (6x6)
    double H[6][6], L[6][6] = {};
    int k = 0;
    for (int a = 0; a < 6; ++a)
        for (int bb = a; bb < 6; ++bb) H[a][bb] = H[bb][a] = s.H[k++];
    double dmax = 0.0;
    for (int a = 0; a < 6; ++a) dmax = std::max(dmax, H[a][a]);
    for (int j = 0; j < 6; ++j) {
        double d = H[j][j];
        for (int q = 0; q < j; ++q) d -= L[j][q] * L[j][q];
        if (!(d > 1e-12 * dmax)) return set_err(c, RGBID_E_DEGENERATE, "filtered Hessian not positive definite");
        L[j][j] = std::sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double e = H[i][j];
            for (int q = 0; q < j; ++q) e -= L[i][q] * L[j][q];
            L[i][j] = e / L[j][j];
        }
    }
    for (int col = 0; col < 6; ++col) {
        double y[6], x[6];
        for (int i = 0; i < 6; ++i) {
            double e = (i == col) ? 1.0 : 0.0;
            for (int q = 0; q < i; ++q) e -= L[i][q] * y[q];
            y[i] = e / L[i][i];
        }
        for (int i = 5; i >= 0; --i) {
            double e = y[i];
            for (int q = i + 1; q < 6; ++q) e -= L[q][i] * x[q];
            x[i] = e / L[i][i];
        }
        for (int i = 0; i < 6; ++i) Sigma[6 * i + col] = x[i];
    }
    return RGBID_OK;
}

rgbid_status rgbid_keyframe_reset(rgbid_ctx* c, rgbid_kf* kf, const float* W_dev,
                                  size_t pitch_elems)
{
    if (!c) return RGBID_E_ARG;
    if (!kf || !W_dev) return set_err(c, RGBID_E_ARG, "NULL keyframe or image");
    if (kf->device != c->device) return set_err(c, RGBID_E_ARG, "keyframe on another device");
    if (pitch_elems < (size_t)kf->cam.width) return set_err(c, RGBID_E_ARG, "pitch < width");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_copy_valid(c->stream, W_dev, (long long)pitch_elems, kf->cam.width,
                                kf->cam.height, kf->W));
    HIPCHK(c, launch_fill(c->stream, kf->C, kf->cam.width * kf->cam.height, 1.0f));
    return RGBID_OK;
}

rgbid_status rgbid_set_profiling(rgbid_ctx* c, int on)
{
    if (!c) return RGBID_E_ARG;
    c->profiling = on != 0;
    for (int i = 0; i < kMaxLevels * 4; ++i) {
        c->prof_ms[i] = 0.0;
        c->prof_n[i] = 0;
    }
    return RGBID_OK;
}

rgbid_status rgbid_kernel_times(const rgbid_ctx* c, double* ms_total, long long* launches)
{
    if (!c || !ms_total || !launches) return RGBID_E_ARG;
    for (int i = 0; i < kMaxLevels * 4; ++i) {
        ms_total[i] = c->prof_ms[i];
        launches[i] = c->prof_n[i];
    }
    return RGBID_OK;
}

void rgbid_keyframe_free(rgbid_kf* kf)
{
    if (!kf) return;
    (void)hipSetDevice(kf->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(kf->base);
    delete kf;
}

}  // extern "C"

// ====================================================================== pose maps, warm start

namespace {

void rot_exp(const double th[3], double R[9])
{
    const double n = std::sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    const double S[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
    double S2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += S[3 * i + k] * S[3 * k + j];
            S2[3 * i + j] = acc;
        }
    const double a = n < 1e-8 ? 1.0 : std::sin(n) / n;
    const double b = n < 1e-8 ? 0.5 : (1.0 - std::cos(n)) / (n * n);
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * S[i] + b * S2[i];
}

rgbid_status net_reserve(rgbid_ctx* c, rgbid_net* net, int n)
{
    if (n <= net->cap) return RGBID_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (net->act_base) HIPCHK(c, hipFree(net->act_base));
    net->act_base = nullptr;
    net->cap = 0;
    const int cap = std::max(n, 64);
    size_t off[16], total = 0;
    int k = 0;
    auto add = [&](size_t bytes) { off[k++] = total; total = align_up(total + bytes, 256); };
    for (int l = 0; l < 4; ++l) add((size_t)cap * kCnnCh[l + 1] * kCnnHs[l + 1] * kCnnWs[l + 1] * 4);
    for (int l = 0; l < 4; ++l) add((size_t)cap * kCnnCh[l + 1] * kCnnHs[l + 1] * kCnnWs[l + 1] * 4);
    add((size_t)cap * 128 * 4);
    add((size_t)cap * 6 * 4);
    add((size_t)cap * 6 * 4);
    add((size_t)cap * 4);
    add((size_t)cap * 6 * 4);
    HIPCHK(c, hipMalloc(&net->act_base, total));
    char* b = static_cast<char*>(net->act_base);
    for (int l = 0; l < 4; ++l) net->buf.act[l] = reinterpret_cast<float*>(b + off[l]);
    for (int l = 0; l < 4; ++l) net->buf.dz[l] = reinterpret_cast<float*>(b + off[4 + l]);
    net->buf.pooled = reinterpret_cast<float*>(b + off[8]);
    net->buf.out = reinterpret_cast<float*>(b + off[9]);
    net->buf.dout = reinterpret_cast<float*>(b + off[10]);
    net->buf.loss_n = reinterpret_cast<float*>(b + off[11]);
    net->buf.target = reinterpret_cast<float*>(b + off[12]);
    net->cap = cap;
    return RGBID_OK;
}

rgbid_status net_targets(rgbid_ctx* c, rgbid_net* net, int n, const double* xi)
{
    char* stage;
    rgbid_status st;
    if ((st = stage_begin(c, (size_t)n * 6 * sizeof(float), &stage)) != RGBID_OK) return st;
    float* t = reinterpret_cast<float*>(stage);
    for (int i = 0; i < n * 6; ++i) t[i] = (float)(xi[i] / kXiScale[i % 6]);
    HIPCHK(c, hipMemcpyAsync(net->buf.target, t, (size_t)n * 6 * sizeof(float),
                             hipMemcpyHostToDevice, c->stream));
    return stage_end(c);
}

rgbid_status net_loss(rgbid_ctx* c, rgbid_net* net, int n, double* loss)
{
    rgbid_status st;
    if ((st = ensure_down(c, (size_t)n * sizeof(float))) != RGBID_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->h_down, net->buf.loss_n, (size_t)n * sizeof(float),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const float* l = static_cast<const float*>(c->h_down);
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += l[i];
    *loss = s / n;
    return RGBID_OK;
}

// The inference buffers for n samples: GEMM-order weights, then the limb
// activations, then the n x 6 output.
size_t net_wg_elems()
{
    size_t e = 0;
    for (int l = 0; l < 4; ++l) e += (size_t)kCnnCh[l + 1] * cnn_gemm_k(l);
    return e;
}

rgbid_status net_infer_reserve(rgbid_ctx* c, rgbid_net* net, int n)
{
    if (n <= net->inf_cap) return RGBID_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (net->inf_base) HIPCHK(c, hipFree(net->inf_base));
    net->inf_base = nullptr;
    net->inf_cap = 0;
    net->wg_step = -1;
    const int cap = std::max(n, 64);
    const size_t total = align_up(net_wg_elems() * 2, 256) + align_up(cnn_limb_bytes(cap), 256) +
                         align_up((size_t)cap * 6 * 4, 256);
    HIPCHK(c, hipMalloc(&net->inf_base, total));
    net->inf_cap = cap;
    return RGBID_OK;
}

// Normalised outputs of the matrix-core forward for pairs (A[i], B[i]) in
// device memory (n x 6 floats); enqueued, not synchronised.
rgbid_status net_forward_pyr(rgbid_ctx* c, rgbid_net* net, int n, const rgbid_pyr* const* A,
                             const rgbid_pyr* const* B, float** out_dev)
{
    rgbid_status st;
    if ((st = net_infer_reserve(c, net, n)) != RGBID_OK) return st;
    char* ib = static_cast<char*>(net->inf_base);
    unsigned short* wg = reinterpret_cast<unsigned short*>(ib);
    unsigned short* limbs = reinterpret_cast<unsigned short*>(ib + align_up(net_wg_elems() * 2, 256));
    float* out = reinterpret_cast<float*>(ib + align_up(net_wg_elems() * 2, 256) +
                                          align_up(cnn_limb_bytes(net->inf_cap), 256));
    if (net->wg_step != net->step) {
        HIPCHK(c, cnn_gemm_weights(c->stream, net->buf, wg));
        net->wg_step = net->step;
    }
    if ((st = ensure(c, c->frames, std::max(n * sizeof(CnnInput), sizeof(PyrFrame)))) != RGBID_OK)
        return st;
    char* stage;
    if ((st = stage_begin(c, n * sizeof(CnnInput), &stage)) != RGBID_OK) return st;
    CnnInput* in = reinterpret_cast<CnnInput*>(stage);
    for (int i = 0; i < n; ++i) {
        if (!A[i] || !B[i]) return set_err(c, RGBID_E_ARG, "NULL pyramid %d", i);
        int la = -1, lb = -1;
        for (int l = 0; l < A[i]->levels; ++l)
            if (A[i]->w[l] == kCnnW && A[i]->h[l] == kCnnH) la = l;
        for (int l = 0; l < B[i]->levels; ++l)
            if (B[i]->w[l] == kCnnW && B[i]->h[l] == kCnnH) lb = l;
        if (la < 0 || lb < 0) return set_err(c, RGBID_E_SHAPE, "pair %d has no 80x60 level", i);
        if (B[i]->f16 != A[i]->f16) return set_err(c, RGBID_E_SHAPE, "pair %d mixes formats", i);
        in[i].A = A[i]->iw[la];
        in[i].B = B[i]->iw[lb];
        in[i].f16 = A[i]->f16;
        in[i].pad = 0;
    }
    HIPCHK(c, hipMemcpyAsync(c->frames.p, in, n * sizeof(CnnInput), hipMemcpyHostToDevice, c->stream));
    if ((st = stage_end(c)) != RGBID_OK) return st;
    HIPCHK(c, cnn_forward_mfma(c->stream, net->buf, wg, static_cast<const CnnInput*>(c->frames.p),
                               n, limbs, out));
    *out_dev = out;
    return RGBID_OK;
}

}  // namespace

extern "C" {

void rgbid_pose_exp(const double xi[6], rgbid_pose* T)
{
    if (!xi || !T) return;
    rot_exp(xi + 3, T->R);
    for (int i = 0; i < 3; ++i) T->t[i] = xi[i];
}

void rgbid_pose_log(const rgbid_pose* T, double xi[6])
{
    if (!xi || !T) return;
    const double* R = T->R;
    double cth = (R[0] + R[4] + R[8] - 1.0) / 2.0;
    cth = std::min(1.0, std::max(-1.0, cth));
    const double n = std::acos(cth);
    const double f = n < 1e-8 ? 0.5 : n / (2.0 * std::sin(n));
    xi[0] = T->t[0];
    xi[1] = T->t[1];
    xi[2] = T->t[2];
    xi[3] = f * (R[7] - R[5]);
    xi[4] = f * (R[2] - R[6]);
    xi[5] = f * (R[3] - R[1]);
}

size_t rgbid_warmstart_param_count(void) { return (size_t)kCnnParams; }

rgbid_status rgbid_warmstart_create(rgbid_ctx* c, const float* params, rgbid_net** out)
{
    if (!c) return RGBID_E_ARG;
    if (!out || !params) return set_err(c, RGBID_E_ARG, "NULL parameters or output");
    *out = nullptr;
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_net* net = new (std::nothrow) rgbid_net();
    if (!net) return set_err(c, RGBID_E_NOMEM, "host allocation failed");
    net->device = c->device;
    net->wg_step = -1;
    const size_t P = kCnnParams, f = align_up(P * 4, 256);
    const size_t total = 5 * f + align_up(P * 2, 256);
    hipError_t e = hipMalloc(&net->base, total);
    if (e != hipSuccess) {
        delete net;
        return set_err(c, RGBID_E_NOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    }
    char* b = static_cast<char*>(net->base);
    net->buf.w = reinterpret_cast<float*>(b);
    net->buf.m = reinterpret_cast<float*>(b + f);
    net->buf.v = reinterpret_cast<float*>(b + 2 * f);
    net->buf.grad = reinterpret_cast<float*>(b + 3 * f);
    net->buf.decay = reinterpret_cast<float*>(b + 4 * f);
    net->buf.wbf = reinterpret_cast<__hip_bfloat16*>(b + 5 * f);
    std::vector<float> decay(P, 0.0f);
    for (int l = 0; l < 10; l += 2)
        for (int i = kCnnOff[l]; i < kCnnOff[l + 1]; ++i) decay[i] = 1.0f;
    e = hipMemcpy(net->buf.w, params, P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(net->buf.decay, decay.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(net->buf.m, 0, 2 * f, c->stream);
    if (e == hipSuccess) e = cnn_refresh_bf16(c->stream, net->buf);
    if (e != hipSuccess) {
        (void)hipFree(net->base);
        delete net;
        return set_err(c, RGBID_E_DEVICE, "warm-start init failed: %s", hipGetErrorString(e));
    }
    *out = net;
    return RGBID_OK;
}

void rgbid_warmstart_free(rgbid_net* net)
{
    if (!net) return;
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    if (net->act_base) (void)hipFree(net->act_base);
    if (net->inf_base) (void)hipFree(net->inf_base);
    (void)hipFree(net->base);
    delete net;
}

rgbid_status rgbid_warmstart_get_params(rgbid_ctx* c, const rgbid_net* net, float* params)
{
    if (!c) return RGBID_E_ARG;
    if (!net || !params) return set_err(c, RGBID_E_ARG, "NULL network or output");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(params, net->buf.w, (size_t)kCnnParams * 4, hipMemcpyDeviceToHost));
    return RGBID_OK;
}

rgbid_status rgbid_warmstart_input(rgbid_ctx* c, int n, const rgbid_pyr* const* A,
                                   const rgbid_pyr* const* B, float* x_dev)
{
    if (!c) return RGBID_E_ARG;
    if (n < 1 || !A || !B || !x_dev) return set_err(c, RGBID_E_ARG, "bad arguments");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    if ((st = ensure(c, c->frames, std::max(n * sizeof(CnnInput), sizeof(PyrFrame)))) != RGBID_OK)
        return st;
    char* stage;
    if ((st = stage_begin(c, n * sizeof(CnnInput), &stage)) != RGBID_OK) return st;
    CnnInput* in = reinterpret_cast<CnnInput*>(stage);
    for (int i = 0; i < n; ++i) {
        if (!A[i] || !B[i]) return set_err(c, RGBID_E_ARG, "NULL pyramid %d", i);
        int la = -1, lb = -1;
        for (int l = 0; l < A[i]->levels; ++l)
            if (A[i]->w[l] == kCnnW && A[i]->h[l] == kCnnH) la = l;
        for (int l = 0; l < B[i]->levels; ++l)
            if (B[i]->w[l] == kCnnW && B[i]->h[l] == kCnnH) lb = l;
        if (la < 0 || lb < 0) return set_err(c, RGBID_E_SHAPE, "pair %d has no 80x60 level", i);
        in[i].A = A[i]->iw[la];
        in[i].B = B[i]->iw[lb];
        in[i].f16 = A[i]->f16;
        if (B[i]->f16 != A[i]->f16) return set_err(c, RGBID_E_SHAPE, "pair %d mixes formats", i);
    }
    HIPCHK(c, hipMemcpyAsync(c->frames.p, in, n * sizeof(CnnInput), hipMemcpyHostToDevice, c->stream));
    if ((st = stage_end(c)) != RGBID_OK) return st;
    HIPCHK(c, cnn_input(c->stream, static_cast<const CnnInput*>(c->frames.p), n, x_dev));
    return RGBID_OK;
}

rgbid_status rgbid_warmstart_forward(rgbid_ctx* c, rgbid_net* net, int n, const float* x_dev,
                                     double* xi_out)
{
    if (!c) return RGBID_E_ARG;
    if (!net || n < 1 || !x_dev || !xi_out) return set_err(c, RGBID_E_ARG, "bad arguments");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    if ((st = net_reserve(c, net, n)) != RGBID_OK) return st;
    HIPCHK(c, cnn_forward(c->stream, net->buf, n, x_dev));
    if ((st = ensure_down(c, (size_t)n * 6 * sizeof(float))) != RGBID_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->h_down, net->buf.out, (size_t)n * 6 * sizeof(float),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const float* o = static_cast<const float*>(c->h_down);
    for (int i = 0; i < n * 6; ++i) xi_out[i] = (double)o[i] * kXiScale[i % 6];
    return RGBID_OK;
}

rgbid_status rgbid_warmstart_forward_pyr(rgbid_ctx* c, rgbid_net* net, int n,
                                         const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                                         double* xi_out)
{
    if (!c) return RGBID_E_ARG;
    if (!net || n < 1 || !A || !B || !xi_out) return set_err(c, RGBID_E_ARG, "bad arguments");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    float* out = nullptr;
    if ((st = net_forward_pyr(c, net, n, A, B, &out)) != RGBID_OK) return st;
    if ((st = ensure_down(c, (size_t)n * 6 * sizeof(float))) != RGBID_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->h_down, out, (size_t)n * 6 * sizeof(float), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const float* o = static_cast<const float*>(c->h_down);
    for (int i = 0; i < n * 6; ++i) xi_out[i] = (double)o[i] * kXiScale[i % 6];
    return RGBID_OK;
}

rgbid_status rgbid_warmstart_predict(rgbid_ctx* c, rgbid_net* net, int n,
                                     const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                                     float* x_scratch, rgbid_pose* init_out)
{
    (void)x_scratch;   // the matrix-core path reads the pyramids itself
    if (!c) return RGBID_E_ARG;
    if (!init_out) return set_err(c, RGBID_E_ARG, "NULL output");
    if (n < 1) return set_err(c, RGBID_E_ARG, "bad arguments");
    std::vector<double> xi((size_t)n * 6);
    rgbid_status st;
    if ((st = rgbid_warmstart_forward_pyr(c, net, n, A, B, xi.data())) != RGBID_OK) return st;
    for (int i = 0; i < n; ++i) rgbid_pose_exp(&xi[6 * i], &init_out[i]);
    return RGBID_OK;
}

rgbid_status rgbid_align_batch_warm(rgbid_ctx* c, rgbid_net* net, int n,
                                    const rgbid_pyr* const* A, const rgbid_pyr* const* B,
                                    const rgbid_align_params* P, rgbid_pose* out,
                                    rgbid_align_stats* stats)
{
    if (!c) return RGBID_E_ARG;
    if (!net || !out) return set_err(c, RGBID_E_ARG, "NULL network or output");
    std::string why;
    if (!params_ok(P, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    if (n < 1 || !A || !B) return set_err(c, RGBID_E_ARG, "need n >= 1 and pyramid arrays");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    float* twist = nullptr;
    if ((st = net_forward_pyr(c, net, n, A, B, &twist)) != RGBID_OK) return st;
    std::vector<Step> sched;
    for (int l = P->levels - 1; l >= 0; --l)
        if (P->iters[l] > 0) sched.push_back(Step{l, P->iters[l]});
    return run_batch(c, n, A, B, nullptr, P, sched, 1, out, stats, nullptr, false, twist);
}

rgbid_status rgbid_warmstart_gradient(rgbid_ctx* c, rgbid_net* net, int n, const float* x_dev,
                                      const double* xi, double* loss, float* grad_host)
{
    if (!c) return RGBID_E_ARG;
    if (!net || n < 1 || !x_dev || !xi) return set_err(c, RGBID_E_ARG, "bad arguments");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    if ((st = net_reserve(c, net, n)) != RGBID_OK) return st;
    if ((st = net_targets(c, net, n, xi)) != RGBID_OK) return st;
    HIPCHK(c, cnn_forward(c->stream, net->buf, n, x_dev));
    HIPCHK(c, cnn_backward(c->stream, net->buf, n, x_dev, net->buf.target));
    if (loss && (st = net_loss(c, net, n, loss)) != RGBID_OK) return st;
    if (grad_host) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(grad_host, net->buf.grad, (size_t)kCnnParams * 4, hipMemcpyDeviceToHost));
    }
    return RGBID_OK;
}

rgbid_status rgbid_warmstart_train_step(rgbid_ctx* c, rgbid_net* net, int n, const float* x_dev,
                                        const double* xi, double lr, double wd, double* loss)
{
    if (!c) return RGBID_E_ARG;
    if (!net || n < 1 || !x_dev || !xi) return set_err(c, RGBID_E_ARG, "bad arguments");
    if (!(lr > 0.0) || wd < 0.0) return set_err(c, RGBID_E_ARG, "lr must be > 0, wd >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    if ((st = net_reserve(c, net, n)) != RGBID_OK) return st;
    if ((st = net_targets(c, net, n, xi)) != RGBID_OK) return st;
    HIPCHK(c, cnn_forward(c->stream, net->buf, n, x_dev));
    HIPCHK(c, cnn_backward(c->stream, net->buf, n, x_dev, net->buf.target));
    net->step += 1;
    HIPCHK(c, cnn_adamw(c->stream, net->buf, (float)lr, (float)wd, net->step));
    if (loss && (st = net_loss(c, net, n, loss)) != RGBID_OK) return st;
    return RGBID_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ sensor input path

namespace {

bool camera_ok(const rgbid_camera* c)
{
    return c && c->width > 0 && c->height > 0 && (long long)c->width * c->height < (1ll << 24) &&
           c->fx > 0 && c->fy > 0 && std::isfinite(c->cx) && std::isfinite(c->cy);
}

LensF lens_f(const rgbid_camera& c, const double* k)
{
    LensF L;
    L.w = c.width;
    L.h = c.height;
    L.fx = (float)c.fx;
    L.fy = (float)c.fy;
    L.cx = (float)c.cx;
    L.cy = (float)c.cy;
    for (int i = 0; i < 5; ++i) L.k[i] = k ? (float)k[i] : 0.0f;
    return L;
}

void reg_pose(RegisterArgs& a, const rgbid_camera& camA, const rgbid_pose& T)
{
    a.tx = (float)(camA.fx * T.t[0] + camA.cx * T.t[2]);
    a.ty = (float)(camA.fy * T.t[1] + camA.cy * T.t[2]);
    a.tz = (float)T.t[2];
    for (int i = 0; i < 9; ++i) a.R.m[i] = (float)T.R[i];
}

}  // namespace

extern "C" {

rgbid_status rgbid_undistort(rgbid_ctx* c, const rgbid_lens* lens, const float* src,
                             size_t pitch_elems, int is_depth, float* dst)
{
    if (!c) return RGBID_E_ARG;
    if (!lens || !src || !dst) return set_err(c, RGBID_E_ARG, "NULL argument");
    if (!camera_ok(&lens->cam)) return set_err(c, RGBID_E_ARG, "bad camera");
    if (pitch_elems < (size_t)lens->cam.width) return set_err(c, RGBID_E_ARG, "pitch < width");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_undistort(c->stream, src, (long long)pitch_elems, lens_f(lens->cam, lens->k),
                               is_depth ? 1 : 0, dst));
    return RGBID_OK;
}

rgbid_status rgbid_register(rgbid_ctx* c, const rgbid_camera* camA, const float* WA,
                            size_t pitch_elems, const rgbid_camera* camB, const rgbid_pose* T,
                            float* WB)
{
    if (!c) return RGBID_E_ARG;
    if (!WA || !WB || !T) return set_err(c, RGBID_E_ARG, "NULL argument");
    if (!camera_ok(camA) || !camera_ok(camB)) return set_err(c, RGBID_E_ARG, "bad camera");
    if (pitch_elems < (size_t)camA->width) return set_err(c, RGBID_E_ARG, "pitch < width");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    if ((st = ensure(c, c->reg, (size_t)camA->width * camA->height * 4)) != RGBID_OK) return st;
    RegisterArgs a{};
    a.src = WA;
    a.pitch = (long long)pitch_elems;
    a.raw = 0;
    a.A = lens_f(*camA, nullptr);
    a.B = lens_f(*camB, nullptr);
    reg_pose(a, *camA, *T);
    a.Wt = static_cast<unsigned*>(c->reg.p);
    a.Wout = WB;
    HIPCHK(c, launch_register(c->stream, a));
    return RGBID_OK;
}

rgbid_status rgbid_preprocess(rgbid_ctx* c, const rgbid_sensor* S, const float* I_raw,
                              size_t pitch_I, const float* Z_raw, size_t pitch_Z, float* I_out,
                              float* W_out)
{
    if (!c) return RGBID_E_ARG;
    if (!S || !I_raw || !Z_raw || !I_out || !W_out) return set_err(c, RGBID_E_ARG, "NULL argument");
    if (!camera_ok(&S->color.cam) || !camera_ok(&S->depth.cam)) return set_err(c, RGBID_E_ARG, "bad camera");
    if (pitch_I < (size_t)S->color.cam.width || pitch_Z < (size_t)S->depth.cam.width)
        return set_err(c, RGBID_E_ARG, "pitch < width");
    if (!std::isfinite(S->beta0) || !std::isfinite(S->beta1))
        return set_err(c, RGBID_E_ARG, "non-finite depth correction");
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_status st;
    const rgbid_camera& cd = S->depth.cam;
    if ((st = ensure(c, c->reg, (size_t)cd.width * cd.height * 4)) != RGBID_OK) return st;
    RegisterArgs a{};
    a.src = Z_raw;
    a.pitch = (long long)pitch_Z;
    a.raw = 1;
    a.A = lens_f(cd, S->depth.k);
    a.B = lens_f(S->color.cam, S->color.k);
    a.D.beta0 = (float)S->beta0;
    a.D.beta1 = (float)S->beta1;
    a.D.p0x = S->p0x;
    a.D.p0y = S->p0y;
    a.D.spatial = S->spatial ? 1 : 0;
    for (int i = 0; i < 9; ++i) {
        a.D.q0[i] = (float)S->q0[i];
        a.D.q1[i] = (float)S->q1[i];
    }
    reg_pose(a, cd, S->T_dc);
    a.Wt = static_cast<unsigned*>(c->reg.p);
    a.Wout = W_out;
    a.Iraw = I_raw;
    a.pitchI = (long long)pitch_I;
    a.Iout = I_out;
    HIPCHK(c, launch_register(c->stream, a));
    return RGBID_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tracking front-end
// Sequence-level policy of sec. 7.1 / 7.2 on top of the calls above: the
// per-pixel work is the alignment, covisibility, covariance and fusion
// kernels; this part only keeps poses (FP64, host) and chooses which frames
// are the reference frame and the keyframe.

struct rgbid_tracker {
    int device = 0;
    rgbid_camera cam{};
    int levels = 0;
    rgbid_format storage = RGBID_F32;
    rgbid_tracker_params p{};
    rgbid_pyr* slot[3] = {nullptr, nullptr, nullptr};   // frame pyramids
    int rf = -1, kfs = -1;        // slots of the reference frame and of the keyframe's frame
    rgbid_kf* kf = nullptr;
    float* maps = nullptr;        // 2 * buffer dense FP32 inverse-depth maps
    std::vector<int> free_maps;
    struct Rec {
        int map;
        rgbid_pose T_w;
        double tol;
    };
    std::vector<Rec> recorded;    // frames of the active keyframe, oldest first
    std::vector<Rec> pending;     // frames of the previous keyframe, next to fuse first
    rgbid_pose T_w_rf{}, T_w_kf{}, T_rf_prev{}, T_prev2_prev{};
    double S_rf_prev[36] = {};
    long long k = -1;
};

namespace {

rgbid_pose pose_identity()
{
    rgbid_pose T{};
    T.R[0] = T.R[4] = T.R[8] = 1.0;
    return T;
}

// a * b (T_A^C = T_A^B T_B^C)
rgbid_pose pose_mul(const rgbid_pose& a, const rgbid_pose& b)
{
    rgbid_pose c{};
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += a.R[3 * i + q] * b.R[3 * q + j];
            c.R[3 * i + j] = s;
        }
        double s = a.t[i];
        for (int q = 0; q < 3; ++q) s += a.R[3 * i + q] * b.t[q];
        c.t[i] = s;
    }
    return c;
}

rgbid_pose pose_inv(const rgbid_pose& a)
{
    rgbid_pose c{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.R[3 * i + j] = a.R[3 * j + i];
    for (int i = 0; i < 3; ++i)
        c.t[i] = -(c.R[3 * i] * a.t[0] + c.R[3 * i + 1] * a.t[1] + c.R[3 * i + 2] * a.t[2]);
    return c;
}

// out = J S J^T for 6x6 row-major matrices (out may not alias S)
void sandwich_add(const double J[36], const double S[36], double out[36])
{
    double JS[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int q = 0; q < 6; ++q) s += J[6 * i + q] * S[6 * q + j];
            JS[6 * i + j] = s;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int q = 0; q < 6; ++q) s += JS[6 * i + q] * J[6 * j + q];
            out[6 * i + j] += s;
        }
}

// [v]x written into the 3x3 block at (r, c) of a 6x6 row-major matrix, scaled
void put_skew(double M[36], int r, int c, const double v[3], double s)
{
    M[6 * r + c + 1] += -s * v[2];
    M[6 * r + c + 2] += s * v[1];
    M[6 * (r + 1) + c] += s * v[2];
    M[6 * (r + 1) + c + 2] += -s * v[0];
    M[6 * (r + 2) + c] += -s * v[1];
    M[6 * (r + 2) + c + 1] += s * v[0];
}

// The alignment's step xi = (v, theta) updates T <- exp(xi)^-1 T (sec. 6.2);
// to first order that is the left perturbation dtheta = -theta,
// dt = -v + [t]x theta, so Sigma_left = M Sigma_xi M^T.
void xi_cov_to_left(const rgbid_pose& T, const double Sxi[36], double out[36])
{
    double M[36] = {};
    for (int i = 0; i < 3; ++i) {
        M[6 * i + i] = -1.0;
        M[6 * (i + 3) + i + 3] = -1.0;
    }
    put_skew(M, 0, 3, T.t, 1.0);
    std::memset(out, 0, 36 * sizeof(double));
    sandwich_add(M, Sxi, out);
}

// Covariance of T_A^B = (T_W^A)^-1 T_W^B from left-perturbation covariances
// of T_W^A and T_W^B (appendix on covariance propagation):
//   J_A = -[[R_A^T, R_A^T [t_A - t_B]x], [0, R_A^T]],  J_B = diag(R_A^T, R_A^T).
void relative_covariance(const rgbid_pose& Twa, const double Sa[36], const rgbid_pose& Twb,
                         const double Sb[36], double out[36])
{
    double Ja[36] = {}, Jb[36] = {};
    double RaT[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) RaT[3 * i + j] = Twa.R[3 * j + i];
    const double d[3] = {Twa.t[0] - Twb.t[0], Twa.t[1] - Twb.t[1], Twa.t[2] - Twb.t[2]};
    // R_A^T [d]x, column by column: (R_A^T [d]x)_{ij} = sum_q RaT_iq [d]x_qj
    double K[9] = {0.0, -d[2], d[1], d[2], 0.0, -d[0], -d[1], d[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += RaT[3 * i + q] * K[3 * q + j];
            Ja[6 * i + j] = -RaT[3 * i + j];
            Ja[6 * i + j + 3] = -s;
            Ja[6 * (i + 3) + j + 3] = -RaT[3 * i + j];
            Jb[6 * i + j] = RaT[3 * i + j];
            Jb[6 * (i + 3) + j + 3] = RaT[3 * i + j];
        }
    std::memset(out, 0, 36 * sizeof(double));
    sandwich_add(Ja, Sa, out);
    sandwich_add(Jb, Sb, out);
}

int take_map(rgbid_tracker* t)
{
    const int m = t->free_maps.back();
    t->free_maps.pop_back();
    return m;
}

}  // namespace

extern "C" {

void rgbid_tracker_default_params(rgbid_tracker_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    rgbid_default_params(&p->align);
    p->rf_threshold = 0.8;
    p->kf_threshold = 0.7;
    p->covis_level = 2;
    p->tol_sigmas = 3.0;
    p->buffer = 8;
    p->covariance = 1;
}

void rgbid_tracker_free(rgbid_tracker* t)
{
    if (!t) return;
    (void)hipSetDevice(t->device);
    (void)hipDeviceSynchronize();
    for (auto* s : t->slot)
        if (s) rgbid_pyramid_free(s);
    if (t->kf) rgbid_keyframe_free(t->kf);
    if (t->maps) (void)hipFree(t->maps);
    delete t;
}

rgbid_status rgbid_tracker_create(rgbid_ctx* c, const rgbid_camera* cam, int levels,
                                  rgbid_format storage, const rgbid_tracker_params* P,
                                  rgbid_tracker** out)
{
    if (!c) return RGBID_E_ARG;
    if (!out) return set_err(c, RGBID_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cam || !P) return set_err(c, RGBID_E_ARG, "NULL camera or parameters");
    std::string why;
    if (!params_ok(&P->align, why)) return set_err(c, RGBID_E_ARG, "%s", why.c_str());
    if (levels < P->align.levels || levels > kMaxLevels)
        return set_err(c, RGBID_E_ARG, "levels must lie in [align.levels, 8]");
    if (P->covis_level < 0 || P->covis_level >= levels)
        return set_err(c, RGBID_E_ARG, "covis_level outside the pyramid");
    if (!(P->rf_threshold >= 0.0 && P->rf_threshold <= 1.0 && P->kf_threshold >= 0.0 &&
          P->kf_threshold <= 1.0))
        return set_err(c, RGBID_E_ARG, "thresholds must lie in [0, 1]");
    if (!(P->tol_sigmas > 0.0)) return set_err(c, RGBID_E_ARG, "tol_sigmas must be > 0");
    if (P->buffer < 0 || P->buffer > 64) return set_err(c, RGBID_E_ARG, "buffer outside 0..64");
    if (storage != RGBID_F32 && storage != RGBID_F16) return set_err(c, RGBID_E_ARG, "unknown storage");
    if (cam->width < 1 || cam->height < 1 || !(cam->fx > 0 && cam->fy > 0))
        return set_err(c, RGBID_E_ARG, "bad camera");
    if ((cam->width >> (levels - 1)) < 1 || (cam->height >> (levels - 1)) < 1)
        return set_err(c, RGBID_E_ARG, "level %d would be empty", levels - 1);
    HIPCHK(c, hipSetDevice(c->device));
    rgbid_tracker* t = new (std::nothrow) rgbid_tracker();
    if (!t) return set_err(c, RGBID_E_NOMEM, "host allocation failed");
    t->device = c->device;
    t->cam = *cam;
    t->levels = levels;
    t->storage = storage;
    t->p = *P;
    if (P->buffer > 0) {
        const size_t np = (size_t)cam->width * cam->height;
        hipError_t e = hipMalloc(&t->maps, 2 * (size_t)P->buffer * np * sizeof(float));
        if (e != hipSuccess) {
            delete t;
            return set_err(c, RGBID_E_NOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
        }
        for (int m = 2 * P->buffer - 1; m >= 0; --m) t->free_maps.push_back(m);
    }
    *out = t;
    return RGBID_OK;
}

const rgbid_kf* rgbid_tracker_keyframe(const rgbid_tracker* t) { return t ? t->kf : nullptr; }

rgbid_status rgbid_track(rgbid_ctx* c, rgbid_tracker* t, const float* I_dev, const float* W_dev,
                         size_t pitch_elems, rgbid_track_result* out)
{
    if (!c) return RGBID_E_ARG;
    if (!t || !I_dev || !W_dev || !out) return set_err(c, RGBID_E_ARG, "NULL argument");
    if (t->device != c->device) return set_err(c, RGBID_E_ARG, "tracker on another device");
    if (pitch_elems < (size_t)t->cam.width) return set_err(c, RGBID_E_ARG, "pitch < width");
    HIPCHK(c, hipSetDevice(c->device));
    const rgbid_tracker_params& P = t->p;
    std::memset(out, 0, sizeof(*out));
    rgbid_status st;
    // a pyramid slot that is neither the reference frame nor the keyframe's
    int s = 0;
    while (s == t->rf || s == t->kfs) ++s;
    if (!t->slot[s]) {
        if ((st = rgbid_pyramid(c, &t->cam, t->levels, t->storage, I_dev, W_dev, pitch_elems,
                                &t->slot[s])) != RGBID_OK)
            return st;
    } else if ((st = rgbid_pyramid_update(c, t->slot[s], I_dev, W_dev, pitch_elems)) != RGBID_OK) {
        return st;
    }
    const long long k = t->k + 1;
    out->frame = k;
    const rgbid_pose I = pose_identity();
    if (k == 0) {
        if (t->kf) {
            if ((st = rgbid_keyframe_reset(c, t->kf, W_dev, pitch_elems)) != RGBID_OK) return st;
        } else if ((st = rgbid_keyframe_init(c, &t->cam, W_dev, pitch_elems, &t->kf)) != RGBID_OK) {
            return st;
        }
        t->rf = t->kfs = s;
        t->T_w_rf = t->T_w_kf = t->T_rf_prev = t->T_prev2_prev = I;
        std::memset(t->S_rf_prev, 0, sizeof(t->S_rf_prev));
        out->T_w_k = out->T_rf_k = out->T_prev_k = I;
        out->covis_rf = out->covis_kf = 1.0;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        t->k = k;
        return RGBID_OK;
    }
    // constant-velocity guess (sec. 7.1) and the alignment to the reference
    const rgbid_pose init = pose_mul(t->T_rf_prev, t->T_prev2_prev);
    rgbid_pose T_rf_k;
    const rgbid_pyr* const A1[1] = {t->slot[t->rf]};
    const rgbid_pyr* const B1[1] = {t->slot[s]};
    if ((st = rgbid_align_batch(c, 1, A1, B1, &init, &P.align, &T_rf_k, &out->stats)) != RGBID_OK)
        return st;
    const double tol = std::max(P.tol_sigmas * out->stats.sigma_W, 1e-12);
    double S_rf_k[36] = {};
    if (P.covariance) {
        double Sxi[36];
        st = rgbid_covariance(c, t->slot[t->rf], t->slot[s], &T_rf_k, &P.align, nullptr, Sxi, nullptr);
        if (st == RGBID_OK) {
            xi_cov_to_left(T_rf_k, Sxi, S_rf_k);
            relative_covariance(t->T_rf_prev, t->S_rf_prev, T_rf_k, S_rf_k, out->Sigma_odo);
            std::memcpy(out->Sigma_rf_k, S_rf_k, sizeof(S_rf_k));
        } else if (st != RGBID_E_DEGENERATE) {
            return st;
        }
        out->cov_status = st;
    }
    const rgbid_pose T_prev_k = pose_mul(pose_inv(t->T_rf_prev), T_rf_k);
    const rgbid_pose T_w_k = pose_mul(t->T_w_rf, T_rf_k);
    // keyframe (sec. 7.2): switch, or fuse this frame and one buffered frame
    const rgbid_pose T_kf_k = pose_mul(pose_inv(t->T_w_kf), T_w_k);
    if ((st = rgbid_covisibility(c, t->slot[t->kfs], t->slot[s], P.covis_level, &T_kf_k, tol,
                                 &out->covis_kf, nullptr)) != RGBID_OK)
        return st;
    if (out->covis_kf < P.kf_threshold) {
        out->kf_switched = 1;
        t->kfs = s;
        t->T_w_kf = T_w_k;
        if ((st = rgbid_keyframe_reset(c, t->kf, W_dev, pitch_elems)) != RGBID_OK) return st;
        for (const auto& r : t->pending) t->free_maps.push_back(r.map);
        t->pending.assign(t->recorded.rbegin(), t->recorded.rend());
        t->recorded.clear();
    } else {
        if ((st = rgbid_fuse(c, t->kf, W_dev, pitch_elems, &T_kf_k, tol, &out->n_fused)) != RGBID_OK)
            return st;
        if (!t->pending.empty()) {
            const auto r = t->pending.front();
            t->pending.erase(t->pending.begin());
            const rgbid_pose T_kf_j = pose_mul(pose_inv(t->T_w_kf), r.T_w);
            const size_t np = (size_t)t->cam.width * t->cam.height;
            if ((st = rgbid_fuse(c, t->kf, t->maps + (size_t)r.map * np, (size_t)t->cam.width,
                                 &T_kf_j, r.tol, &out->n_fused_buffer)) != RGBID_OK)
                return st;
            t->free_maps.push_back(r.map);
        }
    }
    if (P.buffer > 0) {
        if ((int)t->recorded.size() == P.buffer) {
            t->free_maps.push_back(t->recorded.front().map);
            t->recorded.erase(t->recorded.begin());
        }
        const int m = take_map(t);
        const size_t np = (size_t)t->cam.width * t->cam.height;
        HIPCHK(c, launch_copy_valid(c->stream, W_dev, (long long)pitch_elems, t->cam.width,
                                    t->cam.height, t->maps + (size_t)m * np));
        t->recorded.push_back(rgbid_tracker::Rec{m, T_w_k, tol});
    }
    // reference frame (sec. 7.1 with the covisibility criterion of sec. 7.2)
    if ((st = rgbid_covisibility(c, t->slot[t->rf], t->slot[s], P.covis_level, &T_rf_k, tol,
                                 &out->covis_rf, nullptr)) != RGBID_OK)
        return st;
    out->T_w_k = T_w_k;
    out->T_rf_k = T_rf_k;
    out->T_prev_k = T_prev_k;
    t->T_prev2_prev = T_prev_k;
    if (out->covis_rf < P.rf_threshold) {
        out->rf_switched = 1;
        t->rf = s;
        t->T_w_rf = T_w_k;
        t->T_rf_prev = I;
        std::memset(t->S_rf_prev, 0, sizeof(t->S_rf_prev));
    } else {
        t->T_rf_prev = T_rf_k;
        std::memcpy(t->S_rf_prev, S_rf_k, sizeof(S_rf_k));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    t->k = k;
    return RGBID_OK;
}

}  // extern "C"
