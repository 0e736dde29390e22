// Host side of the C ABI: argument validation, work decomposition, per-device
// workspace and error reporting.  Every check here runs before anything is
// enqueued, so an invalid call leaves the device untouched.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "sb_internal.hpp"

namespace sb {

static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// Per-device scratch: the sticky flag word, the loss partials, the ordering
// buffers and the adjoint's two-phase chain-rule buffer (grown on demand, kept
// until the process ends).
struct DeviceState {
    unsigned* flags = nullptr;
    double* partials = nullptr;
    void* order_buf = nullptr;
    size_t order_bytes = 0;
    float* d5 = nullptr;
    size_t d5_bytes = 0;
};

static std::mutex g_mu;
static std::vector<DeviceState> g_dev;

static int device_state(DeviceState** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SB_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    DeviceState& ds = g_dev[dev];
    if (!ds.flags) {
        e = hipMalloc(&ds.flags, 256);
        if (e != hipSuccess) return fail(SB_ERR_HIP, "hipMalloc(flags): %s", hipGetErrorString(e));
        e = hipMemset(ds.flags, 0, 256);
        if (e != hipSuccess) return fail(SB_ERR_HIP, "hipMemset(flags): %s", hipGetErrorString(e));
        e = hipMalloc(&ds.partials, sizeof(double) * loss_blocks());
        if (e != hipSuccess) return fail(SB_ERR_HIP, "hipMalloc(partials): %s", hipGetErrorString(e));
    }
    *out = &ds;
    return SB_OK;
}

// ---- validation ----
struct Shape {
    int64_t B = 0, F = 0, S = 0, T = 0;
    int M = 0;
};

// kernel, basis, position mode and term count (the ball model); M = coefficients per attribute
static int validate_model(const sb_config* cfg, int64_t& M) {
    if (!cfg) return fail(SB_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->kernel != SB_KERNEL_UNIFORM && cfg->kernel != SB_KERNEL_GAUSS)
        return fail(SB_ERR_INVALID_ARG, "unknown kernel %d", cfg->kernel);
    if (cfg->basis < SB_BASIS_STATIC || cfg->basis > SB_BASIS_GAUSS)
        return fail(SB_ERR_INVALID_ARG, "unknown basis %d", cfg->basis);
    if (cfg->pos_mode != SB_POS_ADD && cfg->pos_mode != SB_POS_MUL)
        return fail(SB_ERR_INVALID_ARG, "unknown pos_mode %d", cfg->pos_mode);
    if (cfg->basis == SB_BASIS_FOURIER && (cfg->n_terms < 1 || cfg->n_terms > SB_MAX_FOURIER))
        return fail(SB_ERR_SHAPE, "n_terms %d outside 1..%d for the Fourier basis", cfg->n_terms, SB_MAX_FOURIER);
    if (cfg->basis == SB_BASIS_GAUSS && (cfg->n_terms < 1 || cfg->n_terms > SB_MAX_GAUSS_BASES))
        return fail(SB_ERR_SHAPE, "n_terms %d outside 1..%d for the Gaussian basis", cfg->n_terms,
                    SB_MAX_GAUSS_BASES);
    M = cfg->basis == SB_BASIS_FOURIER ? 2 * cfg->n_terms
      : cfg->basis == SB_BASIS_GAUSS   ? 3 * cfg->n_terms : 0;
    return SB_OK;
}

static int validate_config(const sb_config* cfg, Shape& sh) {
    int64_t M = 0;
    const int st = validate_model(cfg, M);
    if (st) return st;
    if (cfg->n_sensors < 1) return fail(SB_ERR_SHAPE, "n_sensors must be >= 1 (got %d)", cfg->n_sensors);
    if (cfg->n_samples < 1 || cfg->n_samples > (1 << 28))
        return fail(SB_ERR_SHAPE, "n_samples must be in 1..2^28 (got %d)", cfg->n_samples);
    if (!isfinite(cfg->c) || !isfinite(cfg->fs) || !isfinite(cfg->t0))
        return fail(SB_ERR_NONFINITE, "c, fs and t0 must be finite");
    if (!(cfg->c > 0.0) || !(cfg->fs > 0.0)) return fail(SB_ERR_INVALID_ARG, "c and fs must be > 0");
    sh.S = cfg->n_sensors;
    sh.T = cfg->n_samples;
    sh.M = M;
    return SB_OK;
}

static int validate_batch(const sb_batch* batch, Shape& sh) {
    if (!batch) return fail(SB_ERR_INVALID_ARG, "batch is NULL");
    if (batch->n_scenes < 1 || batch->n_scenes > SB_MAX_SCENES)
        return fail(SB_ERR_SHAPE, "n_scenes %d outside 1..%d", batch->n_scenes, SB_MAX_SCENES);
    if (batch->reserved != 0) return fail(SB_ERR_INVALID_ARG, "batch.reserved must be 0");
    if (!batch->ball_offset || !batch->frame_offset)
        return fail(SB_ERR_INVALID_ARG, "ball_offset / frame_offset is NULL");
    if (batch->ball_offset[0] != 0 || batch->frame_offset[0] != 0)
        return fail(SB_ERR_SHAPE, "offsets must start at 0");
    for (int i = 0; i < batch->n_scenes; ++i) {
        if (batch->ball_offset[i + 1] < batch->ball_offset[i] ||
            batch->frame_offset[i + 1] < batch->frame_offset[i])
            return fail(SB_ERR_SHAPE, "offsets of scene %d decrease", i);
        if (batch->ball_offset[i + 1] - batch->ball_offset[i] > (int64_t)INT32_MAX - 4096)
            return fail(SB_ERR_SHAPE, "scene %d has too many balls", i);
    }
    sh.B = batch->ball_offset[batch->n_scenes];
    sh.F = batch->frame_offset[batch->n_scenes];
    if (sh.F > (int64_t)INT32_MAX) return fail(SB_ERR_SHAPE, "too many frames");
    if (sh.T > 0 && sh.S > 0 && sh.F > (int64_t)(INT64_MAX / 8) / (sh.S * sh.T))
        return fail(SB_ERR_SHAPE, "signal size overflows");
    return SB_OK;
}

// Tuning knobs (slingbag_tune): forward column length, adjoint occupancy target
// and adjoint item count.  They change speed, not results (beyond the order of
// floating-point atomics).
struct Tuning {
    int fwd_ucap = SB_FWD_COLUMN_SHARED_SHORT;   // uniform sphere: 64 or 128 samples per wave's LDS
                                                 // column, or one of the shared columns
    int fwd_gauss_ucap = SB_FWD_GAUSS_LANE;   // Gaussian ball: 128 (4-wave blocks), 256 (2-wave
                                              // blocks) or a lane per sample
    int adj_occ = 4;           // 2, 3 or 4 blocks (waves per SIMD) per CU for the adjoint
    int adj_items = 8192;      // adjoint items the sensor split aims for
};
static Tuning g_tune;   // guarded by g_mu

static Tuning tuning() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tune;
}

static void set_tuning(const Tuning& t) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune = t;
}

static TileCfg pick_forward_tiles(int kernel, const Tuning& tu) {
    TileCfg tc;
    const bool long_col = kernel != SB_KERNEL_UNIFORM && tu.fwd_gauss_ucap == 256;
    tc.nw = long_col ? 2 : 4;
    tc.g = 64 * tc.nw;
    tc.ucap = kernel == SB_KERNEL_UNIFORM ? tu.fwd_ucap : tu.fwd_gauss_ucap;
    tc.shared = kernel == SB_KERNEL_UNIFORM
                    ? (tu.fwd_ucap == SB_FWD_COLUMN_SHARED || tu.fwd_ucap == SB_FWD_COLUMN_SHARED_SHORT)
                    : tu.fwd_gauss_ucap == SB_FWD_GAUSS_LANE;
    if (tc.shared) {
        tc.nw = 1;     // 64-sensor blocks: the block's four waves share each of them
        tc.g = 256;
        tc.ucap = kernel != SB_KERNEL_UNIFORM ? 512 : (tu.fwd_ucap == SB_FWD_COLUMN_SHARED_SHORT ? 92 : 132);
    }
    return tc;
}

static TileCfg pick_adjoint_tiles(int kernel, const Tuning& tu) {
    TileCfg tc;
    tc.nw = tu.adj_occ;
    tc.g = 256;
    tc.ucap = kernel == SB_KERNEL_UNIFORM ? 128 : 384;
    return tc;
}

static void fill_common(OpParams& p, const sb_config* cfg, const sb_batch* batch, const Shape& sh) {
    memset(&p, 0, sizeof p);
    p.B = sh.B;
    p.S = (int32_t)sh.S;
    p.T = (int32_t)sh.T;
    p.basis = cfg->basis;
    p.pos_mode = cfg->pos_mode;
    p.n_terms = cfg->basis == SB_BASIS_STATIC ? 0 : cfg->n_terms;
    p.M = sh.M;
    p.inv_delta = cfg->fs / cfg->c;
    p.two_inv_delta = 2.0 * p.inv_delta;
    p.t0fs = cfg->t0 * cfg->fs;
    p.delta = (float)(cfg->c / cfg->fs);
    p.n_scenes = batch->n_scenes;
    for (int i = 0; i < batch->n_scenes; ++i) {
        Scene& s = p.scenes[i];
        s.ball0 = batch->ball_offset[i];
        s.n_balls = (int32_t)(batch->ball_offset[i + 1] - batch->ball_offset[i]);
        s.frame0 = (int32_t)batch->frame_offset[i];
        s.n_frames = (int32_t)(batch->frame_offset[i + 1] - batch->frame_offset[i]);
    }
}

// Forward items: (scene, frame, chunk of tc.g balls, block of 64*nw sensors).
static void fill_forward(OpParams& p, const sb_config* cfg, const sb_batch* batch, const Shape& sh,
                         const TileCfg& tc) {
    fill_common(p, cfg, batch, sh);
    p.n_sblocks = (int32_t)((sh.S + 64 * tc.nw - 1) / (64 * tc.nw));
    // Large launches stage each (frame, chunk) once for several sensor blocks, keeping
    // at least kFwdItemsPerSlot items per resident block (about 512 on the chip).
    constexpr int64_t kFwdItemsPerSlot = 16, kFwdSlots = 512;
    int64_t chunk_frames = 0;
    for (int i = 0; i < batch->n_scenes; ++i) {
        const Scene& s = p.scenes[i];
        chunk_frames += (int64_t)s.n_frames * ((s.n_balls + tc.g - 1) / tc.g);
    }
    int64_t per = chunk_frames * p.n_sblocks / (kFwdItemsPerSlot * kFwdSlots);
    per = per < 1 ? 1 : (per > p.n_sblocks ? p.n_sblocks : per);
    p.sb_per_item = (int32_t)per;
    p.n_sitems = (p.n_sblocks + p.sb_per_item - 1) / p.sb_per_item;
    int64_t items = 0;
    for (int i = 0; i < batch->n_scenes; ++i) {
        Scene& s = p.scenes[i];
        s.n_groups = (s.n_balls + tc.g - 1) / tc.g;
        s.item0 = items;
        items += (int64_t)s.n_frames * s.n_groups * p.n_sitems;
    }
    p.n_items = items;
}

constexpr int64_t kAdjMaxSplitHost = 256;   // sensors per adjoint item at most (LDS staging)

// Adjoint items: (scene, chunk of 256 balls, split of the sensors); frames inside.
// The sensors are split so that there are enough items to fill the chip.
static void fill_adjoint(OpParams& p, const sb_config* cfg, const sb_batch* batch, const Shape& sh,
                         const Tuning& tu) {
    fill_common(p, cfg, batch, sh);
    int64_t chunks = 0;
    for (int i = 0; i < batch->n_scenes; ++i) {
        Scene& s = p.scenes[i];
        s.n_groups = (s.n_balls + 255) / 256;
        if (s.n_frames > 0) chunks += s.n_groups;
    }
    int64_t d5 = 0;          // two-phase chain rule: [frame][5][ball] per scene, concatenated
    for (int i = 0; i < batch->n_scenes; ++i) {
        Scene& s = p.scenes[i];
        s.d5_0 = d5;
        d5 += (int64_t)s.n_frames * 5 * s.n_balls;
    }
    const int64_t target = tu.adj_items;
    int64_t n_split = chunks > 0 ? (target + chunks - 1) / chunks : 1;
    const int64_t max_split = sh.S >= 8 ? sh.S / 8 : 1;
    if (n_split > max_split) n_split = max_split;
    const int64_t min_split = (sh.S + kAdjMaxSplitHost - 1) / kAdjMaxSplitHost;   // kernel's LDS bound
    if (n_split < min_split) n_split = min_split;
    if (n_split < 1) n_split = 1;
    p.s_per_split = (int32_t)((sh.S + n_split - 1) / n_split);
    p.n_sblocks = (int32_t)((sh.S + p.s_per_split - 1) / p.s_per_split);
    int64_t items = 0;
    for (int i = 0; i < batch->n_scenes; ++i) {
        Scene& s = p.scenes[i];
        s.item0 = items;
        if (s.n_frames > 0) items += (int64_t)s.n_groups * p.n_sblocks;
    }
    p.n_items = items;
}

static int hip_fail(hipError_t e, const char* what) {
    return fail(SB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Floats of the adjoint's two-phase chain-rule buffer for this problem (0: the
// kernels apply the chain rule themselves).
static int64_t d5_floats(const sb_config* cfg, const sb_batch* batch, const Shape& sh) {
    OpParams q;
    memset(&q, 0, sizeof q);
    q.basis = cfg->basis;
    q.M = sh.M;
    if (!adjoint_two_phase(q)) return 0;
    int64_t n = 0;
    for (int i = 0; i < batch->n_scenes; ++i)
        n += (batch->frame_offset[i + 1] - batch->frame_offset[i]) * 5 *
             (batch->ball_offset[i + 1] - batch->ball_offset[i]);
    return n;
}

// Grows the per-device chain-rule buffer to `floats` entries.  Growing waits for
// `stream` (the old buffer may still be read) and allocates, so it cannot happen
// under graph capture (a plan allocates a buffer of its own before capturing).
static int reserve_d5(DeviceState* ds, int64_t floats, hipStream_t s) {
    const size_t need = (size_t)floats * sizeof(float);
    std::lock_guard<std::mutex> lk(g_mu);
    if (ds->d5_bytes >= need) return SB_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(SB_ERR_INVALID_ARG, "the adjoint's chain-rule buffer (%zu bytes) cannot grow under graph "
                    "capture: call slingbag_adjoint once on this problem before capturing, or use a plan", need);
    hipError_t e = hipSuccess;
    if (ds->d5) {
        e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipFree(ds->d5);
        if (e != hipSuccess) return hip_fail(e, "release chain-rule buffer");
        ds->d5 = nullptr;
        ds->d5_bytes = 0;
    }
    e = hipMalloc(&ds->d5, need);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(chain-rule buffer)");
    ds->d5_bytes = need;
    return SB_OK;
}

// Opt-in event timing of the main kernel launches (slingbag_timing).  Each
// launch of kind k is bracketed by two events recorded on its own stream; the
// pool holds kTimingSlots pairs per kind and recording stops when it is full.
enum { kTimeForward = 0, kTimeAdjoint = 1, kTimeLoss = 2, kTimeAdam = 3, kTimeKinds = 4 };
constexpr int kTimingSlots = 8192;
struct Timing {
    bool enabled = false;
    int device = -1;
    std::vector<hipEvent_t> ev[kTimeKinds];   // 2 per slot
    int used[kTimeKinds] = {0, 0, 0, 0};
};
static Timing g_timing;

// Set by slingbag_plan_create while it captures: the plan's own chain-rule buffer, which
// the captured adjoint uses instead of the per-device one (the per-device buffer may be
// replaced by a later, larger call; a graph must keep the address it was captured with).
static thread_local float* g_capture_d5 = nullptr;

// A plan captured while timing is on times its launches too.  During the capture
// each mark is an empty marker kernel; afterwards an event record node (with a
// placeholder event) is added after every marker, ahead of the marker's successor,
// and every replay points those nodes at a fresh pair of events from the pool, so
// the launches of a replayed graph are timed like direct ones.
__global__ void plan_mark_kernel() {}

struct CaptureTiming {
    hipEvent_t ev[kTimeKinds][2] = {};         // placeholders
    hipGraphNode_t node[kTimeKinds][2] = {};   // the event record nodes that record them
    std::vector<int> marks;                    // kind * 2 + which, in capture order
    bool failed = false;
};
static thread_local CaptureTiming* g_capture = nullptr;   // set by slingbag_plan_create

static void time_mark(int kind, int which, hipStream_t st) {
    if (!g_timing.enabled) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return;
    if (cs != hipStreamCaptureStatusNone) {
        if (g_capture && g_capture->ev[kind][which]) {
            hipLaunchKernelGGL(plan_mark_kernel, dim3(1), dim3(64), 0, st);
            if (hipGetLastError() == hipSuccess)
                g_capture->marks.push_back(kind * 2 + which);
            else
                g_capture->failed = true;
        }
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int slot = g_timing.used[kind];
    if (slot >= kTimingSlots) return;
    (void)hipEventRecord(g_timing.ev[kind][2 * slot + which], st);
    if (which == 1) g_timing.used[kind] = slot + 1;
}

// Times `fn` (one launch sequence on stream s) `reps` times after one warm-up run.
template <typename Fn>
static int time_ms(hipStream_t s, int reps, Fn fn, float* ms_out) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    int st = fn();
    if (st == SB_OK) {
        (void)hipEventRecord(a, s);
        for (int i = 0; i < reps && st == SB_OK; ++i) st = fn();
        (void)hipEventRecord(b, s);
        e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(ms_out, a, b);
        if (e != hipSuccess && st == SB_OK) st = hip_fail(e, "autotune timing");
        *ms_out /= (float)reps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

}  // namespace sb

using namespace sb;

extern "C" {

int slingbag_version(void) { return (1 << 16) | 1; }

const char* slingbag_last_error(void) { return g_last_error.c_str(); }

int slingbag_forward(const sb_config* cfg, const sb_batch* batch, const float* balls,
                     const float* deform, const float* frame_t, const float* sensors,
                     float* signals, void* stream) {
    Shape sh;
    int st = validate_config(cfg, sh);
    if (st) return st;
    if ((st = validate_batch(batch, sh))) return st;
    if (!frame_t && sh.F > 0) return fail(SB_ERR_INVALID_ARG, "frame_t is NULL");
    if (!sensors) return fail(SB_ERR_INVALID_ARG, "sensors is NULL");
    if (!signals && sh.F > 0) return fail(SB_ERR_INVALID_ARG, "signals is NULL");
    if (!balls && sh.B > 0) return fail(SB_ERR_INVALID_ARG, "balls is NULL");
    if (cfg->basis != SB_BASIS_STATIC && !deform && sh.B > 0)
        return fail(SB_ERR_INVALID_ARG, "deform is NULL for a deformed basis");
    DeviceState* ds;
    if ((st = device_state(&ds))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_fill(signals, sh.F * sh.S * sh.T, 0.f, s);
    if (e != hipSuccess) return hip_fail(e, "fill(signals)");
    if (sh.B == 0 || sh.F == 0) return SB_OK;
    const TileCfg tc = pick_forward_tiles(cfg->kernel, tuning());
    OpParams p;
    fill_forward(p, cfg, batch, sh, tc);
    p.balls = balls;
    p.deform = deform;
    p.frame_t = frame_t;
    p.sensors = sensors;
    p.signals = signals;
    p.flags = ds->flags;
    time_mark(kTimeForward, 0, s);
    e = launch_forward(p, tc, cfg->kernel, s);
    time_mark(kTimeForward, 1, s);
    if (e != hipSuccess) return hip_fail(e, "forward kernel");
    return SB_OK;
}

int slingbag_loss(const sb_config* cfg, const sb_batch* batch, const float* signals,
                  const float* measured, float* residual, double* loss, void* stream) {
    Shape sh;
    int st = validate_config(cfg, sh);
    if (st) return st;
    if ((st = validate_batch(batch, sh))) return st;
    if (!loss) return fail(SB_ERR_INVALID_ARG, "loss is NULL");
    const int64_t n = sh.F * sh.S * sh.T;
    if (n > 0 && (!signals || !measured || !residual))
        return fail(SB_ERR_INVALID_ARG, "signals / measured / residual is NULL");
    DeviceState* ds;
    if ((st = device_state(&ds))) return st;
    time_mark(kTimeLoss, 0, (hipStream_t)stream);
    hipError_t e = launch_loss(signals, measured, residual, n, ds->partials, loss_blocks(), loss,
                               (hipStream_t)stream);
    time_mark(kTimeLoss, 1, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "loss kernels");
    return SB_OK;
}

int slingbag_loss_noalloc(const sb_config* cfg, const sb_batch* batch, const float* signals,
                          const float* measured, float* residual, double* loss, void* stream) {
    Shape sh;
    int st = validate_config(cfg, sh);
    if (st) return st;
    if ((st = validate_batch(batch, sh))) return st;
    if (!loss) return fail(SB_ERR_INVALID_ARG, "loss is NULL");
    const int64_t n = sh.F * sh.S * sh.T;
    if (n > 0 && (!signals || !measured || !residual))
        return fail(SB_ERR_INVALID_ARG, "signals / measured / residual is NULL");
    // the reduction always runs loss_blocks() blocks, one partial each, whatever n
    if (loss_blocks() > noalloc_partials_capacity())
        return fail(SB_ERR_SHAPE, "loss needs %d partials, the fixed scratch holds %d", loss_blocks(),
                    noalloc_partials_capacity());
    double* partials = nullptr;
    hipError_t e = noalloc_partials(&partials);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(loss scratch)");
    e = launch_loss(signals, measured, residual, n, partials, loss_blocks(), loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "loss kernels");
    return SB_OK;
}

int slingbag_adjoint(const sb_config* cfg, const sb_batch* batch, const float* balls,
                     const float* deform, const float* frame_t, const float* sensors,
                     const float* residual, float* grad_balls, float* grad_deform, void* stream) {
    Shape sh;
    int st = validate_config(cfg, sh);
    if (st) return st;
    if ((st = validate_batch(batch, sh))) return st;
    if (sh.B > 0 && (!balls || !grad_balls)) return fail(SB_ERR_INVALID_ARG, "balls / grad_balls is NULL");
    if (!sensors) return fail(SB_ERR_INVALID_ARG, "sensors is NULL");
    if (sh.F > 0 && (!frame_t || !residual)) return fail(SB_ERR_INVALID_ARG, "frame_t / residual is NULL");
    if (cfg->basis != SB_BASIS_STATIC && sh.B > 0 && (!deform || !grad_deform))
        return fail(SB_ERR_INVALID_ARG, "deform / grad_deform is NULL for a deformed basis");
    DeviceState* ds;
    if ((st = device_state(&ds))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_fill(grad_balls, 5 * sh.B, 0.f, s);
    if (e == hipSuccess && cfg->basis != SB_BASIS_STATIC)
        e = launch_fill(grad_deform, 5 * (int64_t)sh.M * sh.B, 0.f, s);
    if (e != hipSuccess) return hip_fail(e, "fill(grads)");
    if (sh.B == 0 || sh.F == 0) return SB_OK;
    const Tuning tu = tuning();
    const TileCfg tc = pick_adjoint_tiles(cfg->kernel, tu);
    OpParams p;
    fill_adjoint(p, cfg, batch, sh, tu);
    p.balls = balls;
    p.deform = deform;
    p.frame_t = frame_t;
    p.sensors = sensors;
    p.residual = residual;
    p.grad_balls = grad_balls;
    p.grad_deform = grad_deform;
    p.flags = ds->flags;
    const int64_t n5 = d5_floats(cfg, batch, sh);
    if (n5 > 0) {
        if (g_capture_d5) {
            p.d5 = g_capture_d5;
        } else {
            if ((st = reserve_d5(ds, n5, s))) return st;
            p.d5 = ds->d5;
        }
        e = launch_fill(p.d5, n5, 0.f, s);
        if (e != hipSuccess) return hip_fail(e, "fill(chain-rule buffer)");
    }
    time_mark(kTimeAdjoint, 0, s);
    e = launch_adjoint(p, tc, cfg->kernel, s);
    if (e == hipSuccess && p.d5) e = launch_chain_rule(p, s);
    time_mark(kTimeAdjoint, 1, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel");
    return SB_OK;
}

int slingbag_adam(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                  float beta1, float beta2, float eps, int32_t step, float lo, float hi, void* stream) {
    if (n < 0) return fail(SB_ERR_SHAPE, "n must be >= 0");
    if (n > 0 && (!param || !grad || !m || !v)) return fail(SB_ERR_INVALID_ARG, "NULL Adam buffer");
    if (step < 1) return fail(SB_ERR_INVALID_ARG, "step must be >= 1 (got %d)", step);
    if (!isfinite(lr) || !isfinite(eps) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return fail(SB_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    if (isnan(lo) || isnan(hi) || !(lo <= hi)) return fail(SB_ERR_INVALID_ARG, "Adam bounds need lo <= hi");
    time_mark(kTimeAdam, 0, (hipStream_t)stream);
    hipError_t e = launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step, lo, hi, (hipStream_t)stream);
    time_mark(kTimeAdam, 1, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adam kernel");
    return SB_OK;
}

static int validate_grid(const sb_grid* g) {
    if (!g) return fail(SB_ERR_INVALID_ARG, "grid is NULL");
    if (g->reserved != 0) return fail(SB_ERR_INVALID_ARG, "grid.reserved must be 0");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(SB_ERR_SHAPE, "grid dimensions must be >= 1 (got %d x %d x %d)", g->nx, g->ny, g->nz);
    if ((int64_t)g->nx * g->ny * g->nz > ((int64_t)1 << 31) - 1)
        return fail(SB_ERR_SHAPE, "grid has more than 2^31 - 1 voxels");
    if (!isfinite(g->x0) || !isfinite(g->y0) || !isfinite(g->z0) || !isfinite(g->h))
        return fail(SB_ERR_NONFINITE, "grid origin and pitch must be finite");
    if (!(g->h > 0.0)) return fail(SB_ERR_INVALID_ARG, "grid pitch must be > 0");
    return SB_OK;
}

int slingbag_voxelize(const sb_config* cfg, const sb_grid* grid, int64_t n_balls, const float* balls,
                      const float* deform, float t, float* volume, void* stream) {
    int64_t M = 0;
    int st = validate_model(cfg, M);
    if (st) return st;
    if ((st = validate_grid(grid))) return st;
    if (n_balls < 0 || n_balls > ((int64_t)1 << 31) - 1) return fail(SB_ERR_SHAPE, "n_balls outside 0..2^31-1");
    if (!isfinite(t)) return fail(SB_ERR_NONFINITE, "frame time must be finite");
    if (!volume) return fail(SB_ERR_INVALID_ARG, "volume is NULL");
    if (n_balls > 0 && !balls) return fail(SB_ERR_INVALID_ARG, "balls is NULL");
    if (n_balls > 0 && cfg->basis != SB_BASIS_STATIC && !deform)
        return fail(SB_ERR_INVALID_ARG, "deform is NULL for a deformed basis");
    DeviceState* ds;
    if ((st = device_state(&ds))) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nvox = (int64_t)grid->nx * grid->ny * grid->nz;
    hipError_t e = launch_fill(volume, nvox, 0.f, s);
    if (e != hipSuccess) return hip_fail(e, "fill(volume)");
    if (n_balls == 0) return SB_OK;
    OpParams p;
    memset(&p, 0, sizeof p);
    p.balls = balls;
    p.deform = deform;
    p.flags = ds->flags;
    p.B = n_balls;
    p.basis = cfg->basis;
    p.pos_mode = cfg->pos_mode;
    p.n_terms = cfg->basis == SB_BASIS_STATIC ? 0 : cfg->n_terms;
    p.M = (int32_t)M;
    p.inv_delta = 1.0;           // deform_ball then returns the size in metres
    p.two_inv_delta = 2.0;
    e = launch_voxelize(p, cfg->kernel, grid->nx, grid->ny, grid->nz, grid->x0, grid->y0, grid->z0, grid->h, t,
                        volume, s);
    if (e != hipSuccess) return hip_fail(e, "voxelize kernel");
    return SB_OK;
}

int slingbag_map(const sb_grid* grid, const float* volume, float* map_xy, float* map_yz, float* map_xz,
                 void* stream) {
    int st = validate_grid(grid);
    if (st) return st;
    if (!volume) return fail(SB_ERR_INVALID_ARG, "volume is NULL");
    hipError_t e = launch_map(volume, grid->nx, grid->ny, grid->nz, map_xy, map_yz, map_xz, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "map kernels");
    return SB_OK;
}

int slingbag_order(const sb_batch* batch, const float* balls, int32_t* perm, void* stream) {
    Shape sh;
    int st = validate_batch(batch, sh);
    if (st) return st;
    if (sh.B > (int64_t)INT32_MAX) return fail(SB_ERR_SHAPE, "too many balls to order (%lld)", (long long)sh.B);
    if (sh.B > 0 && (!balls || !perm)) return fail(SB_ERR_INVALID_ARG, "balls / perm is NULL");
    if (sh.B == 0) return SB_OK;
    DeviceState* ds;
    if ((st = device_state(&ds))) return st;
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)sh.B;
    const size_t keys_bytes = ((size_t)n * 8 + 255) & ~(size_t)255;
    const size_t idx_bytes = ((size_t)n * 4 + 255) & ~(size_t)255;
    const size_t need = 2 * keys_bytes + idx_bytes + radix_sort_scratch_bytes(n);
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ds->order_bytes < need) {
            if (ds->order_buf) {
                e = hipStreamSynchronize(s);
                if (e == hipSuccess) e = hipFree(ds->order_buf);
                if (e != hipSuccess) return hip_fail(e, "release ordering scratch");
                ds->order_buf = nullptr;
                ds->order_bytes = 0;
            }
            e = hipMalloc(&ds->order_buf, need);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(ordering scratch)");
            ds->order_bytes = need;
        }
    }
    // keys, their ping-pong copy, the indices' ping-pong copy (the indices start
    // in perm, where the sort leaves them), the radix tables
    char* base = (char*)ds->order_buf;
    unsigned long long* keys = (unsigned long long*)base;
    unsigned long long* keys_tmp = (unsigned long long*)(base + keys_bytes);
    int* idx_tmp = (int*)(base + 2 * keys_bytes);
    void* tables = base + 2 * keys_bytes + idx_bytes;
    e = launch_morton_keys(balls, sh.B, batch->ball_offset, batch->n_scenes, keys, (int*)perm, s);
    if (e == hipSuccess) e = radix_sort_pairs(keys, keys_tmp, (int*)perm, idx_tmp, tables, n, s);
    if (e != hipSuccess) return hip_fail(e, "ordering kernels");
    return SB_OK;
}

int slingbag_permute(const float* src, float* dst, int64_t rows, int64_t n, const int32_t* perm,
                     void* stream) {
    if (rows < 0 || n < 0) return fail(SB_ERR_SHAPE, "rows and n must be >= 0");
    if (rows * n == 0) return SB_OK;
    if (!src || !dst || !perm) return fail(SB_ERR_INVALID_ARG, "src / dst / perm is NULL");
    if (src == dst) return fail(SB_ERR_INVALID_ARG, "dst must not alias src");
    hipError_t e = launch_gather_rows(src, dst, rows, n, perm, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "permute kernel");
    return SB_OK;
}

int slingbag_tune(int key, int value) {
    std::lock_guard<std::mutex> lk(g_mu);
    switch (key) {
        case SB_TUNE_FWD_COLUMN:
            if (value != 64 && value != 128 && value != SB_FWD_COLUMN_SHARED && value != SB_FWD_COLUMN_SHARED_SHORT)
                return fail(SB_ERR_INVALID_ARG,
                            "forward column must be 64, 128, SB_FWD_COLUMN_SHARED or SB_FWD_COLUMN_SHARED_SHORT");
            g_tune.fwd_ucap = value;
            return SB_OK;
        case SB_TUNE_FWD_GAUSS_COLUMN:
            if (value != 128 && value != 256 && value != SB_FWD_GAUSS_LANE)
                return fail(SB_ERR_INVALID_ARG, "Gaussian forward column must be 128, 256 or SB_FWD_GAUSS_LANE");
            g_tune.fwd_gauss_ucap = value;
            return SB_OK;
        case SB_TUNE_ADJ_OCCUPANCY:
            if (value < 2 || value > 4) return fail(SB_ERR_INVALID_ARG, "adjoint occupancy must be 2..4");
            g_tune.adj_occ = value;
            return SB_OK;
        case SB_TUNE_ADJ_ITEMS:
            if (value < 1 || value > (1 << 22)) return fail(SB_ERR_INVALID_ARG, "adjoint items out of range");
            g_tune.adj_items = value;
            return SB_OK;
        default:
            return fail(SB_ERR_INVALID_ARG, "unknown tuning key %d", key);
    }
}

int slingbag_autotune(const sb_config* cfg, const sb_batch* batch, const float* balls,
                      const float* deform, const float* frame_t, const float* sensors, float* signals,
                      float* grad_balls, float* grad_deform, int32_t* choice, void* stream) {
    Shape sh;
    int st = validate_config(cfg, sh);
    if (st) return st;
    if ((st = validate_batch(batch, sh))) return st;
    if (!choice) return fail(SB_ERR_INVALID_ARG, "choice is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int reps = 2;
    const Tuning saved = tuning();
    Tuning cur = saved;          // the candidate being timed, published to the calls below
    float best = 3.0e38f, ms = 0.f;
    // the column knob of the problem's kernel: 64 / 128 / the two shared columns (uniform
    // sphere), 128 / 256 (Gaussian ball)
    const bool uni = cfg->kernel == SB_KERNEL_UNIFORM;
    int& col_knob = uni ? cur.fwd_ucap : cur.fwd_gauss_ucap;
    int best_col = col_knob;
    for (int col : {64, 128, 256, SB_FWD_COLUMN_SHARED, SB_FWD_COLUMN_SHARED_SHORT}) {
        if (uni ? col == 256 : (col == 64 || col == SB_FWD_COLUMN_SHARED_SHORT)) continue;   // Gaussian: 128, 256, lane
        col_knob = col;
        set_tuning(cur);
        st = time_ms(s, reps, [&] { return slingbag_forward(cfg, batch, balls, deform, frame_t, sensors, signals, stream); }, &ms);
        if (st) { set_tuning(saved); return st; }
        if (ms < best) { best = ms; best_col = col; }
    }
    col_knob = best_col;
    set_tuning(cur);
    // the forward output serves as a finite residual for timing the adjoint
    st = slingbag_forward(cfg, batch, balls, deform, frame_t, sensors, signals, stream);
    if (st) { set_tuning(saved); return st; }
    best = 3.0e38f;
    int best_occ = cur.adj_occ, best_items = cur.adj_items;
    for (int occ : {2, 3, 4}) {
        for (int items : {2048, 4096, 8192, 16384}) {
            cur.adj_occ = occ;
            cur.adj_items = items;
            set_tuning(cur);
            st = time_ms(s, reps, [&] { return slingbag_adjoint(cfg, batch, balls, deform, frame_t, sensors, signals,
                                                                 grad_balls, grad_deform, stream); }, &ms);
            if (st) { set_tuning(saved); return st; }
            if (ms < best) { best = ms; best_occ = occ; best_items = items; }
        }
    }
    cur.adj_occ = best_occ;
    cur.adj_items = best_items;
    set_tuning(cur);
    choice[0] = best_col;
    choice[1] = best_occ;
    choice[2] = best_items;
    return SB_OK;
}

int slingbag_tune_get(int key, int* value) {
    if (!value) return fail(SB_ERR_INVALID_ARG, "value is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    switch (key) {
        case SB_TUNE_FWD_COLUMN: *value = g_tune.fwd_ucap; return SB_OK;
        case SB_TUNE_FWD_GAUSS_COLUMN: *value = g_tune.fwd_gauss_ucap; return SB_OK;
        case SB_TUNE_ADJ_OCCUPANCY: *value = g_tune.adj_occ; return SB_OK;
        case SB_TUNE_ADJ_ITEMS: *value = g_tune.adj_items; return SB_OK;
        default: return fail(SB_ERR_INVALID_ARG, "unknown tuning key %d", key);
    }
}

int slingbag_timing(int enable) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    if (enable && g_timing.device != dev) {
        for (int k = 0; k < kTimeKinds; ++k) {
            for (hipEvent_t ev : g_timing.ev[k]) (void)hipEventDestroy(ev);
            g_timing.ev[k].assign(2 * kTimingSlots, nullptr);
            for (auto& ev : g_timing.ev[k]) {
                e = hipEventCreate(&ev);
                if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
            }
            g_timing.used[k] = 0;
        }
        g_timing.device = dev;
    }
    g_timing.enabled = enable != 0;
    return SB_OK;
}

int slingbag_timing_read(double* total_ms, int64_t* launches) {
    if (!total_ms || !launches) return fail(SB_ERR_INVALID_ARG, "NULL output");
    std::lock_guard<std::mutex> lk(g_mu);
    for (int k = 0; k < kTimeKinds; ++k) {
        double sum = 0.0;
        const int n = g_timing.device >= 0 ? g_timing.used[k] : 0;
        for (int i = 0; i < n; ++i) {
            hipError_t e = hipEventSynchronize(g_timing.ev[k][2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, g_timing.ev[k][2 * i], g_timing.ev[k][2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            sum += ms;
        }
        total_ms[k] = sum;
        launches[k] = n;
        if (g_timing.device >= 0) g_timing.used[k] = 0;
    }
    return SB_OK;
}

struct sb_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float* d5 = nullptr;         // the plan's own two-phase chain-rule buffer (or null)
    int device = -1;
    bool timed = false;          // captured with timing on: the nodes below exist
    bool on_pool = false;        // the nodes currently record pool events (not the placeholders)
    CaptureTiming tm;
};

// Destroys the placeholder events of a plan's timing record.
static void release_capture_timing(CaptureTiming& tm) {
    for (int k = 0; k < kTimeKinds; ++k)
        for (int w = 0; w < 2; ++w)
            if (tm.ev[k][w]) {
                (void)hipEventDestroy(tm.ev[k][w]);
                tm.ev[k][w] = nullptr;
            }
}

// After the capture: walk the captured chain (one stream: every node has at most one
// dependent), and after the i-th marker kernel insert an event record node for the
// i-th mark, on which the marker's successor then also depends.
static int add_timing_nodes(hipGraph_t graph, CaptureTiming& tm) {
    size_t n = 0;
    hipError_t e = hipGraphGetRootNodes(graph, nullptr, &n);
    if (e != hipSuccess) return hip_fail(e, "hipGraphGetRootNodes");
    if (n != 1) return fail(SB_ERR_HIP, "captured plan has %zu root nodes, expected one chain", n);
    hipGraphNode_t node = nullptr;
    if ((e = hipGraphGetRootNodes(graph, &node, &n)) != hipSuccess) return hip_fail(e, "hipGraphGetRootNodes");
    std::vector<hipGraphNode_t> chain;
    while (node) {
        chain.push_back(node);
        size_t nd = 0;
        if ((e = hipGraphNodeGetDependentNodes(node, nullptr, &nd)) != hipSuccess)
            return hip_fail(e, "hipGraphNodeGetDependentNodes");
        if (nd > 1) return fail(SB_ERR_HIP, "captured plan is not a chain");
        hipGraphNode_t next = nullptr;
        if (nd == 1 && (e = hipGraphNodeGetDependentNodes(node, &next, &nd)) != hipSuccess)
            return hip_fail(e, "hipGraphNodeGetDependentNodes");
        node = nd == 1 ? next : nullptr;
    }
    size_t mi = 0;
    for (size_t i = 0; i < chain.size(); ++i) {
        hipGraphNodeType ty;
        if ((e = hipGraphNodeGetType(chain[i], &ty)) != hipSuccess) return hip_fail(e, "hipGraphNodeGetType");
        if (ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        if ((e = hipGraphKernelNodeGetParams(chain[i], &kp)) != hipSuccess)
            return hip_fail(e, "hipGraphKernelNodeGetParams");
        if (kp.func != reinterpret_cast<void*>(plan_mark_kernel)) continue;
        if (mi >= tm.marks.size()) return fail(SB_ERR_HIP, "more timing markers in the plan than marks");
        const int k = tm.marks[mi] / 2, w = tm.marks[mi] % 2;
        ++mi;
        hipGraphNode_t ev = nullptr;
        if ((e = hipGraphAddEventRecordNode(&ev, graph, &chain[i], 1, tm.ev[k][w])) != hipSuccess)
            return hip_fail(e, "hipGraphAddEventRecordNode");
        if (i + 1 < chain.size() && (e = hipGraphAddDependencies(graph, &ev, &chain[i + 1], 1)) != hipSuccess)
            return hip_fail(e, "hipGraphAddDependencies");
        tm.node[k][w] = ev;
    }
    if (mi != tm.marks.size()) return fail(SB_ERR_HIP, "timing markers of the plan not found");
    return SB_OK;
}

// Before a replay: point the plan's timing nodes at the next pool slot of each kind
// (timing on) or back at the placeholders (timing off, or the pool full).
static int retarget_timing_nodes(sb_plan* plan) {
    if (!plan->timed) return SB_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    const bool on = g_timing.enabled && g_timing.device == plan->device && dev == plan->device;
    if (!on && !plan->on_pool) return SB_OK;
    bool any_pool = false;
    for (int k = 0; k < kTimeKinds; ++k) {
        if (!plan->tm.node[k][0] || !plan->tm.node[k][1]) continue;
        hipEvent_t a = plan->tm.ev[k][0], b = plan->tm.ev[k][1];
        const int slot = g_timing.used[k];
        const bool take = on && slot < kTimingSlots;
        if (take) {
            a = g_timing.ev[k][2 * slot];
            b = g_timing.ev[k][2 * slot + 1];
        }
        hipError_t e = hipGraphExecEventRecordNodeSetEvent(plan->exec, plan->tm.node[k][0], a);
        if (e == hipSuccess) e = hipGraphExecEventRecordNodeSetEvent(plan->exec, plan->tm.node[k][1], b);
        if (e != hipSuccess) return hip_fail(e, "hipGraphExecEventRecordNodeSetEvent");
        if (take) {
            g_timing.used[k] = slot + 1;
            any_pool = true;
        }
    }
    plan->on_pool = any_pool;
    return SB_OK;
}

int slingbag_plan_create(const sb_config* cfg, const sb_batch* batch, const float* balls,
                         const float* deform, const float* frame_t, const float* sensors,
                         const float* measured, float* signals, float* residual, double* loss,
                         float* grad_balls, float* grad_deform, void* stream, sb_plan** out) {
    if (!out) return fail(SB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Shape sh;
    int st = validate_config(cfg, sh);
    if (st) return st;
    if ((st = validate_batch(batch, sh))) return st;
    if (!stream) return fail(SB_ERR_INVALID_ARG, "graph capture needs a non-null stream");
    DeviceState* ds;
    if ((st = device_state(&ds))) return st;   // per-device buffers exist before capture
    hipStream_t s = (hipStream_t)stream;
    // the plan's own chain-rule buffer, allocated before the capture and kept by the plan
    const int64_t n5 = d5_floats(cfg, batch, sh);
    float* plan_d5 = nullptr;
    if (n5 > 0) {
        hipError_t ea = hipMalloc(&plan_d5, (size_t)n5 * sizeof(float));
        if (ea != hipSuccess) return hip_fail(ea, "hipMalloc(plan chain-rule buffer)");
    }
    // with timing on, the timed launches are captured between event record nodes
    CaptureTiming tm;
    const bool timed = g_timing.enabled;
    hipError_t e = hipSuccess;
    auto release = [&]() {
        release_capture_timing(tm);
        if (plan_d5) (void)hipFree(plan_d5);
    };
    if (timed) {
        for (int k : {(int)kTimeForward, (int)kTimeLoss, (int)kTimeAdjoint})
            for (int w = 0; w < 2 && e == hipSuccess; ++w) e = hipEventCreate(&tm.ev[k][w]);
        if (e != hipSuccess) {
            release();
            return hip_fail(e, "hipEventCreate(plan timing)");
        }
    }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "hipStreamBeginCapture");
    }
    g_capture = timed ? &tm : nullptr;
    g_capture_d5 = plan_d5;
    st = slingbag_forward(cfg, batch, balls, deform, frame_t, sensors, signals, stream);
    if (st == SB_OK) st = slingbag_loss(cfg, batch, signals, measured, residual, loss, stream);
    if (st == SB_OK)
        st = slingbag_adjoint(cfg, batch, balls, deform, frame_t, sensors, residual, grad_balls, grad_deform, stream);
    g_capture = nullptr;
    g_capture_d5 = nullptr;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st == SB_OK && tm.failed) st = fail(SB_ERR_HIP, "capturing the plan's timing markers failed");
    if (st == SB_OK && e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
    if (st == SB_OK && timed) st = add_timing_nodes(graph, tm);
    if (st != SB_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        release();
        return st;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        release();
        return hip_fail(e, "hipGraphInstantiate");
    }
    sb_plan* plan = new sb_plan;
    plan->graph = graph;
    plan->exec = exec;
    plan->d5 = plan_d5;
    plan->timed = timed;
    plan->tm = tm;
    (void)hipGetDevice(&plan->device);
    *out = plan;
    return SB_OK;
}

int slingbag_plan_run(sb_plan* plan, void* stream) {
    if (!plan || !plan->exec) return fail(SB_ERR_INVALID_ARG, "plan is NULL");
    int st = retarget_timing_nodes(plan);
    if (st) return st;
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SB_OK;
}

int slingbag_plan_destroy(sb_plan* plan) {
    if (!plan) return SB_OK;
    hipError_t e = hipSuccess;
    if (plan->exec) e = hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    release_capture_timing(plan->tm);
    if (plan->d5) {
        const hipError_t ef = hipFree(plan->d5);
        if (e == hipSuccess) e = ef;
    }
    delete plan;
    if (e != hipSuccess) return hip_fail(e, "hipGraphExecDestroy");
    return SB_OK;
}

int slingbag_check(void* stream, uint32_t* flags) {
    DeviceState* ds;
    int st = device_state(&ds);
    if (st) return st;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    unsigned f = 0;
    e = hipMemcpy(&f, ds->flags, sizeof f, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(flags)");
    e = hipMemset(ds->flags, 0, sizeof f);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(flags)");
    if (flags) *flags = f;
    if (f & (SB_FLAG_GEOMETRY | SB_FLAG_NONFINITE))
        return fail(SB_ERR_DEVICE_FLAG, "device flags 0x%x raised (geometry=%d, nonfinite=%d)", f,
                    (f & SB_FLAG_GEOMETRY) ? 1 : 0, (f & SB_FLAG_NONFINITE) ? 1 : 0);
    return SB_OK;
}

}  // extern "C"
