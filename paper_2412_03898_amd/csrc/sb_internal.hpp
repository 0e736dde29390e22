// Internal definitions shared by the HIP translation units of libslingbag.
// Not part of the public ABI (that is include/slingbag.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "slingbag.h"

namespace sb {

// One scene of a batch, with the first work item it owns.
struct Scene {
    int64_t ball0;      // first ball (global index)
    int64_t item0;      // first work item of this scene
    int32_t n_balls;
    int32_t frame0;     // first frame (global index)
    int32_t n_frames;
    int32_t n_groups;   // ceil(n_balls / G)
    int64_t d5_0;       // adjoint, two-phase chain rule: first entry of this scene in OpParams::d5
};

// Kernel argument block (passed by value).
struct OpParams {
    const float* balls;      // [5][B]
    const float* deform;     // [5][M][B] or null
    const float* frame_t;    // [F]
    const float* sensors;    // [3][S]
    float* signals;          // forward output [F][S][T]
    const float* residual;   // adjoint input  [F][S][T]
    float* grad_balls;       // [5][B]
    float* grad_deform;      // [5][M][B]
    unsigned* flags;         // device flag word
    // Adjoint with a two-phase chain rule (deformed bases with more coefficients than
    // the kernels keep in registers): per scene, [frame][5][ball] derivatives of the loss
    // with respect to the deformed attributes, summed over the sensor splits by the
    // adjoint kernels and turned into parameter gradients by chain_rule_kernel.  Null:
    // the adjoint kernels apply the chain rule themselves.
    float* d5;
    int64_t B;               // total balls (row stride of balls/deform)
    int64_t n_items;
    double inv_delta;        // fs / c   (samples per metre)
    double two_inv_delta;    // 2 fs / c
    double t0fs;             // t0 * fs  (sample index of the time origin)
    float delta;             // c / fs   (metres per sample)
    int32_t S, T;
    int32_t basis, pos_mode, n_terms, M;
    int32_t n_sblocks;       // forward: sensor blocks per (frame, chunk); adjoint: sensor splits
    int32_t sb_per_item;     // forward: sensor blocks per work item (the chunk is staged once for them)
    int32_t n_sitems;        // forward: items per (frame, chunk) = ceil(n_sblocks / sb_per_item)
    int32_t s_per_split;     // adjoint: sensors per split
    int32_t n_scenes;
    Scene scenes[SB_MAX_SCENES];
};

// A deformed ball at one frame as staged in LDS (40 bytes).  The size is kept in
// FP64 because the inside/outside decisions of the window boundaries (where the
// N-wave's derivative jumps) are taken in FP64, the oracle's precision.
struct BallF {
    double x, y, z;
    double rho;              // R_f / delta: radius (uniform) or std (Gaussian) in samples; < 0: skip
    float amp;               // P_f
    float rhof;              // (float)rho
};

// Gaussian-ball traces are cut where |r - c t| > kGaussCut * a (+ half a sample).
constexpr float kGaussCut = 6.0f;

// Work item -> (scene, local frame, group, first sensor block).  Items of one scene
// are ordered frame-major, then group, then sensor block.
struct Item {
    int scene, frame, group, sblock;
};

__device__ inline Item decode_item(const OpParams& p, int64_t item) {
    int i = 0;
    while (i + 1 < p.n_scenes && p.scenes[i + 1].item0 <= item) ++i;
    const Scene& sc = p.scenes[i];
    int64_t local = item - sc.item0;
    Item it;
    it.scene = i;
    it.sblock = (int)(local % p.n_sitems) * p.sb_per_item;     // first sensor block of the item
    int64_t q = local / p.n_sitems;
    it.group = (int)(q % sc.n_groups);
    it.frame = (int)(q / sc.n_groups);
    return it;
}

// Adjoint work item -> (scene, chunk of 256 balls, sensor split); items of one
// scene are ordered split-major so that consecutive items share residual rows.
struct ItemA {
    int scene, chunk, split;
};

__device__ inline ItemA decode_item_adj(const OpParams& p, int64_t item) {
    int i = 0;
    while (i + 1 < p.n_scenes && p.scenes[i + 1].item0 <= item) ++i;
    const Scene& sc = p.scenes[i];
    const int64_t local = item - sc.item0;
    ItemA it;
    it.scene = i;
    it.chunk = (int)(local % sc.n_groups);
    it.split = (int)(local / sc.n_groups);
    return it;
}

// Basis values of the frame: Fourier cos(2 pi k t), sin(2 pi k t) for k = 1..K (FP64).
__device__ inline void fourier_basis(float t, int K, double* fb) {
    for (int k = 1; k <= K; ++k) {
        double s, c;
        sincospi(2.0 * k * (double)t, &s, &c);
        fb[2 * (k - 1)] = c;
        fb[2 * (k - 1) + 1] = s;
    }
}

// Same values computed cooperatively: lane k < 2K of the calling wave writes entry
// k of an LDS array (the values are the same for every lane of a frame).  Kept out
// of line: the kernels call it once per frame, and inlined, the FP64 constants of
// sincospi are hoisted out of their loops into registers that the pair loops need.
__device__ __noinline__ void fourier_basis_lanes(float t, int K, double* fb, int lane) {
    if (lane < 2 * K) {
        const int k = lane / 2 + 1;
        double s, c;
        sincospi(2.0 * k * (double)t, &s, &c);
        fb[lane] = (lane & 1) ? s : c;
    }
}

// H of attribute a of ball b at time t (Eq. 2 or the Fourier series), in FP64 so
// that deformed positions and sizes carry no FP32 rounding into the arrival time.
// Eq. 2 sum of one attribute (coefficients d, stride B).  Out of line for the same
// reason as fourier_basis_lanes (the FP64 constants of exp).
__device__ __noinline__ double gauss_basis_H(const float* d, int64_t B, int n_terms, float t) {
    double h = 0.0;
    for (int n = 0; n < n_terms; ++n) {
        const double w = d[(int64_t)(3 * n) * B];
        const double th = d[(int64_t)(3 * n + 1) * B];
        const double sg = d[(int64_t)(3 * n + 2) * B];
        const double dt = (double)t - th;
        h = fma(w, exp(-dt * dt / (2.0 * sg * sg)), h);
    }
    return h;
}

__device__ inline double eval_H(const OpParams& p, int64_t b, int a, float t, const double* fb) {
    if (p.basis == SB_BASIS_STATIC) return 0.0;
    const float* d = p.deform + (int64_t)a * p.M * p.B + b;
    double h = 0.0;
    if (p.basis == SB_BASIS_FOURIER) {
        for (int m = 0; m < p.M; ++m) h = fma((double)d[(int64_t)m * p.B], fb[m], h);
    } else {
        h = gauss_basis_H(d, p.B, p.n_terms, t);
    }
    return h;
}

// Deformed attributes (Eq. 1) of ball b at time t; positions and size in FP64.
// Returns false (and marks the ball to skip) for invalid attributes.
__device__ inline bool deform_ball(const OpParams& p, int64_t b, float t, const double* fb,
                                   BallF& out) {
    const int64_t B = p.B;
    double base[5];
    for (int a = 0; a < 5; ++a) base[a] = p.balls[(int64_t)a * B + b];
    double pos[3];
    for (int a = 0; a < 3; ++a) {
        const double h = eval_H(p, b, a, t, fb);
        pos[a] = (p.pos_mode == SB_POS_ADD) ? base[a] + h : base[a] * (1.0 + h);
    }
    const double Rf = base[3] * (1.0 + eval_H(p, b, 3, t, fb));
    const double Pf = base[4] * (1.0 + eval_H(p, b, 4, t, fb));
    const bool ok = isfinite(pos[0]) && isfinite(pos[1]) && isfinite(pos[2]) && isfinite(Rf) &&
                    isfinite(Pf) && Rf > 0.0 && Pf >= 0.0;
    out.x = pos[0];
    out.y = pos[1];
    out.z = pos[2];
    out.rho = ok ? Rf * p.inv_delta : -1.0;
    out.rhof = (float)out.rho;
    out.amp = ok ? (float)Pf : 0.f;
    return ok;
}

// FP32 atomic add to global memory, as an instruction the compiler knows to be a
// global one.  An address rebuilt from lane reads is otherwise generic, which makes
// the atomic a FLAT operation; FLAT operations count on the same wait counter as
// LDS operations and may complete out of their order, so after one the compiler can
// only wait for every outstanding LDS operation at once.
__device__ inline void global_atomic_add(float* p, float v) {
    (void)__builtin_amdgcn_global_atomic_fadd_f32(
        (__attribute__((address_space(1))) float*)(p), v);
}

__device__ inline void raise_flag(unsigned* flags, unsigned bit) {
    atomicOr(flags, bit);
}


// Canonical grid for ball ordering and grouping: positions in [-1 m, 1 m) are
// quantised to 2^-18 m (3.8 um), 19 bits per axis.  Balls sorted by the Morton
// key of this grid (slingbag_order) make every grid cell at every level k (side
// 2^(k-18) m) a contiguous run of balls.
constexpr double kGridOrigin = -1.0;
constexpr double kGridQuantum = 1.0 / 262144.0;   // 2^-18 m
constexpr int kGridBits = 19;

__host__ __device__ inline uint32_t grid_coord(double x) {
    double q = floor((x - kGridOrigin) / kGridQuantum);
    q = q < 0.0 ? 0.0 : (q > (double)((1u << kGridBits) - 1) ? (double)((1u << kGridBits) - 1) : q);
    return (uint32_t)q;
}

// Ball-sensor distance: FP32 square root refined by one Newton step in FP64
// (relative error ~1e-15, well below the FP64 decisions' needs).  `ri` receives
// the FP32 reciprocal of the distance (relative error ~1e-7), which the
// amplitude factors 1/r use.
__device__ inline double dist64(double dx, double dy, double dz, float& ri) {
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const float rf = __builtin_amdgcn_sqrtf((float)r2);
    ri = __builtin_amdgcn_rcpf(rf);
    const double r0 = (double)rf;
    const float e = (float)fma(-r0, r0, r2);
    return fma((double)(e * ri), 0.5, r0);
}
__device__ inline double dist64(double dx, double dy, double dz) {
    float ri;
    return dist64(dx, dy, dz, ri);
}

// Window of one (ball, sensor) pair, as every kernel places it (inline, in its own
// pair loop).  tau = (r - c t0)/delta is the arrival sample; the window starts at
// sample k_lo = floor(tau - h + 1/2) (h = rho for the uniform sphere, kGaussCut*rho
// for the Gaussian ball) so that boundary 0, x_0 = tau - k_lo + 1/2, lies in
// [h, h + 1), and spans W = floor(2h) + 2 samples, so that boundary W lies below -h:
// every nonzero sample is inside.  For the uniform sphere the boundaries strictly
// inside (-rho, rho) are m = 1..m_hi, m_hi = ceil(x_0 + rho) - 1; that decision is
// taken in FP64.  A pair is used only when the sensor lies outside the uniform ball
// (r > 0 for the Gaussian ball) and |k_lo| stays far inside int32.

// Wave-wide reductions (all 64 lanes participate).
__device__ inline float wave_min(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}
__device__ inline float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}
__device__ inline int wave_max_i(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// Wave-wide reductions over DPP lane moves (no LDS round trip); every lane of
// the wave must be active.  Quad and row mirrors reduce each row of 16 lanes,
// then the four row results are read as scalars.
template <int CTRL>
__device__ inline int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <typename T, typename Op>
__device__ inline T wave_reduce_dpp(T v, Op op) {
    static_assert(sizeof(T) == 4, "32-bit values");
    auto mv = [](T x, auto ctrl) {
        const int r = dpp_move<decltype(ctrl)::value>(__builtin_bit_cast(int, x));
        return __builtin_bit_cast(T, r);
    };
    v = op(v, mv(v, std::integral_constant<int, 0xB1>{}));    // quad_perm [1,0,3,2]
    v = op(v, mv(v, std::integral_constant<int, 0x4E>{}));    // quad_perm [2,3,0,1]
    v = op(v, mv(v, std::integral_constant<int, 0x141>{}));   // row_half_mirror
    v = op(v, mv(v, std::integral_constant<int, 0x140>{}));   // row_mirror
    const T r0 = __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const T r1 = __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const T r2 = __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const T r3 = __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return op(op(r0, r1), op(r2, r3));
}
__device__ inline float wave_min_all(float v) {
    return wave_reduce_dpp(v, [](float a, float b) { return fminf(a, b); });
}
__device__ inline float wave_max_all(float v) {
    return wave_reduce_dpp(v, [](float a, float b) { return fmaxf(a, b); });
}
__device__ inline int wave_max_all(int v) {
    return wave_reduce_dpp(v, [](int a, int b) { return max(a, b); });
}

// Compiler-level ordering point for LDS traffic between lanes of one wave (the
// hardware executes a wave's LDS instructions in order).
__device__ inline void wave_lds_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Distance range [dmin, dmax] from point s to the axis-aligned box [lo, hi].
__device__ inline void box_distance_range(const float* lo, const float* hi, double sx, double sy,
                                          double sz, double& dmin, double& dmax) {
    const double s[3] = {sx, sy, sz};
    double n2 = 0.0, f2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double l = lo[a], h = hi[a];
        const double dn = s[a] < l ? l - s[a] : (s[a] > h ? s[a] - h : 0.0);
        const double df = fmax(fabs(s[a] - l), fabs(s[a] - h));
        n2 += dn * dn;
        f2 += df * df;
    }
    dmin = sqrt(n2);
    dmax = sqrt(f2);
}

// ---- host-side launchers (defined in the .hip files) ----
struct TileCfg {
    int nw;      // forward: sensors per item block / 64 (waves per block but for the shared column)
    int g;       // forward: balls per chunk
    int ucap;    // forward: tile length in samples; adjoint: residual row length
    int shared = 0;   // forward, uniform sphere: one column per sensor shared by the block's waves
};

hipError_t launch_forward(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st);
hipError_t launch_adjoint(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st);
bool adjoint_two_phase(const OpParams& p);     // does launch_adjoint need OpParams::d5?
hipError_t launch_chain_rule(const OpParams& p, hipStream_t st);
hipError_t launch_morton_keys(const float* balls, int64_t B, const int64_t* ball_offset_host,
                              int n_scenes, unsigned long long* keys, int* idx, hipStream_t st);
// Stable sort of (key, value) pairs by the low 62 key bits; the result lands back
// in keys / vals, keys_tmp and vals_tmp hold n elements each, scratch holds
// radix_sort_scratch_bytes(n).
size_t radix_sort_scratch_bytes(int n);
hipError_t radix_sort_pairs(unsigned long long* keys, unsigned long long* keys_tmp, int* vals, int* vals_tmp,
                            void* scratch, int n, hipStream_t st);
hipError_t launch_gather_rows(const float* src, float* dst, int64_t rows, int64_t B, const int* perm,
                              hipStream_t st);
hipError_t launch_fill(float* ptr, int64_t n, float v, hipStream_t st);
hipError_t launch_loss(const float* y, const float* d, float* r, int64_t n, double* partials,
                       int n_blocks, double* loss, hipStream_t st);
int loss_blocks();
hipError_t noalloc_partials(double** out);   // device address of the fixed partials array
int noalloc_partials_capacity();
hipError_t launch_voxelize(const OpParams& p, int kernel, int nx, int ny, int nz, double x0, double y0,
                           double z0, double h, float t, float* vol, hipStream_t st);
hipError_t launch_map(const float* vol, int nx, int ny, int nz, float* xy, float* yz, float* xz, hipStream_t st);
hipError_t launch_adam(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, float lo, float hi, hipStream_t st);

}  // namespace sb
