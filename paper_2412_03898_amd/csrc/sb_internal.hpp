// Internal definitions shared by the HIP translation units of libslingbag.
// Not part of the public ABI (that is include/slingbag.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
    int64_t B;               // total balls (row stride of balls/deform)
    int64_t n_items;
    double inv_delta;        // fs / c   (samples per metre)
    double t0fs;             // t0 * fs  (sample index of the time origin)
    float delta;             // c / fs   (metres per sample)
    int32_t S, T;
    int32_t basis, pos_mode, n_terms, M;
    int32_t n_sblocks;       // sensor blocks per (frame, group)
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

// Work item -> (scene, local frame, group, sensor block).  Items of one scene are
// ordered frame-major, then group, then sensor block.
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
    it.sblock = (int)(local % p.n_sblocks);
    int64_t q = local / p.n_sblocks;
    it.group = (int)(q % sc.n_groups);
    it.frame = (int)(q / sc.n_groups);
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

// H of attribute a of ball b at time t (Eq. 2 or the Fourier series), in FP64 so
// that deformed positions and sizes carry no FP32 rounding into the arrival time.
__device__ inline double eval_H(const OpParams& p, int64_t b, int a, float t, const double* fb) {
    if (p.basis == SB_BASIS_STATIC) return 0.0;
    const float* d = p.deform + (int64_t)a * p.M * p.B + b;
    double h = 0.0;
    if (p.basis == SB_BASIS_FOURIER) {
        for (int m = 0; m < p.M; ++m) h = fma((double)d[(int64_t)m * p.B], fb[m], h);
    } else {
        for (int n = 0; n < p.n_terms; ++n) {
            const double w = d[(int64_t)(3 * n) * p.B];
            const double th = d[(int64_t)(3 * n + 1) * p.B];
            const double sg = d[(int64_t)(3 * n + 2) * p.B];
            const double dt = (double)t - th;
            h = fma(w, exp(-dt * dt / (2.0 * sg * sg)), h);
        }
    }
    return h;
}

// dH/d(coefficient m) of attribute a of ball b at time t.
__device__ inline float eval_dH(const OpParams& p, int64_t b, int a, int m, float t, const double* fb) {
    if (p.basis == SB_BASIS_FOURIER) return (float)fb[m];
    const float* d = p.deform + (int64_t)a * p.M * p.B + b;
    int n = m / 3, which = m - 3 * n;
    float w = d[(int64_t)(3 * n) * p.B];
    float th = d[(int64_t)(3 * n + 1) * p.B];
    float sg = d[(int64_t)(3 * n + 2) * p.B];
    float dt = t - th;
    float e = expf(-dt * dt / (2.f * sg * sg));
    if (which == 0) return e;
    if (which == 1) return w * e * dt / (sg * sg);
    return w * e * dt * dt / (sg * sg * sg);
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

__device__ inline void raise_flag(unsigned* flags, unsigned bit) {
    atomicOr(flags, bit);
}


// Stage the deformed balls of one group (Eq. 1, recomputed per frame) into LDS
// and find the centre of their bounding box.  Ends with a block barrier.
template <int NW, int G>
__device__ inline void stage_group(const OpParams& p, const Scene& sc, int group, float t,
                                   BallF* sball, double* sred, double* scen, int& nb) {
    const int tid = threadIdx.x;
    const int64_t first = sc.ball0 + (int64_t)group * G;
    nb = min(G, sc.n_balls - group * G);
    double fb[2 * SB_MAX_FOURIER];
    if (p.basis == SB_BASIS_FOURIER) fourier_basis(t, p.n_terms, fb);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = tid; i < G; i += 64 * NW) {
        BallF bl;
        if (i < nb) {
            if (!deform_ball(p, first + i, t, fb, bl)) raise_flag(p.flags, SB_FLAG_NONFINITE);
        } else {
            bl.x = bl.y = bl.z = 0.0;
            bl.rho = -1.0;
            bl.rhof = -1.f;
            bl.amp = 0.f;
        }
        sball[i] = bl;
        if (bl.rho >= 0.0) {
            lo[0] = fmin(lo[0], bl.x); hi[0] = fmax(hi[0], bl.x);
            lo[1] = fmin(lo[1], bl.y); hi[1] = fmax(hi[1], bl.y);
            lo[2] = fmin(lo[2], bl.z); hi[2] = fmax(hi[2], bl.z);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], off));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], off));
        }
    }
    const int wid = tid >> 6, lane = tid & 63;
    if (lane == 0)
        for (int a = 0; a < 3; ++a) { sred[wid * 6 + a] = lo[a]; sred[wid * 6 + 3 + a] = hi[a]; }
    __syncthreads();
    if (tid == 0) {
        for (int a = 0; a < 3; ++a) {
            double l = sred[a], h = sred[3 + a];
            for (int w = 1; w < NW; ++w) { l = fmin(l, sred[w * 6 + a]); h = fmax(h, sred[w * 6 + 3 + a]); }
            scen[a] = (l <= h) ? 0.5 * (l + h) : 0.0;
        }
    }
    __syncthreads();
}

// Tile origin of a lane: arrival sample of the group centre minus half the tile,
// clamped so that k_lo - o and k_lo + W stay far inside int32 for in-range pairs.
__device__ inline int tile_origin(const OpParams& p, const double* scen, double sx, double sy,
                                  double sz, int ucap) {
    const double cx = scen[0] - sx, cy = scen[1] - sy, cz = scen[2] - sz;
    const double tau_c = sqrt(cx * cx + cy * cy + cz * cz) * p.inv_delta - p.t0fs;
    return (int)fmin(fmax(floor(tau_c) - (double)(ucap / 2), -5.0e8), 5.0e8);
}

// Window of one (ball, sensor) pair.  tau = (r - c t0)/delta is the arrival
// sample; the window starts at sample k_lo = floor(tau - h + 1/2) (h = rho for the
// uniform sphere, kGaussCut*rho for the Gaussian ball) so that boundary 0,
// x_0 = tau - k_lo + 1/2, lies in [h, h + 1), and spans W = floor(2h) + 2 samples,
// so that boundary W lies below -h: every nonzero sample is inside.  All in FP64.
template <int KERNEL>
struct PairWin {
    double r;        // ball-sensor distance
    double a0;       // x_0
    int klo, W;
    bool ok;         // sensor outside the uniform ball (or r > 0 for the Gaussian ball)
    bool in_range;   // |k_lo| and W small enough for int32 sample arithmetic
};

template <int KERNEL>
__device__ inline PairWin<KERNEL> pair_window(const OpParams& p, const BallF& bl, double dx,
                                              double dy, double dz) {
    PairWin<KERNEL> w;
    w.r = sqrt(dx * dx + dy * dy + dz * dz);
    const double h = (KERNEL == SB_KERNEL_UNIFORM) ? bl.rho : (double)kGaussCut * bl.rho;
    w.ok = (KERNEL == SB_KERNEL_UNIFORM) ? (w.r > bl.rho * (double)p.delta) : (w.r > 0.0);
    const double tau = w.r * p.inv_delta - p.t0fs;
    const double kl = floor(tau - h + 0.5);
    w.in_range = fabs(kl) < 5.0e8 && h < 1.0e6;
    w.klo = w.in_range ? (int)kl : 0;
    w.W = w.in_range ? (int)(2.0 * h) + 2 : 0;
    w.a0 = tau - kl + 0.5;
    return w;
}

// ---- host-side launchers (defined in the .hip files) ----
struct TileCfg {
    int nw;      // waves per block (64 sensors each)
    int g;       // balls per group
    int ucap;    // tile length in samples
};

hipError_t launch_forward(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st);
hipError_t launch_adjoint(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st);
hipError_t launch_fill(float* ptr, int64_t n, float v, hipStream_t st);
hipError_t launch_loss(const float* y, const float* d, float* r, int64_t n, double* partials,
                       int n_blocks, double* loss, hipStream_t st);
int loss_blocks();
hipError_t launch_adam(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, hipStream_t st);

}  // namespace sb
