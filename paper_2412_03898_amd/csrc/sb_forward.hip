// Forward operator: per (ball, sensor, frame) scatter of a short sampled trace.
//
// Work item = (scene, frame, group of G consecutive balls, block of 64*NW sensors).
// A block stages its group's deformed balls (Eq. 1, recomputed here) in LDS and
// finds the group's bounding-box centre.  Each wave owns 64 sensors, one per lane,
// and each lane owns one column of the wave's LDS trace tile: samples
// [o, o + UCAP) of its sensor, with o centred on the arrival time from the group
// centre.  Balls are wave-uniform; each lane adds the ball's window into its own
// column (no LDS atomics, no bank conflicts: column c lives in bank c mod 32).
// After the group, each lane adds the touched part of its column to the global
// trace with FP32 atomics.  A window that does not fit the tile (a spread-out
// group) is added to global memory directly.
//
// Trace of one ball in sample units (tau = (r - c t0)/delta, rho = R_f/delta):
// with boundaries x_m = tau - k_lo + 1/2 - m, m = 0..W, between samples,
//   uniform:  sample j = C (Q_j - Q_{j+1}),  Q_m = clamp(x_m, -rho, rho)^2,
//             C = P_f delta / (4 r)
//   gaussian: sample j = K (E_{j+1} - E_j),  E_m = exp(-x_m^2 / (2 rho^2)),
//             K = P_f rho^2 delta / (2 r)
// which is the interval mean of the N-wave P(r - ct)/(2r) (resp. of the Gaussian
// ball's outgoing term) over each sample interval.

#include "sb_internal.hpp"

namespace sb {

template <int KERNEL>
__device__ inline float trace_coef(const BallF& bl, double r, float delta) {
    if (KERNEL == SB_KERNEL_UNIFORM) return (float)((double)bl.amp * (double)delta / (4.0 * r));
    return (float)((double)bl.amp * bl.rho * bl.rho * (double)delta / (2.0 * r));
}

template <int NW, int G, int UCAP, int KERNEL>
__global__ __launch_bounds__(64 * NW) void forward_kernel(OpParams p) {
    __shared__ BallF sball[G];
    __shared__ float tile[NW][UCAP][64];
    __shared__ double sred[NW * 6];
    __shared__ double scen[3];

    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    float* col = &tile[wid][0][lane];
    for (int k = 0; k < UCAP; ++k) col[k * 64] = 0.f;

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const Item it = decode_item(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int gf = sc.frame0 + it.frame;
        const float t = p.frame_t[gf];
        __syncthreads();   // previous item's readers of sball/scen are done
        int nb;
        stage_group<NW, G>(p, sc, it.group, t, sball, sred, scen, nb);

        const int s = it.sblock * 64 * NW + wid * 64 + lane;
        const bool active = s < p.S;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        if (active) { sx = p.sensors[s]; sy = p.sensors[p.S + s]; sz = p.sensors[2 * p.S + s]; }
        const int o = tile_origin(p, scen, sx, sy, sz, UCAP);
        int kmin = UCAP, kmax = -1;
        float* out_row = p.signals + ((int64_t)gf * p.S + (active ? s : 0)) * p.T;
        bool clipped = false;

        for (int bi = 0; bi < nb; ++bi) {
            const BallF bl = sball[bi];
            if (bl.rho < 0.0 || !active) continue;
            const PairWin<KERNEL> w = pair_window<KERNEL>(p, bl, bl.x - sx, bl.y - sy, bl.z - sz);
            if (!w.ok) {
                raise_flag(p.flags, SB_FLAG_GEOMETRY);
                continue;
            }
            if (!w.in_range) {          // arrival far outside any record: nothing to add
                clipped = true;
                continue;
            }
            const float rho = bl.rhof;
            const float C = trace_coef<KERNEL>(bl, w.r, p.delta);
            const int W = w.W;
            const int tl = w.klo - o;
            float x = (float)w.a0;
            if (tl >= 0 && tl + W <= UCAP) {
                float* c = col + tl * 64;
                kmin = min(kmin, tl);
                kmax = max(kmax, tl + W - 1);
                if (KERNEL == SB_KERNEL_UNIFORM) {
                    float Qp = rho * rho;
                    for (int j = 0; j < W; ++j) {
                        x -= 1.f;
                        const float q = __builtin_amdgcn_fmed3f(x, -rho, rho);
                        const float Q = q * q;
                        c[j * 64] += C * (Qp - Q);
                        Qp = Q;
                    }
                } else {
                    const float ce = -1.f / (2.f * rho * rho);
                    float Ep = expf(x * x * ce);
                    for (int j = 0; j < W; ++j) {
                        x -= 1.f;
                        const float E = expf(x * x * ce);
                        c[j * 64] += C * (E - Ep);
                        Ep = E;
                    }
                }
            } else {
                // window outside the tile: add straight to the global trace
                float Qp = rho * rho;
                const float ce = -1.f / (2.f * rho * rho);
                float Ep = (KERNEL == SB_KERNEL_UNIFORM) ? 0.f : expf(x * x * ce);
                for (int j = 0; j < W; ++j) {
                    x -= 1.f;
                    float v;
                    if (KERNEL == SB_KERNEL_UNIFORM) {
                        const float q = __builtin_amdgcn_fmed3f(x, -rho, rho);
                        const float Q = q * q;
                        v = C * (Qp - Q);
                        Qp = Q;
                    } else {
                        const float E = expf(x * x * ce);
                        v = C * (E - Ep);
                        Ep = E;
                    }
                    const int k = w.klo + j;
                    if (v != 0.f) {
                        if (k >= 0 && k < p.T) unsafeAtomicAdd(out_row + k, v);
                        else clipped = true;
                    }
                }
            }
        }
        // flush the touched part of this lane's column, leaving it zero
        for (int k = kmin; k <= kmax; ++k) {
            const float v = col[k * 64];
            col[k * 64] = 0.f;
            const int kg = o + k;
            if (v != 0.f) {
                if (kg >= 0 && kg < p.T) unsafeAtomicAdd(out_row + kg, v);
                else clipped = true;
            }
        }
        if (clipped) raise_flag(p.flags, SB_FLAG_CLIPPED);
    }
}

template <int NW, int G, int UCAP, int KERNEL>
static hipError_t launch_fwd_t(const OpParams& p, hipStream_t st) {
    int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((forward_kernel<NW, G, UCAP, KERNEL>), dim3((unsigned)grid), dim3(64 * NW), 0,
                       st, p);
    return hipGetLastError();
}

hipError_t launch_forward(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st) {
    // the host's work decomposition (n_sblocks, n_groups) must match the instance
    if (kernel == SB_KERNEL_UNIFORM) {
        if (tc.nw == 4 && tc.g == 256 && tc.ucap == 64) return launch_fwd_t<4, 256, 64, 0>(p, st);
        if (tc.nw == 2 && tc.g == 128 && tc.ucap == 96) return launch_fwd_t<2, 128, 96, 0>(p, st);
        if (tc.nw == 4 && tc.g == 128 && tc.ucap == 64) return launch_fwd_t<4, 128, 64, 0>(p, st);
    } else {
        if (tc.nw == 4 && tc.g == 128 && tc.ucap == 96) return launch_fwd_t<4, 128, 96, 1>(p, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace sb
