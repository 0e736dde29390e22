// Adjoint: gradient of 1/2 |y - d|^2 with respect to every ball attribute and
// deformation coefficient, given the residual y - d.
//
// Work item = (scene, chunk of 256 consecutive balls, split of the sensors).
// A block of four waves takes the chunk and ranks its balls by size, so that
// each wave holds 64 balls of similar size (similar window lengths keep the
// lanes of a wave busy for the same number of samples); lane = ball.  For
// every frame of the scene the lane deforms its ball (Eq. 1, recomputed here),
// and for every sensor of the split the wave stages the residual samples around
// its balls' arrival times in an LDS row (64 consecutive samples per coalesced
// load; the next sensor's row is fetched while the current one is used).  Each
// lane gathers its window from the row and accumulates the five derivatives of
// the loss with respect to its deformed ball in registers: no cross-lane
// reductions and no atomics until the chain rule at the end of the item.
//
// Sums by parts over the window boundaries x_m (residual differences
// dr_m = r_m - r_{m-1}, r_{-1} = r_W = 0).  Uniform sphere: boundaries m = 1..m_hi
// lie strictly inside (-rho, rho) (decided in FP64); the clamped ones
// telescope, so with
//   S_w = sum_in x_m^2 dr_m - rho^2 S_r,  S_t = sum_in x_m dr_m,  S_r = r_{m_hi} - r_0
// and C = P_f delta / (4r):  G_v = C S_w,  G_tau = 2 C S_t,  G_rho = -2 rho C S_r.
// Gaussian ball: all boundaries, E_m = exp(-x_m^2 / (2 rho^2)), K = P_f rho^2 delta/(2r),
// S_n = sum x_m^n E_m dr_m:  G_v = -K S0,  G_tau = K/rho^2 S1,
// G_rho = -2K/rho S0 - K/rho^3 S2.
// Then dL/dr = G_tau/delta - G_v/r, dL/dR_f = G_rho/delta, dL/dP_f = G_v/P_f and
// dL/dx_f = dL/dr (x_f - s)/r; the chain rule through Eq. 1 (and Eq. 2 or the
// Fourier series) gives the parameter gradients.

#include "sb_internal.hpp"

namespace sb {

constexpr int kAdjChunk = 256;   // balls per block item (4 waves x 64 lanes)

// Per-lane gather of one pair's window from a row reader rd(m) = residual at
// sample k_lo + m.  Returns the three sums of the uniform sphere (Sw, St, Sr) or
// of the Gaussian ball (S0, S1, S2).
template <int KERNEL, typename Reader>
__device__ inline void gather_window(const PairWin<KERNEL>& w, float rho, Reader rd, float& A,
                                     float& Bs, float& Cs) {
    float x = (float)w.a0;
    if (KERNEL == SB_KERNEL_UNIFORM) {
        const float r0 = rd(0);
        float rp = r0, sw = 0.f, st = 0.f;
        for (int m = 1; m <= w.m_hi; ++m) {
            x -= 1.f;
            const float rm = rd(m);
            const float dr = rm - rp;
            rp = rm;
            sw = fmaf(x * x, dr, sw);
            st = fmaf(x, dr, st);
        }
        const float sr = rp - r0;
        A = fmaf(-rho * rho, sr, sw);
        Bs = st;
        Cs = sr;
    } else {
        const float ce = -1.4426950408889634f / (2.f * rho * rho);   // exp2 scale
        float rp = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
        for (int m = 0; m <= w.W; ++m) {
            const float rm = (m < w.W) ? rd(m) : 0.f;
            const float dr = rm - rp;
            rp = rm;
            const float e = __builtin_amdgcn_exp2f(x * x * ce) * dr;
            s0 += e;
            s1 = fmaf(x, e, s1);
            s2 = fmaf(x * x, e, s2);
            x -= 1.f;
        }
        A = s0;
        Bs = s1;
        Cs = s2;
    }
}

template <int UROW, int KERNEL, int MREG>
__global__ __launch_bounds__(256) void adjoint_kernel(OpParams p) {
    static_assert(UROW % 64 == 0, "row length must be a multiple of 64");
    constexpr int NQ = UROW / 64;
    __shared__ float rowbuf[4][UROW];
    __shared__ float sR[kAdjChunk];
    __shared__ int sperm[kAdjChunk];

    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    float* const row = rowbuf[wid];
    const float delta = p.delta;
    const float inv_delta_f = (float)p.inv_delta;

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const ItemA it = decode_item_adj(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int nb = min(kAdjChunk, sc.n_balls - it.chunk * kAdjChunk);
        const int64_t first = sc.ball0 + (int64_t)it.chunk * kAdjChunk;
        const int s_begin = it.split * p.s_per_split;
        const int s_end = min(p.S, s_begin + p.s_per_split);

        // ---- rank the chunk's balls by base size; wave w takes ranks 64w..64w+63
        __syncthreads();
        const float Ri = tid < nb ? p.balls[3 * p.B + first + tid] : 3.0e38f;
        sR[tid] = Ri;
        __syncthreads();
        int rank = 0;
        for (int j = 0; j < kAdjChunk; ++j) {
            const float Rj = sR[j];
            rank += (Rj < Ri) || (Rj == Ri && j < tid);
        }
        sperm[rank] = tid;
        __syncthreads();
        const int li = sperm[wid * 64 + lane];
        const bool valid = li < nb;
        const int64_t b = first + (valid ? li : 0);

        float gb[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        float gd[5][MREG > 0 ? MREG : 1];
        for (int a = 0; a < 5; ++a)
            for (int m = 0; m < (MREG > 0 ? MREG : 1); ++m) gd[a][m] = 0.f;

        for (int f = 0; f < sc.n_frames; ++f) {
            const int gf = sc.frame0 + f;
            const float t = p.frame_t[gf];
            BallF bl;
            bool live = false;
            if (valid) {
                double fb[2 * SB_MAX_FOURIER];
                if (p.basis == SB_BASIS_FOURIER) fourier_basis(t, p.n_terms, fb);
                live = deform_ball(p, b, t, fb, bl);
                if (!live) raise_flag(p.flags, SB_FLAG_NONFINITE);
            }
            // bounding box (rounded outwards) and largest size of the wave's live balls
            float lo[3], hi[3];
            lo[0] = live ? __double2float_rd(bl.x) : 3.0e38f;
            lo[1] = live ? __double2float_rd(bl.y) : 3.0e38f;
            lo[2] = live ? __double2float_rd(bl.z) : 3.0e38f;
            hi[0] = live ? __double2float_ru(bl.x) : -3.0e38f;
            hi[1] = live ? __double2float_ru(bl.y) : -3.0e38f;
            hi[2] = live ? __double2float_ru(bl.z) : -3.0e38f;
            float rmax = live ? bl.rhof : 0.f;
            for (int a = 0; a < 3; ++a) { lo[a] = wave_min(lo[a]); hi[a] = wave_max(hi[a]); }
            rmax = wave_max(rmax);
            if (!(lo[0] <= hi[0])) continue;           // no live ball in this wave
            const double hmax = (KERNEL == SB_KERNEL_UNIFORM) ? (double)rmax : (double)kGaussCut * rmax;

            const float* res_frame = p.residual + (int64_t)gf * p.S * p.T;
            float g5[5] = {0.f, 0.f, 0.f, 0.f, 0.f};

            // row origin of a sensor: every window of the wave starts at or after o + 1
            auto origin = [&](int s) -> int {
                double dmin, dmax;
                box_distance_range(lo, hi, (double)p.sensors[s], (double)p.sensors[p.S + s],
                                   (double)p.sensors[2 * p.S + s], dmin, dmax);
                const double ofl = floor(dmin * p.inv_delta - p.t0fs - hmax - 1.0) - 1.0;
                return (int)fmin(fmax(ofl, -5.0e8), 5.0e8);
            };
            float pf[NQ];
            int o_next = 0;
            if (s_begin < s_end) {
                o_next = origin(s_begin);
                const float* rr = res_frame + (int64_t)s_begin * p.T;
                for (int q = 0; q < NQ; ++q) {
                    const int k = o_next + q * 64 + lane;
                    pf[q] = (k >= 0 && k < p.T) ? rr[k] : 0.f;
                }
            }
            for (int s = s_begin; s < s_end; ++s) {
                const int o = o_next;
                wave_lds_sync();
                for (int q = 0; q < NQ; ++q) row[q * 64 + lane] = pf[q];
                wave_lds_sync();
                if (s + 1 < s_end) {            // fetch the next sensor's row
                    o_next = origin(s + 1);
                    const float* rr = res_frame + (int64_t)(s + 1) * p.T;
                    for (int q = 0; q < NQ; ++q) {
                        const int k = o_next + q * 64 + lane;
                        pf[q] = (k >= 0 && k < p.T) ? rr[k] : 0.f;
                    }
                }
                if (!live) continue;
                const double sx = p.sensors[s], sy = p.sensors[p.S + s], sz = p.sensors[2 * p.S + s];
                const double dx = bl.x - sx, dy = bl.y - sy, dz = bl.z - sz;
                const PairWin<KERNEL> w = pair_window<KERNEL>(p, bl.rho, dx, dy, dz);
                if (!w.ok) {
                    raise_flag(p.flags, SB_FLAG_GEOMETRY);
                    continue;
                }
                if (!w.in_range) continue;      // the window reads only zeros
                const float rho = bl.rhof;
                const int tl = w.klo - o;
                float A, Bs, Cs;
                if (tl >= 0 && tl + w.W <= UROW) {
                    const float* rw = row + tl;
                    gather_window<KERNEL>(w, rho, [&](int m) { return rw[m]; }, A, Bs, Cs);
                } else {
                    const float* rr = res_frame + (int64_t)s * p.T;
                    const int klo = w.klo, T = p.T;
                    gather_window<KERNEL>(
                        w, rho, [&](int m) { const int k = klo + m; return (k >= 0 && k < T) ? rr[k] : 0.f; },
                        A, Bs, Cs);
                }
                const float rf = (float)w.r;
                const float inv_r = __builtin_amdgcn_rcpf(rf);
                float dLdr, dLdR, dLdP;
                if (KERNEL == SB_KERNEL_UNIFORM) {
                    const float Cr = delta * 0.25f * inv_r;   // C / P_f
                    const float C = bl.amp * Cr;
                    const float Gv = C * A, Gt = 2.f * C * Bs, Gr = -2.f * rho * C * Cs;
                    dLdr = Gt * inv_delta_f - Gv * inv_r;
                    dLdR = Gr * inv_delta_f;
                    dLdP = Cr * A;
                } else {
                    const float Kr = rho * rho * delta * 0.5f * inv_r;   // K / P_f
                    const float K = bl.amp * Kr;
                    const float Gv = -K * A;
                    const float Gt = K / (rho * rho) * Bs;
                    const float Ga = -2.f * K / rho * A - K / (rho * rho * rho) * Cs;
                    dLdr = Gt * inv_delta_f - Gv * inv_r;
                    dLdR = Ga * inv_delta_f;
                    dLdP = -Kr * A;
                }
                g5[0] = fmaf(dLdr, (float)dx * inv_r, g5[0]);
                g5[1] = fmaf(dLdr, (float)dy * inv_r, g5[1]);
                g5[2] = fmaf(dLdr, (float)dz * inv_r, g5[2]);
                g5[3] += dLdR;
                g5[4] += dLdP;
            }
            // chain rule through Eq. 1 (and Eq. 2 / the Fourier series) for this frame
            if (live) {
                double fb[2 * SB_MAX_FOURIER];
                if (p.basis == SB_BASIS_FOURIER) fourier_basis(t, p.n_terms, fb);
                float base[5];
                for (int a = 0; a < 5; ++a) base[a] = p.balls[(int64_t)a * p.B + b];
                for (int a = 0; a < 5; ++a) {
                    const bool additive = (a < 3 && p.pos_mode == SB_POS_ADD);
                    const float h = (float)eval_H(p, b, a, t, fb);
                    gb[a] += additive ? g5[a] : g5[a] * (1.f + h);
                    const float gs = additive ? g5[a] : g5[a] * base[a];
                    if (MREG > 0) {
                        for (int m = 0; m < MREG; ++m) gd[a][m] = fmaf(gs, (float)fb[m], gd[a][m]);
                    } else if (p.basis != SB_BASIS_STATIC) {
                        for (int m = 0; m < p.M; ++m)
                            unsafeAtomicAdd(p.grad_deform + ((int64_t)a * p.M + m) * p.B + b,
                                            gs * eval_dH(p, b, a, m, t, fb));
                    }
                }
            }
        }
        if (valid) {
            for (int a = 0; a < 5; ++a) {
                unsafeAtomicAdd(p.grad_balls + (int64_t)a * p.B + b, gb[a]);
                if (MREG > 0)
                    for (int m = 0; m < MREG; ++m)
                        unsafeAtomicAdd(p.grad_deform + ((int64_t)a * p.M + m) * p.B + b, gd[a][m]);
            }
        }
    }
}

template <int UROW, int KERNEL, int MREG>
static hipError_t launch_adj_t(const OpParams& p, hipStream_t st) {
    int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((adjoint_kernel<UROW, KERNEL, MREG>), dim3((unsigned)grid), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_adjoint(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st) {
    // register accumulators for the Fourier coefficients when they fit (K <= 2)
    const bool reg = p.basis == SB_BASIS_FOURIER && p.M == 4;
    if (tc.ucap == 128) {
        if (kernel == SB_KERNEL_UNIFORM)
            return reg ? launch_adj_t<128, 0, 4>(p, st) : launch_adj_t<128, 0, 0>(p, st);
        return reg ? launch_adj_t<128, 1, 4>(p, st) : launch_adj_t<128, 1, 0>(p, st);
    }
    if (tc.ucap == 192 && kernel == SB_KERNEL_GAUSS)
        return reg ? launch_adj_t<192, 1, 4>(p, st) : launch_adj_t<192, 1, 0>(p, st);
    return hipErrorInvalidValue;
}

}  // namespace sb
