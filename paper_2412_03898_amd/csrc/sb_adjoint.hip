// Adjoint: gradient of 1/2 |y - d|^2 with respect to every ball attribute and
// deformation coefficient, given the residual y - d.
//
// Two kernels.  The uniform sphere's (adjoint_uniform_kernel, further below) sums
// each window in closed form from prefix sums of a staged residual row.  The
// Gaussian ball's (adjoint_gauss_kernel) gathers every window boundary:
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
// dr_m = r_m - r_{m-1}, r_{-1} = r_W = 0), E_m = exp(-x_m^2 / (2 rho^2)),
// K = P_f rho^2 delta/(2r), S_n = sum x_m^n E_m dr_m:  G_v = -K S0,
// G_tau = K/rho^2 S1, G_rho = -2K/rho S0 - K/rho^3 S2.
// Then dL/dr = G_tau/delta - G_v/r, dL/dR_f = G_rho/delta, dL/dP_f = G_v/P_f and
// dL/dx_f = dL/dr (x_f - s)/r; the chain rule through Eq. 1 (and Eq. 2 or the
// Fourier series) gives the parameter gradients.

#include "sb_internal.hpp"

namespace sb {

constexpr int kAdjChunk = 256;   // balls per block item (4 waves x 64 lanes)
constexpr int kAdjMaxSplit = 256;   // sensors per item at most

template <int UROW, int MREG, int OCC>
__global__ __launch_bounds__(256, OCC) void adjoint_gauss_kernel(OpParams p) {
    static_assert(UROW % 64 == 0, "row length must be a multiple of 64");
    constexpr int NQ = UROW / 64;
    __shared__ float rowbuf[4][UROW];
    __shared__ float sR[kAdjChunk];
    __shared__ int sperm[kAdjChunk];
    // per wave, per sensor of the split: row origin and coordinates
    __shared__ int s_org[4][kAdjMaxSplit];
    __shared__ float s_sx[4][kAdjMaxSplit], s_sy[4][kAdjMaxSplit], s_sz[4][kAdjMaxSplit];
    __shared__ double s_fb[4][2 * SB_MAX_FOURIER];     // Fourier basis of the wave's frame

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
        const int ns = min(p.S - s_begin, p.s_per_split);     // sensors of this split (<= kAdjMaxSplit)

        // ---- rank the chunk's balls by base size; wave w takes ranks 64w..64w+63.
        // (key, index) must be a strict total order so that the ranks form a
        // permutation: a NaN or +inf size (a ball that deform_ball skips) takes the
        // padding key, ordered by index before the padding threads.
        __syncthreads();
        float Ri = 3.0e38f;
        if (tid < nb) {
            const float R = p.balls[3 * p.B + first + tid];
            Ri = R < 3.0e38f ? R : 3.0e38f;
        }
        sR[tid] = Ri;
        __syncthreads();
        int rank = 0;
#pragma unroll 8
        for (int j = 0; j < kAdjChunk; ++j) {
            const float Rj = sR[j];
            rank += (Rj < Ri) || (Rj == Ri && j < tid);
        }
        sperm[rank] = tid;
        __syncthreads();
        const int li = sperm[wid * 64 + lane];
        const bool valid = li < nb;
        const int64_t b = first + (valid ? li : 0);
        // sensor coordinates of the split (float, as given)
        for (int j = lane; j < ns; j += 64) {
            s_sx[wid][j] = p.sensors[s_begin + j];
            s_sy[wid][j] = p.sensors[p.S + s_begin + j];
            s_sz[wid][j] = p.sensors[2 * p.S + s_begin + j];
        }

        float gb[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        float gd[5][MREG > 0 ? MREG : 1];
        for (int a = 0; a < 5; ++a)
            for (int m = 0; m < (MREG > 0 ? MREG : 1); ++m) gd[a][m] = 0.f;

        for (int f = 0; f < sc.n_frames; ++f) {
            const int gf = sc.frame0 + f;
            const float t = p.frame_t[gf];
            const double* fb = s_fb[wid];
            wave_lds_sync();
            if (p.basis == SB_BASIS_FOURIER) fourier_basis_lanes(t, p.n_terms, s_fb[wid], lane);
            wave_lds_sync();
            BallF bl;
            bool live = false;
            if (valid) {
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
            const double hmax = (double)kGaussCut * rmax;
            // row origins of all sensors of the split, one sensor per lane: every
            // window of the wave starts at or after o + 1
            wave_lds_sync();
            for (int j = lane; j < ns; j += 64) {
                double dmin, dmax;
                box_distance_range(lo, hi, (double)s_sx[wid][j], (double)s_sy[wid][j], (double)s_sz[wid][j],
                                   dmin, dmax);
                const double ofl = floor(dmin * p.inv_delta - p.t0fs - hmax - 1.0) - 1.0;
                s_org[wid][j] = (int)fmin(fmax(ofl, -5.0e8), 5.0e8);
            }
            wave_lds_sync();

            // per-ball constants of this frame
            const float rho = live ? bl.rhof : 0.f;
            const double h = (double)kGaussCut * bl.rho;
            const double h_half = h - 0.5;
            const double r_in = 0.0;                           // the sensor must not sit at the centre
            const int W = live ? (int)(2.0 * h) + 2 : 0;
            const bool w_ok = live && h < 1.0e6;
            const float* res_frame = p.residual + (int64_t)gf * p.S * p.T;
            float g5[5] = {0.f, 0.f, 0.f, 0.f, 0.f};

            float pf[NQ];
            {
                const int o0 = s_org[wid][0];
                const float* rr = res_frame + (int64_t)s_begin * p.T;
                for (int q = 0; q < NQ; ++q) {
                    const int k = o0 + q * 64 + lane;
                    pf[q] = (k >= 0 && k < p.T) ? rr[k] : 0.f;
                }
            }
            for (int j = 0; j < ns; ++j) {
                const int o = s_org[wid][j];
                wave_lds_sync();
                for (int q = 0; q < NQ; ++q) row[q * 64 + lane] = pf[q];
                wave_lds_sync();
                if (j + 1 < ns) {               // fetch the next sensor's row
                    const int on = s_org[wid][j + 1];
                    const float* rr = res_frame + (int64_t)(s_begin + j + 1) * p.T;
                    for (int q = 0; q < NQ; ++q) {
                        const int k = on + q * 64 + lane;
                        pf[q] = (k >= 0 && k < p.T) ? rr[k] : 0.f;
                    }
                }
                const double dx = bl.x - (double)s_sx[wid][j];
                const double dy = bl.y - (double)s_sy[wid][j];
                const double dz = bl.z - (double)s_sz[wid][j];
                const double r = dist64(dx, dy, dz);
                const double tau = fma(r, p.inv_delta, -p.t0fs);
                const double kl = floor(tau - h_half);
                const double a0d = tau - kl + 0.5;
                const bool geo = w_ok && r > r_in;
                if (w_ok && !(r > r_in)) raise_flag(p.flags, SB_FLAG_GEOMETRY);
                const bool use = geo && fabs(kl) < 5.0e8;
                const int klo = use ? (int)kl : 0;
                const int tl = klo - o;
                const bool in_row = tl >= 0 && tl + W <= UROW;
                const float* rres = res_frame + (int64_t)(s_begin + j) * p.T;
                float A = 0.f, Bs = 0.f, Cs = 0.f;
                if (use) {
                    float x = (float)a0d;
                    {
                        // every boundary m = 0..W (r_{-1} = r_W = 0)
                        const float ce = -1.4426950408889634f / (2.f * rho * rho);   // exp2 scale
                        float rp = 0.f;
                        if (in_row) {
                            // eight boundaries per batch, their samples read together (indices
                            // clamped into the window; boundaries past W contribute nothing)
                            const float* rw = row + tl;          // samples 0..W-1 lie in the row
                            // E_m advances by E_{m+1} = E_m g_m, g_{m+1} = g_m q (x steps by -1),
                            // restarted exactly at every batch: E enters the sums multiplied,
                            // not differenced, so eight steps of FP32 rounding stay near 1e-6
                            const float q = __builtin_amdgcn_exp2f(2.f * ce);
                            // batches whose eight boundaries all lie before W: no clamping or
                            // masking (r_{m-1} of the first boundary is the previous batch's last)
                            int m0 = 0;
                            for (; m0 + 8 <= W; m0 += 8) {
                                float v[8];
#pragma unroll
                                for (int u = 0; u < 8; ++u) v[u] = rw[m0 + u];
                                float E = __builtin_amdgcn_exp2f(x * x * ce);
                                float g = __builtin_amdgcn_exp2f(fmaf(-2.f, x, 1.f) * ce);
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    const float dr = v[u] - rp;
                                    rp = v[u];
                                    const float e = E * dr;
                                    A += e;
                                    Bs = fmaf(x, e, Bs);
                                    Cs = fmaf(x * x, e, Cs);
                                    x -= 1.f;
                                    E *= g;
                                    g *= q;
                                }
                            }
                            // the last one or two batches, up to boundary W
                            for (; m0 <= W; m0 += 8) {
                                float v[8];
#pragma unroll
                                for (int u = 0; u < 8; ++u) v[u] = rw[min(m0 + u, W - 1)];
                                float E = __builtin_amdgcn_exp2f(x * x * ce);
                                float g = __builtin_amdgcn_exp2f(fmaf(-2.f, x, 1.f) * ce);
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    const int m = m0 + u;
                                    const float rm = (m < W) ? v[u] : 0.f;
                                    const float dr = (m <= W) ? rm - rp : 0.f;
                                    rp = rm;
                                    const float e = E * dr;
                                    A += e;
                                    Bs = fmaf(x, e, Bs);
                                    Cs = fmaf(x * x, e, Cs);
                                    x -= 1.f;
                                    E *= g;
                                    g *= q;
                                }
                            }
                        } else {
                            // boundaries straight from global memory, eight loads in flight at
                            // a time (no load of a batch waits on another; boundaries past W
                            // add nothing)
                            for (int m0 = 0; m0 <= W; m0 += 8) {
                                float v[8];
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    const int k = klo + m0 + u;
                                    v[u] = (m0 + u < W && k >= 0 && k < p.T) ? rres[k] : 0.f;
                                }
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    const float dr = (m0 + u <= W) ? v[u] - rp : 0.f;
                                    rp = v[u];
                                    const float e = __builtin_amdgcn_exp2f(x * x * ce) * dr;
                                    A += e;
                                    Bs = fmaf(x, e, Bs);
                                    Cs = fmaf(x * x, e, Cs);
                                    x -= 1.f;
                                }
                            }
                        }
                    }
                }
                if (use) {
                    const float rf = (float)r;
                    const float inv_r = __builtin_amdgcn_rcpf(rf);
                    float dLdr, dLdR, dLdP;
                    {
                        const float Kr = rho * rho * delta * 0.5f * inv_r;   // K / P_f
                        const float K = bl.amp * Kr;
                        dLdr = K / (rho * rho) * Bs * inv_delta_f + K * A * inv_r;
                        dLdR = (-2.f * K / rho * A - K / (rho * rho * rho) * Cs) * inv_delta_f;
                        dLdP = -Kr * A;
                    }
                    g5[0] = fmaf(dLdr, (float)dx * inv_r, g5[0]);
                    g5[1] = fmaf(dLdr, (float)dy * inv_r, g5[1]);
                    g5[2] = fmaf(dLdr, (float)dz * inv_r, g5[2]);
                    g5[3] += dLdR;
                    g5[4] += dLdP;
                }
            }
            // chain rule through Eq. 1 (and Eq. 2 / the Fourier series) for this frame, or
            // (two-phase) this split's share of dL/d(deformed attributes) to the scratch
            if (live) {
                if (MREG == 0 && p.d5) {
                    float* const dst = p.d5 + sc.d5_0 + (int64_t)f * 5 * sc.n_balls + (b - sc.ball0);
                    for (int a = 0; a < 5; ++a) global_atomic_add(dst + (int64_t)a * sc.n_balls, g5[a]);
                } else {
                    float base[5];
                    for (int a = 0; a < 5; ++a) base[a] = p.balls[(int64_t)a * p.B + b];
                    for (int a = 0; a < 5; ++a) {
                        const bool additive = (a < 3 && p.pos_mode == SB_POS_ADD);
                        const float hh = (float)eval_H(p, b, a, t, fb);
                        gb[a] += additive ? g5[a] : g5[a] * (1.f + hh);
                        if (MREG > 0) {
                            const float gs = additive ? g5[a] : g5[a] * base[a];
                            for (int m = 0; m < MREG; ++m) gd[a][m] = fmaf(gs, (float)fb[m], gd[a][m]);
                        }
                    }
                }
            }
        }
        if (valid && !(MREG == 0 && p.d5)) {
            for (int a = 0; a < 5; ++a) {
                global_atomic_add(p.grad_balls + (int64_t)a * p.B + b, gb[a]);
                if (MREG > 0)
                    for (int m = 0; m < MREG; ++m)
                        global_atomic_add(p.grad_deform + ((int64_t)a * p.M + m) * p.B + b, gd[a][m]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Uniform sphere, prefix-sum form.  Writing x_m = x_0 - m and summing by parts
// once more (x_m - x_{m+1} = 1), with M = m_hi and r_m the residual at sample
// k_lo + m:
//   S_t = x_M r_M - x_1 r_0 + T0,   S_w(inside) = x_M^2 r_M - x_1^2 r_0 + (2 x_0 - 1) T0 - 2 T1,
//   T0 = sum_{m=1}^{M-1} r_m,       T1 = sum_{m=1}^{M-1} m r_m,
// (all zero when M = 0).  With exclusive prefix sums P0[k] = sum_{i<k} row_i and
// P1[k] = sum_{i<k} i row_i of a staged residual row, T0 and T1 cost two LDS
// reads per pair whatever the window length.
//
// Work item as above, but lane = ball in chunk order (no ranking: the cost no
// longer depends on the window length) and the row is shared by the block: the
// row origin of each sensor comes from the bounding box of the whole chunk.
// Sensors are taken four at a time: wave w stages sensor 4g + w (its residual
// row and the FP64 prefix sums, by a DPP scan over the wave), one barrier, then
// every wave evaluates its balls against the four staged sensors.  The slots are
// double-buffered, so one barrier per four sensors suffices.
constexpr int kPfxRow = 128;      // staged residual samples per sensor

// A sensor of the work item's split, with the row origin of the current frame.
struct SensorRow {
    double x, y, z;
    int org;
    int pad;
};

struct PfxSlot {
    double2 pfx[kPfxRow + 1];     // (P0[k], P1[k]), k = 0..kPfxRow
    double rowd[kPfxRow];         // the samples, widened once here rather than per pair
};

// Inclusive prefix sum over the 64 lanes of a wave (every lane active): row
// shifts by 1, 2, 4, 8 within each row of 16 lanes, then the row totals are
// broadcast to the rows above (DPP row_bcast:15 and row_bcast:31).
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_add_step(double v) {
    const uint64_t bits = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)bits, CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(bits >> 32), CTRL, ROW_MASK, 0xF, true);
    return v + __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline double wave_incl_scan(double v) {
    v = dpp_add_step<0x111, 0xF>(v);   // row_shr:1
    v = dpp_add_step<0x112, 0xF>(v);   // row_shr:2
    v = dpp_add_step<0x114, 0xF>(v);   // row_shr:4
    v = dpp_add_step<0x118, 0xF>(v);   // row_shr:8
    v = dpp_add_step<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add_step<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Stage one sensor's residual row: lane l holds samples o + 2l and o + 2l + 1.
__device__ inline void stage_prefix(PfxSlot& sl, float e0, float e1, int lane) {
    const int i0 = 2 * lane;
    *reinterpret_cast<double2*>(&sl.rowd[i0]) = make_double2((double)e0, (double)e1);
    const double s0 = (double)e0 + (double)e1;
    const double s1 = (double)i0 * (double)e0 + (double)(i0 + 1) * (double)e1;
    const double I0 = wave_incl_scan(s0), I1 = wave_incl_scan(s1);
    const double E0 = I0 - s0, E1 = I1 - s1;
    sl.pfx[i0 + 1] = make_double2(E0 + (double)e0, E1 + (double)i0 * (double)e0);
    sl.pfx[i0 + 2] = make_double2(I0, I1);
    if (lane == 0) sl.pfx[0] = make_double2(0.0, 0.0);
}

template <int MREG, int OCC>
__global__ __launch_bounds__(256, OCC) void adjoint_uniform_kernel(OpParams p) {
    static_assert(kPfxRow == 128, "two samples per lane");
    __shared__ PfxSlot slots[2][4];
    __shared__ SensorRow s_sen[kAdjMaxSplit];          // sensors of the split, row origins
    __shared__ double s_fb[2 * SB_MAX_FOURIER];
    __shared__ float s_red[4][8];

    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const float delta = p.delta;
    const float inv_delta_f = (float)p.inv_delta;
    bool geometry = false, nonfinite = false;

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const ItemA it = decode_item_adj(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int nb = min(kAdjChunk, sc.n_balls - it.chunk * kAdjChunk);
        const int64_t first = sc.ball0 + (int64_t)it.chunk * kAdjChunk;
        const int s_begin = it.split * p.s_per_split;
        const int ns = min(p.S - s_begin, p.s_per_split);     // sensors of this split (<= kAdjMaxSplit)
        const bool valid = tid < nb;
        const int64_t b = first + (valid ? tid : 0);

        __syncthreads();                 // the previous item is done with the sensor arrays
        for (int j = tid; j < ns; j += 256) {
            s_sen[j].x = p.sensors[s_begin + j];
            s_sen[j].y = p.sensors[p.S + s_begin + j];
            s_sen[j].z = p.sensors[2 * p.S + s_begin + j];
        }

        float gb[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        float gd[5][MREG > 0 ? MREG : 1];
        for (int a = 0; a < 5; ++a)
            for (int m = 0; m < (MREG > 0 ? MREG : 1); ++m) gd[a][m] = 0.f;

        for (int f = 0; f < sc.n_frames; ++f) {
            const int gf = sc.frame0 + f;
            const float t = p.frame_t[gf];
            __syncthreads();             // the previous frame is done with s_fb, the row origins, slots
            if (p.basis == SB_BASIS_FOURIER && wid == 0) fourier_basis_lanes(t, p.n_terms, s_fb, lane);
            __syncthreads();
            BallF bl;
            bool live = false;
            if (valid) {
                live = deform_ball(p, b, t, s_fb, bl);
                nonfinite |= !live;
            }
            // bounding box (rounded outwards) and largest size of the chunk's live balls
            float red[7];
            red[0] = live ? __double2float_rd(bl.x) : 3.0e38f;
            red[1] = live ? __double2float_rd(bl.y) : 3.0e38f;
            red[2] = live ? __double2float_rd(bl.z) : 3.0e38f;
            red[3] = live ? __double2float_ru(bl.x) : -3.0e38f;
            red[4] = live ? __double2float_ru(bl.y) : -3.0e38f;
            red[5] = live ? __double2float_ru(bl.z) : -3.0e38f;
            red[6] = live ? bl.rhof : 0.f;
            for (int a = 0; a < 3; ++a) red[a] = wave_min_all(red[a]);
            for (int a = 3; a < 7; ++a) red[a] = wave_max_all(red[a]);
            if (lane == 0)
                for (int a = 0; a < 7; ++a) s_red[wid][a] = red[a];
            __syncthreads();
            float lo[3], hi[3], rmax = 0.f;
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(fminf(s_red[0][a], s_red[1][a]), fminf(s_red[2][a], s_red[3][a]));
                hi[a] = fmaxf(fmaxf(s_red[0][3 + a], s_red[1][3 + a]), fmaxf(s_red[2][3 + a], s_red[3][3 + a]));
            }
            rmax = fmaxf(fmaxf(s_red[0][6], s_red[1][6]), fmaxf(s_red[2][6], s_red[3][6]));
            if (!(lo[0] <= hi[0])) continue;           // no live ball in the chunk (same in every thread)
            const double hmax = (double)rmax;
            // row origins: every window of the chunk starts at or after o + 1
            for (int j = tid; j < ns; j += 256) {
                double dmin, dmax;
                box_distance_range(lo, hi, s_sen[j].x, s_sen[j].y, s_sen[j].z, dmin, dmax);
                const double ofl = floor(dmin * p.inv_delta - p.t0fs - hmax - 1.0) - 1.0;
                s_sen[j].org = (int)fmin(fmax(ofl, -5.0e8), 5.0e8);
            }
            __syncthreads();

            // per-ball constants of this frame
            const float rho = live ? bl.rhof : 0.f;
            const double rhod = live ? bl.rho : 0.0;
            const double c1 = p.t0fs + (rhod - 0.5);          // window start: floor(r / delta - c1)
            const double nrr = -rhod * rhod;
            const double r_in = rhod * (double)delta;          // sensor must be farther than this
            const bool w_ok = live && rhod < 1.0e6;
            const int W = w_ok ? (int)(2.0 * rhod) + 2 : 0;
            // a window lies in the staged row iff 0 <= k_lo - o <= kPfxRow - W
            const bool w_fits = W <= kPfxRow;
            const int row_span = w_fits ? kPfxRow - W : 0;
            const float* res_frame = p.residual + (int64_t)gf * p.S * p.T;
            // per-pair sums in FP64: the pair's offsets and closed forms are FP64
            // already, so no conversion is spent on them
            double h5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

            auto load_pair = [&](int j, float& e0, float& e1) {
                const int k = s_sen[j].org + 2 * lane;
                const float* rr = res_frame + (int64_t)(s_begin + j) * p.T;
                e0 = (k >= 0 && k < p.T) ? rr[k] : 0.f;
                e1 = (k + 1 >= 0 && k + 1 < p.T) ? rr[k + 1] : 0.f;
            };
            float e0 = 0.f, e1 = 0.f;
            if (wid < ns) load_pair(wid, e0, e1);
            const int ngroups = (ns + 3) >> 2;
            SensorRow sen_next = s_sen[0];       // the next pair's sensor, read one pair ahead
            for (int g = 0; g < ngroups; ++g) {
                const int buf = g & 1;
                if (4 * g + wid < ns) stage_prefix(slots[buf][wid], e0, e1, lane);
                if (4 * g + 4 + wid < ns) load_pair(4 * g + 4 + wid, e0, e1);
                __syncthreads();
                const int nu = min(4, ns - 4 * g);
                for (int u = 0; u < nu; ++u) {
                    const int j = 4 * g + u;
                    const PfxSlot& sl = slots[buf][u];
                    const SensorRow sen = sen_next;
                    sen_next = s_sen[min(j + 1, ns - 1)];
                    const double dx = bl.x - sen.x;
                    const double dy = bl.y - sen.y;
                    const double dz = bl.z - sen.z;
                    float inv_r;
                    const double r = dist64(dx, dy, dz, inv_r);
                    const double uw = fma(r, p.inv_delta, -c1);    // tau - rho + 1/2
                    const double kl = floor(uw);
                    const double a0d = (uw - kl) + rhod;             // x_0 = tau - k_lo + 1/2
                    const double x1 = a0d - 1.0;
                    const bool geo = w_ok && r > r_in;
                    geometry |= w_ok && !geo;
                    const bool use = geo && fabs(kl) < 5.0e8;
                    const int klo = use ? (int)kl : 0;
                    const int tl = klo - sen.org;
                    const bool in_row = use && w_fits && (unsigned)tl <= (unsigned)row_span;
                    // inside boundaries m = 1..M, M = ceil(x_1 + rho) (decided in FP64)
                    const int M = use ? (int)ceil(x1 + rhod) : 0;
                    // prefix form (lanes outside the row read row entry 0 and discard it);
                    // byte offsets from the slot base keep the address arithmetic to shifts
                    const int t0 = in_row ? tl : 0, iM = in_row ? tl + M : 0;
                    const char* const slb = reinterpret_cast<const char*>(&sl);
                    constexpr int kRowOff = (int)offsetof(PfxSlot, rowd);
                    const double r0 = *reinterpret_cast<const double*>(slb + kRowOff + (t0 << 3));
                    const double rM = *reinterpret_cast<const double*>(slb + kRowOff + (iM << 3));
                    const double2 pa = *reinterpret_cast<const double2*>(slb + ((t0 + 1) << 4));
                    const double2 pb = *reinterpret_cast<const double2*>(slb + (iM << 4));
                    const double T0 = pb.x - pa.x;
                    const double T1 = (pb.y - pa.y) - (double)t0 * T0;
                    const double xM = a0d - (double)M;
                    double St = fma(xM, rM, fma(-x1, r0, T0));
                    double Sw = fma(xM * xM, rM, fma(-x1 * x1, r0, fma(2.0 * a0d - 1.0, T0, -2.0 * T1)));
                    double Sr = rM - r0;
                    // windows outside the staged row: boundaries straight from global memory
                    // (a window without an inside boundary, M < 1, contributes nothing and is
                    // skipped below)
                    const bool glob = use && !in_row;
                    {
                        if (glob) {
                            // the same closed form, summing r_1..r_{M-1} straight from the
                            // residual row in global memory, eight loads in flight at a time
                            const float* rres = res_frame + (int64_t)(s_begin + j) * p.T;
                            auto at = [&](int m) {
                                const int k = klo + m;
                                return (k >= 0 && k < p.T) ? rres[k] : 0.f;
                            };
                            float q0, qM;
                            double g0 = 0.0, g1 = 0.0;
                            if (klo >= 0 && klo + M + 8 < p.T) {
                                // window and one batch beyond it inside the record (the usual
                                // case): one base address, immediate offsets, every load of a
                                // batch unconditional and the samples past the window masked
                                const float* w = rres + klo;
                                q0 = w[0];
                                qM = w[M];
                                // FP32 sums of at most a window's samples, widened for the
                                // closed form
                                float h0 = 0.f, h1 = 0.f;
                                for (int m0 = 1; m0 < M; m0 += 8) {
                                    float v[8];
#pragma unroll
                                    for (int u = 0; u < 8; ++u) v[u] = w[m0 + u];
                                    float b0 = 0.f, b1 = 0.f;     // sum r and sum u r over the batch
#pragma unroll
                                    for (int u = 0; u < 8; ++u) {
                                        const float x = (m0 + u < M) ? v[u] : 0.f;
                                        b0 += x;
                                        b1 = fmaf((float)u, x, b1);
                                    }
                                    h0 += b0;
                                    h1 = fmaf((float)m0, b0, h1 + b1);
                                }
                                g0 = h0;
                                g1 = h1;
                            } else {
                                q0 = at(0);
                                qM = at(M);
                                for (int m0 = 1; m0 < M; m0 += 8) {
                                    float v[8];
#pragma unroll
                                    for (int u = 0; u < 8; ++u) v[u] = (m0 + u < M) ? at(m0 + u) : 0.f;
#pragma unroll
                                    for (int u = 0; u < 8; ++u) {
                                        g0 += (double)v[u];
                                        g1 = fma((double)(m0 + u), (double)v[u], g1);
                                    }
                                }
                            }
                            St = fma(xM, (double)qM, fma(-x1, (double)q0, g0));
                            Sw = fma(xM * xM, (double)qM, fma(-x1 * x1, (double)q0, fma(2.0 * a0d - 1.0, g0, -2.0 * g1)));
                            Sr = (double)qM - (double)q0;
                        }
                    }
                    if (M >= 1) {                                // implies use
                        // C = P_f delta / (4 r); constant factors (P_f delta / 4, -2 rho / delta,
                        // delta / 4) are applied once per frame below
                        const double ri = (double)inv_r;
                        const double A = fma(nrr, Sr, Sw);
                        const double q = fma(p.two_inv_delta, St, -A * ri);   // dL/dr / (C)
                        const double qr = q * ri * ri;                       // times 1/r for the direction
                        h5[0] = fma(qr, dx, h5[0]);
                        h5[1] = fma(qr, dy, h5[1]);
                        h5[2] = fma(qr, dz, h5[2]);
                        h5[3] = fma(ri, Sr, h5[3]);
                        h5[4] = fma(ri, A, h5[4]);
                    }
                }
            }
            // per-frame factors of the accumulated sums: dL/dx_f = (P_f delta/4) sum q dx/r^2,
            // dL/dR_f = -(2 rho/delta)(P_f delta/4) sum Sr/r, dL/dP_f = (delta/4) sum A/r
            float g5[5];
            {
                const float cp = live ? bl.amp * delta * 0.25f : 0.f;
                g5[0] = (float)h5[0] * cp;
                g5[1] = (float)h5[1] * cp;
                g5[2] = (float)h5[2] * cp;
                g5[3] = (float)h5[3] * (-2.f * rho * inv_delta_f * cp);
                g5[4] = (float)h5[4] * (delta * 0.25f);
            }
            // chain rule through Eq. 1 (and Eq. 2 / the Fourier series) for this frame, or
            // (two-phase) this split's share of dL/d(deformed attributes) to the scratch
            if (live) {
                if (MREG == 0 && p.d5) {
                    float* const dst = p.d5 + sc.d5_0 + (int64_t)f * 5 * sc.n_balls + (b - sc.ball0);
                    for (int a = 0; a < 5; ++a) global_atomic_add(dst + (int64_t)a * sc.n_balls, g5[a]);
                } else {
                    float base[5];
                    for (int a = 0; a < 5; ++a) base[a] = p.balls[(int64_t)a * p.B + b];
                    for (int a = 0; a < 5; ++a) {
                        const bool additive = (a < 3 && p.pos_mode == SB_POS_ADD);
                        const float hh = (float)eval_H(p, b, a, t, s_fb);
                        gb[a] += additive ? g5[a] : g5[a] * (1.f + hh);
                        if (MREG > 0) {
                            const float gs = additive ? g5[a] : g5[a] * base[a];
                            for (int m = 0; m < MREG; ++m) gd[a][m] = fmaf(gs, (float)s_fb[m], gd[a][m]);
                        }
                    }
                }
            }
        }
        if (valid && !(MREG == 0 && p.d5)) {
            for (int a = 0; a < 5; ++a) {
                global_atomic_add(p.grad_balls + (int64_t)a * p.B + b, gb[a]);
                if (MREG > 0)
                    for (int m = 0; m < MREG; ++m)
                        global_atomic_add(p.grad_deform + ((int64_t)a * p.M + m) * p.B + b, gd[a][m]);
            }
        }
    }
    if (geometry) raise_flag(p.flags, SB_FLAG_GEOMETRY);
    if (nonfinite) raise_flag(p.flags, SB_FLAG_NONFINITE);
}

template <int MREG, int OCC>
static hipError_t launch_adj_u(const OpParams& p, hipStream_t st) {
    int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((adjoint_uniform_kernel<MREG, OCC>), dim3((unsigned)grid), dim3(256), 0, st, p);
    return hipGetLastError();
}

template <int OCC>
static hipError_t launch_adj_um(const OpParams& p, hipStream_t st) {
    const bool reg = p.basis == SB_BASIS_FOURIER && p.M == 4;
    return reg ? launch_adj_u<4, OCC>(p, st) : launch_adj_u<0, OCC>(p, st);
}

template <int UROW, int MREG, int OCC>
static hipError_t launch_adj_t(const OpParams& p, hipStream_t st) {
    int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((adjoint_gauss_kernel<UROW, MREG, OCC>), dim3((unsigned)grid), dim3(256), 0, st, p);
    return hipGetLastError();
}

template <int UROW, int OCC>
static hipError_t launch_adj_m(const OpParams& p, hipStream_t st) {
    // register accumulators for the Fourier coefficients when they fit (K <= 2); with them
    // the kernel needs 168 registers, so it is held to three blocks per compute unit (at
    // four it spills 55)
    const bool reg = p.basis == SB_BASIS_FOURIER && p.M == 4;
    return reg ? launch_adj_t<UROW, 4, (OCC > 3 ? 3 : OCC)>(p, st) : launch_adj_t<UROW, 0, OCC>(p, st);
}

// Second phase of the two-phase chain rule: one thread per ball.  From the summed
// derivatives of the loss with respect to the ball's deformed attributes at every frame
// of its scene (OpParams::d5), the gradients of its base attributes (Eq. 1: dx_f/dx = 1
// for an additive position, 1 + H otherwise) and of every deformation coefficient
// (dattr_f/dcoef = dH/dcoef times 1 for an additive position, times the base attribute
// otherwise; Fourier: cos 2 pi k t, sin 2 pi k t; Eq. 2: e_n, w_n e_n (t - theta_n) /
// sigma_n^2, w_n e_n (t - theta_n)^2 / sigma_n^3 with e_n = exp(-(t - theta_n)^2 /
// (2 sigma_n^2))), summed over the frames in FP64 and stored (each ball's entries are
// written by its thread only).
__global__ __launch_bounds__(256) void chain_rule_kernel(OpParams p) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p.B) return;
    int i = 0;
    while (i + 1 < p.n_scenes && p.scenes[i + 1].ball0 <= b) ++i;
    const Scene& sc = p.scenes[i];
    if (sc.n_frames <= 0 || b - sc.ball0 >= sc.n_balls) return;
    const int64_t nb = sc.n_balls;
    const float* const g = p.d5 + sc.d5_0 + (b - sc.ball0);
    const int M = p.M, N = p.n_terms;
    for (int a = 0; a < 5; ++a) {
        const bool additive = a < 3 && p.pos_mode == SB_POS_ADD;
        const double base = p.balls[(int64_t)a * p.B + b];
        const float* const d = p.deform + (int64_t)a * M * p.B + b;
        float* const gdef = p.grad_deform + (int64_t)a * M * p.B + b;
        double gbase = 0.0;
        if (p.basis == SB_BASIS_FOURIER) {
            double acc[2 * SB_MAX_FOURIER];
            for (int m = 0; m < M; ++m) acc[m] = 0.0;
            for (int f = 0; f < sc.n_frames; ++f) {
                const double ga = g[((int64_t)f * 5 + a) * nb];
                if (ga == 0.0) continue;
                double fb[2 * SB_MAX_FOURIER];
                fourier_basis(p.frame_t[sc.frame0 + f], N, fb);
                double h = 0.0;
                for (int m = 0; m < M; ++m) h = fma((double)d[(int64_t)m * p.B], fb[m], h);
                gbase += additive ? ga : ga * (1.0 + h);
                const double gs = additive ? ga : ga * base;
                for (int m = 0; m < M; ++m) acc[m] = fma(gs, fb[m], acc[m]);
            }
            for (int m = 0; m < M; ++m) gdef[(int64_t)m * p.B] = (float)acc[m];
        } else {
            // Eq. 2, one basis at a time: its three coefficients summed over the frames
            // (dL/dbase needs H, the sum over all bases, at every frame: a first pass)
            if (!additive) {
                for (int f = 0; f < sc.n_frames; ++f) {
                    const double ga = g[((int64_t)f * 5 + a) * nb];
                    if (ga == 0.0) continue;
                    gbase += ga * (1.0 + gauss_basis_H(d, p.B, N, p.frame_t[sc.frame0 + f]));
                }
            } else {
                for (int f = 0; f < sc.n_frames; ++f) gbase += g[((int64_t)f * 5 + a) * nb];
            }
            for (int n = 0; n < N; ++n) {
                const double w = d[(int64_t)(3 * n) * p.B];
                const double th = d[(int64_t)(3 * n + 1) * p.B];
                const double sg = d[(int64_t)(3 * n + 2) * p.B];
                double aw = 0.0, at = 0.0, as = 0.0;
                for (int f = 0; f < sc.n_frames; ++f) {
                    const double ga = g[((int64_t)f * 5 + a) * nb];
                    if (ga == 0.0) continue;
                    const double gs = additive ? ga : ga * base;
                    const double dt = (double)p.frame_t[sc.frame0 + f] - th;
                    const double e = exp(-dt * dt / (2.0 * sg * sg));
                    aw = fma(gs, e, aw);
                    at = fma(gs, w * e * dt / (sg * sg), at);
                    as = fma(gs, w * e * dt * dt / (sg * sg * sg), as);
                }
                gdef[(int64_t)(3 * n) * p.B] = (float)aw;
                gdef[(int64_t)(3 * n + 1) * p.B] = (float)at;
                gdef[(int64_t)(3 * n + 2) * p.B] = (float)as;
            }
        }
        p.grad_balls[(int64_t)a * p.B + b] = (float)gbase;
    }
}

hipError_t launch_chain_rule(const OpParams& p, hipStream_t st) {
    if (p.B <= 0) return hipSuccess;
    const int64_t blocks = (p.B + 255) / 256;
    hipLaunchKernelGGL(chain_rule_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p);
    return hipGetLastError();
}

// Deformed bases whose coefficients the adjoint kernels do not keep in registers (all
// but the 2-harmonic Fourier series) take the two-phase chain rule.
bool adjoint_two_phase(const OpParams& p) {
    return p.basis != SB_BASIS_STATIC && !(p.basis == SB_BASIS_FOURIER && p.M == 4);
}

// tc.ucap: residual row length; tc.nw: blocks per CU requested from the compiler (occupancy)
hipError_t launch_adjoint(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st) {
    if (kernel == SB_KERNEL_UNIFORM && tc.ucap == kPfxRow) {
        if (tc.nw == 2) return launch_adj_um<2>(p, st);
        if (tc.nw == 3) return launch_adj_um<3>(p, st);
        if (tc.nw == 4) return launch_adj_um<4>(p, st);
    }
    if (kernel == SB_KERNEL_GAUSS && tc.ucap == 384) {
        if (tc.nw == 2) return launch_adj_m<384, 2>(p, st);
        if (tc.nw == 3) return launch_adj_m<384, 3>(p, st);
        if (tc.nw == 4) return launch_adj_m<384, 4>(p, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace sb
