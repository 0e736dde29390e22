// Adjoint: gradient of 1/2 |y - d|^2 with respect to every ball attribute and
// deformation coefficient, given the residual y - d.
//
// Same work items and staging as the forward.  Each lane loads its sensor's
// residual samples [o, o + UCAP) into its LDS column, then for each
// wave-uniform ball gathers the residual over the ball's window and forms the
// derivative of the sampled trace with respect to the arrival time, the size
// and the pressure (summation by parts over the window boundaries, so each
// boundary is evaluated once).  The 64 lanes' contributions are reduced across
// the wave into per-ball accumulators in LDS; after the group, one thread per
// ball applies the chain rule through Eq. 1 (and Eq. 2 / the Fourier series)
// and adds the result to the global gradients.
//
// With dr_m = r_m - r_{m-1} (residual samples of the window, r_{-1} = r_W = 0)
// and in_m = [|x_m| < rho] decided in FP64:
//   uniform:  G_v = C sum Q_m dr_m,  G_tau = 2C sum in_m x_m dr_m,
//             G_rho = -2 rho C sum in_m dr_m
//   gaussian: G_v = -K S0,  G_tau = K/rho^2 S1,  G_rho = -2K/rho S0 - K/rho^3 S2,
//             S_n = sum x_m^n E_m dr_m
// and dL/dr = G_tau/delta - G_v/r, dL/dR_f = G_rho/delta, dL/dP_f = G_v/P_f,
// dL/dx_f = dL/dr (x_f - s)/r.

#include "sb_internal.hpp"

namespace sb {

__device__ inline float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int NW, int G, int UCAP, int KERNEL>
__global__ __launch_bounds__(64 * NW) void adjoint_kernel(OpParams p) {
    __shared__ BallF sball[G];
    __shared__ float tile[NW][UCAP][64];
    __shared__ float acc[G][5];
    __shared__ double sred[NW * 6];
    __shared__ double scen[3];

    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    float* col = &tile[wid][0][lane];

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const Item it = decode_item(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int gf = sc.frame0 + it.frame;
        const float t = p.frame_t[gf];
        __syncthreads();   // previous item's chain-rule readers of acc/sball are done
        for (int i = tid; i < G * 5; i += 64 * NW) (&acc[0][0])[i] = 0.f;
        int nb;
        stage_group<NW, G>(p, sc, it.group, t, sball, sred, scen, nb);

        const int s = it.sblock * 64 * NW + wid * 64 + lane;
        const bool active = s < p.S;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        if (active) { sx = p.sensors[s]; sy = p.sensors[p.S + s]; sz = p.sensors[2 * p.S + s]; }
        const int o = tile_origin(p, scen, sx, sy, sz, UCAP);
        const float* res_row = p.residual + ((int64_t)gf * p.S + (active ? s : 0)) * p.T;
        for (int k = 0; k < UCAP; ++k) {
            const int kg = o + k;
            col[k * 64] = (active && kg >= 0 && kg < p.T) ? res_row[kg] : 0.f;
        }

        for (int bi = 0; bi < nb; ++bi) {
            const BallF bl = sball[bi];
            if (bl.rho < 0.0) continue;
            float gx = 0.f, gy = 0.f, gz = 0.f, gR = 0.f, gP = 0.f;
            if (active) {
                const double dx = bl.x - sx, dy = bl.y - sy, dz = bl.z - sz;
                const PairWin<KERNEL> w = pair_window<KERNEL>(p, bl, dx, dy, dz);
                if (!w.ok) {
                    raise_flag(p.flags, SB_FLAG_GEOMETRY);
                } else if (w.in_range) {   // otherwise the window reads only zeros
                    const float rho = bl.rhof;
                    const int W = w.W;
                    const int tl = w.klo - o;
                    const bool in_tile = tl >= 0 && tl + W <= UCAP;
                    const float* c = col + (in_tile ? tl : 0) * 64;
                    float x = (float)w.a0;
                    float rp = 0.f;
                    float dLdr, dLdR, dLdP;
                    const float rf = (float)w.r;
                    if (KERNEL == SB_KERNEL_UNIFORM) {
                        // boundaries m_lo..m_hi lie strictly inside (-rho, rho)
                        const int m_lo = (int)floor(w.a0 - bl.rho) + 1;
                        const int m_hi = (int)ceil(w.a0 + bl.rho) - 1;
                        float Sw = 0.f, St = 0.f, Sr = 0.f;
                        for (int m = 0; m <= W; ++m) {
                            float rm = 0.f;
                            if (m < W) {
                                if (in_tile) rm = c[m * 64];
                                else {
                                    const int kg = w.klo + m;
                                    rm = (kg >= 0 && kg < p.T) ? res_row[kg] : 0.f;
                                }
                            }
                            const float dr = rm - rp;
                            rp = rm;
                            const bool in = (m >= m_lo) && (m <= m_hi);
                            const float q = in ? x : (m < m_lo ? rho : -rho);
                            Sw = fmaf(q * q, dr, Sw);
                            St = fmaf(in ? x : 0.f, dr, St);
                            Sr += in ? dr : 0.f;
                            x -= 1.f;
                        }
                        const float C = (float)((double)bl.amp * (double)p.delta / (4.0 * w.r));
                        const float Gv = C * Sw, Gt = 2.f * C * St, Gr = -2.f * rho * C * Sr;
                        dLdr = Gt / p.delta - Gv / rf;
                        dLdR = Gr / p.delta;
                        dLdP = (p.delta / (4.f * rf)) * Sw;
                    } else {
                        float S0 = 0.f, S1 = 0.f, S2 = 0.f;
                        const float ce = -1.f / (2.f * rho * rho);
                        for (int m = 0; m <= W; ++m) {
                            float rm = 0.f;
                            if (m < W) {
                                if (in_tile) rm = c[m * 64];
                                else {
                                    const int kg = w.klo + m;
                                    rm = (kg >= 0 && kg < p.T) ? res_row[kg] : 0.f;
                                }
                            }
                            const float dr = rm - rp;
                            rp = rm;
                            const float E = expf(x * x * ce) * dr;
                            S0 += E;
                            S1 = fmaf(x, E, S1);
                            S2 = fmaf(x * x, E, S2);
                            x -= 1.f;
                        }
                        const float Kr = rho * rho * p.delta / (2.f * rf);   // K / P_f
                        const float K = bl.amp * Kr;
                        const float Gv = -K * S0;
                        const float Gt = K / (rho * rho) * S1;
                        const float Ga = -2.f * K / rho * S0 - K / (rho * rho * rho) * S2;
                        dLdr = Gt / p.delta - Gv / rf;
                        dLdR = Ga / p.delta;
                        dLdP = -Kr * S0;
                    }
                    gx = dLdr * (float)(dx / w.r);
                    gy = dLdr * (float)(dy / w.r);
                    gz = dLdr * (float)(dz / w.r);
                    gR = dLdR;
                    gP = dLdP;
                }
            }
            gx = wave_sum(gx);
            gy = wave_sum(gy);
            gz = wave_sum(gz);
            gR = wave_sum(gR);
            gP = wave_sum(gP);
            if (lane < 5) {
                const float v = lane == 0 ? gx : lane == 1 ? gy : lane == 2 ? gz : lane == 3 ? gR : gP;
                atomicAdd(&acc[bi][lane], v);
            }
        }
        __syncthreads();

        // chain rule through Eq. 1 (and Eq. 2 / Fourier) for this frame
        double fb[2 * SB_MAX_FOURIER];
        if (p.basis == SB_BASIS_FOURIER) fourier_basis(t, p.n_terms, fb);
        const int64_t first = sc.ball0 + (int64_t)it.group * G;
        for (int i = tid; i < nb; i += 64 * NW) {
            if (sball[i].rho < 0.0) continue;
            const int64_t b = first + i;
            for (int a = 0; a < 5; ++a) {
                const float g = acc[i][a];
                const bool additive = (a < 3 && p.pos_mode == SB_POS_ADD);
                const float h = (float)eval_H(p, b, a, t, fb);
                unsafeAtomicAdd(p.grad_balls + (int64_t)a * p.B + b, additive ? g : g * (1.f + h));
                if (p.basis != SB_BASIS_STATIC) {
                    const float base = p.balls[(int64_t)a * p.B + b];
                    for (int m = 0; m < p.M; ++m) {
                        const float dh = eval_dH(p, b, a, m, t, fb);
                        unsafeAtomicAdd(p.grad_deform + ((int64_t)a * p.M + m) * p.B + b,
                                        additive ? g * dh : g * base * dh);
                    }
                }
            }
        }
    }
}

template <int NW, int G, int UCAP, int KERNEL>
static hipError_t launch_adj_t(const OpParams& p, hipStream_t st) {
    int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((adjoint_kernel<NW, G, UCAP, KERNEL>), dim3((unsigned)grid), dim3(64 * NW), 0,
                       st, p);
    return hipGetLastError();
}

hipError_t launch_adjoint(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st) {
    // the host's work decomposition (n_sblocks, n_groups) must match the instance
    if (kernel == SB_KERNEL_UNIFORM) {
        if (tc.nw == 4 && tc.g == 256 && tc.ucap == 64) return launch_adj_t<4, 256, 64, 0>(p, st);
        if (tc.nw == 2 && tc.g == 128 && tc.ucap == 96) return launch_adj_t<2, 128, 96, 0>(p, st);
        if (tc.nw == 4 && tc.g == 128 && tc.ucap == 64) return launch_adj_t<4, 128, 64, 0>(p, st);
    } else {
        if (tc.nw == 4 && tc.g == 128 && tc.ucap == 96) return launch_adj_t<4, 128, 96, 1>(p, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace sb
