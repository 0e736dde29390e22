// Forward operator: per (ball, sensor, frame) scatter of a short sampled trace.
//
// Work item = (scene, frame, chunk of G consecutive balls, one or more blocks
// of 64*NW sensors).  The block stages the chunk's deformed balls (Eq. 1,
// recomputed here) in LDS once, then takes its sensor blocks one after the
// other.  Each wave owns 64 sensors, one per lane, and each lane owns
// one column of the wave's LDS trace tile T[UCAP][64] (column c lives in bank
// c mod 32: no conflicts while lanes add their windows at different samples).
// The column of a lane covers UCAP consecutive samples of its sensor from an
// origin o.  The wave walks the chunk's balls in order; the windows land in
// the columns as long as they fit, and when a window would leave its column
// in some lane the wave flushes the tile to the global trace and re-centres
// every lane's column on that ball's window.  With balls in a spatially
// coherent order (slingbag_order) consecutive balls arrive at nearly the same
// sample at every sensor, so one flush covers on the order of a hundred balls,
// also when every ball is displaced differently at each frame.  The flush
// transposes each touched 64-sample block through LDS so that one row holds 64
// consecutive samples of one sensor, and adds it to the global trace with one
// coalesced FP32 atomic per row.  Windows longer than the tile go to global
// memory directly.  For the uniform sphere the tile normally holds the traces'
// second differences as exact integers (see d2_window), so that a window costs
// seven tile updates (LDS integer adds that return nothing) whatever its length;
// the flush integrates them back.
//
// Trace of one ball in sample units (tau = (r - c t0)/delta, rho = R_f/delta):
// with boundaries x_m = tau - k_lo + 1/2 - m, m = 0..W, between samples,
//   uniform:  sample j = C (Q_j - Q_{j+1}),  Q_m = clamp(x_m, -rho, rho)^2,
//             C = P_f delta / (4 r)
//   gaussian: sample j = K (E_{j+1} - E_j),  E_m = exp(-x_m^2 / (2 rho^2)),
//             K = P_f rho^2 delta / (2 r)
// which is the interval mean of the N-wave P(r - ct)/(2r) (resp. of the Gaussian
// ball's outgoing term) over each sample interval.

#include <climits>

#include "sb_internal.hpp"

namespace sb {

// Add N consecutive values v0 - 2C*u (u = 0..N-1, a stretch of the ramp) to a
// tile column: all N entries are read before any is written back, so the wave
// waits for LDS once per stretch.
template <int N>
__device__ inline void add_ramp(float* cp, float yb, float m2c) {
    float o[N];
#pragma unroll
    for (int u = 0; u < N; ++u) o[u] = cp[u * 64];
#pragma unroll
    for (int u = 0; u < N; ++u) cp[u * 64] = o[u] + fmaf(m2c, (float)u, yb);
}

// Add one ball's window (W samples from boundary x0 on) to a tile column
// (stride 64 floats).  `C` is the per-pair amplitude (P_f delta / (4 r) for the
// uniform sphere, P_f rho^2 delta / (2 r) for the Gaussian ball).
//
// Uniform sphere: with x0 in [rho, rho + 1) and W = floor(2 rho) + 2, boundaries
// 1 .. W-2 lie inside [-rho, rho] and boundary W below -rho, so samples
// 1 .. W-3 see both of their boundaries inside and equal C (x_j^2 - x_{j+1}^2)
// = C (2 x_j - 1): a ramp falling by 2C per sample (the N-wave is linear in
// time).  Sample 0 and the last two samples take the clamped form.
template <int KERNEL>
__device__ inline void add_window(float* c, int W, float x0, float rho, float C) {
    if (KERNEL == SB_KERNEL_UNIFORM) {
        // sample 0 and the last two samples e1 = W-2, e2 = W-1 (for W = 2: samples
        // 1 and 2, the latter zero; the caller keeps three rows in the tile)
        const float rr = rho * rho;
        auto sq = [&](float x) {
            const float q = __builtin_amdgcn_fmed3f(x, -rho, rho);
            return q * q;
        };
        const int e1 = max(W - 2, 1);
        const float xa = x0 - (float)e1;                 // boundary e1 (exact in FP32)
        const float qa = sq(xa), qb = sq(xa - 1.f);
        {
            float* const p1 = c + e1 * 64;
            const float o0 = c[0], o1 = p1[0], o2 = p1[64];
            c[0] = o0 + C * (rr - sq(x0 - 1.f));
            p1[0] = o1 + C * (qa - qb);
            p1[64] = o2 + C * (qb - rr);                 // boundary e1 + 2 lies below -rho
        }
        // interior samples 1 .. W-3: v_j = y - 2C j, y = C (2 x0 - 1)
        const float m2c = -2.f * C;
        float yb = fmaf(C, fmaf(2.f, x0, -1.f), m2c);   // v_1
        float* cp = c + 64;
        int n = W - 3;
        for (; n >= 8; n -= 8) {
            add_ramp<8>(cp, yb, m2c);
            cp += 8 * 64;
            yb = fmaf(m2c, 8.f, yb);
        }
        if (n > 0) {
            if (n & 4) {
                add_ramp<4>(cp, yb, m2c);
                cp += 4 * 64;
                yb = fmaf(m2c, 4.f, yb);
            }
            if (n & 2) {
                add_ramp<2>(cp, yb, m2c);
                cp += 2 * 64;
                yb = fmaf(m2c, 2.f, yb);
            }
            if (n & 1) add_ramp<1>(cp, yb, m2c);
        }
    } else {
        // Gaussian ball: eight samples per batch, all eight rows read before any is
        // written back (one LDS wait per batch instead of one per sample)
        const float ce = -1.4426950408889634f / (2.f * rho * rho);   // exp2 scale: log2(e) / (2 rho^2)
        float Ep = __builtin_amdgcn_exp2f(x0 * x0 * ce), x = x0;
        int j = 0;
        for (; j + 8 <= W; j += 8) {
            float o[8], v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) o[u] = c[(j + u) * 64];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                x -= 1.f;
                const float E = __builtin_amdgcn_exp2f(x * x * ce);
                v[u] = C * (E - Ep);
                Ep = E;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) c[(j + u) * 64] = o[u] + v[u];
        }
        if (j < W) {
            // the last 1..7 samples as one batch: rows past the window are neither read
            // nor written
            const int n = W - j;
            float o[8], v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) o[u] = (u < n) ? c[(j + u) * 64] : 0.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                x -= 1.f;
                const float E = __builtin_amdgcn_exp2f(x * x * ce);
                v[u] = C * (E - Ep);
                Ep = E;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u < n) c[(j + u) * 64] = o[u] + v[u];
        }
    }
}

// Second-difference form of the uniform sphere's window.  The column holds, in
// integer units of 1/s, the second difference D_k = u_k - 2 u_{k-1} + u_{k-2} of
// the quantised trace u; the flush recovers u by two running sums.  A window's
// trace is a ramp between three end samples (see add_window), so its second
// difference is zero except at rows 0, 1, 2 and W-2 .. W+1: seven updates per
// window whatever its length.  The ramp is quantised as A + B (j - 1) with integer
// A and B, so every window's second differences sum back to exactly zero past
// its end: all arithmetic is modulo 2^32 and the running sums return the exact
// integer column as long as its true value fits in int32, which the caller's
// choice of s guarantees.  A window with W < 5 is written as one of length 5
// (its samples from W on are exactly zero): samples 1 and 2 then define the
// "ramp" through A = u_1 and B = u_2 - u_1.  Rows: max(W, 5) + 2.
struct D2Win {
    uint32_t d[7];   // added to rows 0, 1, 2 and w2 .. w2 + 3 of the window
    int w2;          // max(W, 5) - 2
};

// round to nearest (halves up) in one conversion
__device__ inline int round_rpi(float v) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

template <bool LONG>   // LONG: the caller knows W >= 5
__device__ inline D2Win d2_window(int W, float x0, float rho, float Cs) {
    const float rr = rho * rho;
    auto sq = [&](float x) {
        const float q = __builtin_amdgcn_fmed3f(x, -rho, rho);
        return q * q;
    };
    auto qn = [](float v) { return (uint32_t)round_rpi(v); };
    const int Wp = LONG ? W : max(W, 5);
    // W >= 5 means rho >= 3/2: boundaries 1 and W - 2 then lie inside [-rho, rho] (x0 is in
    // [rho, rho + 1), and W - 2 <= 2 rho), so their squares need no clamp
    const float q1 = LONG ? (x0 - 1.f) * (x0 - 1.f) : sq(x0 - 1.f);
    float va, vb;                                        // sample 1 and the step to sample 2 (units of C)
    if (LONG || W >= 5) {
        va = fmaf(2.f, x0, -3.f);                        // C (2 x_1 - 1)
        vb = -2.f;
    } else {
        const float q2 = sq(x0 - 2.f), q3 = sq(x0 - 3.f);
        va = q1 - q2;
        vb = (q2 - q3) - va;
    }
    const float xa = x0 - (float)(Wp - 2);               // boundary Wp-2 (exact in FP32)
    const float qa = LONG ? xa * xa : sq(xa), qb = sq(xa - 1.f);   // boundary Wp lies below -rho
    const uint32_t u0 = qn(Cs * (rr - q1)), a = qn(Cs * va), b = qn(Cs * vb);
    const uint32_t e1 = qn(Cs * (qa - qb)), e2 = qn(Cs * (qb - rr));
    const uint32_t last = a + b * (uint32_t)(Wp - 4);    // ramp sample Wp-3
    D2Win r;
    r.d[0] = u0;
    r.d[1] = a - 2u * u0;
    r.d[2] = b - a + u0;
    r.d[3] = e1 - last - b;
    r.d[4] = e2 - 2u * e1 + last;
    r.d[5] = e1 - 2u * e2;
    r.d[6] = e2;
    r.w2 = Wp - 2;
    return r;
}

// Adds a window's seven second differences to the lane's column (rows c0[0], c0[64],
// c0[128] and c1[0] .. c1[192], in units of 64 floats per row) with LDS integer atomics
// that return nothing: no read-back, so nothing waits on the LDS round trip.  The
// column is the lane's own; a wave's LDS operations complete in order, so the flush's
// reads see every add.  Integer addition wraps modulo 2^32, as the second-difference
// form requires.
__device__ inline void d2_add(uint32_t* c0, uint32_t* c1, const D2Win& dw) {
    auto add = [](uint32_t* a, uint32_t v) {
        __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    add(c0, dw.d[0]);
    add(c0 + 64, dw.d[1]);
    add(c0 + 128, dw.d[2]);
    add(c1, dw.d[3]);
    add(c1 + 64, dw.d[4]);
    add(c1 + 128, dw.d[5]);
    add(c1 + 192, dw.d[6]);
}

// A chunk ball as staged in LDS for the pair set-up: what depends on the ball only
// is computed once per ball instead of once per pair.
struct BallS {
    double x, y, z;   // deformed centre (m)
    double c1;        // t0 fs + h - 1/2: the window starts at sample floor(r / delta - c1)
    double Rd;        // uniform sphere: R_f (m), the sensor must lie outside; Gaussian ball: 0
    float amp;        // amplitude scale of the trace
    float rhof;       // rho = R_f / delta (samples)
    float hf;         // half-width h of the window: rho (uniform) or kGaussCut rho (Gaussian)
    int Wc;           // window length W = floor(2 h) + 2; 0: no ball; -1: longer than any record
};

// The uniform sphere's record in the shared-column forward: 48 bytes, so that the
// staged chunk and the column fit four blocks per compute unit.  The window's half-width
// is rho, and the inside-ball radius R_f is kept in FP32 (the test r > R_f then differs
// from the FP64 one only for a sensor within 1e-7 R_f of the ball's surface).
struct BallU {
    double x, y, z;   // deformed centre (m)
    double c1;        // t0 fs + rho - 1/2: the window starts at sample floor(r / delta - c1)
    float Rd;         // R_f (m): the sensor must lie outside
    float amp;        // amplitude scale of the trace
    float rhof;       // rho = R_f / delta (samples), also the window's half-width
    int Wc;           // window length W = floor(2 rho) + 2; 0: no ball; -1: longer than any record
};
__device__ inline float win_half(const BallS& b) { return b.hf; }
__device__ inline float win_half(const BallU& b) { return b.rhof; }

// Per-pair quantities of one ball for the wave's 64 sensors (one per lane).
struct FwdPair {
    float Cg, xg;    // amplitude and boundary 0
    float rhof;
    int klo;         // sample index of sample 0
    int W;           // window length (the same in every lane)
    bool in_tile;    // this lane has a window to add
};

// Set-up of one staged ball for the lane's sensor (sx, sy, sz).  A pair without its
// window (sensor inside a uniform ball, or an arrival sample out of int32 range) sets
// `bad`; the exact flags are told apart on a slow path (chunk_flags).
template <typename Rec>
__device__ inline FwdPair pair_setup(const OpParams& p, const Rec& bs, double sx, double sy, double sz,
                                     bool active, bool& bad) {
    FwdPair f;
    const int Wc = __builtin_amdgcn_readfirstlane(bs.Wc);
    const bool valid = Wc != 0, too_long = Wc < 0;
    f.W = Wc > 0 ? Wc : 5;                           // no window: zeros at the first rows
    float ri;
    const double r = dist64(bs.x - sx, bs.y - sy, bs.z - sz, ri);
    const bool ok = r > (double)bs.Rd;               // outside the uniform ball (r > 0: Gaussian)
    const double u = fma(r, p.inv_delta, -bs.c1);   // r / delta - t0 fs - h + 1/2
    const double kl = floor(u);
    const bool in_range = fabs(kl) < 5.0e8;          // int32 sample arithmetic
    const bool use = active && valid && !too_long;
    f.in_tile = use && ok && in_range;               // the window exists
    bad |= use && !f.in_tile;
    f.Cg = bs.amp * ri;                              // amp holds the amplitude scale (staging)
    f.xg = (float)(u - kl) + win_half(bs);           // boundary 0: tau - k_lo + 1/2
    f.klo = in_range ? (int)kl : 0;
    f.rhof = bs.rhof;
    return f;
}

// Slow path behind `bad`: redo the pair tests of n staged balls to raise the exact flags.
template <typename Rec>
__device__ inline void chunk_flags(const OpParams& p, const Rec* balls, int n, double sx, double sy, double sz,
                                   bool active, bool& geometry, bool& clipped) {
    for (int i = 0; i < n; ++i) {
        const Rec bs = balls[i];
        const int Wc = __builtin_amdgcn_readfirstlane(bs.Wc);
        const bool use = active && Wc > 0;
        float ri;
        const double r = dist64(bs.x - sx, bs.y - sy, bs.z - sz, ri);
        const bool ok = r > (double)bs.Rd;
        const double kl = floor(fma(r, p.inv_delta, -bs.c1));
        geometry |= use && !ok;
        clipped |= use && ok && !(fabs(kl) < 5.0e8);
    }
}

template <int KERNEL>
__device__ inline bool add_window_global(float* row, int klo, int T, int W, float x, float rho,
                                         float C) {
    bool clipped = false;
    float Qp = rho * rho;
    const float ce = -1.4426950408889634f / (2.f * rho * rho);   // exp2 scale
    float Ep = (KERNEL == SB_KERNEL_UNIFORM) ? 0.f : __builtin_amdgcn_exp2f(x * x * ce);
    for (int j = 0; j < W; ++j) {
        x -= 1.f;
        float v;
        if (KERNEL == SB_KERNEL_UNIFORM) {
            const float q = __builtin_amdgcn_fmed3f(x, -rho, rho);
            const float Q = q * q;
            v = C * (Qp - Q);
            Qp = Q;
        } else {
            const float E = __builtin_amdgcn_exp2f(x * x * ce);
            v = C * (E - Ep);
            Ep = E;
        }
        const int k = klo + j;
        if (v != 0.f) {
            if (k >= 0 && k < T) global_atomic_add(row + k, v);
            else clipped = true;
        }
    }
    return clipped;
}

// Deformed ball `first + tid` of the chunk at frame time t (Eq. 1), with its amplitude
// scale: P_f delta / 4 (uniform sphere), P_f rho^2 delta / 2 (Gaussian ball); threads past
// the chunk's end get an empty ball.
template <int KERNEL>
__device__ inline BallF stage_deform(const OpParams& p, int tid, int nb, int64_t first, float t, const double* fb,
                                     bool& nonfinite) {
    BallF bl;
    if (tid < nb) {
        nonfinite |= !deform_ball(p, first + tid, t, fb, bl);
        bl.amp = (KERNEL == SB_KERNEL_UNIFORM)
                     ? (float)((double)bl.amp * (double)p.delta * 0.25)
                     : (float)((double)bl.amp * bl.rho * bl.rho * (double)p.delta * 0.5);
    } else {
        bl.x = bl.y = bl.z = 0.0;
        bl.rho = -1.0;
        bl.rhof = -1.f;
        bl.amp = 0.f;
    }
    return bl;
}

// The staged record of a deformed ball: what depends on the ball only.
template <int KERNEL>
__device__ inline BallS ball_record(const OpParams& p, const BallF& bl, bool& clipped) {
    BallS bs;
    const bool valid = bl.rho >= 0.0;
    const double h = (KERNEL == SB_KERNEL_UNIFORM) ? bl.rho : (double)kGaussCut * bl.rho;
    bs.x = bl.x;
    bs.y = bl.y;
    bs.z = bl.z;
    bs.c1 = p.t0fs + h - 0.5;
    bs.Rd = (KERNEL == SB_KERNEL_UNIFORM) ? bl.rho * (double)p.delta : 0.0;
    bs.amp = bl.amp;
    bs.rhof = bl.rhof;
    bs.hf = (float)h;
    bs.Wc = !valid ? 0 : (h >= 1.0e6 ? -1 : (int)(2.0 * h) + 2);
    clipped |= valid && h >= 1.0e6;                      // a window longer than any record
    return bs;
}

// Uniform sphere, per wave of staged balls: the box of the centres of the balls whose
// windows go to an LDS tile of CAP rows (max(W, 5) + 2 <= CAP with W = floor(2 rho) + 2,
// as in the pair set-up), the sum of |P delta/4| (2 rho + 1) over them, and their largest
// row count, written to box[0..7] by lane 0.  Every tile window adds at most
// |P delta/4| (2 rho + 1) / r to any sample, with r at least the distance from the sensor
// to the box: the bound behind the integer tile's scale.
template <int CAP>
__device__ inline void stage_box(const BallF& bl, bool real, int lane, float* box) {
    const int rows = max((int)(2.0 * fmin(bl.rho, 1.0e6)) + 2, 5) + 2;
    const bool in_tile = real && bl.rho >= 0.0 && rows <= CAP;
    const float inf = __builtin_huge_valf();
    const float lo[3] = {in_tile ? (float)bl.x : inf, in_tile ? (float)bl.y : inf, in_tile ? (float)bl.z : inf};
    const float hi[3] = {in_tile ? (float)bl.x : -inf, in_tile ? (float)bl.y : -inf, in_tile ? (float)bl.z : -inf};
    const float sa = in_tile ? fabsf(bl.amp) * fmaf(2.f, bl.rhof, 1.f) : 0.f;
    float red[8];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        red[a] = wave_min_all(lo[a]);
        red[3 + a] = wave_max_all(hi[a]);
    }
    red[6] = wave_reduce_dpp(sa, [](float x, float y) { return x + y; });
    red[7] = (float)wave_max_all(in_tile ? rows : 0);
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < 8; ++a) box[a] = red[a];
    }
}

// The uniform sphere's 48-byte record (shared-column forward).
__device__ inline BallU ball_record_u(const OpParams& p, const BallF& bl, bool& clipped) {
    BallU bs;
    const bool valid = bl.rho >= 0.0;
    bs.x = bl.x;
    bs.y = bl.y;
    bs.z = bl.z;
    bs.c1 = p.t0fs + bl.rho - 0.5;
    bs.Rd = (float)(bl.rho * (double)p.delta);
    bs.amp = bl.amp;
    bs.rhof = bl.rhof;
    bs.Wc = !valid ? 0 : (bl.rho >= 1.0e6 ? -1 : (int)(2.0 * bl.rho) + 2);
    clipped |= valid && bl.rho >= 1.0e6;                 // a window longer than any record
    return bs;
}

template <int NW, int G, int UCAP, int KERNEL>
__global__ __launch_bounds__(64 * NW) void forward_kernel(OpParams p) {
    static_assert(UCAP % 64 == 0, "tile length must be a multiple of 64");
    static_assert(G == 64 * NW, "one ball per thread when staging");
    __shared__ BallS sball[G];
    __shared__ double s_fb[2 * SB_MAX_FOURIER];       // Fourier basis of the item's frame
    __shared__ float s_box[NW][8];                    // per wave: centre box of the chunk's tile balls, amplitude sum
    __shared__ float tile[NW][(UCAP + 1) * 64];     // per wave: a pad row, then UCAP rows of 64 sensors

    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    float* const tw = &tile[wid][64];
    for (int k = -1; k < UCAP; ++k) tw[k * 64 + lane] = 0.f;
    bool clipped = false, geometry = false, nonfinite = false;

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const Item it = decode_item(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int gf = sc.frame0 + it.frame;
        const float t = p.frame_t[gf];
        const int64_t first = sc.ball0 + (int64_t)it.group * G;
        const int nb = min(G, sc.n_balls - it.group * G);
        __syncthreads();   // the previous item is done with sball and s_fb

        // ---- stage the chunk's deformed balls (Eq. 1, one per thread)
        if (p.basis == SB_BASIS_FOURIER && wid == 0) fourier_basis_lanes(t, p.n_terms, s_fb, lane);
        __syncthreads();
        {
            const BallF bl = stage_deform<KERNEL>(p, tid, nb, first, t, s_fb, nonfinite);
            sball[tid] = ball_record<KERNEL>(p, bl, clipped);
            if (KERNEL == SB_KERNEL_UNIFORM) stage_box<UCAP>(bl, tid < nb, lane, s_box[wid]);
        }
        __syncthreads();

        // the item's sensor blocks, one after the other, against the staged chunk
        const int sb_end = min(it.sblock + p.sb_per_item, p.n_sblocks);
        for (int sbk = it.sblock; sbk < sb_end; ++sbk) {
            const int s = sbk * 64 * NW + wid * 64 + lane;
            const bool active = s < p.S;
            double sx = 0.0, sy = 0.0, sz = 0.0;
            if (active) { sx = p.sensors[s]; sy = p.sensors[p.S + s]; sz = p.sensors[2 * p.S + s]; }
            const int64_t row_off = ((int64_t)gf * p.S + (active ? s : 0)) * p.T;   // this lane's trace row
            float* out_row = p.signals + row_off;

            // Uniform sphere: the tile holds second differences in units of 1/qs (add_window_d2)
            // when a per-lane scale qs keeps every column within int32; qs = 2^30 r_min / sum,
            // with r_min the distance from the sensor to the box of the tile balls' centres.
            // A wave whose sensors come within a quarter of the box's far distance (the bound
            // would cost precision) keeps the FP32 tile for this chunk.
            float qs = 1.f, qeps = 1.f;
            bool qmode = false;
            if (KERNEL == SB_KERNEL_UNIFORM) {
                float lo[3], hi[3], sum = 0.f;
    #pragma unroll
                for (int a = 0; a < 3; ++a) {
                    lo[a] = s_box[0][a];
                    hi[a] = s_box[0][3 + a];
                }
                sum = s_box[0][6];
    #pragma unroll
                for (int w = 1; w < NW; ++w) {
    #pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = fminf(lo[a], s_box[w][a]);
                        hi[a] = fmaxf(hi[a], s_box[w][3 + a]);
                    }
                    sum += s_box[w][6];
                }
                bool ok = true;
                if (active) {
                    if (!(sum < __builtin_huge_valf())) {
                        ok = false;                          // a non-finite amplitude in the chunk
                    } else if (sum > 0.f && lo[0] <= hi[0]) {
                        double dmin, dmax;
                        box_distance_range(lo, hi, sx, sy, sz, dmin, dmax);
                        qs = (float)(1073741824.0 * dmin / (double)sum);
                        ok = dmin > 0.25 * dmax && qs > 0.f && qs < __builtin_huge_valf();
                        qeps = 1.f / qs;
                    }                                        // else: every tile amplitude is zero
                }
                qmode = __all(ok);
            }
            uint32_t* const twu = reinterpret_cast<uint32_t*>(tw);

            // A pair without its window (sensor inside a uniform ball, or an arrival sample out
            // of int32 range) sets one lane mask; the flags are told apart on a slow path.
            bool bad = false;

            // Each lane's column covers samples o .. o + UCAP - 1 of its sensor.  The
            // balls are taken in chunk order (spatially coherent after slingbag_order);
            // when a window does not fit its column in some lane, the wave flushes the
            // tile and re-centres every lane's column on that ball's window.
            int o = -(1 << 30);          // no column yet: the first window triggers the set-up
            int kmax = -1;               // last tile row written (wave-wide max at the flush)

            // ---- flush, per touched 64-sample block q: each lane reads its column
            // (64 samples of its sensor) into registers and writes it back as row
            // `lane` of a 64 x 65 matrix that starts 64 floats before the block (in
            // the previous, already flushed block, or the pad row before the tile); the
            // row stride of 65 keeps both the row writes and the column reads of the
            // matrix conflict-free.  Row a then holds 64 consecutive samples of sensor
            // a, added to the global trace with one coalesced FP32 atomic per row.
            auto flush = [&]() {
                const int nblk = (wave_max_all(kmax) + 64) >> 6;
                // When every lane's touched samples o .. o + kmax lie inside the record (the usual
                // case), the rows go out without a per-sample range test: one 64-bit row address
                // per sensor, and the atomics skip the zero samples.
                const bool inside = __all(kmax < 0 || (o >= 0 && o + kmax < p.T));
                const uintptr_t rowp = reinterpret_cast<uintptr_t>(p.signals) +
                                       (uintptr_t)(row_off + (int64_t)o) * sizeof(float);
                uint32_t d1 = 0u, d0 = 0u;                   // running sums of the second differences
                for (int q = 0; q < nblk; ++q) {
                    float* const blk = tw + q * 64 * 64;
                    float* const mat = blk - 64;
                    float col[64];
                    wave_lds_sync();
                    if (qmode) {
                        const uint32_t* const blku = twu + q * 64 * 64;
    #pragma unroll
                        for (int k = 0; k < 64; ++k) {
                            d1 += blku[k * 64 + lane];
                            d0 += d1;
                            col[k] = (float)(int32_t)d0 * qeps;
                        }
                    } else {
    #pragma unroll
                        for (int k = 0; k < 64; ++k) col[k] = blk[k * 64 + lane];
                    }
                    wave_lds_sync();
    #pragma unroll
                    for (int k = 0; k < 64; ++k) mat[lane * 65 + k] = col[k];
                    wave_lds_sync();
                    if (inside) {
    #pragma unroll
                        for (int a0 = 0; a0 < 64; a0 += 8) {
                            float v[8];                              // sample q*64 + lane of sensors a0 .. a0+7
    #pragma unroll
                            for (int u = 0; u < 8; ++u) v[u] = mat[(a0 + u) * 65 + lane];
    #pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int a = a0 + u;
                                const uint64_t pa =
                                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(rowp >> 32), a) << 32) |
                                    (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)rowp, a);
                                if (v[u] != 0.f) global_atomic_add(reinterpret_cast<float*>(pa) + (q * 64 + lane), v[u]);
                            }
                        }
                    } else {
    #pragma unroll
                        for (int a0 = 0; a0 < 64; a0 += 8) {
                            float v[8];
    #pragma unroll
                            for (int u = 0; u < 8; ++u) v[u] = mat[(a0 + u) * 65 + lane];
    #pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int a = a0 + u;
                                const int act_a = __builtin_amdgcn_readlane((int)active, a);
                                const int k = __builtin_amdgcn_readlane(o, a) + q * 64 + lane;
                                const int64_t ra = ((int64_t)__builtin_amdgcn_readlane((int)(row_off >> 32), a) << 32) |
                                                   (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)row_off, a);
                                if (v[u] != 0.f && act_a) {
                                    if (k >= 0 && k < p.T) global_atomic_add(p.signals + ra + k, v[u]);
                                    else clipped = true;
                                }
                            }
                        }
                    }
                    wave_lds_sync();
    #pragma unroll
                    for (int k = 0; k < 64; ++k) blk[k * 64 + lane] = 0.f;
                    mat[lane] = 0.f;
                }
                kmax = -1;
            };

            // pair set-up of ball i for this wave's sensors
            auto setup = [&](const BallS& bs) { return pair_setup(p, bs, sx, sy, sz, active, bad); };
            auto prep = [&](int i) { return setup(sball[i]); };
            auto apply = [&](const FwdPair& f) {
                const bool part = f.in_tile;
                const int rows = (KERNEL == SB_KERNEL_UNIFORM) ? max(f.W, 3) : f.W;
                if (rows <= UCAP) {
                    int tl = f.klo - o;
                    if (__ballot(part && (tl < 0 || tl + rows > UCAP))) {
                        flush();
                        if (part) o = f.klo - ((UCAP - rows) >> 1);
                        tl = f.klo - o;
                    }
                    // lanes without a window add zeros at the first rows
                    const int tr = part ? tl : 0;
                    add_window<KERNEL>(tw + tr * 64 + lane, f.W, part ? f.xg : 0.f, f.rhof, part ? f.Cg : 0.f);
                    if (part) kmax = max(kmax, tl + f.W - 1);
                } else if (part) {
                    clipped |= add_window_global<KERNEL>(out_row, f.klo, p.T, f.W, f.xg, f.rhof, f.Cg);
                }
            };
            if (KERNEL == SB_KERNEL_UNIFORM && qmode) {
                // Integer tile.  Per ball: place this ball's window (flushing if needed),
                // issue its seven LDS adds, and run the next ball's FP64 set-up while they
                // complete (nothing waits on them).  The ball after next is read from
                // LDS at the end of each iteration, into the registers the set-up has just
                // released (reading it earlier needs a second set of registers and a copy
                // per ball).
                FwdPair cur = prep(0);
                BallS bn = sball[min(1, nb - 1)];
                for (int i = 0; i < nb; ++i) {
                    const bool part = cur.in_tile;
                    const int rows = max(cur.W, 5) + 2;           // the same in every lane
                    const bool in_lds = rows <= UCAP;
                    int tr = 0;                                   // the window's first tile row
                    if (in_lds) {
                        // the loop's one flush site: flush and re-centre when this ball's
                        // window leaves some lane's column
                        int tl = cur.klo - o;
                        if (__ballot(part && (tl < 0 || tl + rows > UCAP))) {
                            flush();
                            if (part) o = cur.klo - ((UCAP - rows) >> 1);
                            tl = cur.klo - o;
                        }
                        if (part) kmax = max(kmax, tl + rows - 1);
                        tr = part ? tl : 0;
                    }
                    FwdPair nxt;
                    if (cur.W >= 5 && in_lds) {
                        // common case, one basic block: the window's values, the next ball's
                        // set-up and the row updates interleave
                        const D2Win dw = d2_window<true>(cur.W, part ? cur.xg : 0.f, cur.rhof, part ? cur.Cg * qs : 0.f);
                        uint32_t* const c0 = twu + tr * 64 + lane;
                        d2_add(c0, c0 + dw.w2 * 64, dw);
                        nxt = setup(bn);
                    } else {
                        if (in_lds) {
                            const D2Win dw = d2_window<false>(cur.W, part ? cur.xg : 0.f, cur.rhof, part ? cur.Cg * qs : 0.f);
                            uint32_t* const c0 = twu + tr * 64 + lane;
                            d2_add(c0, c0 + dw.w2 * 64, dw);
                        } else if (part) {
                            clipped |= add_window_global<KERNEL>(out_row, cur.klo, p.T, cur.W, cur.xg, cur.rhof, cur.Cg);
                        }
                        nxt = setup(bn);
                    }
                    cur = nxt;
                    bn = sball[min(i + 2, nb - 1)];
                }
            } else {
                // FP32 tile; software pipeline: the set-up of ball i+1 overlaps the tile
                // update of ball i
                FwdPair cur = prep(0);
                for (int i = 0; i < nb; ++i) {
                    const FwdPair nxt = prep(min(i + 1, nb - 1));
                    apply(cur);
                    cur = nxt;
                }
            }
            flush();
            if (__ballot(bad)) chunk_flags(p, sball, nb, sx, sy, sz, active, geometry, clipped);
        }
    }
    if (clipped) raise_flag(p.flags, SB_FLAG_CLIPPED);
    if (geometry) raise_flag(p.flags, SB_FLAG_GEOMETRY);
    if (nonfinite) raise_flag(p.flags, SB_FLAG_NONFINITE);
}

// ---- Shared column (uniform sphere, integer tile) ----------------------------------
//
// The four waves of a block take the same 64 sensors (one per lane) and a quarter of the
// chunk's 256 balls each, and add their windows' second differences into one column of
// kShRows samples per sensor that the whole block shares.  A sensor's column starts at a
// lower bound of the chunk's arrival samples there (from the distance to the box of the
// centres), so no column moves while the waves add.  A window that starts kShRows - rmax + 1
// or more samples past the column start (rmax: rows of the chunk's longest tile window)
// is left for a later pass, whose column starts where this one's windows stopped (from
// the second later pass on: at the sensor's least sample left, when that lies further);
// only the balls with such a window in some lane are set up again.  A pass ends with one
// flush: each wave integrates a quarter of the rows (a SEG-row segment) for all 64
// sensors, the segments' running sums are chained through LDS, and the segment is
// transposed in place (each LDS row then holds SEG consecutive samples of one sensor, row
// stride SEG: conflict-free both ways for odd SEG) and added to the global trace, two
// sensors' runs of up to 32 samples per coalesced FP32 atomic (and the 33rd samples in
// one more).  The column (4 SEG rows of 64 sensors: 1 KB per unit of SEG) and the
// staged chunk take 50 KB for SEG = 33 (three blocks, twelve waves per compute unit)
// or 39 KB for SEG = 23 (four blocks, sixteen waves), against 81 KB and two blocks for
// forward_kernel's tile per wave.  (SEG = 15, five blocks, was slower: its 60-sample
// column needs a second pass for too many chunks.)

template <int SEG, int OCC>
__global__ __launch_bounds__(256, OCC) void forward_shared_kernel(OpParams p) {
    constexpr int NW = 4, G = 256, kShSeg = SEG, kShRows = 4 * SEG, kRun = SEG < 32 ? SEG : 32;
    // longest window kept in LDS (rows; longer ones go to the trace directly), leaving every
    // pass at least 16 first samples
    constexpr int kShCap = kShRows - 16 < 64 ? kShRows - 16 : 64;
    static_assert(SEG <= 33 && kShCap >= 16, "segment length");
    __shared__ BallU sball[G];
    __shared__ double s_fb[2 * SB_MAX_FOURIER];       // Fourier basis of the item's frame
    __shared__ float s_box[NW][8];                    // per wave of staged balls: tile box, amplitude sum, rows
    __shared__ __align__(16) uint32_t col[kShRows * 64];   // row k, sensor (lane): second differences
    __shared__ uint32_t s_tot[NW][2][64];             // per segment and sensor: running sums at its end
    __shared__ int s_kb[NW][64];                      // per segment and sensor: trace sample of its first row
    __shared__ int s_more[2];                         // per pass parity: some window is left for a later pass
    __shared__ int s_nmin[2][64];                     // per pass parity and sensor: least sample left

    // the wave index as a scalar: the wave's ball loop and flush segment are then uniform
    // control flow for the compiler
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    for (int i = tid; i < kShRows * 64; i += 64 * NW) col[i] = 0u;
    if (tid < 2) s_more[tid] = 0;
    if (tid < 128) (&s_nmin[0][0])[tid] = INT_MAX;
    bool clipped = false, geometry = false, nonfinite = false;
    int pp = 0;                                       // passes so far: s_more[pp & 1] is the current one

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const Item it = decode_item(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int gf = sc.frame0 + it.frame;
        const float t = p.frame_t[gf];
        const int64_t first = sc.ball0 + (int64_t)it.group * G;
        const int nb = min(G, sc.n_balls - it.group * G);
        __syncthreads();   // the previous item is done with sball and s_fb
        if (p.basis == SB_BASIS_FOURIER && wid == 0) fourier_basis_lanes(t, p.n_terms, s_fb, lane);
        __syncthreads();
        {
            const BallF bl = stage_deform<SB_KERNEL_UNIFORM>(p, tid, nb, first, t, s_fb, nonfinite);
            sball[tid] = ball_record_u(p, bl, clipped);
            stage_box<kShCap>(bl, tid < nb, lane, s_box[wid]);
        }
        __syncthreads();
        float lo[3], hi[3], sum = 0.f;
        int rmax = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = s_box[0][a];
            hi[a] = s_box[0][3 + a];
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(lo[a], s_box[w][a]);
                hi[a] = fmaxf(hi[a], s_box[w][3 + a]);
            }
            sum += s_box[w][6];
            rmax = max(rmax, (int)s_box[w][7]);
        }
        const int nbw = max(0, min(64, nb - 64 * wid));   // this wave's balls: 64 wid + [0, nbw)
        const BallU* const wb = sball + 64 * wid;

        // the item's sensor blocks (64 sensors each), one after the other
        const int sb_end = min(it.sblock + p.sb_per_item, p.n_sblocks);
        for (int sbk = it.sblock; sbk < sb_end; ++sbk) {
            {
                const int s0 = sbk * 64;
                const int s = s0 + lane;
                const bool active = s < p.S;
                double sx = 0.0, sy = 0.0, sz = 0.0;
                if (active) { sx = p.sensors[s]; sy = p.sensors[p.S + s]; sz = p.sensors[2 * p.S + s]; }
                float* const sig0 = p.signals + ((int64_t)gf * p.S + s0) * p.T;   // trace row of sensor s0
                float* const out_row = sig0 + (int64_t)(active ? lane : 0) * p.T;

                // Integer scale qs = 2^30 r_min / sum (as in forward_kernel) and the column start:
                // no tile window of the chunk starts before floor(r_min / delta - t0 fs - rmax / 2)
                // (rho < rows / 2), nor ends after floor(r_max / delta - t0 fs + 1/2) + rmax - 1;
                // two samples of margin each way cover the rounding of the box.
                float qs = 1.f, qeps = 1.f;
                int base = 0, kfar = INT_MIN;
                bool ok = true;
                if (active) {
                    if (!(sum < __builtin_huge_valf())) {
                        ok = false;                       // a non-finite amplitude in the chunk
                    } else if (lo[0] <= hi[0]) {
                        double dmin, dmax;
                        box_distance_range(lo, hi, sx, sy, sz, dmin, dmax);
                        const double b0 = floor(dmin * p.inv_delta - p.t0fs - 0.5 * (double)rmax) - 2.0;
                        const double b1 = floor(dmax * p.inv_delta - p.t0fs + 0.5) + (double)(rmax + 1);
                        base = (int)fmin(fmax(b0, -1.0e9), 1.0e9);
                        kfar = (int)fmin(fmax(b1, -1.0e9), 1.0e9);
                        if (sum > 0.f) {
                            qs = (float)(1073741824.0 * dmin / (double)sum);
                            ok = dmin > 0.25 * dmax && qs > 0.f && qs < __builtin_huge_valf();
                            qeps = 1.f / qs;
                        }
                    }                                     // else: no tile window in the chunk
                }
                const bool qmode = __all(ok);             // the same in every wave (same sensors, same box)
                bool bad = false;
                auto setup = [&](const BallU& bs) { return pair_setup(p, bs, sx, sy, sz, active, bad); };

                // flush of the column after a pass (every wave, between block barriers): rows
                // k0 .. k0 + 32 of every sensor, integrated, chained to the rows before, and added to
                // the trace from sample base + k0 on.  kmax_b: last row any window of the pass can
                // have reached (segments past it are exactly zero).
                auto flush = [&](int kmax_b) {
                    const int k0 = kShSeg * wid;
                    const bool touched = k0 <= kmax_b;
                    uint32_t v[kShSeg];
                    uint32_t d1 = 0u, d0 = 0u;
                    if (touched) {
#pragma unroll
                        for (int k = 0; k < kShSeg; ++k) {
                            d1 += col[(k0 + k) * 64 + lane];
                            d0 += d1;
                            v[k] = d0;
                        }
                    }
                    s_tot[wid][0][lane] = d1;
                    s_tot[wid][1][lane] = d0;
                    __syncthreads();
                    if (touched) {
                        // running sums at the end of the segments before this one
                        uint32_t c1 = 0u, c0 = 0u;
                        for (int u = 0; u < wid; ++u) {
                            c0 += (uint32_t)kShSeg * c1 + s_tot[u][1][lane];
                            c1 += s_tot[u][0][lane];
                        }
                        // the segment, transposed in place: LDS row a (stride 33) holds the 33
                        // samples of sensor a
                        float* const seg = reinterpret_cast<float*>(col + k0 * 64);
                        uint32_t c = c0 + c1;
#pragma unroll
                        for (int k = 0; k < kShSeg; ++k) {
                            seg[lane * kShSeg + k] = (float)(int32_t)(v[k] + c) * qeps;
                            c += c1;
                        }
                        const int kb = base + k0;         // trace sample of this sensor's row k0
                        s_kb[wid][lane] = kb;
                        wave_lds_sync();
                        // atomic i adds samples kb + j, j < kRun, of sensors 2i (lanes j) and 2i + 1
                        // (lanes 32 + j): one 32-bit byte offset per lane from the pair's row
                        const int half = lane >> 5, j = lane & 31;
                        const bool jv = j < kRun;
                        const int nact = p.S - s0;        // sensors of the group inside the record's S
                        const bool inside = __all(!active || (kb >= 0 && kb <= p.T - kShSeg)) && p.T < (1 << 28);
                        const int* const kbv = &s_kb[wid][half];
                        const float* const sv = seg + half * kShSeg + (jv ? j : 0);
                        if (inside) {
                            const uint32_t lane_b = (uint32_t)(half * p.T + j) * 4u;
#pragma unroll 1
                            for (int i0 = 0; i0 < 32; i0 += 8) {
                                float vv[8];
                                int kk[8];
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    vv[u] = jv ? sv[2 * (i0 + u) * kShSeg] : 0.f;
                                    kk[u] = kbv[2 * (i0 + u)];
                                }
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    char* const rowp = reinterpret_cast<char*>(sig0 + (int64_t)(2 * (i0 + u)) * p.T);
                                    if (vv[u] != 0.f)
                                        global_atomic_add(reinterpret_cast<float*>(rowp + (lane_b + (uint32_t)kk[u] * 4u)), vv[u]);
                                }
                            }
                        } else {
#pragma unroll 1
                            for (int i = 0; i < 32; ++i) {
                                const float vi = jv ? sv[2 * i * kShSeg] : 0.f;
                                const int a = 2 * i + half;
                                const int k = kbv[2 * i] + j;
                                if (vi != 0.f && a < nact) {
                                    if (k >= 0 && k < p.T) global_atomic_add(sig0 + (int64_t)a * p.T + k, vi);
                                    else clipped = true;
                                }
                            }
                        }
                        // the 33rd sample of every sensor (lane = sensor)
                        if (kShSeg > 32) {
                            const float vl = seg[lane * kShSeg + 32];
                            const int k = kb + 32;
                            if (vl != 0.f && active) {
                                if (k >= 0 && k < p.T) global_atomic_add(out_row + k, vl);
                                else clipped = true;
                            }
                        }
                        wave_lds_sync();
                        uint4* const z = reinterpret_cast<uint4*>(col + k0 * 64);
#pragma unroll
                        for (int q = 0; q < (kShSeg * 64 + 255) / 256; ++q)
                            if (q * 64 + lane < kShSeg * 16) z[q * 64 + lane] = make_uint4(0u, 0u, 0u, 0u);
                    }
                    __syncthreads();                      // the column is zero again
                };

                if (qmode) {
                    const int span = kShRows + 1 - rmax;  // first samples of one pass's windows
                    int lim = base + span;                // windows starting before lim fit this pass
                    uint64_t left = 0;                    // the wave's balls with a window left for later
                    for (int pass = 0;; ++pass) {
                        int nmin = INT_MAX;                   // later passes: least sample left (this lane)
                        if (pass == 0 && nbw > 0) {
                            // every ball of the wave; the next ball's FP64 set-up runs while this
                            // ball's seven LDS adds complete (as in forward_kernel)
                            FwdPair cur = setup(wb[0]);
                            BallU bn = wb[min(1, nbw - 1)];
                            for (int i = 0; i < nbw; ++i) {
                                const bool part = cur.in_tile;
                                const int rows = max(cur.W, 5) + 2;       // the same in every lane
                                const bool in_lds = rows <= kShCap;
                                const int tl = cur.klo - base;
                                const bool fit = part && in_lds && tl >= 0 && cur.klo < lim;
                                const bool later = part && in_lds && cur.klo >= lim;
                                const bool direct = part && (!in_lds || tl < 0);
                                if (__ballot(later)) left |= 1ull << i;
                                const int tr = fit ? tl : 0;            // lanes without a window add zeros
                                FwdPair nxt;
                                if (cur.W >= 5 && in_lds) {
                                    const D2Win dw = d2_window<true>(cur.W, fit ? cur.xg : 0.f, cur.rhof, fit ? cur.Cg * qs : 0.f);
                                    uint32_t* const c0 = col + tr * 64 + lane;
                                    d2_add(c0, c0 + dw.w2 * 64, dw);
                                    nxt = setup(bn);
                                } else {
                                    if (in_lds) {
                                        const D2Win dw = d2_window<false>(cur.W, fit ? cur.xg : 0.f, cur.rhof, fit ? cur.Cg * qs : 0.f);
                                        uint32_t* const c0 = col + tr * 64 + lane;
                                        d2_add(c0, c0 + dw.w2 * 64, dw);
                                    }
                                    nxt = setup(bn);
                                }
                                if (__ballot(direct)) {
                                    if (direct) clipped |= add_window_global<SB_KERNEL_UNIFORM>(out_row, cur.klo, p.T, cur.W, cur.xg, cur.rhof, cur.Cg);
                                }
                                cur = nxt;
                                bn = wb[min(i + 2, nbw - 1)];
                            }
                        } else if (pass > 0) {
                            // the balls with a window left over, again; every such window is an LDS one
                            uint64_t m = left;
                            left = 0;
                            while (m) {
                                const int i = (int)__builtin_ctzll(m);
                                m &= m - 1;
                                const FwdPair f = setup(wb[i]);
                                const int tl = f.klo - base;
                                const bool fit = f.in_tile && tl >= 0 && f.klo < lim;
                                const bool later = f.in_tile && f.klo >= lim;
                                if (__ballot(later)) left |= 1ull << i;
                                if (later) nmin = min(nmin, f.klo);
                                const D2Win dw = d2_window<false>(f.W, fit ? f.xg : 0.f, f.rhof, fit ? f.Cg * qs : 0.f);
                                uint32_t* const c0 = col + (fit ? tl : 0) * 64 + lane;
                                d2_add(c0, c0 + dw.w2 * 64, dw);
                            }
                        }
                        if (left != 0 && lane == 0) s_more[pp & 1] = 1;
                        if (nmin != INT_MAX) atomicMin(&s_nmin[pp & 1][lane], nmin);
                        const int kmax_b = __builtin_amdgcn_readfirstlane(
                            wave_max_all(kfar == INT_MIN ? -1 : min(kfar - base, kShRows - 1)));
                        __syncthreads();                  // every window of the pass is in the column
                        const bool more = s_more[pp & 1] != 0;
                        const int nnext = s_nmin[pp & 1][lane];
                        if (wid == 0) {                   // the other parity was read last in the pass before
                            s_nmin[(pp + 1) & 1][lane] = INT_MAX;
                            if (lane == 0) s_more[(pp + 1) & 1] = 0;
                        }
                        flush(kmax_b);
                        ++pp;
                        if (!more) break;                 // the same in every wave
                        base = nnext == INT_MAX ? lim : max(lim, nnext);
                        lim = base + span;
                    }
                } else {
                    // no integer scale for these sensors: every window straight to the trace
                    for (int i = 0; i < nbw; ++i) {
                        const FwdPair f = setup(wb[i]);
                        if (f.in_tile) clipped |= add_window_global<SB_KERNEL_UNIFORM>(out_row, f.klo, p.T, f.W, f.xg, f.rhof, f.Cg);
                    }
                }
                if (__ballot(bad)) chunk_flags(p, wb, nbw, sx, sy, sz, active, geometry, clipped);
            }
        }
    }
    if (clipped) raise_flag(p.flags, SB_FLAG_CLIPPED);
    if (geometry) raise_flag(p.flags, SB_FLAG_GEOMETRY);
    if (nonfinite) raise_flag(p.flags, SB_FLAG_NONFINITE);
}

// ---- Gaussian ball, a lane per sample ------------------------------------------------
//
// A Gaussian ball's window is long (≈100 samples for the heart phantom's balls), so a
// tile of 64 sensors needs some 256 rows per wave, and forward_kernel then fits one
// two-wave block per compute unit.  Here a lane takes a sample instead: a wave walks its
// sensors one at a time, and for each it first sets up the chunk's 256 pairs (lane = ball,
// four rounds; results to a per-wave LDS table), then adds each ball's window to a
// per-wave LDS row of the sensor's samples, 63 samples per step (one exponential per lane:
// a sample's second boundary comes from the next lane; read, add, write: the row is the
// wave's own), and finally adds the row to the global trace with coalesced FP32 atomics.  The row starts at the chunk's earliest window at that sensor; a window that
// would leave it flushes the row and restarts it at that window, and a window longer than
// the row goes to the trace directly (still 64 consecutive samples per atomic).  The
// block (staged chunk, four tables and four rows) takes 37 KB: four blocks, sixteen
// waves per compute unit.

// The Gaussian ball's record (48 bytes; no inside test: any sensor off the centre).
struct BallG {
    double x, y, z;   // deformed centre (m)
    double c1;        // t0 fs + h - 1/2, h = kGaussCut rho: the window starts at floor(r / delta - c1)
    float amp;        // amplitude scale of the trace: P_f rho^2 delta / 2
    float rhof;       // rho = a_f / delta (samples)
    float hf;         // half-width h of the window
    int Wc;           // window length W = floor(2 h) + 2; 0: no ball; -1: longer than any record
};

// A pair of the lane's ball with the wave's current sensor, as the window loop reads it.
struct GPair {
    int klo;          // sample index of sample 0; INT_MIN: no window
    float xg;         // boundary 0: tau - k_lo + 1/2
    float C;          // amplitude P_f rho^2 delta / (2 r)
    float ce;         // exp2 scale -log2(e) / (2 rho^2)
};

constexpr int kGRow = 512;        // samples per wave's row

__global__ __launch_bounds__(256, 4) void forward_gauss_lane_kernel(OpParams p) {
    constexpr int NW = 4, G = 256;
    __shared__ BallG sball[G];
    __shared__ double s_fb[2 * SB_MAX_FOURIER];       // Fourier basis of the item's frame
    __shared__ __align__(16) GPair s_pair[NW][G];     // per wave: the current sensor's pairs
    __shared__ float s_row[NW][kGRow + 64];           // per wave: the current sensor's samples from `base`
                                                      // (64 samples of padding: the last step of a
                                                      // window adds zeros past its end)

    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    float* const row = s_row[wid];
    for (int k = lane; k < kGRow + 64; k += 64) row[k] = 0.f;
    GPair* const tab = s_pair[wid];
    bool clipped = false, geometry = false, nonfinite = false;
    // samples that fell outside the record, as a lane value (a flag carried as a lane mask
    // through the window loops costs scalar mask updates in every block)
    uint32_t clip_w = 0u;

    for (int64_t item = blockIdx.x; item < p.n_items; item += gridDim.x) {
        const Item it = decode_item(p, item);
        const Scene& sc = p.scenes[it.scene];
        const int gf = sc.frame0 + it.frame;
        const float t = p.frame_t[gf];
        const int64_t first = sc.ball0 + (int64_t)it.group * G;
        const int nb = min(G, sc.n_balls - it.group * G);
        __syncthreads();   // the previous item is done with sball and s_fb
        if (p.basis == SB_BASIS_FOURIER && wid == 0) fourier_basis_lanes(t, p.n_terms, s_fb, lane);
        __syncthreads();
        {
            BallF bl = stage_deform<SB_KERNEL_GAUSS>(p, tid, nb, first, t, s_fb, nonfinite);
            BallG bs;
            const bool valid = bl.rho >= 0.0;
            const double h = (double)kGaussCut * bl.rho;
            bs.x = bl.x;
            bs.y = bl.y;
            bs.z = bl.z;
            bs.c1 = p.t0fs + h - 0.5;
            bs.amp = bl.amp;
            bs.rhof = bl.rhof;
            bs.hf = (float)h;
            bs.Wc = !valid ? 0 : (h >= 1.0e6 ? -1 : (int)(2.0 * h) + 2);
            clipped |= valid && h >= 1.0e6;               // a window longer than any record
            sball[tid] = bs;
        }
        __syncthreads();

        // the wave's sensors of the item's 64-sensor blocks: 16 per block, one at a time
        const int sb_end = min(it.sblock + p.sb_per_item, p.n_sblocks);
        for (int sbk = it.sblock; sbk < sb_end; ++sbk) {
            const int s_lo = sbk * 64 + wid * 16, s_hi = min(s_lo + 16, p.S);
            for (int s = s_lo; s < s_hi; ++s) {
                const double sx = p.sensors[s], sy = p.sensors[p.S + s], sz = p.sensors[2 * p.S + s];
                float* const out_row = p.signals + ((int64_t)gf * p.S + s) * p.T;

                // ---- set-up of the chunk's pairs with this sensor (lane = ball)
                int kmin = INT_MAX, kend = INT_MIN;       // first sample and end of the row windows
#pragma unroll
                for (int r = 0; r < G / 64; ++r) {
                    const int b = 64 * r + lane;
                    const BallG bs = sball[b];
                    GPair g;
                    g.klo = INT_MIN;
                    g.xg = 0.f;
                    g.C = 0.f;
                    g.ce = 0.f;
                    if (b < nb && bs.Wc > 0) {
                        float ri;
                        const double dist = dist64(bs.x - sx, bs.y - sy, bs.z - sz, ri);
                        const double u = fma(dist, p.inv_delta, -bs.c1);   // r / delta - t0 fs - h + 1/2
                        const double kl = floor(u);
                        const bool ok = dist > 0.0;
                        geometry |= !ok;
                        clipped |= ok && !(fabs(kl) < 5.0e8);
                        if (ok && fabs(kl) < 5.0e8) {
                            g.klo = (int)kl;
                            g.xg = (float)(u - kl) + bs.hf;
                            g.C = bs.amp * ri;
                            g.ce = -1.4426950408889634f / (2.f * bs.rhof * bs.rhof);
                            if (bs.Wc <= kGRow) {
                                kmin = min(kmin, g.klo);
                                kend = max(kend, g.klo + bs.Wc);
                            }
                        }
                    }
                    tab[b] = g;
                }
                int base = __builtin_amdgcn_readfirstlane(-wave_max_all(-max(kmin, -INT_MAX)));
                const int kend_all = __builtin_amdgcn_readfirstlane(wave_max_all(kend));
                // every row window of the chunk fits the row from `base` (the usual case)
                const bool one_row = kend_all != INT_MIN && (int64_t)kend_all - base <= kGRow;
                int kmax = one_row ? kend_all - base - 1 : -1;   // last row written
                wave_lds_sync();

                // adds the row (samples base .. base + kmax) to the trace and clears it
                auto flush = [&]() {
                    for (int k0 = 0; k0 <= kmax; k0 += 64) {
                        const int k = k0 + lane;
                        const float v = row[k];
                        row[k] = 0.f;
                        const int ks = base + k;
                        if (v != 0.f) {
                            if (ks >= 0 && ks < p.T) global_atomic_add(out_row + ks, v);
                            else clip_w = 1u;
                        }
                    }
                    kmax = -1;
                };

                // ---- the windows (lane = sample)
                // a window longer than the row: straight to the trace, 64 samples per step
                auto direct = [&](const GPair& g, int klo, int W) {
                    for (int j0 = 0; j0 < W; j0 += 64) {
                        const int j = j0 + lane;
                        const float x = g.xg - (float)j;
                        const float v = g.C * (__builtin_amdgcn_exp2f((x - 1.f) * (x - 1.f) * g.ce) -
                                               __builtin_amdgcn_exp2f(x * x * g.ce));
                        const int ks = klo + j;
                        if (j < W && v != 0.f) {
                            if (ks >= 0 && ks < p.T) global_atomic_add(out_row + ks, v);
                            else clip_w = 1u;
                        }
                    }
                };
                // a window into the row from row sample tl on, 63 samples per step: lane i
                // evaluates the Gaussian at boundary j0 + i, and sample j0 + i (i < 63) takes the
                // next boundary's value from lane i + 1
                auto to_row = [&](const GPair& g, int W, int tl) {
                    float x = g.xg - (float)lane;         // boundary j0 + lane (exact: integer steps)
                    if (W <= 2 * 63) {
                        // one or two steps: both steps' row entries are read before either is
                        // written, so the wave waits for LDS once per window.  A step writes
                        // only its n <= 63 samples, so lane 63 of the first step, which reads
                        // the second step's first entry, writes nothing.
                        const bool two = W > 63;          // the same in every lane
                        float* const r0 = row + tl + lane;
                        const float o0 = r0[0];
                        const float o1 = two ? r0[63] : 0.f;
                        const float E0 = __builtin_amdgcn_exp2f(x * x * g.ce);
                        const float E1 = __builtin_amdgcn_exp2f((x - 63.f) * (x - 63.f) * g.ce);
                        const float N0 = __builtin_bit_cast(
                            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, E0), 0x130, 0xF, 0xF, false));
                        const float N1 = __builtin_bit_cast(
                            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, E1), 0x130, 0xF, 0xF, false));
                        if (lane < min(63, W)) r0[0] = o0 + g.C * (N0 - E0);
                        if (two && lane < W - 63) r0[63] = o1 + g.C * (N1 - E1);
                        return;
                    }
                    for (int j0 = 0; j0 < W; j0 += 63) {
                        const float E = __builtin_amdgcn_exp2f(x * x * g.ce);
                        const float En = __builtin_bit_cast(
                            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, E), 0x130, 0xF, 0xF, false));
                        const int n = min(63, W - j0);    // samples of this step
                        row[tl + j0 + lane] += lane < n ? g.C * (En - E) : 0.f;   // < kGRow + 64
                        x -= 63.f;
                    }
                };
                if (one_row) {
                    // the next ball's pair and window length are read one ball ahead
                    GPair gn = tab[0];                    // the same address in every lane
                    int Wn = sball[0].Wc;
                    for (int b = 0; b < nb; ++b) {
                        const GPair g = gn;
                        const int klo = __builtin_amdgcn_readfirstlane(g.klo);
                        const int W = __builtin_amdgcn_readfirstlane(Wn);
                        gn = tab[min(b + 1, nb - 1)];
                        Wn = sball[min(b + 1, nb - 1)].Wc;
                        if (klo == INT_MIN) continue;
                        if (W > kGRow) direct(g, klo, W);
                        else to_row(g, W, klo - base);
                    }
                } else {
                    for (int b = 0; b < nb; ++b) {
                        const GPair g = tab[b];
                        const int klo = __builtin_amdgcn_readfirstlane(g.klo);
                        if (klo == INT_MIN) continue;
                        const int W = __builtin_amdgcn_readfirstlane(sball[b].Wc);
                        if (W > kGRow) {
                            direct(g, klo, W);
                            continue;
                        }
                        int tl = klo - base;
                        if (tl < 0 || tl + W > kGRow) {
                            flush();
                            base = klo;
                            tl = 0;
                        }
                        to_row(g, W, tl);
                        kmax = max(kmax, tl + W - 1);
                    }
                }
                flush();
                wave_lds_sync();                          // the table is read before the next sensor's set-up
            }
        }
    }
    if (clipped || clip_w) raise_flag(p.flags, SB_FLAG_CLIPPED);
    if (geometry) raise_flag(p.flags, SB_FLAG_GEOMETRY);
    if (nonfinite) raise_flag(p.flags, SB_FLAG_NONFINITE);
}

template <int NW, int G, int UCAP, int KERNEL>
static hipError_t launch_fwd_t(const OpParams& p, hipStream_t st) {
    static_assert(G == 64 * NW, "one ball per thread in the sub-group compaction");
    int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((forward_kernel<NW, G, UCAP, KERNEL>), dim3((unsigned)grid), dim3(64 * NW), 0,
                       st, p);
    return hipGetLastError();
}

hipError_t launch_forward(const OpParams& p, const TileCfg& tc, int kernel, hipStream_t st) {
    // the host's work decomposition (n_sblocks, n_groups) must match the instance
    if (kernel == SB_KERNEL_GAUSS && tc.shared) {
        if (tc.nw != 1 || tc.g != 256) return hipErrorInvalidValue;   // sensor blocks of 64, chunks of 256
        const int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
        if (grid <= 0) return hipSuccess;
        hipLaunchKernelGGL(forward_gauss_lane_kernel, dim3((unsigned)grid), dim3(256), 0, st, p);
        return hipGetLastError();
    }
    if (kernel == SB_KERNEL_UNIFORM && tc.shared) {
        if (tc.nw != 1 || tc.g != 256) return hipErrorInvalidValue;   // sensor blocks of 64, chunks of 256
        const int64_t grid = p.n_items < (int64_t)(1 << 20) ? p.n_items : (int64_t)(1 << 20);
        if (grid <= 0) return hipSuccess;
        if (tc.ucap == 132)
            hipLaunchKernelGGL((forward_shared_kernel<33, 3>), dim3((unsigned)grid), dim3(256), 0, st, p);
        else if (tc.ucap == 92)
            hipLaunchKernelGGL((forward_shared_kernel<23, 4>), dim3((unsigned)grid), dim3(256), 0, st, p);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (kernel == SB_KERNEL_UNIFORM) {
        if (tc.nw == 4 && tc.g == 256 && tc.ucap == 128) return launch_fwd_t<4, 256, 128, 0>(p, st);
        if (tc.nw == 4 && tc.g == 256 && tc.ucap == 64) return launch_fwd_t<4, 256, 64, 0>(p, st);
    } else {
        if (tc.nw == 4 && tc.g == 256 && tc.ucap == 128) return launch_fwd_t<4, 256, 128, 1>(p, st);
        if (tc.nw == 2 && tc.g == 128 && tc.ucap == 256) return launch_fwd_t<2, 128, 256, 1>(p, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace sb
