/*
 * FP64 CPU oracle of the point-cloud photoacoustic forward operator, its L2
 * data loss and the gradient of that loss.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * library: it is written from the definitions below, plainly and slowly.
 *
 * What is computed (paper Sec. 2.1-2.2, Eq. 1-2; the radiator itself is only
 * cited by the paper, so the textbook solution is used):
 *
 *  Source.  Ball b at frame time t_f has centre x_f, size R_f and peak
 *  pressure P_f.  Uniform sphere: p0(x) = P_f 1[|x - x_f| <= R_f].  Gaussian
 *  ball (Sec. 2.1): p0(x) = P_f exp(-|x - x_f|^2 / (2 R_f^2)), R_f the std.
 *
 *  Pressure at a point sensor at distance r from the centre (spherically
 *  symmetric initial pressure, zero initial velocity, speed c; d'Alembert for
 *  r*p):  p(r,t) = [ (r-ct) f(|r-ct|) + (r+ct) f(|r+ct|) ] / (2r),
 *  f the radial profile of p0.  Uniform sphere, r > R: the N-wave
 *  P (r-ct)/(2r) for |r-ct| <= R.
 *
 *  Sampling.  Sample k (time t_k = t0 + k/fs) is the average of p over
 *  [t_k - dt/2, t_k + dt/2].  With u = r - c t and delta = c dt this is
 *  (1/delta) * integral of (P/2r) s f(s) ds over s in [u_k - delta/2, u_k + delta/2]
 *  (plus the same for s = r + c t).
 *    uniform:  v_k = P/(4 r delta) * (B - A)(B + A),
 *              A = clamp(u_k - delta/2, -R, R), B = clamp(u_k + delta/2, -R, R)
 *    gaussian: v_k = [G(u_k + delta/2) - G(u_k - delta/2)]/delta + same at w_k = r + c t_k,
 *              G(s) = -(P R^2 / (2 r)) exp(-s^2 / (2 R^2))
 *  Signal y[f][j][k] = sum over the scene's balls of v_k(ball, frame f, sensor j).
 *  Contributions with k outside [0, T) are dropped.
 *
 *  Deformation (Eq. 1): R_f = R (1 + H^R(t_f)), P_f = P (1 + H^P(t_f)),
 *  position x_f = x (1 + H^x(t_f)) per coordinate (multiplicative, Eq. 1) or
 *  x_f = x + H^x(t_f) (additive offset).  H is either
 *    Gaussian basis (Eq. 2): H(t) = sum_n w_n exp(-(t - theta_n)^2 / (2 sigma_n^2))
 *    Fourier:                H(t) = sum_k a_k cos(2 pi k t) + b_k sin(2 pi k t)
 *    static:                 H = 0.
 *
 *  Loss (Sec. 2.2, "L2 loss"): L = 1/2 sum (y - d)^2 over all frames of all
 *  scenes, residual rho = y - d.  Gradient: exact derivative of L with respect
 *  to every ball attribute and deformation coefficient (clamp derivatives at
 *  exact ties take the clamped branch).
 *
 * Layouts (all double, contiguous):
 *   balls [5][B] rows x, y, z, R, P;  deform [5][M][B];  sensors [3][S];
 *   frame_t [F];  signals/residual [F][S][T];  ball_offset/frame_offset [n+1].
 * Fourier coefficient m of an attribute: m = 2(k-1) -> cos(2 pi k t), m = 2(k-1)+1 -> sin.
 * Gaussian-basis coefficient m: m = 3n -> w_n, 3n+1 -> theta_n, 3n+2 -> sigma_n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define SBO_OK 0
#define SBO_ERR_ARG (-1)
#define SBO_ERR_NONFINITE (-3)
#define SBO_ERR_GEOMETRY (-4)

typedef struct {
    int32_t kernel;       /* 0 uniform sphere, 1 gaussian ball */
    int32_t basis;        /* 0 static, 1 fourier, 2 gaussian basis */
    int32_t pos_mode;     /* 0 additive offset, 1 multiplicative */
    int32_t n_terms;      /* harmonics K (fourier) or bases N (gaussian) */
    int32_t n_sensors;
    int32_t n_samples;
    int32_t n_threads;    /* 0: OpenMP default */
    int32_t pad_;
    double c, fs, t0;
    double gauss_window;  /* gaussian ball: samples with |r - c t_k| > gauss_window*R + delta
                             are skipped (their value is below exp(-gauss_window^2/2) of the
                             peak); <= 0 evaluates every sample of the record */
} sbo_problem;

static const double PI = 3.14159265358979323846;

static int n_coef(const sbo_problem* p) {
    if (p->basis == 1) return 2 * p->n_terms;
    if (p->basis == 2) return 3 * p->n_terms;
    return 0;
}

/* H of attribute a of ball b at time t (Eq. 2 or the Fourier series). */
static double deform_H(const sbo_problem* p, const double* deform, int64_t B, int64_t b,
                       int a, double t) {
    int M = n_coef(p);
    double h = 0.0;
    if (p->basis == 1) {
        for (int k = 1; k <= p->n_terms; ++k) {
            double ak = deform[((int64_t)a * M + 2 * (k - 1)) * B + b];
            double bk = deform[((int64_t)a * M + 2 * (k - 1) + 1) * B + b];
            h += ak * cos(2.0 * PI * k * t) + bk * sin(2.0 * PI * k * t);
        }
    } else if (p->basis == 2) {
        for (int n = 0; n < p->n_terms; ++n) {
            double w = deform[((int64_t)a * M + 3 * n) * B + b];
            double th = deform[((int64_t)a * M + 3 * n + 1) * B + b];
            double sg = deform[((int64_t)a * M + 3 * n + 2) * B + b];
            h += w * exp(-(t - th) * (t - th) / (2.0 * sg * sg));
        }
    }
    return h;
}

/* dH/d(coefficient m) of attribute a of ball b at time t. */
static double deform_dH(const sbo_problem* p, const double* deform, int64_t B, int64_t b,
                        int a, int m, double t) {
    int M = n_coef(p);
    if (p->basis == 1) {
        int k = m / 2 + 1;
        return (m % 2 == 0) ? cos(2.0 * PI * k * t) : sin(2.0 * PI * k * t);
    }
    if (p->basis == 2) {
        int n = m / 3, which = m % 3;
        double w = deform[((int64_t)a * M + 3 * n) * B + b];
        double th = deform[((int64_t)a * M + 3 * n + 1) * B + b];
        double sg = deform[((int64_t)a * M + 3 * n + 2) * B + b];
        double e = exp(-(t - th) * (t - th) / (2.0 * sg * sg));
        if (which == 0) return e;
        if (which == 1) return w * e * (t - th) / (sg * sg);
        return w * e * (t - th) * (t - th) / (sg * sg * sg);
    }
    return 0.0;
}

/* Deformed attributes (Eq. 1) of ball b at time t: out = x_f, y_f, z_f, R_f, P_f. */
static void deformed(const sbo_problem* p, const double* balls, const double* deform,
                     int64_t B, int64_t b, double t, double out[5]) {
    for (int a = 0; a < 5; ++a) {
        double base = balls[(int64_t)a * B + b];
        double h = (p->basis == 0) ? 0.0 : deform_H(p, deform, B, b, a, t);
        if (a < 3 && p->pos_mode == 0) out[a] = base + h;
        else out[a] = base * (1.0 + h);
    }
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Sample value and its partial derivatives (d/dr, d/dR, d/dP) for one ball at distance r,
   with u = r - c t_k and w = r + c t_k. */
static void sample_uniform(double u, double r, double R, double P, double delta,
                           double* v, double* dr, double* dR, double* dP) {
    double h = 0.5 * delta;
    double A = clampd(u - h, -R, R), Bv = clampd(u + h, -R, R);
    double C = P / (4.0 * r * delta);
    double q = (Bv - A) * (Bv + A);
    *v = C * q;
    if (dr) {
        double inB = fabs(u + h) < R ? 1.0 : 0.0;
        double inA = fabs(u - h) < R ? 1.0 : 0.0;
        *dr = -(*v) / r + 2.0 * C * (Bv * inB - A * inA);
        *dR = 2.0 * R * C * ((1.0 - inB) - (1.0 - inA));
        *dP = q / (4.0 * r * delta);
    }
}

static double gG(double s, double r, double a, double P) {   /* antiderivative G(s) */
    return -(P * a * a / (2.0 * r)) * exp(-s * s / (2.0 * a * a));
}
static double gg(double s, double r, double a, double P) {   /* G'(s) = (P/2r) s e^{-s^2/2a^2} */
    return (P / (2.0 * r)) * s * exp(-s * s / (2.0 * a * a));
}
static double gGa(double s, double r, double a, double P) {  /* dG/da */
    return -(P / (2.0 * r)) * exp(-s * s / (2.0 * a * a)) * (2.0 * a + s * s / a);
}

static void sample_gauss(double u, double w, double r, double a, double P, double delta,
                         double* v, double* dr, double* da, double* dP) {
    double h = 0.5 * delta;
    double val = (gG(u + h, r, a, P) - gG(u - h, r, a, P)
                  + gG(w + h, r, a, P) - gG(w - h, r, a, P)) / delta;
    *v = val;
    if (dr) {
        *dr = -val / r + (gg(u + h, r, a, P) - gg(u - h, r, a, P)
                          + gg(w + h, r, a, P) - gg(w - h, r, a, P)) / delta;
        *da = (gGa(u + h, r, a, P) - gGa(u - h, r, a, P)
               + gGa(w + h, r, a, P) - gGa(w - h, r, a, P)) / delta;
        *dP = (P != 0.0) ? val / P
                         : (gG(u + h, r, a, 1.0) - gG(u - h, r, a, 1.0)
                            + gG(w + h, r, a, 1.0) - gG(w - h, r, a, 1.0)) / delta;
    }
}

/* Sample index range [*k0, *k1] (inclusive, clipped to the record) outside which the
   ball's contribution at distance r is exactly zero (uniform) or negligible (gaussian). */
static void window(const sbo_problem* p, double r, double R, int64_t* k0, int64_t* k1) {
    double delta = p->c / p->fs;
    int64_t T = p->n_samples;
    double half;
    if (p->kernel == 0) half = R + 0.5 * delta;
    else if (p->gauss_window > 0.0) half = p->gauss_window * R + 0.5 * delta;
    else { *k0 = 0; *k1 = T - 1; return; }
    double kc = (r - p->c * p->t0) / delta;          /* u_k = delta (kc - k) */
    int64_t lo = (int64_t)floor(kc - half / delta) - 1;
    int64_t hi = (int64_t)ceil(kc + half / delta) + 1;
    *k0 = lo < 0 ? 0 : lo;
    *k1 = hi > T - 1 ? T - 1 : hi;
}

static int check_problem(const sbo_problem* p, int n_scenes, const int64_t* bo, const int64_t* fo) {
    if (!p || !bo || !fo || n_scenes < 1) return SBO_ERR_ARG;
    if (p->kernel < 0 || p->kernel > 1 || p->basis < 0 || p->basis > 2) return SBO_ERR_ARG;
    if (p->basis != 0 && p->n_terms < 1) return SBO_ERR_ARG;
    if (p->n_sensors < 1 || p->n_samples < 1 || !(p->c > 0) || !(p->fs > 0)) return SBO_ERR_ARG;
    if (bo[0] != 0 || fo[0] != 0) return SBO_ERR_ARG;
    for (int i = 0; i < n_scenes; ++i)
        if (bo[i + 1] < bo[i] || fo[i + 1] < fo[i]) return SBO_ERR_ARG;
    return SBO_OK;
}

/* Deformed attributes of all balls at frame g: out [5][B_total] (test helper). */
int sbo_deformed(const sbo_problem* p, int n_scenes, const int64_t* ball_offset,
                 const int64_t* frame_offset, const double* balls, const double* deform,
                 const double* frame_t, int64_t frame, double* out) {
    int st = check_problem(p, n_scenes, ball_offset, frame_offset);
    if (st) return st;
    int64_t B = ball_offset[n_scenes];
    for (int i = 0; i < n_scenes; ++i) {
        if (frame < frame_offset[i] || frame >= frame_offset[i + 1]) continue;
        for (int64_t b = ball_offset[i]; b < ball_offset[i + 1]; ++b) {
            double a5[5];
            deformed(p, balls, deform, B, b, frame_t[frame], a5);
            for (int a = 0; a < 5; ++a) out[(int64_t)a * B + b] = a5[a];
        }
    }
    return SBO_OK;
}

int sbo_forward(const sbo_problem* p, int n_scenes, const int64_t* ball_offset,
                const int64_t* frame_offset, const double* balls, const double* deform,
                const double* frame_t, const double* sensors, double* signals) {
    int st = check_problem(p, n_scenes, ball_offset, frame_offset);
    if (st) return st;
    const int64_t B = ball_offset[n_scenes], F = frame_offset[n_scenes];
    const int64_t S = p->n_sensors, T = p->n_samples;
    const double delta = p->c / p->fs;
    int nt = p->n_threads > 0 ? p->n_threads : omp_get_max_threads();
    memset(signals, 0, sizeof(double) * (size_t)(F * S * T));
    double* attr = (double*)malloc(sizeof(double) * 5 * (size_t)(B > 0 ? B : 1));
    int err = SBO_OK;
    for (int i = 0; i < n_scenes; ++i) {
        for (int64_t f = frame_offset[i]; f < frame_offset[i + 1]; ++f) {
            const double t = frame_t[f];
            for (int64_t b = ball_offset[i]; b < ball_offset[i + 1]; ++b) {
                double a5[5];
                deformed(p, balls, deform, B, b, t, a5);
                for (int a = 0; a < 5; ++a) attr[(int64_t)a * B + b] = a5[a];
                for (int a = 0; a < 5; ++a) if (!isfinite(a5[a])) err = SBO_ERR_NONFINITE;
                if (!(a5[3] > 0.0) || a5[4] < 0.0) err = SBO_ERR_NONFINITE;
            }
            if (err) break;
            int geo = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1) reduction(| : geo)
            for (int64_t j = 0; j < S; ++j) {
                const double sx = sensors[j], sy = sensors[S + j], sz = sensors[2 * S + j];
                double* row = signals + (f * S + j) * T;
                for (int64_t b = ball_offset[i]; b < ball_offset[i + 1]; ++b) {
                    const double x = attr[b], y = attr[B + b], z = attr[2 * B + b];
                    const double R = attr[3 * B + b], P = attr[4 * B + b];
                    const double r = sqrt((x - sx) * (x - sx) + (y - sy) * (y - sy) + (z - sz) * (z - sz));
                    if (p->kernel == 0 ? !(r > R) : !(r > 0.0)) { geo = 1; continue; }
                    int64_t k0, k1;
                    window(p, r, R, &k0, &k1);
                    for (int64_t k = k0; k <= k1; ++k) {
                        const double tk = p->t0 + (double)k / p->fs;
                        const double u = r - p->c * tk, w = r + p->c * tk;
                        double v;
                        if (p->kernel == 0) sample_uniform(u, r, R, P, delta, &v, 0, 0, 0);
                        else sample_gauss(u, w, r, R, P, delta, &v, 0, 0, 0);
                        row[k] += v;
                    }
                }
            }
            if (geo) { err = SBO_ERR_GEOMETRY; break; }
        }
        if (err) break;
    }
    free(attr);
    return err;
}

/* residual = y - d; returns L = 1/2 sum residual^2, summed in index order. */
double sbo_loss(const double* y, const double* d, int64_t n, double* residual) {
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = y[i] - d[i];
        if (residual) residual[i] = r;
        L += 0.5 * r * r;
    }
    return L;
}

/* Gradient of L = 1/2 |y(theta) - d|^2 given residual = y - d:
   grad_balls [5][B], grad_deform [5][M][B] (both overwritten). */
int sbo_adjoint(const sbo_problem* p, int n_scenes, const int64_t* ball_offset,
                const int64_t* frame_offset, const double* balls, const double* deform,
                const double* frame_t, const double* sensors, const double* residual,
                double* grad_balls, double* grad_deform) {
    int st = check_problem(p, n_scenes, ball_offset, frame_offset);
    if (st) return st;
    const int64_t B = ball_offset[n_scenes];
    const int64_t S = p->n_sensors, T = p->n_samples;
    const int M = n_coef(p);
    const double delta = p->c / p->fs;
    int nt = p->n_threads > 0 ? p->n_threads : omp_get_max_threads();
    memset(grad_balls, 0, sizeof(double) * 5 * (size_t)B);
    if (M > 0 && grad_deform) memset(grad_deform, 0, sizeof(double) * 5 * (size_t)M * (size_t)B);
    int err = SBO_OK;
    for (int i = 0; i < n_scenes; ++i) {
        int bad = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16) reduction(| : bad)
        for (int64_t b = ball_offset[i]; b < ball_offset[i + 1]; ++b) {
            for (int64_t f = frame_offset[i]; f < frame_offset[i + 1]; ++f) {
                const double t = frame_t[f];
                double a5[5];
                deformed(p, balls, deform, B, b, t, a5);
                const double R = a5[3], P = a5[4];
                if (!(R > 0.0) || P < 0.0) { bad |= 2; continue; }
                /* dL/d(x_f, y_f, z_f, R_f, P_f) */
                double g[5] = {0, 0, 0, 0, 0};
                for (int64_t j = 0; j < S; ++j) {
                    const double sx = sensors[j], sy = sensors[S + j], sz = sensors[2 * S + j];
                    const double dx = a5[0] - sx, dy = a5[1] - sy, dz = a5[2] - sz;
                    const double r = sqrt(dx * dx + dy * dy + dz * dz);
                    if (p->kernel == 0 ? !(r > R) : !(r > 0.0)) { bad |= 1; continue; }
                    int64_t k0, k1;
                    window(p, r, R, &k0, &k1);
                    const double* res = residual + (f * S + j) * T;
                    double gr = 0.0, gR = 0.0, gP = 0.0;
                    for (int64_t k = k0; k <= k1; ++k) {
                        const double tk = p->t0 + (double)k / p->fs;
                        const double u = r - p->c * tk, w = r + p->c * tk;
                        double v, dvr, dvR, dvP;
                        if (p->kernel == 0) sample_uniform(u, r, R, P, delta, &v, &dvr, &dvR, &dvP);
                        else sample_gauss(u, w, r, R, P, delta, &v, &dvr, &dvR, &dvP);
                        gr += res[k] * dvr;
                        gR += res[k] * dvR;
                        gP += res[k] * dvP;
                    }
                    g[0] += gr * dx / r;
                    g[1] += gr * dy / r;
                    g[2] += gr * dz / r;
                    g[3] += gR;
                    g[4] += gP;
                }
                /* chain rule through Eq. 1 to the static attributes and coefficients */
                for (int a = 0; a < 5; ++a) {
                    const double base = balls[(int64_t)a * B + b];
                    const double h = (p->basis == 0) ? 0.0 : deform_H(p, deform, B, b, a, t);
                    const int additive = (a < 3 && p->pos_mode == 0);
                    grad_balls[(int64_t)a * B + b] += g[a] * (additive ? 1.0 : 1.0 + h);
                    for (int m = 0; m < M; ++m) {
                        const double dh = deform_dH(p, deform, B, b, a, m, t);
                        grad_deform[((int64_t)a * M + m) * B + b] += g[a] * (additive ? dh : base * dh);
                    }
                }
            }
        }
        if (bad & 2) { err = SBO_ERR_NONFINITE; break; }
        if (bad & 1) { err = SBO_ERR_GEOMETRY; break; }
    }
    return err;
}

/*
 * Voxel grid of the initial pressure (the point cloud viewed as an image,
 * Sec. 2.1 and the maximum amplitude projections of Sec. 3).
 *
 *  vol[k][j][i] = sum over balls b of P_b phi(d), d = distance from the centre
 *  of voxel (i,j,k), (x0 + i h, y0 + j h, z0 + k h), to the ball centre;
 *  phi = 1[d <= R_b] (uniform sphere) or exp(-d^2 / (2 R_b^2)) (Gaussian ball,
 *  evaluated out to `gauss_window` R_b; <= 0 means every voxel).
 *  Inputs are the (already deformed) attributes in FP64, one array per
 *  attribute.  Planes k are independent, so they are split over threads; each
 *  voxel's sum runs over the balls in order.  The voxel centre and the squared
 *  distance are the plain expressions x0 + i h and dx^2 + dy^2 + dz^2.
 */
int sbo_voxelize(int kernel, int64_t n, const double* x, const double* y, const double* z,
                 const double* R, const double* P, int32_t nx, int32_t ny, int32_t nz,
                 double x0, double y0, double z0, double h, double gauss_window, int32_t n_threads,
                 double* vol) {
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || n < 0) return SBO_ERR_ARG;
    memset(vol, 0, sizeof(double) * (size_t)nx * ny * nz);
    if (n_threads > 0) omp_set_num_threads(n_threads);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < nz; ++k) {
        const double zc = z0 + (double)k * h;
        for (int64_t b = 0; b < n; ++b) {
            /* balls with non-finite or invalid attributes contribute nothing */
            if (!isfinite(x[b]) || !isfinite(y[b]) || !isfinite(z[b]) || !isfinite(R[b]) || !isfinite(P[b]) ||
                !(R[b] > 0.0) || !(P[b] >= 0.0))
                continue;
            const double reach = (kernel == 0) ? R[b]
                               : (gauss_window > 0.0 ? gauss_window * R[b] : INFINITY);
            const double dz = zc - z[b];
            if (fabs(dz) > reach) continue;
            /* every (i, j) whose centre is within reach in x and y */
            int64_t i0 = 0, i1 = nx - 1, j0 = 0, j1 = ny - 1;
            if (isfinite(reach)) {
                const double lo_i = floor((x[b] - reach - x0) / h) - 1, hi_i = ceil((x[b] + reach - x0) / h) + 1;
                const double lo_j = floor((y[b] - reach - y0) / h) - 1, hi_j = ceil((y[b] + reach - y0) / h) + 1;
                if (lo_i > i0) i0 = (int64_t)lo_i;
                if (hi_i < i1) i1 = (int64_t)hi_i;
                if (lo_j > j0) j0 = (int64_t)lo_j;
                if (hi_j < j1) j1 = (int64_t)hi_j;
            }
            for (int64_t j = j0; j <= j1; ++j) {
                const double dy = (y0 + (double)j * h) - y[b];
                for (int64_t i = i0; i <= i1; ++i) {
                    const double dx = (x0 + (double)i * h) - x[b];
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    double v;
                    if (kernel == 0) v = (d2 <= R[b] * R[b]) ? P[b] : 0.0;
                    else v = (d2 <= reach * reach) ? P[b] * exp(-d2 / (2.0 * R[b] * R[b])) : 0.0;
                    vol[((int64_t)k * ny + j) * nx + i] += v;
                }
            }
        }
    }
    return SBO_OK;
}

/*
 * Tie voxels of the uniform-sphere grid: voxels whose centre lies so close to
 * some ball's surface that the inside test d^2 <= R^2 depends on how d^2 is
 * rounded.  Two FP64 evaluations of d^2 (any order of the operations, with or
 * without fused multiply-adds) differ by at most a few units in the last place
 * of the coordinates and of d^2; a voxel counts as a tie when
 *   |d^2 - R^2| <= 64 eps (R^2 + 2 R L),   eps = 2^-52,
 * L the largest coordinate magnitude of the voxel centre and the ball centre.
 * mask[k][j][i] is set to 1 for ties (0 elsewhere); returns the tie count.
 */
int64_t sbo_voxel_ties(int64_t n, const double* x, const double* y, const double* z, const double* R,
                       int32_t nx, int32_t ny, int32_t nz, double x0, double y0, double z0, double h,
                       unsigned char* mask) {
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || n < 0) return -1;
    memset(mask, 0, (size_t)nx * ny * nz);
    const double eps = 2.220446049250313e-16;
    int64_t count = 0;
    for (int64_t b = 0; b < n; ++b) {
        if (!isfinite(x[b]) || !isfinite(y[b]) || !isfinite(z[b]) || !isfinite(R[b]) || !(R[b] > 0.0)) continue;
        const double reach = R[b] * 1.001;
        const double lo_i = floor((x[b] - reach - x0) / h) - 1, hi_i = ceil((x[b] + reach - x0) / h) + 1;
        const double lo_j = floor((y[b] - reach - y0) / h) - 1, hi_j = ceil((y[b] + reach - y0) / h) + 1;
        const double lo_k = floor((z[b] - reach - z0) / h) - 1, hi_k = ceil((z[b] + reach - z0) / h) + 1;
        const int64_t i0 = lo_i > 0 ? (int64_t)lo_i : 0, i1 = hi_i < nx - 1 ? (int64_t)hi_i : nx - 1;
        const int64_t j0 = lo_j > 0 ? (int64_t)lo_j : 0, j1 = hi_j < ny - 1 ? (int64_t)hi_j : ny - 1;
        const int64_t k0 = lo_k > 0 ? (int64_t)lo_k : 0, k1 = hi_k < nz - 1 ? (int64_t)hi_k : nz - 1;
        for (int64_t k = k0; k <= k1; ++k)
            for (int64_t j = j0; j <= j1; ++j)
                for (int64_t i = i0; i <= i1; ++i) {
                    const double cx = x0 + (double)i * h, cy = y0 + (double)j * h, cz = z0 + (double)k * h;
                    const double dx = cx - x[b], dy = cy - y[b], dz = cz - z[b];
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    double L = fabs(cx);
                    const double cand[5] = {fabs(cy), fabs(cz), fabs(x[b]), fabs(y[b]), fabs(z[b])};
                    for (int c = 0; c < 5; ++c) L = cand[c] > L ? cand[c] : L;
                    const double tol = 64.0 * eps * (R[b] * R[b] + 2.0 * R[b] * L);
                    unsigned char* m = mask + ((size_t)k * ny + j) * nx + i;
                    if (fabs(d2 - R[b] * R[b]) <= tol && !*m) {
                        *m = 1;
                        ++count;
                    }
                }
    }
    return count;
}
