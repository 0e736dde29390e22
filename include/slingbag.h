/*
 * slingbag.h - C ABI of the MI355X (gfx950) library for the differentiable
 * point-cloud photoacoustic forward operator of 4D SlingBAG and its adjoint.
 *
 * The problem (paper Sec. 2.1-2.2): a dynamic scene is a cloud of balls, each
 * with a position mu, a size a0 and a peak initial pressure p0, whose
 * attributes at normalised frame time t are deformed by Eq. 1 with a
 * deformation function H(t) (Eq. 2, or a Fourier series).  For every frame,
 * the pressure trace that each deformed ball radiates is summed into every
 * sensor's time samples (the "forward"); the predicted frames are compared
 * with the measured frames by an L2 loss; and the gradient of that loss with
 * respect to every ball attribute and deformation coefficient drives each
 * iterative-reconstruction step (the "adjoint").
 *
 * Physics used for one ball (the paper cites its radiator without giving it;
 * this is the textbook solution of the wave equation for a spherically
 * symmetric initial pressure with zero initial velocity, speed c):
 *   uniform sphere (radius R, pressure P), sensor at distance r > R:
 *     p(r, t) = P (r - c t) / (2 r)   for |r - c t| <= R, else 0   (the N-wave)
 *   Gaussian ball (std a, peak P):
 *     p(r, t) = P / (2r) [ (r-ct) e^{-(r-ct)^2/2a^2} + (r+ct) e^{-(r+ct)^2/2a^2} ]
 *   Sample k of a sensor (time t_k = t0 + k/fs) is the mean of p over
 *   [t_k - 1/(2 fs), t_k + 1/(2 fs)].  Samples with k outside [0, T) are dropped.
 *   The Gaussian ball's (r + ct) term is below the float range for every
 *   sensor outside the ball and is not evaluated; its trace is cut where
 *   |r - c t| exceeds 6 a + c/(2 fs) (relative truncation below 2e-8).
 *
 * Deformation (Eq. 1): R_f = R (1 + H^R(t_f)), P_f = P (1 + H^P(t_f)); each
 * coordinate x_f = x (1 + H^x(t_f)) (SB_POS_MUL, Eq. 1) or x_f = x + H^x(t_f)
 * (SB_POS_ADD).  H is the Gaussian-basis sum of Eq. 2
 * (SB_BASIS_GAUSS), a Fourier series sum_k a_k cos(2 pi k t) + b_k sin(2 pi k t)
 * (SB_BASIS_FOURIER), or zero (SB_BASIS_STATIC).
 *
 * Loss (Sec. 2.2, L2 loss): L = 1/2 sum over all frames, sensors, samples of
 * (y - d)^2; residual = y - d is the gradient of L with respect to y.
 *
 * Units: SI (metres, seconds, m/s, Hz).  Memory: every array argument is a
 * DEVICE pointer owned by the caller (e.g. allocated by PyTorch) unless marked
 * HOST; the library never frees or keeps caller memory.  All arrays are
 * contiguous float32 structure-of-arrays:
 *   balls      [5][B_total]       rows x, y, z, R (radius, or std a), P
 *   deform     [5][M][B_total]    per attribute x, y, z, R, P: M coefficients
 *                                 FOURIER: M = 2K, coefficient 2(k-1) multiplies
 *                                   cos(2 pi k t), 2(k-1)+1 multiplies sin(2 pi k t)
 *                                 GAUSS:   M = 3N, coefficient 3n is w_n, 3n+1
 *                                   theta_n, 3n+2 sigma_n (Eq. 2)
 *   frame_t    [F_total]          normalised frame times
 *   sensors    [3][S]             rows x, y, z
 *   signals, measured, residual   [F_total][S][T]
 * A batch is n_scenes independent scenes, concatenated: scene i owns balls
 * [ball_offset[i], ball_offset[i+1]) and frames [frame_offset[i],
 * frame_offset[i+1]); all scenes share the sensors, c, fs, t0 and T.
 *
 * Calls are asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 * Host-side validation runs before anything is enqueued; an invalid argument
 * returns a negative status and enqueues nothing.  Conditions that only the
 * device can see (a sensor inside a uniform ball, a non-finite or
 * non-positive deformed size, a negative deformed pressure) skip the affected
 * ball and raise a sticky device flag, read back by slingbag_check().
 *
 * Concurrency: the library keeps one set of scratch buffers per device (the
 * flag word, the loss partials, the ordering buffers), shared by every stream
 * of that device and bound into every captured plan.  Calls (and plan
 * replays) on one device must therefore not overlap in time: issue them on one
 * stream, or order the streams.  Host-side state (tuning knobs, timing, the
 * per-thread error message) is guarded, so entry points may be called from
 * several host threads.
 */
#ifndef SLINGBAG_H
#define SLINGBAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (returned by every entry point) ---- */
#define SB_OK               0
#define SB_ERR_INVALID_ARG  (-1)   /* null pointer, unknown enum, bad scalar */
#define SB_ERR_SHAPE        (-2)   /* offsets not a prefix sum, too many scenes/terms, size overflow */
#define SB_ERR_NONFINITE    (-3)   /* non-finite c, fs or t0 */
#define SB_ERR_GEOMETRY     (-4)   /* reserved, not returned: geometry violations are found on the
                                      device and reported as SB_FLAG_GEOMETRY by slingbag_check */
#define SB_ERR_HIP          (-5)   /* a HIP runtime call failed (message in slingbag_last_error) */
#define SB_ERR_DEVICE_FLAG  (-6)   /* slingbag_check found a device-side violation */
#define SB_ERR_UNSUPPORTED  (-7)   /* valid request the library does not implement */

/* ---- device flag bits (slingbag_check) ---- */
#define SB_FLAG_GEOMETRY    1u     /* a sensor lay inside a uniform ball (pair skipped) */
#define SB_FLAG_NONFINITE   2u     /* a deformed attribute was non-finite, R_f <= 0 or P_f < 0 (ball skipped) */
#define SB_FLAG_CLIPPED     4u     /* some trace fell partly outside [0, T) (dropped; informational) */

/* ---- enums ---- */
#define SB_KERNEL_UNIFORM   0      /* uniform sphere of radius R */
#define SB_KERNEL_GAUSS     1      /* Gaussian ball of std R (Sec. 2.1) */
#define SB_BASIS_STATIC     0      /* H = 0 */
#define SB_BASIS_FOURIER    1      /* H = sum_k a_k cos 2 pi k t + b_k sin 2 pi k t */
#define SB_BASIS_GAUSS      2      /* H = sum_n w_n exp(-(t - theta_n)^2 / (2 sigma_n^2)), Eq. 2 */
#define SB_POS_ADD          0      /* x_f = x + H^x(t) */
#define SB_POS_MUL          1      /* x_f = x (1 + H^x(t)), Eq. 1 */

/* ---- limits ---- */
#define SB_MAX_SCENES       32
#define SB_MAX_FOURIER      8      /* harmonics K */
#define SB_MAX_GAUSS_BASES  128    /* bases N per attribute */

typedef struct sb_config {
    int32_t kernel;      /* SB_KERNEL_* */
    int32_t basis;       /* SB_BASIS_* */
    int32_t pos_mode;    /* SB_POS_* */
    int32_t n_terms;     /* K (FOURIER) or N (GAUSS); ignored for STATIC */
    int32_t n_sensors;   /* S >= 1 */
    int32_t n_samples;   /* 1 <= T <= 2^28 */
    double  c;           /* speed of sound, > 0 */
    double  fs;          /* sample rate, > 0 */
    double  t0;          /* time of sample 0, finite */
} sb_config;

typedef struct sb_batch {
    int32_t        n_scenes;      /* 1 .. SB_MAX_SCENES */
    int32_t        reserved;      /* must be 0 */
    const int64_t* ball_offset;   /* HOST [n_scenes+1], ball_offset[0] = 0, non-decreasing */
    const int64_t* frame_offset;  /* HOST [n_scenes+1], frame_offset[0] = 0, non-decreasing */
} sb_batch;

/* Forward operator (Sec. 2.2: the radiator applied to each ball's time-varying
 * attributes, Eq. 1-2).  Writes signals[f][s][k] = sum over the balls of f's
 * scene of the sampled trace of that ball at sensor s (every entry is
 * overwritten; frames of empty scenes become zero).  deform may be NULL only
 * for SB_BASIS_STATIC.  Scratch: none beyond a per-device flag word.
 * Precision: FP64 geometry and FP32 samples; for the uniform sphere the
 * per-chunk accumulation normally runs in integers at 2^-30 of the chunk's
 * amplitude bound (about 1e-6 relative L2 against an FP64 evaluation), so the
 * result depends at that level on which balls share a chunk of 256 (ball
 * order) and on the FP32 atomic order. */
int slingbag_forward(const sb_config* cfg, const sb_batch* batch,
                     const float* balls, const float* deform, const float* frame_t,
                     const float* sensors, float* signals, void* stream);

/* L2 data loss (Sec. 2.2).  residual[i] = signals[i] - measured[i] for all
 * F_total*S*T entries (residual may alias signals or measured), and *loss
 * (a DEVICE double) = 1/2 sum residual^2, reduced in a fixed order (the
 * result does not depend on timing).  Scratch: a fixed per-device buffer of
 * block partials (16 KB), allocated on the first call on the device. */
int slingbag_loss(const sb_config* cfg, const sb_batch* batch,
                  const float* signals, const float* measured, float* residual,
                  double* loss, void* stream);

/* slingbag_loss for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and error behaviour, bit-identical residual and
 * *loss, but no allocation of any kind.  The block partials live in a fixed
 * device array of 2,048 doubles (16 KiB), which each device that loads the
 * library holds until the process ends; the reduction always uses 2,048
 * blocks, so every signal size fits (a larger need would return
 * SB_ERR_SHAPE).  Every partial is rewritten by each call, so nothing carries
 * over from the last call.  All calls on one device share that array: calls
 * that overlap in time on one device (on different streams, or replays of
 * graphs that captured this call) race and return wrong losses; order them. */
int slingbag_loss_noalloc(const sb_config* cfg, const sb_batch* batch,
                          const float* signals, const float* measured, float* residual,
                          double* loss, void* stream);

/* Adjoint (Sec. 2.2: gradient of the L2 loss with respect to all baseline
 * attributes and deformation parameters).  Given residual = dL/dsignals,
 * writes grad_balls [5][B_total] = dL/dballs and grad_deform [5][M][B_total]
 * = dL/ddeform (both overwritten; grad_deform may be NULL only for STATIC).
 * Per-frame deformed attributes are recomputed here, never stored.  The
 * 2-harmonic Fourier series (and STATIC) apply the chain rule inside the
 * adjoint kernel; every other basis sums the derivatives with respect to each
 * ball's deformed attributes at every frame (5 floats per ball and frame) in a
 * per-device buffer, allocated on first use and grown as needed (growing
 * cannot happen under graph capture: call slingbag_adjoint once on the problem
 * before capturing it), and applies the chain rule once per ball in a second
 * kernel.  A plan allocates a buffer of its own (see slingbag_plan_create). */
int slingbag_adjoint(const sb_config* cfg, const sb_batch* batch,
                     const float* balls, const float* deform, const float* frame_t,
                     const float* sensors, const float* residual,
                     float* grad_balls, float* grad_deform, void* stream);

/* Ball order (performance only: every result is independent of the order of
 * the balls within a scene).  Writes perm (DEVICE int32 [B_total]) such that
 * placing ball perm[i] at position i sorts every scene's balls along the
 * Morton (Z-order) curve of a fixed grid (2^-18 m cells over [-1 m, 1 m)^3,
 * positions outside are clamped to its faces); perm stays within each
 * scene's range and is stable for equal keys.  Ordered balls let the forward
 * group neighbours into short arrival windows and the adjoint stage compact
 * residual rows.  Apply perm to every per-ball array (balls, deform,
 * optimiser state) with slingbag_permute.  Scratch: a per-device buffer
 * (keys, indices and radix-sort tables, about 21 bytes per ball), allocated
 * on first use and grown as needed.  B_total must be below 2^31. */
int slingbag_order(const sb_batch* batch, const float* balls, int32_t* perm, void* stream);

/* dst[r][i] = src[r][perm[i]] for r < rows, i < n (DEVICE float arrays of
 * rows*n elements, DEVICE int32 perm of n entries in [0, n)); dst must not
 * alias src. */
int slingbag_permute(const float* src, float* dst, int64_t rows, int64_t n, const int32_t* perm,
                     void* stream);

/* One Adam step of the iterative reconstruction (Sec. 3.2 updates each
 * parameter group - coordinates, peak pressure, size, deformation
 * coefficients - with its own learning rate; the optimiser is not named, Adam
 * is used), followed by a projection onto [lo, hi].  For i < n, with
 * g = grad[i] and t = step >= 1:
 *   m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2;
 *   param = clamp(param - lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps), lo, hi).
 * param, m, v are updated in place (DEVICE, n floats each).  Call once per
 * parameter group.  0 <= beta < 1, eps > 0, lo <= hi (use -INFINITY / INFINITY
 * for no bound; an IR loop keeps peak pressure >= 0 and size > 0 this way). */
int slingbag_adam(float* param, const float* grad, float* m, float* v, int64_t n,
                  float lr, float beta1, float beta2, float eps, int32_t step, float lo, float hi,
                  void* stream);

/* Waits for `stream`, returns the device flag bits raised since the last
 * check in *flags (HOST, may be NULL) and clears them.  Returns
 * SB_ERR_DEVICE_FLAG if SB_FLAG_GEOMETRY or SB_FLAG_NONFINITE was raised. */
int slingbag_check(void* stream, uint32_t* flags);

/* One IR step as a captured HIP graph (Sec. 2.2: forward, L2 loss and the
 * gradient of every parameter, per iteration).  slingbag_plan_create records
 * slingbag_forward, slingbag_loss (residual = signals - measured, *loss) and
 * slingbag_adjoint (with that residual) on `stream` (must not be NULL) into a
 * graph and instantiates it; slingbag_plan_run replays the whole sequence with
 * one hipGraphLaunch on any stream.  The plan binds the buffers and the tuning
 * knobs of its creation: the caller may change their contents (for instance
 * update balls and deform in place between runs) but not their addresses or
 * the shapes.  No memsets are recorded (outputs are cleared by kernels).  A
 * plan created while timing is on (slingbag_timing) also records an event
 * node before and after its forward, loss and adjoint kernels, and every
 * replay while timing is on times them into the same pool as direct calls.
 * The plan owns the graph, those nodes' own events and, for deformations that
 * take the adjoint's two-phase chain rule, its own chain-rule buffer (5 floats
 * per ball and frame, allocated at creation); slingbag_plan_destroy releases
 * them (NULL is a no-op). */
typedef struct sb_plan sb_plan;
int slingbag_plan_create(const sb_config* cfg, const sb_batch* batch, const float* balls,
                         const float* deform, const float* frame_t, const float* sensors,
                         const float* measured, float* signals, float* residual, double* loss,
                         float* grad_balls, float* grad_deform, void* stream, sb_plan** out);
int slingbag_plan_run(sb_plan* plan, void* stream);
int slingbag_plan_destroy(sb_plan* plan);

/* Tuning knobs, read by every later call on any device (process-wide).  They
 * change speed only; results differ at most by rounding (the order of FP32
 * atomic additions, and the uniform sphere's integer accumulation scale when
 * the column length changes which windows stay in LDS).  The autotuner (python: paper_2412_03898_amd.tune) times the
 * candidates on the caller's own shapes and sets the fastest.
 *   SB_TUNE_FWD_COLUMN     forward LDS column of the uniform sphere: 64 or 128 (each wave
 *                          of a block keeps its own column of that many samples per sensor
 *                          and walks all of the chunk's balls; two blocks per compute unit),
 *                          SB_FWD_COLUMN_SHARED (the block's four waves share one 132-sample
 *                          column per sensor and take a quarter of the balls each; three
 *                          blocks per compute unit) or SB_FWD_COLUMN_SHARED_SHORT (the same
 *                          with a 92-sample column; four blocks per compute unit, more
 *                          passes where a chunk's arrivals spread wider);
 *                          default SB_FWD_COLUMN_SHARED_SHORT
 *   SB_TUNE_FWD_GAUSS_COLUMN  forward layout for the Gaussian ball: a column of 128 samples
 *                          per wave and sensor (blocks of 4 waves) or 256 (blocks of 2 waves,
 *                          for windows that nearly fill 128 rows), or SB_FWD_GAUSS_LANE (a
 *                          lane per sample: each wave takes one sensor at a time and adds
 *                          the windows to a 512-sample LDS row; sixteen waves per compute
 *                          unit); default SB_FWD_GAUSS_LANE
 *   SB_TUNE_ADJ_OCCUPANCY  adjoint blocks per compute unit the compiler targets: 2, 3 or 4
 *                          (both kernels; the Gaussian ball with the 2-harmonic Fourier
 *                          series at most 3); default 4
 *   SB_TUNE_ADJ_ITEMS      adjoint work items the sensor split aims for: 1 .. 2^22;
 *                          default 8192
 * Unknown keys or values return SB_ERR_INVALID_ARG and change nothing. */
#define SB_TUNE_FWD_COLUMN     1
#define SB_TUNE_ADJ_OCCUPANCY  2
#define SB_TUNE_ADJ_ITEMS      3
#define SB_TUNE_FWD_GAUSS_COLUMN 4
#define SB_FWD_COLUMN_SHARED        1   /* values of SB_TUNE_FWD_COLUMN */
#define SB_FWD_COLUMN_SHARED_SHORT  2
#define SB_FWD_GAUSS_LANE           1   /* value of SB_TUNE_FWD_GAUSS_COLUMN */
int slingbag_tune(int key, int value);
int slingbag_tune_get(int key, int* value);

/* Autotuner: runs the forward with every column length of the problem's kernel
 * (SB_TUNE_FWD_COLUMN for the uniform sphere, SB_TUNE_FWD_GAUSS_COLUMN for the
 * Gaussian ball) and the adjoint with every (occupancy, item count) candidate on the caller's own
 * problem (the arguments of slingbag_forward / slingbag_adjoint; signals,
 * grad_balls and grad_deform are overwritten, the forward output serves as
 * the adjoint's residual), times each with HIP events on `stream` (one
 * warm-up and two timed runs), keeps the fastest setting of every knob and
 * writes it to choice[3] (HOST: forward column of the problem's kernel, adjoint
 * occupancy, adjoint items).  Synchronises the stream.  Not for use under graph
 * capture. */
int slingbag_autotune(const sb_config* cfg, const sb_batch* batch, const float* balls,
                      const float* deform, const float* frame_t, const float* sensors, float* signals,
                      float* grad_balls, float* grad_deform, int32_t* choice, void* stream);

/* Opt-in timing of the main kernels with HIP events recorded on each call's
 * own stream around the kernel launch (not around the output clearing).
 * slingbag_timing(1) creates the events on the current device and starts
 * recording; slingbag_timing(0) stops.  slingbag_timing_read waits for the
 * recorded events and returns, per kind [forward, adjoint, loss, adam], the
 * summed kernel milliseconds in total_ms[4] and the launch count in
 * launches[4] (HOST arrays), then resets the counters.  At most 8192 launches
 * per kind are recorded between reads.  Replays of a plan created with timing
 * on count like direct calls (see slingbag_plan_create); other graph captures
 * record no timing. */
int slingbag_timing(int enable);
int slingbag_timing_read(double* total_ms, int64_t* launches);

/* ---- point cloud -> voxel grid and maximum amplitude projections ----
 * Sec. 2.1 and Sec. 3: the reconstruction is viewed by converting the point
 * cloud into a voxel grid and projecting it (MAP images in the XY, YZ and XZ
 * planes).  The grid holds the model's initial pressure p0(x) = sum over balls
 * of P_f phi(|x - x_f|) sampled at voxel centres, phi = 1[d <= R_f] for the
 * uniform sphere (the inside test taken in FP64) or exp(-d^2 / (2 R_f^2)) for
 * the Gaussian ball (cut at 6 R_f). */
typedef struct sb_grid {
    int32_t nx, ny, nz;  /* voxels per axis, each >= 1; nx*ny*nz <= 2^31 */
    int32_t reserved;    /* must be 0 */
    double  x0, y0, z0;  /* centre of voxel (0, 0, 0), metres, finite */
    double  h;           /* voxel pitch, metres, > 0; voxel (i,j,k) is centred at (x0+i h, y0+j h, z0+k h) */
} sb_grid;

/* Voxelise one scene at frame time t: volume[k][j][i] (device, FP32, nz*ny*nx,
 * caller-owned, every entry overwritten) = p0 at the centre of voxel (i,j,k)
 * for the n_balls balls [5][n_balls] (device) deformed by Eq. 1 at t with the
 * coefficients deform [5][M][n_balls] (device; NULL only for SB_BASIS_STATIC).
 * cfg supplies kernel, basis, pos_mode and n_terms (its sensor, sample and
 * time fields are ignored).  Balls with non-finite or invalid attributes are
 * skipped and set SB_FLAG_NONFINITE.  n_balls may be 0 (zero volume).
 * Scratch: none beyond the per-device flag word. */
int slingbag_voxelize(const sb_config* cfg, const sb_grid* grid, int64_t n_balls, const float* balls,
                      const float* deform, float t, float* volume, void* stream);

/* Maximum amplitude projections of a volume [nz][ny][nx] (device): map_xy[j][i]
 * = max over k, map_yz[k][j] = max over i, map_xz[k][i] = max over j (device,
 * FP32, caller-owned; any of the three may be NULL to skip it). */
int slingbag_map(const sb_grid* grid, const float* volume, float* map_xy, float* map_yz,
                 float* map_xz, void* stream);

/* Message for the last non-OK status returned on the calling host thread. */
const char* slingbag_last_error(void);

/* ABI version: (major << 16) | minor. */
int slingbag_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SLINGBAG_H */
