// Point cloud -> voxel grid, and maximum amplitude projections of the grid.
//
// Voxelisation is a scatter: one wave per ball (grid-stride over balls)
// deforms its ball (Eq. 1 at the requested frame time, FP64 positions and
// size), walks the voxels of the ball's bounding box with its 64 lanes, x
// fastest so that consecutive lanes hit consecutive voxels of a row, and adds
// P_f phi(d) to every voxel whose centre lies in the ball's support with a
// float atomic.  The inside test of the uniform sphere (d^2 <= R_f^2) is taken
// in FP64; the Gaussian ball's support is cut at 6 R_f.
//
// Projections: each output element is the maximum along one axis; the XY and
// XZ maps stream the volume with consecutive threads on consecutive x (one
// column or slab line per thread); the YZ map reduces each x row with one wave.

#include "sb_internal.hpp"

namespace sb {

constexpr double kVoxGaussCut = 6.0;

struct GridP {
    int nx, ny, nz;
    double x0, y0, z0, h, inv_h;
};

// voxel index range (clamped to [0, n-1]) covering the centres c0 + i h in [lo, hi],
// one voxel wider on each side so that the rounded 1/h never drops a centre the
// exact distance test accepts
__device__ inline void voxel_range(double lo, double hi, double c0, double inv_h, int n, int& i0, int& i1) {
    const double a = ceil((lo - c0) * inv_h) - 1.0, b = floor((hi - c0) * inv_h) + 1.0;
    i0 = (int)fmin(fmax(a, 0.0), (double)n);
    i1 = (int)fmax(fmin(b, (double)(n - 1)), -1.0);
}

template <int KERNEL>
__global__ __launch_bounds__(256) void voxelize_kernel(OpParams p, GridP g, float t, float* __restrict__ vol) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    __shared__ double s_fb[2 * SB_MAX_FOURIER];
    if (p.basis == SB_BASIS_FOURIER && threadIdx.x < 64) fourier_basis_lanes(t, p.n_terms, s_fb, lane);
    __syncthreads();
    bool nonfinite = false;
    for (int64_t b = wave; b < p.B; b += n_waves) {
        BallF bl;
        const bool ok = deform_ball(p, b, t, s_fb, bl);     // rho = R_f in metres (inv_delta = 1)
        nonfinite |= !ok;
        if (!ok) continue;                                   // the same in every lane of the wave
        const double R = bl.rho;
        const double reach = (KERNEL == SB_KERNEL_UNIFORM) ? R : kVoxGaussCut * R;
        int i0, i1, j0, j1, k0, k1;
        voxel_range(bl.x - reach, bl.x + reach, g.x0, g.inv_h, g.nx, i0, i1);
        voxel_range(bl.y - reach, bl.y + reach, g.y0, g.inv_h, g.ny, j0, j1);
        voxel_range(bl.z - reach, bl.z + reach, g.z0, g.inv_h, g.nz, k0, k1);
        if (i1 < i0 || j1 < j0 || k1 < k0) continue;        // outside the grid
        const int bx = i1 - i0 + 1, by = j1 - j0 + 1;
        const int64_t nbox = (int64_t)bx * by * (k1 - k0 + 1);
        const double reach2 = reach * reach;
        const float amp = bl.amp;
        const float ce = (KERNEL == SB_KERNEL_UNIFORM) ? 0.f : (float)(-1.0 / (2.0 * R * R));
        for (int64_t v = lane; v < nbox; v += 64) {
            const int64_t plane = (int64_t)bx * by;
            const int kk = (int)(v / plane);
            const int rem = (int)(v - (int64_t)kk * plane);
            const int jj = rem / bx, ii = rem - jj * bx;
            const int i = i0 + ii, j = j0 + jj, k = k0 + kk;
            const double dx = fma((double)i, g.h, g.x0) - bl.x;
            const double dy = fma((double)j, g.h, g.y0) - bl.y;
            const double dz = fma((double)k, g.h, g.z0) - bl.z;
            const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
            if (d2 <= reach2) {
                const float val = (KERNEL == SB_KERNEL_UNIFORM) ? amp : amp * __expf((float)d2 * ce);
                global_atomic_add(vol + ((int64_t)k * g.ny + j) * g.nx + i, val);
            }
        }
    }
    if (nonfinite && lane == 0) raise_flag(p.flags, SB_FLAG_NONFINITE);
}

hipError_t launch_voxelize(const OpParams& p, int kernel, int nx, int ny, int nz, double x0, double y0,
                           double z0, double h, float t, float* vol, hipStream_t st) {
    if (p.B <= 0) return hipSuccess;
    GridP g{nx, ny, nz, x0, y0, z0, h, 1.0 / h};
    int64_t blocks = (p.B + 3) / 4;                          // one wave per ball
    if (blocks > 65536) blocks = 65536;
    if (kernel == SB_KERNEL_UNIFORM)
        hipLaunchKernelGGL(voxelize_kernel<SB_KERNEL_UNIFORM>, dim3((unsigned)blocks), dim3(256), 0, st, p, g, t, vol);
    else
        hipLaunchKernelGGL(voxelize_kernel<SB_KERNEL_GAUSS>, dim3((unsigned)blocks), dim3(256), 0, st, p, g, t, vol);
    return hipGetLastError();
}

// map_xy[j][i] = max_k vol[k][j][i]  (one thread per (i, j))
__global__ __launch_bounds__(256) void map_xy_kernel(const float* __restrict__ vol, int nx, int ny, int nz,
                                                     float* __restrict__ out) {
    const int64_t n = (int64_t)nx * ny;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        float m = vol[c];
        for (int k = 1; k < nz; ++k) m = fmaxf(m, vol[(int64_t)k * n + c]);
        out[c] = m;
    }
}

// map_xz[k][i] = max_j vol[k][j][i]  (one thread per (i, k))
__global__ __launch_bounds__(256) void map_xz_kernel(const float* __restrict__ vol, int nx, int ny, int nz,
                                                     float* __restrict__ out) {
    const int64_t n = (int64_t)nx * nz;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = c / nx, i = c - k * nx;
        const float* col = vol + k * (int64_t)ny * nx + i;
        float m = col[0];
        for (int j = 1; j < ny; ++j) m = fmaxf(m, col[(int64_t)j * nx]);
        out[c] = m;
    }
}

// map_yz[k][j] = max_i vol[k][j][i]  (one wave per x row)
__global__ __launch_bounds__(256) void map_yz_kernel(const float* __restrict__ vol, int nx, int ny, int nz,
                                                     float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t rows = (int64_t)ny * nz;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < rows; r += n_waves) {
        const float* row = vol + r * nx;
        float m = -3.4e38f;
        for (int i = lane; i < nx; i += 64) m = fmaxf(m, row[i]);
        m = wave_max_all(m);
        if (lane == 0) out[r] = m;
    }
}

static int64_t stream_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return b < 1 ? 1 : (b > 16384 ? 16384 : b);
}

hipError_t launch_map(const float* vol, int nx, int ny, int nz, float* xy, float* yz, float* xz, hipStream_t st) {
    if (xy) hipLaunchKernelGGL(map_xy_kernel, dim3((unsigned)stream_blocks((int64_t)nx * ny)), dim3(256), 0, st,
                               vol, nx, ny, nz, xy);
    if (xz) hipLaunchKernelGGL(map_xz_kernel, dim3((unsigned)stream_blocks((int64_t)nx * nz)), dim3(256), 0, st,
                               vol, nx, ny, nz, xz);
    if (yz) {
        int64_t blocks = ((int64_t)ny * nz + 3) / 4;
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL(map_yz_kernel, dim3((unsigned)blocks), dim3(256), 0, st, vol, nx, ny, nz, yz);
    }
    return hipGetLastError();
}

}  // namespace sb
