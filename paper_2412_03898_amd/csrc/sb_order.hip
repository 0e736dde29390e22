// Ball ordering (performance only; results do not depend on ball order): Morton
// keys of the canonical grid with the scene index in the top bits, a stable
// radix sort of (key, index), and a row gather that applies the permutation to
// any [rows][B] array.

#include <hipcub/hipcub.hpp>

#include "sb_internal.hpp"

namespace sb {

struct SceneOffsets {
    int64_t off[SB_MAX_SCENES + 1];
};

// spread the low 19 bits of v so that bit i moves to bit 3i
__device__ inline unsigned long long spread3(uint32_t v) {
    unsigned long long x = v & 0x7ffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(256) void morton_keys_kernel(const float* __restrict__ balls, int64_t B,
                                                          SceneOffsets so, int n_scenes,
                                                          unsigned long long* __restrict__ keys,
                                                          int* __restrict__ idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += stride) {
        int sc = 0;
        while (sc + 1 < n_scenes && so.off[sc + 1] <= b) ++sc;
        const unsigned long long m = spread3(grid_coord(balls[b])) | (spread3(grid_coord(balls[B + b])) << 1) |
                                     (spread3(grid_coord(balls[2 * B + b])) << 2);
        keys[b] = ((unsigned long long)sc << 57) | m;
        idx[b] = (int)b;
    }
}

__global__ __launch_bounds__(256) void gather_rows_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                          int64_t rows, int64_t B, const int* __restrict__ perm) {
    const int64_t n = rows * B;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t r = i / B, c = i - r * B;
        dst[i] = src[r * B + perm[c]];
    }
}

hipError_t launch_morton_keys(const float* balls, int64_t B, const int64_t* ball_offset_host,
                              int n_scenes, unsigned long long* keys, int* idx, hipStream_t st) {
    SceneOffsets so;
    for (int i = 0; i <= n_scenes; ++i) so.off[i] = ball_offset_host[i];
    int64_t blocks = (B + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(morton_keys_kernel, dim3((unsigned)blocks), dim3(256), 0, st, balls, B, so, n_scenes,
                       keys, idx);
    return hipGetLastError();
}

hipError_t sort_pairs(void* temp, size_t& temp_bytes, const unsigned long long* kin,
                      unsigned long long* kout, const int* vin, int* vout, int n, hipStream_t st) {
    return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, kin, kout, vin, vout, n, 0, 62, st);
}

hipError_t launch_gather_rows(const float* src, float* dst, int64_t rows, int64_t B, const int* perm,
                              hipStream_t st) {
    const int64_t n = rows * B;
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, rows, B, perm);
    return hipGetLastError();
}

}  // namespace sb
