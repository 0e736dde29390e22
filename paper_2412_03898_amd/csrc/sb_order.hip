// Ball ordering (performance only; results do not depend on ball order): Morton
// keys of the canonical grid with the scene index in the top bits, a stable
// radix sort of (key, index), and a row gather that applies the permutation to
// any [rows][B] array.

#include <utility>

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

// ---------------------------------------------------------------------------
// Stable least-significant-digit radix sort of (62-bit key, int32 value) pairs,
// eight bits per pass.  Each pass:
//   1. radix_hist_kernel: block i counts the digits of tile i (kSortTile
//      consecutive elements) into hist[i][256];
//   2. three small kernels turn hist into exclusive output offsets,
//      off[i][d] = (elements of all tiles with a digit below d)
//                + (elements of tiles before i with digit d),
//      scanning the [tiles][256] table down its columns in groups of
//      kScanRows tiles;
//   3. radix_scatter_kernel: block i ranks its tile's elements among equal
//      digits in index order (a wave splits its 64 lanes by digit with eight
//      ballots; the waves of a round and the rounds of a tile follow index
//      order) and writes each pair to off[i][d] + rank.
// Equal digits keep their input order in every pass, so the sort is stable.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                            // rounds of 256 elements per tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadix = 256;
constexpr int kSortBits = 62;                             // scene index in bits 57..61
constexpr int kSortPasses = (kSortBits + 7) / 8;
constexpr int kScanRows = 32;                             // tiles per column-scan block

static_assert(kSortPasses % 2 == 0, "the sorted pairs land back in the input buffers");

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const unsigned long long* __restrict__ keys,
                                                                  int n, int shift, int* __restrict__ hist) {
    __shared__ int cnt[kRadix];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kSortThreads + tid;
        if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & (kRadix - 1))], 1);
    }
    __syncthreads();
    hist[(int64_t)blockIdx.x * kRadix + tid] = cnt[tid];
}

// part[g][d] = sum of hist[i][d] over the tiles i of group g
__global__ __launch_bounds__(kRadix) void radix_colsum_kernel(const int* __restrict__ hist, int n_tiles,
                                                              int* __restrict__ part) {
    const int d = threadIdx.x;
    const int i0 = blockIdx.x * kScanRows, i1 = min(n_tiles, i0 + kScanRows);
    int s = 0;
    for (int i = i0; i < i1; ++i) s += hist[(int64_t)i * kRadix + d];
    part[(int64_t)blockIdx.x * kRadix + d] = s;
}

// One block: part[g][d] becomes the output offset of group g's first element
// with digit d (digit base plus the groups before g).
__global__ __launch_bounds__(kRadix) void radix_top_kernel(int* __restrict__ part, int n_groups) {
    __shared__ int tot[kRadix];
    const int d = threadIdx.x;
    int s = 0;
    for (int g = 0; g < n_groups; ++g) {
        const int c = part[(int64_t)g * kRadix + d];
        part[(int64_t)g * kRadix + d] = s;
        s += c;
    }
    tot[d] = s;
    __syncthreads();
    int below = 0;
    for (int e = 0; e < d; ++e) below += tot[e];
    for (int g = 0; g < n_groups; ++g) part[(int64_t)g * kRadix + d] += below;
}

// hist[i][d] becomes the output offset of tile i's first element with digit d
__global__ __launch_bounds__(kRadix) void radix_down_kernel(int* __restrict__ hist, int n_tiles,
                                                            const int* __restrict__ part) {
    const int d = threadIdx.x;
    const int i0 = blockIdx.x * kScanRows, i1 = min(n_tiles, i0 + kScanRows);
    int run = part[(int64_t)blockIdx.x * kRadix + d];
    for (int i = i0; i < i1; ++i) {
        const int c = hist[(int64_t)i * kRadix + d];
        hist[(int64_t)i * kRadix + d] = run;
        run += c;
    }
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const unsigned long long* __restrict__ kin, const int* __restrict__ vin, unsigned long long* __restrict__ kout,
    int* __restrict__ vout, int n, int shift, const int* __restrict__ off) {
    __shared__ int s_run[kRadix];          // next output position per digit
    __shared__ int s_cnt[4][kRadix];       // per wave of the round: elements per digit
    const int tid = threadIdx.x, wid = tid >> 6;
    s_run[tid] = off[(int64_t)blockIdx.x * kRadix + tid];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        for (int w = 0; w < 4; ++w) s_cnt[w][tid] = 0;
        const int64_t i = base + r * kSortThreads + tid;
        const bool valid = i < n;
        const unsigned long long key = valid ? kin[i] : 0ull;
        const int val = valid ? vin[i] : 0;
        const int d = (int)((key >> shift) & (kRadix - 1));
        // lanes of this wave holding the same digit
        unsigned long long same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const unsigned long long ones = __ballot((d >> b) & 1);
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
        __syncthreads();                   // counts cleared; s_run holds the earlier rounds
        if (valid && below == 0) s_cnt[wid][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int pos = s_run[d] + below;
            for (int w = 0; w < wid; ++w) pos += s_cnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();                   // every lane has read s_run
        s_run[tid] += s_cnt[0][tid] + s_cnt[1][tid] + s_cnt[2][tid] + s_cnt[3][tid];
    }
}

size_t radix_sort_scratch_bytes(int n) {
    const int64_t tiles = ((int64_t)n + kSortTile - 1) / kSortTile;
    const int64_t groups = (tiles + kScanRows - 1) / kScanRows;
    return (size_t)(tiles + groups) * kRadix * sizeof(int);
}

hipError_t radix_sort_pairs(unsigned long long* keys, unsigned long long* keys_tmp, int* vals, int* vals_tmp,
                            void* scratch, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int tiles = (int)(((int64_t)n + kSortTile - 1) / kSortTile);
    const int groups = (tiles + kScanRows - 1) / kScanRows;
    int* hist = (int*)scratch;
    int* part = hist + (int64_t)tiles * kRadix;
    unsigned long long* ka = keys;
    unsigned long long* kb = keys_tmp;
    int* va = vals;
    int* vb = vals_tmp;
    for (int pass = 0; pass < kSortPasses; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(tiles), dim3(kSortThreads), 0, st, ka, n, shift, hist);
        hipLaunchKernelGGL(radix_colsum_kernel, dim3(groups), dim3(kRadix), 0, st, hist, tiles, part);
        hipLaunchKernelGGL(radix_top_kernel, dim3(1), dim3(kRadix), 0, st, part, groups);
        hipLaunchKernelGGL(radix_down_kernel, dim3(groups), dim3(kRadix), 0, st, hist, tiles, part);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(tiles), dim3(kSortThreads), 0, st, ka, va, kb, vb, n, shift,
                           hist);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return hipSuccess;
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
