// L2 data loss (Sec. 2.2): residual = y - d, loss = 1/2 sum residual^2.
// HBM-streaming pass with a fixed grid; each block writes one FP64 partial and a
// single block adds the partials in index order, so the scalar does not depend
// on scheduling.  Also the plain fill kernel used to clear outputs (a kernel
// rather than a memset so that the sequence can be captured in a graph).

#include <mutex>
#include <vector>

#include "sb_internal.hpp"

namespace sb {

constexpr int kLossThreads = 256;
constexpr int kLossBlocks = 2048;

int loss_blocks() { return kLossBlocks; }

// Block partials of slingbag_loss_noalloc: a fixed device array, so that the call
// allocates nothing (each device that loads the library holds one copy, 16 KiB, until
// the process ends).  In host code `scratch` names a host-side stand-in, not device
// memory: its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed to kernels.
constexpr int kNoallocPartials = 2048;
static __device__ __align__(256) double scratch[kNoallocPartials];
static_assert(kLossBlocks <= kNoallocPartials, "one partial per loss block");

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_addr;   // per device: device address of `scratch`

int noalloc_partials_capacity() { return kNoallocPartials; }

hipError_t noalloc_partials(double** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

__global__ __launch_bounds__(256) void fill_kernel(float* __restrict__ ptr, int64_t n, float v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = n / 4;
    float4* p4 = reinterpret_cast<float4*>(ptr);
    const float4 v4 = make_float4(v, v, v, v);
    if ((reinterpret_cast<uintptr_t>(ptr) & 15) == 0) {
        for (int64_t j = i; j < n4; j += stride) p4[j] = v4;
        for (int64_t j = n4 * 4 + i; j < n; j += stride) ptr[j] = v;
    } else {
        for (int64_t j = i; j < n; j += stride) ptr[j] = v;
    }
}

hipError_t launch_fill(float* ptr, int64_t n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n / 4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ptr, n, v);
    return hipGetLastError();
}

__global__ __launch_bounds__(kLossThreads) void loss_partial_kernel(const float* y, const float* d,
                                                                    float* r, int64_t n,
                                                                    double* partials) {
    __shared__ double red[kLossThreads / 64];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    const bool vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(d) |
                       reinterpret_cast<uintptr_t>(r)) & 15) == 0;
    int64_t tail0 = 0;
    if (vec) {
        const int64_t n4 = n / 4;
        const float4* y4 = reinterpret_cast<const float4*>(y);
        const float4* d4 = reinterpret_cast<const float4*>(d);
        float4* r4 = reinterpret_cast<float4*>(r);
        for (int64_t j = i0; j < n4; j += stride) {
            const float4 a = y4[j], b = d4[j];
            float4 e;
            e.x = a.x - b.x; e.y = a.y - b.y; e.z = a.z - b.z; e.w = a.w - b.w;
            r4[j] = e;
            acc += (double)e.x * e.x + (double)e.y * e.y + (double)e.z * e.z + (double)e.w * e.w;
        }
        tail0 = n4 * 4;
    }
    for (int64_t j = tail0 + i0; j < n; j += stride) {
        const float e = y[j] - d[j];
        r[j] = e;
        acc += (double)e * e;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kLossThreads / 64; ++w) s += red[w];
        partials[blockIdx.x] = 0.5 * s;
    }
}

__global__ __launch_bounds__(256) void loss_final_kernel(const double* partials, int n, double* loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
}

hipError_t launch_loss(const float* y, const float* d, float* r, int64_t n, double* partials,
                       int n_blocks, double* loss, hipStream_t st) {
    hipLaunchKernelGGL(loss_partial_kernel, dim3(n_blocks), dim3(kLossThreads), 0, st, y, d, r, n,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, partials, n_blocks, loss);
    return hipGetLastError();
}

}  // namespace sb

namespace sb {

// One Adam step over n parameters (bias-corrected; step >= 1).
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ param, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2, float lo, float hi) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float g = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        const float p = param[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        param[i] = fminf(fmaxf(p, lo), hi);      // projection onto [lo, hi]
    }
}

hipError_t launch_adam(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, float lo, float hi, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, st, param, grad, m, v, n, lr,
                       b1, b2, eps, c1, c2, lo, hi);
    return hipGetLastError();
}

}  // namespace sb
