// FP64 reductions over a phi field: sums for conservation and error norms,
// extrema and a count of non-finite values.  Two passes: per-workgroup
// partials, then one workgroup folds them in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/lbm.h"
#include "lbm_internal.h"
#include "lbm_reduce.h"

namespace lbm {

int api_fail(int code, const char *msg);

namespace {

__global__ void __launch_bounds__(kBlock)
k_reduce_part(const double *__restrict__ phi, const double *__restrict__ ref, uint32_t n,
              double *__restrict__ part) {
    double acc[kRed];
    red_init(acc);
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        red_add(acc, phi[i], ref ? ref[i] : 0.0);
    red_block_fold(acc, part + (size_t)blockIdx.x * kRed);
}

__global__ void __launch_bounds__(kBlock)
k_reduce_final(const double *__restrict__ part, int nparts, double *__restrict__ out) {
    double acc[kRed];
    red_init(acc);
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        const double *q = part + (size_t)b * kRed;
#pragma unroll
        for (int i = 0; i < kRed; ++i)
            acc[i] = (i == 4) ? fmin(acc[i], q[i]) : ((i == 5) ? fmax(acc[i], q[i]) : acc[i] + q[i]);
    }
    red_block_fold(acc, out);
}

// acc[j] += sum_b part[b * width + j]
__global__ void __launch_bounds__(kBlock)
k_sum_partials(const double *__restrict__ part, int nparts, int width, double *__restrict__ acc) {
    __shared__ double sh[kBlock];
    for (int j = 0; j < width; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kBlock) v += part[(size_t)b * width + j];
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int s = kBlock / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) acc[j] += sh[0];
        __syncthreads();
    }
}

// Plain copy, the practical bandwidth of a read-once write-once stream and
// the reference for the traffic counters.  The buffer is cut into chunks of
// 1024 x 16 bytes; a workgroup copies whole chunks (four coalesced 16-byte
// loads per lane in flight, then the four stores), one chunk per workgroup
// when the grid covers them all, else looping over them.
__global__ void __launch_bounds__(kBlock)
k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n16) {
    constexpr size_t kChunk = 4 * kBlock;
    const size_t nchunks = (n16 + kChunk - 1) / kChunk;
    for (size_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const size_t i = c * kChunk + threadIdx.x;
        if (i + 3 * kBlock < n16) {
            const uint4 a = src[i], b = src[i + kBlock], d = src[i + 2 * kBlock], e = src[i + 3 * kBlock];
            dst[i] = a; dst[i + kBlock] = b; dst[i + 2 * kBlock] = d; dst[i + 3 * kBlock] = e;
        } else {
            for (size_t j = i; j < n16; j += kBlock) dst[j] = src[j];
        }
    }
}

}  // namespace

hipError_t launch_copy16(const void *src, void *dst, size_t n16, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, st, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *phi, const double *ref, uint32_t n, double *part, int nparts,
                         double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_part, dim3(nparts), dim3(kBlock), 0, st, phi, ref, n, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, part, nparts, out);
    return hipGetLastError();
}

hipError_t launch_reduce_final(const double *part, int nparts, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, part, nparts, out);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int nparts, int width, double *acc, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, st, part, nparts, width, acc);
    return hipGetLastError();
}

}  // namespace lbm

// ---- lbm_reduce_noalloc: the reductions with library-held partials --------
//
// The partial rows live in one file-scope device array instead of memory the
// library allocates.  Each device that runs the call holds its own copy of
// the array at its own address, found once per device with
// hipGetSymbolAddress; host code uses only that address (the array's name in
// host code is a stand-in, not a device pointer).

static __device__ __align__(256) double scratch[lbm::kRedParts * lbm::kRed];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// The address of this device's copy of `scratch` (nullptr and a message on
// failure).  The first call on a device resolves it, with that device current.
double *device_scratch(std::string *err) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { *err = std::string("hipGetDevice: ") + hipGetErrorString(e); return nullptr; }
    if (dev < 0 || dev >= kMaxDevices) { *err = "device index beyond the supported 64"; return nullptr; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_dev[dev] = (double *)ptr;
    }
    return g_scratch_dev[dev];
}

}  // namespace

extern "C" int lbm_reduce_noalloc(const double *phi_dev, const double *ref_dev, size_t n, double *out_dev,
                                  void *stream) {
    using namespace lbm;
    if (!phi_dev || !out_dev) return api_fail(LBM_E_INVALID, "null argument");
    if (n > (size_t)LBM_NOALLOC_MAX_NODES)
        return api_fail(LBM_E_INVALID, "lbm_reduce_noalloc: more than 2^31 - 1 values");
    std::string err;
    double *part = device_scratch(&err);
    if (!part) return api_fail(LBM_E_HIP, err.c_str());
    // the partial-row count of lbm_reduce_async on a context of n nodes, so
    // that both add in the same order
    int parts = (int)std::min<size_t>(kRedParts, (n + kBlock - 1) / kBlock);
    if (parts < 1) parts = 1;
    const hipError_t e = launch_reduce(phi_dev, ref_dev, (uint32_t)n, part, parts, out_dev, (hipStream_t)stream);
    if (e != hipSuccess) return api_fail(LBM_E_HIP, (std::string("reduction: ") + hipGetErrorString(e)).c_str());
    return LBM_OK;
}
