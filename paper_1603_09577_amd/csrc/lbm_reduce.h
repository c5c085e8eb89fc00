// Device helpers of the FP64 reductions (sum, sum of squares, sum of squared
// and absolute differences to a reference, sum of the reference squared,
// min, max, count of non-finite values), shared by the reduction over a phi
// field and the one that forms phi from the state on the fly.  Both
// accumulate node i on thread i mod (grid x workgroup size) in increasing i
// and fold in the same fixed order, so their results are identical.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {

constexpr int kRed = 8;  // sum, sumsq, sum d^2, sum ref^2, min, max, nonfinite, sum |d|

__device__ __forceinline__ void red_init(double *acc) {
    acc[0] = acc[1] = acc[2] = acc[3] = acc[6] = acc[7] = 0.0;
    acc[4] = __builtin_inf();
    acc[5] = -__builtin_inf();
}

__device__ __forceinline__ void red_add(double *acc, double v, double r) {
    if (!__builtin_isfinite(v)) { acc[6] += 1.0; return; }
    const double d = v - r;
    acc[0] += v; acc[1] += v * v; acc[2] += d * d; acc[3] += r * r;
    acc[4] = fmin(acc[4], v); acc[5] = fmax(acc[5], v); acc[7] += fabs(d);
}

__device__ __forceinline__ double red_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double red_wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double red_wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Fold the per-thread values of a workgroup of kBlock threads into out[0..7]
// (written by the first kRed threads).  Called by every thread.
__device__ __forceinline__ void red_block_fold(double *acc, double *out) {
    __shared__ double sh[kRed][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kRed; ++i) {
        double v = acc[i];
        v = (i == 4) ? red_wave_min(v) : ((i == 5) ? red_wave_max(v) : red_wave_sum(v));
        if (lane == 0) sh[i][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < kRed) {
        const int i = threadIdx.x;
        double v = sh[i][0];
        for (int w = 1; w < kBlock / 64; ++w)
            v = (i == 4) ? fmin(v, sh[i][w]) : ((i == 5) ? fmax(v, sh[i][w]) : v + sh[i][w]);
        out[i] = v;
    }
}

}  // namespace lbm
