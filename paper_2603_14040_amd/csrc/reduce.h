// Deterministic block reductions with wave64 shuffles (CDNA wavefront = 64 lanes).
#pragma once
#include <hip/hip_runtime.h>

namespace tph {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of up to 1024 threads; the result is valid in thread 0.
// All threads of the block must call it (it synchronises twice).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    v = wave_sum(v);
    if ((tid & 63) == 0) part[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (tid == 0) {
        const int nw = (nthr + 63) >> 6;
        for (int w = 0; w < nw; ++w) t += part[w];
    }
    __syncthreads();
    return t;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    return v;
}

// Minimum over a block (valid in thread 0); all threads must call it.
__device__ __forceinline__ double block_min(double v) {
    __shared__ double part[16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    v = wave_min(v);
    if ((tid & 63) == 0) part[tid >> 6] = v;
    __syncthreads();
    double t = v;
    if (tid == 0) {
        const int nw = (nthr + 63) >> 6;
        for (int w = 0; w < nw; ++w) t = fmin(t, part[w]);
    }
    __syncthreads();
    return t;
}

}  // namespace tph
