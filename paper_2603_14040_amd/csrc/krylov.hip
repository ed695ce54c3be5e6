// FP64 Krylov vector kernels for flexible GMRES (Sec. "Comparison with
// FGMRES"): multi-vector dot products (with the vector's own norm in the
// same pass), fused axpy + norm (classical Gram-Schmidt with a second pass
// only on cancellation), normalisation and the solution update.  Vectors are flat (vx | vy | p) arrays whose entries
// outside the equation rows are zero, so every kernel is a plain 1D stream.
// Reductions are two-stage with a fixed block count and fixed summation
// order: results are bitwise reproducible run to run (no atomics).
#include "kernels.h"
#include "reduce.h"

namespace tph {

int flat_blocks(size_t n) {
    size_t b = (n + 2047) / 2048;                     // >= 8 elements per thread
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int)b;
}

namespace {

constexpr int kNV = 8;

__global__ __launch_bounds__(256) void k_multidot(const double* __restrict__ V0, size_t vstride, int nv,
                                                 const double* __restrict__ w, size_t n,
                                                 double* __restrict__ partial, int nblk, int norm_slot) {
    double acc[kNV];
#pragma unroll
    for (int v = 0; v < kNV; ++v) acc[v] = 0.0;
    double nacc = 0.0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double wv = w[t];
#pragma unroll
        for (int v = 0; v < kNV; ++v)
            if (v < nv) acc[v] += V0[v * vstride + t] * wv;
        nacc += wv * wv;
    }
#pragma unroll
    for (int v = 0; v < kNV; ++v) {
        if (v < nv) {
            const double s = block_sum(acc[v]);
            if (threadIdx.x == 0) partial[(size_t)v * nblk + blockIdx.x] = s;
        }
    }
    if (norm_slot >= 0) {
        const double s = block_sum(nacc);
        if (threadIdx.x == 0) partial[(size_t)norm_slot * nblk + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_axpy_dot(double* __restrict__ w, const double* __restrict__ V0,
                                                 size_t vstride, int nv, const double* __restrict__ h, size_t n,
                                                 int want_dots, int norm_slot, double* __restrict__ partial,
                                                 int nblk) {
    double hv[kNV];
    double acc[kNV];
#pragma unroll
    for (int v = 0; v < kNV; ++v) {
        hv[v] = v < nv ? h[v] : 0.0;
        acc[v] = 0.0;
    }
    double nacc = 0.0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double vv[kNV];
        double x = w[t];
#pragma unroll
        for (int v = 0; v < kNV; ++v) {
            vv[v] = v < nv ? V0[v * vstride + t] : 0.0;
            x -= hv[v] * vv[v];
        }
        w[t] = x;
        if (want_dots) {
#pragma unroll
            for (int v = 0; v < kNV; ++v) acc[v] += vv[v] * x;
        }
        nacc += x * x;
    }
    if (want_dots) {
#pragma unroll
        for (int v = 0; v < kNV; ++v) {
            if (v < nv) {
                const double s = block_sum(acc[v]);
                if (threadIdx.x == 0) partial[(size_t)v * nblk + blockIdx.x] = s;
            }
        }
    }
    if (norm_slot >= 0) {
        const double s = block_sum(nacc);
        if (threadIdx.x == 0) partial[(size_t)norm_slot * nblk + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_reduce_rows(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out, double* __restrict__ host_out,
                                                    unsigned* __restrict__ host_seq, unsigned seq) {
    const double* row = partial + (size_t)blockIdx.x * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += row[b];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        out[blockIdx.x] = s;
        if (host_out) host_out[blockIdx.x] = s;
        if (host_seq) {
            __threadfence_system();               // the values above reach host memory first
            *(volatile unsigned*)host_seq = seq;
        }
    }
}

__global__ __launch_bounds__(256) void k_scale_rnorm(double* __restrict__ dst, const double* __restrict__ src,
                                                    size_t n, const double* __restrict__ nrm2) {
    const double r = 1.0 / sqrt(nrm2[0]);
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        dst[t] = src[t] * r;
}

__global__ __launch_bounds__(256) void k_scale_rbeta(double* __restrict__ dst, const double* __restrict__ src,
                                                    size_t n, const double* __restrict__ beta) {
    const double r = 1.0 / beta[0];
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        dst[t] = src[t] * r;
}

__global__ __launch_bounds__(256) void k_update_x(double* __restrict__ x, const double* __restrict__ Z0,
                                                 size_t zstride, int k, const double* __restrict__ y, size_t n) {
    double yv[kNV];
#pragma unroll
    for (int v = 0; v < kNV; ++v) yv[v] = v < k ? y[v] : 0.0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double s = x[t];
#pragma unroll
        for (int v = 0; v < kNV; ++v)
            if (v < k) s += yv[v] * Z0[v * zstride + t];
        x[t] = s;
    }
}

__global__ __launch_bounds__(256) void k_p_sum(Geom g, const double* __restrict__ p, double* __restrict__ partial) {
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    double v = 0.0;
    if (i <= g.ny && j <= g.nx) v = p[i * g.pitch + j];
    const double s = block_sum(v);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_p_shift(Geom g, double* __restrict__ p, const double* __restrict__ sum) {
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    if (i > g.ny || j > g.nx) return;
    p[i * g.pitch + j] -= sum[0] / ((double)g.nx * (double)g.ny);
}

}  // namespace

hipError_t launch_multidot(const double* V0, size_t vstride, int nv, const double* w, size_t n, double* partial,
                           int nblk, hipStream_t st, int norm_slot) {
    for (int v0 = 0; v0 < nv; v0 += kNV) {
        const int c = nv - v0 < kNV ? nv - v0 : kNV;
        // the norm slot is an absolute row index; offset it for this chunk's partial base
        const int ns = (v0 == 0 && norm_slot >= 0) ? norm_slot : -1;
        hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(256), 0, st, V0 + v0 * vstride, vstride, c, w, n,
                           partial + (size_t)v0 * nblk, nblk, ns);
    }
    return hipGetLastError();
}

hipError_t launch_axpy_dot(double* w, const double* V0, size_t vstride, int nv, const double* h, size_t n,
                           bool want_dots, int norm_slot, double* partial, int nblk, hipStream_t st) {
    if (nv <= kNV) {
        hipLaunchKernelGGL(k_axpy_dot, dim3(nblk), dim3(256), 0, st, w, V0, vstride, nv, h, n, want_dots ? 1 : 0,
                           norm_slot, partial, nblk);
        return hipGetLastError();
    }
    // more than kNV basis vectors: subtract in chunks, then one dot pass
    for (int v0 = 0; v0 < nv; v0 += kNV) {
        const int c = nv - v0 < kNV ? nv - v0 : kNV;
        const bool last = v0 + c >= nv;
        hipLaunchKernelGGL(k_axpy_dot, dim3(nblk), dim3(256), 0, st, w, V0 + v0 * vstride, vstride, c, h + v0, n, 0,
                           last ? norm_slot : -1, partial, nblk);
    }
    if (want_dots) return launch_multidot(V0, vstride, nv, w, n, partial, nblk, st, -1);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const double* partial, int nblk, int k, double* out, hipStream_t st,
                              double* host_out, unsigned* host_seq, unsigned seq) {
    if (host_seq && k != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce_rows, dim3(k), dim3(256), 0, st, partial, nblk, out, host_out, host_seq, seq);
    return hipGetLastError();
}

hipError_t launch_scale_by_rnorm(double* dst, const double* src, size_t n, const double* nrm2, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_rnorm, dim3(flat_blocks(n)), dim3(256), 0, st, dst, src, n, nrm2);
    return hipGetLastError();
}

hipError_t launch_scale_by_rbeta(double* dst, const double* src, size_t n, const double* beta, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_rbeta, dim3(flat_blocks(n)), dim3(256), 0, st, dst, src, n, beta);
    return hipGetLastError();
}

hipError_t launch_update_x(double* x, const double* Z0, size_t zstride, int k, const double* y, size_t n,
                           hipStream_t st) {
    for (int v0 = 0; v0 < k; v0 += kNV) {
        const int c = k - v0 < kNV ? k - v0 : kNV;
        hipLaunchKernelGGL(k_update_x, dim3(flat_blocks(n)), dim3(256), 0, st, x, Z0 + v0 * zstride, zstride, c,
                           y + v0, n);
    }
    return hipGetLastError();
}

hipError_t launch_p_sum(const Geom& g, const double* p, double* partial, int* nblk_out, hipStream_t st) {
    const dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4);
    if (nblk_out) *nblk_out = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_p_sum, grid, dim3(64, 4), 0, st, g, p, partial);
    return hipGetLastError();
}

hipError_t launch_p_shift(const Geom& g, double* p, const double* sum, hipStream_t st) {
    const dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4);
    hipLaunchKernelGGL(k_p_shift, grid, dim3(64, 4), 0, st, g, p, sum);
    return hipGetLastError();
}

}  // namespace tph
