// FP64 vector kernels of the accelerators (Sec. "Accelerators").
//
// Flexible GMRES (Sec. "Comparison with FGMRES"): multi-vector dot products
// (with the vector's own norm in the same pass), fused axpy + norm
// (classical Gram-Schmidt with a second pass only on cancellation),
// normalisation and the solution update.  Flexible GCR (Alg. "Flexible
// GCR(m)"): one pass that finishes a step - orthogonalises and normalises
// the new direction pair (w, z) and updates x and r.  Anderson acceleration
// (Alg. "Anderson Acceleration(m) with Mixing"): dot products over the
// unknowns only and the mixing combination of the stored iterates.
//
// Residual-type vectors are flat (vx | vy | p) arrays whose entries outside
// the equation rows are zero, so those kernels are plain 1D streams.
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

// One step of flexible GCR after the Gram-Schmidt coefficients are known:
//   w^ = (w - sum_j hw_j W_j) / nu   (orth_w = 0: w is already orthogonal)
//   r -= alpha w^
// and, when z is given, z' = (z - sum_j hz_j Z_j) / nu, x += alpha z'.
// The coefficients travel in the kernel arguments (uniform scalar loads).
__global__ __launch_bounds__(256) void k_gcr_step(const GcrStepArgs a) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < a.n; t += (size_t)gridDim.x * blockDim.x) {
        double wv = a.w[t];
        if (a.orth_w) {
#pragma unroll 4
            for (int j = 0; j < a.i; ++j) wv -= a.hw[j] * a.W0[j * a.stride + t];
        }
        wv *= a.inv_nu;
        a.w[t] = wv;
        a.r[t] -= a.alpha * wv;
        if (a.z) {
            double zv = a.z[t];
#pragma unroll 4
            for (int j = 0; j < a.i; ++j) zv -= a.hz[j] * a.Z0[j * a.stride + t];
            zv *= a.inv_nu;
            a.z[t] = zv;
            a.x[t] += a.alpha * zv;
        }
    }
}

// Dot products of f with up to kNV vectors (and f . f) over the unknowns of a
// three-field solution vector only: vx rows 1..ny, columns 1..nx-1; vy rows
// 1..ny-1, columns 1..nx; p rows 1..ny, columns 1..nx.  Ghost entries (which
// repeat wall-adjacent values) and walls are left out.  Blocks stride over
// the 3 (ny + 2) rows, threads over the columns of a row.
__global__ __launch_bounds__(256) void k_multidot_unknowns(Geom g, size_t fstride, VecSet vs, int nv,
                                                          const double* __restrict__ f,
                                                          double* __restrict__ partial, int nblk, int norm_slot) {
    double acc[kNV];
#pragma unroll
    for (int v = 0; v < kNV; ++v) acc[v] = 0.0;
    double nacc = 0.0;
    const int rows = g.ny + 2;
    for (int q = blockIdx.x; q < 3 * rows; q += gridDim.x) {
        const int fld = q / rows, i = q - fld * rows;
        const int ilast = fld == 1 ? g.ny - 1 : g.ny;
        const int jlast = fld == 0 ? g.nx - 1 : g.nx;
        if (i < 1 || i > ilast) continue;
        const size_t row = (size_t)(kAlign - 1) + fld * fstride + (size_t)i * g.pitch;
        for (int j = 1 + threadIdx.x; j <= jlast; j += blockDim.x) {
            const double fv = f[row + j];
#pragma unroll
            for (int v = 0; v < kNV; ++v)
                if (v < nv) acc[v] += vs.v[v][row + j] * fv;
            nacc += fv * fv;
        }
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

// out = (acc ? out : 0) + sum_v (cx_v X_v + cf_v F_v) over every entry.  out
// may be one of the X_v: each entry is read before it is written, by the
// same thread.
__global__ __launch_bounds__(256) void k_mix(const MixArgs a) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < a.n; t += (size_t)gridDim.x * blockDim.x) {
        double s = a.acc ? a.out[t] : 0.0;
#pragma unroll
        for (int v = 0; v < kNV; ++v)
            if (v < a.nv) s += a.cx[v] * a.X[v][t] + a.cf[v] * a.F[v][t];
        a.out[t] = s;
    }
}

// posts seq to mapped host memory once every earlier kernel on the stream is done
__global__ void k_post_seq(unsigned* __restrict__ host_seq, unsigned seq) {
    __threadfence_system();
    *(volatile unsigned*)host_seq = seq;
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

hipError_t launch_gcr_step(const GcrStepArgs& a, hipStream_t st) {
    if (a.i < 0 || a.i > kMaxRestart) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gcr_step, dim3(flat_blocks(a.n)), dim3(256), 0, st, a);
    return hipGetLastError();
}

int unknown_dot_blocks(const Geom& g) {
    const int rows = 3 * (g.ny + 2);
    return rows < 2048 ? rows : 2048;
}

hipError_t launch_multidot_unknowns(const Geom& g, size_t fstride, const double* const* vecs, int nv,
                                    const double* f, double* partial, int nblk, hipStream_t st, int norm_slot) {
    if (nv == 0 && norm_slot >= 0) {
        VecSet vs{};
        hipLaunchKernelGGL(k_multidot_unknowns, dim3(nblk), dim3(256), 0, st, g, fstride, vs, 0, f, partial, nblk,
                           norm_slot);
        return hipGetLastError();
    }
    for (int v0 = 0; v0 < nv; v0 += kNV) {
        const int c = nv - v0 < kNV ? nv - v0 : kNV;
        VecSet vs{};
        for (int v = 0; v < c; ++v) vs.v[v] = vecs[v0 + v];
        const int ns = (v0 == 0 && norm_slot >= 0) ? norm_slot : -1;
        hipLaunchKernelGGL(k_multidot_unknowns, dim3(nblk), dim3(256), 0, st, g, fstride, vs, c, f,
                           partial + (size_t)v0 * nblk, nblk, ns);
    }
    return hipGetLastError();
}

hipError_t launch_mix(double* out, const double* const* X, const double* cx, const double* const* F,
                      const double* cf, int nv, size_t n, hipStream_t st) {
    for (int v0 = 0; v0 < nv; v0 += kNV) {
        MixArgs a{};
        a.out = out;
        a.n = n;
        a.nv = nv - v0 < kNV ? nv - v0 : kNV;
        a.acc = v0 > 0 ? 1 : 0;
        for (int v = 0; v < a.nv; ++v) {
            a.X[v] = X[v0 + v];
            a.F[v] = F[v0 + v];
            a.cx[v] = cx[v0 + v];
            a.cf[v] = cf[v0 + v];
        }
        hipLaunchKernelGGL(k_mix, dim3(flat_blocks(n)), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_post_seq(unsigned* host_seq, unsigned seq, hipStream_t st) {
    hipLaunchKernelGGL(k_post_seq, dim3(1), dim3(1), 0, st, host_seq, seq);
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
