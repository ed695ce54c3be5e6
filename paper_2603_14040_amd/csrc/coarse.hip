// Coarsest-level solve in FP64 (Ch. 4 "Multigrid Cycles": the coarsest
// correction equation is solved directly).  The dense matrix M = -L of the
// coarsest level (symmetric positive definite) is assembled on the device
// from the rediscretised stencil, inverted once per coefficient set by an
// in-place Gauss-Jordan sweep in a single workgroup, and applied as a dense
// matrix-vector product (one wavefront per row).  Unknown order: vx(i, j)
// row-major (i in [1, ny], j in [1, nx-1]), then vy(i, j) (i in [1, ny-1],
// j in [1, nx]).
#include "kernels.h"
#include "reduce.h"

namespace tph {

int coarse_unknowns(const Geom& g) { return g.ny * (g.nx - 1) + (g.ny - 1) * g.nx; }

namespace {

__device__ __forceinline__ void unknown_to_node(const Geom& g, int m, int& comp, int& i, int& j) {
    const int nvx = g.ny * (g.nx - 1);
    if (m < nvx) {
        comp = 0;
        i = 1 + m / (g.nx - 1);
        j = 1 + m % (g.nx - 1);
    } else {
        m -= nvx;
        comp = 1;
        i = 1 + m / g.nx;
        j = 1 + m % g.nx;
    }
}

// Add coef * field(ci, cj) of an L row into row m of M = -L, resolving walls
// (dropped) and ghosts (mirrored onto the adjacent unknown).
__device__ __forceinline__ void add_ref(const Geom& g, double* row, int comp, int ci, int cj, double coef) {
    const int nvx = g.ny * (g.nx - 1);
    if (comp == 0) {
        if (cj <= 0 || cj >= g.nx) return;
        if (ci == 0) { ci = 1; coef *= g.mir[2]; }
        else if (ci == g.ny + 1) { ci = g.ny; coef *= g.mir[3]; }
        row[(ci - 1) * (g.nx - 1) + (cj - 1)] -= coef;
    } else {
        if (ci <= 0 || ci >= g.ny) return;
        if (cj == 0) { cj = 1; coef *= g.mir[0]; }
        else if (cj == g.nx + 1) { cj = g.nx; coef *= g.mir[1]; }
        row[nvx + (ci - 1) * g.nx + (cj - 1)] -= coef;
    }
}

__global__ void k_coarse_assemble(Geom g, const double* __restrict__ eb, const double* __restrict__ ep,
                                  double* __restrict__ M, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double* row = M + (size_t)m * n;
    for (int q = 0; q < n; ++q) row[q] = 0.0;
    int comp, i, j;
    unknown_to_node(g, m, comp, i, j);
    const int P = g.pitch;
    const int c = i * P + j;
    const double idx2 = 1.0 / (g.dx * g.dx), idy2 = 1.0 / (g.dy * g.dy), idxy = 1.0 / (g.dx * g.dy);
    if (comp == 0) {
        const double er = ep[c + 1], el = ep[c], bt = eb[c], bb = eb[c - P];
        add_ref(g, row, 0, i, j + 1, 2 * er * idx2);
        add_ref(g, row, 0, i, j, -2 * (er + el) * idx2 - (bt + bb) * idy2);
        add_ref(g, row, 0, i, j - 1, 2 * el * idx2);
        add_ref(g, row, 0, i + 1, j, bt * idy2);
        add_ref(g, row, 0, i - 1, j, bb * idy2);
        add_ref(g, row, 1, i, j + 1, bt * idxy);
        add_ref(g, row, 1, i, j, -bt * idxy);
        add_ref(g, row, 1, i - 1, j + 1, -bb * idxy);
        add_ref(g, row, 1, i - 1, j, bb * idxy);
    } else {
        const double et = ep[c + P], eb_ = ep[c], br = eb[c], bl = eb[c - 1];
        add_ref(g, row, 1, i + 1, j, 2 * et * idy2);
        add_ref(g, row, 1, i, j, -2 * (et + eb_) * idy2 - (br + bl) * idx2);
        add_ref(g, row, 1, i - 1, j, 2 * eb_ * idy2);
        add_ref(g, row, 1, i, j + 1, br * idx2);
        add_ref(g, row, 1, i, j - 1, bl * idx2);
        add_ref(g, row, 0, i + 1, j, br * idxy);
        add_ref(g, row, 0, i, j, -br * idxy);
        add_ref(g, row, 0, i + 1, j - 1, -bl * idxy);
        add_ref(g, row, 0, i, j - 1, bl * idxy);
    }
}

// In-place Gauss-Jordan inverse of an SPD matrix (no pivoting needed) in
// memory, one step k per pair of launches over the whole device: the pivot
// launch copies row k (scaled by 1 / M[k][k]) and column k into separate
// vectors, so the elimination launch can overwrite both while every row
// reads the values of the previous step.
__global__ __launch_bounds__(256) void k_gj_pivot(const double* __restrict__ M, int n, int k,
                                                  double* __restrict__ prow, double* __restrict__ pcol) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double rd = 1.0 / M[(size_t)k * n + k];
    prow[t] = t == k ? rd : M[(size_t)k * n + t] * rd;
    pcol[t] = M[(size_t)t * n + k];
}

__global__ __launch_bounds__(256) void k_gj_eliminate(double* __restrict__ M, int n, int k,
                                                      const double* __restrict__ prow,
                                                      const double* __restrict__ pcol) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    double* ri = M + (size_t)i * n;
    if (i == k) {
        ri[j] = prow[j];
        return;
    }
    const double f = pcol[i];
    if (j != k) ri[j] -= f * prow[j];
    else ri[j] = -f * prow[k];
}

// Gauss-Jordan inversion of a small SPD matrix (n <= kGJLds) by one
// workgroup of kGJThreads threads, the matrix held in registers: R =
// kGJThreads / n threads share a row, each owning a run of at most kGJRun
// consecutive entries.  Each step k copies the old row k and column k to
// LDS, then every thread updates its own entries (the same operations as
// the device-wide form: row k scaled by 1 / M[k][k], the others reduced by
// the scaled row), two barriers per step.  Blocks of a batched launch each
// invert their own matrix (mats[blockIdx.x], sizes ns[blockIdx.x]).
constexpr int kGJThreads = 1024;
constexpr int kGJRun = 20;   // max over n <= 136 of ceil(n / floor(1024 / n))
static_assert(kGJThreads >= kGJLds, "one row per thread at least");

__global__ __launch_bounds__(kGJThreads) void k_gauss_jordan_lds(double* const* __restrict__ mats,
                                                                const int* __restrict__ ns) {
    extern __shared__ double lds[];
    const int n = ns[blockIdx.x];
    double* __restrict__ Mg = mats[blockIdx.x];
    double* prow = lds;
    double* pcol = lds + n;
    const int tid = threadIdx.x;
    const int R = kGJThreads / n;                   // threads per row
    const int ch = (n + R - 1) / R;                 // run length
    const int i = tid / R, p = tid - (tid / R) * R;
    const int j0 = p * ch;
    const int cnt = i < n ? (j0 + ch <= n ? ch : (j0 < n ? n - j0 : 0)) : 0;
    double a[kGJRun];
#pragma unroll
    for (int c = 0; c < kGJRun; ++c) a[c] = c < cnt ? Mg[(size_t)i * n + j0 + c] : 0.0;
    for (int k = 0; k < n; ++k) {
#pragma unroll
        for (int c = 0; c < kGJRun; ++c) {
            if (c < cnt) {
                if (i == k) prow[j0 + c] = a[c];
                if (j0 + c == k) pcol[i] = a[c];
            }
        }
        __syncthreads();
        const double rd = 1.0 / pcol[k];
        const double f = cnt > 0 ? pcol[i] : 0.0;
#pragma unroll
        for (int c = 0; c < kGJRun; ++c) {
            if (c < cnt) {
                const int j = j0 + c;
                if (i == k) a[c] = j == k ? rd : a[c] * rd;
                else a[c] = j == k ? -f * rd : a[c] - f * (prow[j] * rd);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < kGJRun; ++c)
        if (c < cnt) Mg[(size_t)i * n + j0 + c] = a[c];
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(Geom g, const double* __restrict__ Minv,
                                                      const T* __restrict__ rx, const T* __restrict__ ry,
                                                      T* __restrict__ ex, T* __restrict__ ey, int n) {
    extern __shared__ double rs[];
    const int tid = threadIdx.x;
    const int P = g.pitch;
    for (int m = tid; m < n; m += blockDim.x) {
        int comp, i, j;
        unknown_to_node(g, m, comp, i, j);
        rs[m] = (double)(comp == 0 ? rx[i * P + j] : ry[i * P + j]);
    }
    __syncthreads();
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwave = blockDim.x >> 6;
    // one wave per row of the inverse; every workgroup holds the whole right-hand side
    for (int m = blockIdx.x * nwave + wave; m < n; m += gridDim.x * nwave) {
        const double* row = Minv + (size_t)m * n;
        double s = 0.0;
        for (int q = lane; q < n; q += 64) s += row[q] * rs[q];
        s = wave_sum(s);
        if (lane == 0) {
            // L e = r  <=>  e = -(-L)^{-1} r
            const T e = (T)(-s);
            int comp, i, j;
            unknown_to_node(g, m, comp, i, j);
            const int c = i * P + j;
            if (comp == 0) {
                ex[c] = e;
                if (i == 1) ex[c - P] = (T)g.mir[2] * e;
                if (i == g.ny) ex[c + P] = (T)g.mir[3] * e;
            } else {
                ey[c] = e;
                if (j == 1) ey[c - 1] = (T)g.mir[0] * e;
                if (j == g.nx) ey[c + 1] = (T)g.mir[1] * e;
            }
        }
    }
}

}  // namespace

hipError_t launch_coarse_assemble(const Geom& g, const double* eb, const double* ep, double* M, hipStream_t st) {
    const int n = coarse_unknowns(g);
    hipLaunchKernelGGL(k_coarse_assemble, dim3((n + 127) / 128), dim3(128), 0, st, g, eb, ep, M, n);
    return hipGetLastError();
}

size_t gauss_jordan_lds_bytes(int n) { return 2 * (size_t)n * sizeof(double); }

hipError_t launch_gauss_jordan_batched(double* const* mats, const int* ns, int count, int nmax, hipStream_t st) {
    const size_t lds = gauss_jordan_lds_bytes(nmax);
    if (nmax > kGJLds) return hipErrorInvalidValue;
    static thread_local int dev_cached = -1;
    static thread_local size_t granted = 64 * 1024;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
    if (dev != dev_cached) {
        dev_cached = dev;
        granted = 64 * 1024;
    }
    if (lds > granted) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_gauss_jordan_lds,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        granted = lds;
    }
    hipLaunchKernelGGL(k_gauss_jordan_lds, dim3(count), dim3(kGJThreads), lds, st, mats, ns);
    return hipGetLastError();
}

hipError_t launch_gauss_jordan(double* M, int n, hipStream_t st, double** table, double* work) {
    if (n <= kGJLds && table) {
        // table: device scratch of one pointer and one int (owned by the caller)
        return launch_gauss_jordan_batched(table, (const int*)(table + 1), 1, n, st);
    }
    if (!work) return hipErrorInvalidValue;
    double* prow = work;
    double* pcol = work + n;
    const dim3 g1((n + 255) / 256), g2((n + 255) / 256, n);
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, g1, dim3(256), 0, st, M, n, k, prow, pcol);
        hipLaunchKernelGGL(k_gj_eliminate, g2, dim3(256), 0, st, M, n, k, prow, pcol);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(const Geom& g, const double* Minv, const T* rx, const T* ry, T* ex, T* ey,
                               hipStream_t st) {
    const int n = coarse_unknowns(g);
    // 4 rows per workgroup: the n^2 inverse streams through the whole device
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3((n + 3) / 4), dim3(256), (size_t)n * sizeof(double), st, g, Minv, rx,
                       ry, ex, ey, n);
    return hipGetLastError();
}

template hipError_t launch_coarse_solve<float>(const Geom&, const double*, const float*, const float*, float*,
                                               float*, hipStream_t);
template hipError_t launch_coarse_solve<double>(const Geom&, const double*, const double*, const double*,
                                                double*, double*, hipStream_t);

}  // namespace tph
