// Inter-level transfers for factor-2 coarsening (Ch. 4 "Restriction and
// Prolongation Operators").
//
// Restriction is the normalised bilinear weighting sum w r / sum w of
// Alg. "4-Color Parallel Restriction" written as a gather: each coarse node
// reads the fine nodes inside its footprint, so no colouring and no atomics
// are needed.  For ratio 2 the hat weights (1 - |r_x|)(1 - |r_y|) reduce to
//   nodes on coinciding lines:   1/2, 1, 1/2   (fine offsets -1, 0, +1)
//   staggered (half-cell) lines: 1/4, 3/4, 3/4, 1/4 (fine 2I-2 .. 2I+1)
// and fine nodes outside the physical domain (ghost rows/columns) are left
// out of both sums.  Prolongation is bilinear (weights 1 or 1/2, 1/2 on
// coinciding lines; 3/4, 1/4 on staggered lines) from the coarse correction
// whose ghosts already hold the mirrored values.
#include "kernels.h"

namespace tph {
namespace {

constexpr int BX = 64;
constexpr int BY = 4;

// weights of the 4-point staggered footprint, fine index 2I-2+q
__device__ __forceinline__ double w4(int q) { return (q == 1 || q == 2) ? 0.75 : 0.25; }
// weights of the 3-point coinciding footprint, fine index 2I-1+q
__device__ __forceinline__ double w3(int q) { return q == 1 ? 1.0 : 0.5; }

__global__ __launch_bounds__(256) void k_restrict_eta(Geom gf, Geom gc, const double* __restrict__ ebf,
                                                     const double* __restrict__ epf, double* __restrict__ ebc,
                                                     double* __restrict__ epc, int geometric) {
    const int J = blockIdx.x * BX + threadIdx.x;
    const int I = blockIdx.y * BY + threadIdx.y;
    if (I > gc.ny || J > gc.nx) return;
    const int Pf = gf.pitch;
    // basic grid: coarse node (I, J) = fine node (2I, 2J); fine nodes in [0, n]
    {
        double s = 0.0, ws = 0.0;
        for (int a = 0; a < 3; ++a) {
            const int i = 2 * I - 1 + a;
            if (i < 0 || i > gf.ny) continue;
            for (int b = 0; b < 3; ++b) {
                const int j = 2 * J - 1 + b;
                if (j < 0 || j > gf.nx) continue;
                const double w = w3(a) * w3(b);
                const double v = ebf[i * Pf + j];
                s += w * (geometric ? log(v) : v);
                ws += w;
            }
        }
        const double m = s / ws;
        ebc[I * gc.pitch + J] = geometric ? exp(m) : m;
    }
    // cell-centre grid: coarse cell (I, J) covers fine cells 2I-1, 2I; fine cells in [1, n]
    if (I >= 1 && J >= 1) {
        double s = 0.0, ws = 0.0;
        for (int a = 0; a < 4; ++a) {
            const int i = 2 * I - 2 + a;
            if (i < 1 || i > gf.ny) continue;
            for (int b = 0; b < 4; ++b) {
                const int j = 2 * J - 2 + b;
                if (j < 1 || j > gf.nx) continue;
                const double w = w4(a) * w4(b);
                const double v = epf[i * Pf + j];
                s += w * (geometric ? log(v) : v);
                ws += w;
            }
        }
        const double m = s / ws;
        epc[I * gc.pitch + J] = geometric ? exp(m) : m;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict_res(Geom gf, Geom gc, const T* __restrict__ tx,
                                                     const T* __restrict__ ty, T* __restrict__ rx,
                                                     T* __restrict__ ry) {
    const int J = blockIdx.x * BX + threadIdx.x + 1;
    const int I = blockIdx.y * BY + threadIdx.y + 1;
    if (I > gc.ny || J > gc.nx) return;
    const int Pf = gf.pitch;
    const int C = I * gc.pitch + J;
    if (J < gc.nx) {
        // vx: staggered in y (rows 2I-2 .. 2I+1 inside [1, ny]), coinciding in x (2J-1 .. 2J+1)
        T s = (T)0;
        T wy = (T)0;
        for (int a = 0; a < 4; ++a) {
            const int i = 2 * I - 2 + a;
            if (i < 1 || i > gf.ny) continue;
            const int c = i * Pf + 2 * J;
            const T row = (T)0.5 * tx[c - 1] + tx[c] + (T)0.5 * tx[c + 1];
            s += (T)w4(a) * row;
            wy += (T)w4(a);
        }
        rx[C] = s / ((T)2 * wy);
    }
    if (I < gc.ny) {
        // vy: coinciding in y (2I-1 .. 2I+1), staggered in x (2J-2 .. 2J+1 inside [1, nx])
        T s = (T)0;
        T wx = (T)0;
        for (int b = 0; b < 4; ++b) {
            const int j = 2 * J - 2 + b;
            if (j < 1 || j > gf.nx) continue;
            const int c = 2 * I * Pf + j;
            const T col = (T)0.5 * ty[c - Pf] + ty[c] + (T)0.5 * ty[c + Pf];
            s += (T)w4(b) * col;
            wx += (T)w4(b);
        }
        ry[C] = s / ((T)2 * wx);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(Geom gf, Geom gc, const T* __restrict__ ecx,
                                                    const T* __restrict__ ecy, T* __restrict__ ex,
                                                    T* __restrict__ ey) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > gf.ny || j > gf.nx) return;
    const int P = gf.pitch;
    const int Pc = gc.pitch;
    const int c = i * P + j;
    if (j < gf.nx) {
        // rows: staggered (3/4 nearest coarse row, 1/4 the next); columns: coinciding
        const int I0 = (i + 1) >> 1;                    // nearest coarse row
        const int I1 = (i & 1) ? I0 - 1 : I0 + 1;       // second coarse row (may be a ghost)
        T v;
        if ((j & 1) == 0) {
            const int J = j >> 1;
            v = (T)0.75 * ecx[I0 * Pc + J] + (T)0.25 * ecx[I1 * Pc + J];
        } else {
            const int J = j >> 1;                        // columns J, J + 1
            v = (T)0.375 * (ecx[I0 * Pc + J] + ecx[I0 * Pc + J + 1]) +
                (T)0.125 * (ecx[I1 * Pc + J] + ecx[I1 * Pc + J + 1]);
        }
        const T e = ex[c] + v;
        ex[c] = e;
        if (i == 1) ex[c - P] = (T)gf.mir[2] * e;
        if (i == gf.ny) ex[c + P] = (T)gf.mir[3] * e;
    }
    if (i < gf.ny) {
        const int J0 = (j + 1) >> 1;
        const int J1 = (j & 1) ? J0 - 1 : J0 + 1;
        T v;
        if ((i & 1) == 0) {
            const int I = i >> 1;
            v = (T)0.75 * ecy[I * Pc + J0] + (T)0.25 * ecy[I * Pc + J1];
        } else {
            const int I = i >> 1;
            v = (T)0.375 * (ecy[I * Pc + J0] + ecy[(I + 1) * Pc + J0]) +
                (T)0.125 * (ecy[I * Pc + J1] + ecy[(I + 1) * Pc + J1]);
        }
        const T e = ey[c] + v;
        ey[c] = e;
        if (j == 1) ey[c - 1] = (T)gf.mir[0] * e;
        if (j == gf.nx) ey[c + 1] = (T)gf.mir[1] * e;
    }
}

}  // namespace

hipError_t launch_restrict_eta(const Geom& gf, const Geom& gc, const double* ebf, const double* epf,
                               double* ebc, double* epc, bool geometric, hipStream_t st) {
    const dim3 grid((gc.nx + 1 + BX - 1) / BX, (gc.ny + 1 + BY - 1) / BY);
    hipLaunchKernelGGL(k_restrict_eta, grid, dim3(BX, BY), 0, st, gf, gc, ebf, epf, ebc, epc, geometric ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_res(const Geom& gf, const Geom& gc, const T* tx, const T* ty, T* rx, T* ry,
                               hipStream_t st) {
    const dim3 grid((gc.nx + BX - 1) / BX, (gc.ny + BY - 1) / BY);
    hipLaunchKernelGGL(k_restrict_res<T>, grid, dim3(BX, BY), 0, st, gf, gc, tx, ty, rx, ry);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const Geom& gf, const Geom& gc, const T* ecx, const T* ecy, T* ex, T* ey,
                              hipStream_t st) {
    const dim3 grid((gf.nx + BX - 1) / BX, (gf.ny + BY - 1) / BY);
    hipLaunchKernelGGL(k_prolong_add<T>, grid, dim3(BX, BY), 0, st, gf, gc, ecx, ecy, ex, ey);
    return hipGetLastError();
}

template hipError_t launch_restrict_res<float>(const Geom&, const Geom&, const float*, const float*, float*,
                                               float*, hipStream_t);
template hipError_t launch_restrict_res<double>(const Geom&, const Geom&, const double*, const double*, double*,
                                                double*, hipStream_t);
template hipError_t launch_prolong_add<float>(const Geom&, const Geom&, const float*, const float*, float*,
                                              float*, hipStream_t);
template hipError_t launch_prolong_add<double>(const Geom&, const Geom&, const double*, const double*, double*,
                                               double*, hipStream_t);

}  // namespace tph
