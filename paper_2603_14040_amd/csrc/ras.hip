// RAS-type temporal-blocking Jacobi smoother (Sec. "The Multigrid Method",
// subsection "RAS-Type Jacobi Smoother", Alg. "RAS-Type Temporal Blocking").
//
// One launch is one outer iteration: the velocity unknowns are split into
// TT x TT tiles whose boundaries sit at rows 1 + si + k TT and columns
// 1 + sj + k TT (the shifts drawn for this outer iteration), one workgroup
// per tile.  A workgroup stages its tile with a halo of one node (both
// velocity components, both viscosities) in LDS, runs `inner` damped Jacobi
// sweeps on the unknowns it owns while the halo keeps the values the outer
// iteration started from, and writes its unknowns (with the ghost mirrors of
// wall-adjacent ones) to the output buffer.  Every unknown has one writer
// and every read comes from the input buffer, so the result does not depend
// on the order in which tiles run.  Bytes per sweep fall by `inner`: e, r
// and eta are read once per launch.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "stencil.h"

namespace tph {
namespace {

// one thread per tile node (both components): the sweeps' dependency chain is
// one update long per thread
template <int TT>
constexpr int ras_threads() { return TT * TT < 1024 ? TT * TT : 1024; }

template <typename T, int TT>
__global__ __launch_bounds__(ras_threads<TT>()) void k_ras_tile(Geom g, int si, int sj, int inner, int zero,
                                                         const T* __restrict__ exi, const T* __restrict__ eyi,
                                                         T* __restrict__ exo, T* __restrict__ eyo,
                                                         const T* __restrict__ rx, const T* __restrict__ ry,
                                                         const T* __restrict__ eb, const T* __restrict__ ep,
                                                         T omega) {
    constexpr int W = TT + 2;                 // LDS window side: the tile and a halo of one node
    constexpr int NQ = TT * TT;
    constexpr int NT = ras_threads<TT>();
    constexpr int K = (NQ + NT - 1) / NT;
    __shared__ T sx[2][W * W];
    __shared__ T sy[2][W * W];
    __shared__ T sb[W * W];
    __shared__ T sp[W * W];

    // tile rows [R0, R1), columns [C0, C1) of the index space [1, ny] x [1, nx]
    const int oi = si ? si - TT : 0, oj = sj ? sj - TT : 0;
    const int R0 = max(1, 1 + oi + (int)blockIdx.y * TT), R1 = min(g.ny + 1, 1 + oi + ((int)blockIdx.y + 1) * TT);
    const int C0 = max(1, 1 + oj + (int)blockIdx.x * TT), C1 = min(g.nx + 1, 1 + oj + ((int)blockIdx.x + 1) * TT);
    const int nr = R1 - R0 + 2, nc = C1 - C0 + 2;   // window rows / columns in use
    const int P = g.pitch;
    const size_t base = (size_t)(R0 - 1) * P + (C0 - 1);

    for (int q = threadIdx.x; q < W * W; q += NT) {
        const int a = q / W, b = q - a * W;
        T vx = (T)0, vy = (T)0, vb = (T)1, vp = (T)1;
        if (a < nr && b < nc) {
            const size_t c = base + (size_t)a * P + b;
            if (!zero) {
                vx = exi[c];
                vy = eyi[c];
            }
            vb = eb[c];
            vp = ep[c];
        }
        sx[0][q] = vx;
        sx[1][q] = vx;
        sy[0][q] = vy;
        sy[1][q] = vy;
        sb[q] = vb;
        sp[q] = vp;
    }
    // the unknowns this thread owns, their right-hand sides and diagonals
    const LevelC<T> kc = level_consts<T>(g);
    int lq[K], gi[K], gj[K];
    bool ox[K], oy[K];
    T rvx[K], rvy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = threadIdx.x + k * NT;
        const int a = q / TT + 1, b = q % TT + 1;
        const int i = R0 - 1 + a, j = C0 - 1 + b;
        const bool in = q < NQ && i < R1 && j < C1;
        ox[k] = in && j <= g.nx - 1;
        oy[k] = in && i <= g.ny - 1;
        lq[k] = a * W + b;
        gi[k] = i;
        gj[k] = j;
        const size_t c = (size_t)i * P + j;
        rvx[k] = ox[k] ? rx[c] : (T)0;
        rvy[k] = oy[k] ? ry[c] : (T)0;
    }
    __syncthreads();
    T dx[K], dy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        dx[k] = ox[k] ? lx_diag(sb, sp, lq[k], W, gi[k], g.ny, kc) : (T)1;
        dy[k] = oy[k] ? ly_diag(sb, sp, lq[k], W, gj[k], g.nx, kc) : (T)1;
    }
    int cur = 0;
    for (int t = 0; t < inner; ++t) {
        const T* X = sx[cur];
        const T* Y = sy[cur];
        T* XN = sx[cur ^ 1];
        T* YN = sy[cur ^ 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int c = lq[k];
            if (ox[k]) {
                const T e = X[c];
                const T v = relax(e, omega, rvx[k] - lx_row(X, Y, sb, sp, c, W, kc.idx, kc.idy), dx[k]);
                XN[c] = v;
                if (gi[k] == 1) XN[c - W] = kc.mirS * v;
                if (gi[k] == g.ny) XN[c + W] = kc.mirN * v;
            }
            if (oy[k]) {
                const T e = Y[c];
                const T v = relax(e, omega, rvy[k] - ly_row(X, Y, sb, sp, c, W, kc.idx, kc.idy), dy[k]);
                YN[c] = v;
                if (gj[k] == 1) YN[c - 1] = kc.mirW * v;
                if (gj[k] == g.nx) YN[c + 1] = kc.mirE * v;
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    const T* X = sx[cur];
    const T* Y = sy[cur];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const size_t c = (size_t)gi[k] * P + gj[k];
        const int q = lq[k];
        if (ox[k]) {
            exo[c] = X[q];
            if (gi[k] == 1) exo[c - P] = X[q - W];
            if (gi[k] == g.ny) exo[c + P] = X[q + W];
        }
        if (oy[k]) {
            eyo[c] = Y[q];
            if (gj[k] == 1) eyo[c - 1] = Y[q - 1];
            if (gj[k] == g.nx) eyo[c + 1] = Y[q + 1];
        }
    }
}

template <typename T, int TT>
hipError_t launch_ras_t(const Geom& g, int si, int sj, int inner, bool zero, const T* exi, const T* eyi, T* exo,
                        T* eyo, const T* rx, const T* ry, const T* eb, const T* ep, T omega, hipStream_t st) {
    const int oi = si ? si - TT : 0, oj = sj ? sj - TT : 0;
    const dim3 grid((g.nx - oj + TT - 1) / TT, (g.ny - oi + TT - 1) / TT);
    hipLaunchKernelGGL((k_ras_tile<T, TT>), grid, dim3(ras_threads<TT>()), 0, st, g, si, sj, inner, zero ? 1 : 0, exi, eyi,
                       exo, eyo, rx, ry, eb, ep, omega);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_ras_tile(const Geom& g, int tile, int si, int sj, int inner, bool zero, const T* exi, const T* eyi,
                           T* exo, T* eyo, const T* rx, const T* ry, const T* eb, const T* ep, T omega,
                           hipStream_t st) {
    if (si < 0 || sj < 0 || si >= tile || sj >= tile || inner < 1 || (!zero && (!exi || !eyi)) || exo == exi ||
        eyo == eyi)
        return hipErrorInvalidValue;
    switch (tile) {
        case 8: return launch_ras_t<T, 8>(g, si, sj, inner, zero, exi, eyi, exo, eyo, rx, ry, eb, ep, omega, st);
        case 16: return launch_ras_t<T, 16>(g, si, sj, inner, zero, exi, eyi, exo, eyo, rx, ry, eb, ep, omega, st);
        case 32: return launch_ras_t<T, 32>(g, si, sj, inner, zero, exi, eyi, exo, eyo, rx, ry, eb, ep, omega, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_ras_tile<float>(const Geom&, int, int, int, int, bool, const float*, const float*, float*,
                                           float*, const float*, const float*, const float*, const float*, float,
                                           hipStream_t);
template hipError_t launch_ras_tile<double>(const Geom&, int, int, int, int, bool, const double*, const double*,
                                            double*, double*, const double*, const double*, const double*,
                                            const double*, double, hipStream_t);

}  // namespace tph
