// Per-cell device bodies of the outer residual and of the preconditioner
// entry / exit, shared by the single-problem kernels (stencil.hip) and the
// batched kernels (batch.hip).  Thread (i, j) owns vx(i, j), vy(i, j) and
// p(i, j) and writes the ghost mirrored from an owned wall-adjacent value.
#pragma once
#include "common.h"
#include "stencil.h"

namespace tph {

// Outer FP64 residual / apply at cell (i, j); returns the sum of squares written.
__device__ __forceinline__ double outer_residual_cell(const Geom& g, const Vec3& x, const Vec3& b, int has_b,
                                                      const double* __restrict__ eb, const double* __restrict__ ep,
                                                      const Vec3& out, int apply, int energy, int bscaled, int i,
                                                      int j) {
    const LevelC<double> k = level_consts<double>(g);
    const int P = g.pitch;
    double acc = 0.0;
    if (i <= g.ny && j <= g.nx) {
        const int c = i * P + j;
        const double* vx = x.vx();
        const double* vy = x.vy();
        const double* p = x.p();
        if (j < g.nx) {
            const double a = lx_row(vx, vy, eb, ep, c, P, k.idx, k.idy) - (p[c + 1] - p[c]) * k.idx;
            const double sq = (energy || bscaled) ? sqrt(-lx_diag(eb, ep, c, P, i, g.ny, k)) : 1.0;
            double bv = has_b ? b.vx()[c] : 0.0;
            if (bscaled) bv *= sq;
            double r = apply ? a : (bv - a);
            if (energy) r *= 1.0 / sq;
            out.vx()[c] = r;
            acc += r * r;
        }
        if (i < g.ny) {
            const double a = ly_row(vx, vy, eb, ep, c, P, k.idx, k.idy) - (p[c + P] - p[c]) * k.idy;
            const double sq = (energy || bscaled) ? sqrt(-ly_diag(eb, ep, c, P, j, g.nx, k)) : 1.0;
            double bv = has_b ? b.vy()[c] : 0.0;
            if (bscaled) bv *= sq;
            double r = apply ? a : (bv - a);
            if (energy) r *= 1.0 / sq;
            out.vy()[c] = r;
            acc += r * r;
        }
        {
            const double a = (vx[c] - vx[c - 1]) * k.idx + (vy[c] - vy[c - P]) * k.idy;
            const double sw = (energy || bscaled) ? sqrt(wp_weight(ep[c], k)) : 1.0;
            double bv = has_b ? b.p()[c] : 0.0;
            if (bscaled) bv /= sw;
            double r = apply ? a : (bv - a);
            if (energy) r *= sw;
            out.p()[c] = r;
            acc += r * r;
        }
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ void precond_in_cell(const Geom& g, const Vec3& v, const double* __restrict__ eb,
                                                const double* __restrict__ ep, int energy, T* __restrict__ rx,
                                                T* __restrict__ ry, int i, int j) {
    if (i > g.ny || j > g.nx) return;
    const LevelC<double> k = level_consts<double>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    if (j < g.nx) {
        double r = v.vx()[c];
        if (energy) r *= sqrt(-lx_diag(eb, ep, c, P, i, g.ny, k));
        rx[c] = (T)r;
    }
    if (i < g.ny) {
        double r = v.vy()[c];
        if (energy) r *= sqrt(-ly_diag(eb, ep, c, P, j, g.nx, k));
        ry[c] = (T)r;
    }
}

template <typename T>
__device__ __forceinline__ void precond_out_cell(const Geom& g, const T* __restrict__ ex, const T* __restrict__ ey,
                                                 const Vec3& v, const double* __restrict__ ep, int energy,
                                                 double alpha, const Vec3& z, int acc, int i, int j) {
    if (i > g.ny || j > g.nx) return;
    const LevelC<double> k = level_consts<double>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    double* zx = z.vx();
    double* zy = z.vy();
    if (j < g.nx) {
        const double e = acc ? zx[c] + (double)ex[c] : (double)ex[c];
        zx[c] = e;
        if (i == 1) zx[c - P] = (double)g.mir[2] * e;
        if (i == g.ny) zx[c + P] = (double)g.mir[3] * e;
    }
    if (i < g.ny) {
        const double e = acc ? zy[c] + (double)ey[c] : (double)ey[c];
        zy[c] = e;
        if (j == 1) zy[c - 1] = (double)g.mir[0] * e;
        if (j == g.nx) zy[c + 1] = (double)g.mir[1] * e;
    }
    // divergence of this step's (cast) velocity correction; walls read as zero
    const double div = ((double)ex[c] - (double)ex[c - 1]) * k.idx + ((double)ey[c] - (double)ey[c - P]) * k.idy;
    double rp = v.p()[c];
    if (energy) rp *= 1.0 / sqrt(wp_weight(ep[c], k));
    const double dp = alpha * ep[c] * (rp - div);
    z.p()[c] = acc ? z.p()[c] + dp : dp;
}

}  // namespace tph
