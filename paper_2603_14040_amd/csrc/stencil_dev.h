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

// Energy-weighted magnitude of the residual rows at cell (i, j): |b| plus the
// absolute terms of A x, scaled as the energy residual; returns the sum of
// their squares.  eps times its root bounds the size of the rounding error
// of b - A x (the floor below which the true residual cannot fall).
__device__ __forceinline__ double residual_magnitude_cell(const Geom& g, const Vec3& x, const Vec3& b,
                                                          const double* __restrict__ eb,
                                                          const double* __restrict__ ep, int i, int j) {
    const LevelC<double> k = level_consts<double>(g);
    const int P = g.pitch;
    double acc = 0.0;
    if (i <= g.ny && j <= g.nx) {
        const int c = i * P + j;
        const double* vx = x.vx();
        const double* vy = x.vy();
        const double* p = x.p();
        if (j < g.nx) {
            const double a = lx_row_abs(vx, vy, eb, ep, c, P, k.idx, k.idy) + (fabs(p[c + 1]) + fabs(p[c])) * k.idx;
            const double r = (fabs(b.vx()[c]) + a) / sqrt(-lx_diag(eb, ep, c, P, i, g.ny, k));
            acc += r * r;
        }
        if (i < g.ny) {
            const double a = ly_row_abs(vx, vy, eb, ep, c, P, k.idx, k.idy) + (fabs(p[c + P]) + fabs(p[c])) * k.idy;
            const double r = (fabs(b.vy()[c]) + a) / sqrt(-ly_diag(eb, ep, c, P, j, g.nx, k));
            acc += r * r;
        }
        {
            const double a = (fabs(vx[c]) + fabs(vx[c - 1])) * k.idx + (fabs(vy[c]) + fabs(vy[c - P])) * k.idy;
            const double r = (fabs(b.p()[c]) + a) * sqrt(wp_weight(ep[c], k));
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

// ---------------------------------------------------------------------------
// Link between two Uzawa steps of the preconditioner (or its last step and
// the Krylov apply), one pass per cell.  With e the V-cycle correction of
// this step and s the step's source (the preconditioner input r at the first
// step, energy-scaled or not; the residual t of the previous step after it):
//   z_new = z_old + e,  z_new_p = z_old_p + alpha eta_p (s_p - D e)
// (z_old = 0 at the first step), written to zout, then either
//   kLinkNext:  t = r - A z_new  -> FP32/FP64 right-hand side of the next
//               V-cycle (velocity) and tp (FP64 pressure part), or
//   kLinkApply: w = A z_new (energy-scaled for a Krylov basis) into wout, or
//   kLinkStore: nothing more (the last step when no apply is wanted).
// z_new at the neighbouring nodes the stencil needs is recomputed from e and
// z_old there (both carry mirrored ghosts and zero walls), so no pass
// waits for another; zout and zold must be different arrays.
// ---------------------------------------------------------------------------
enum { kLinkNext = 0, kLinkApply = 1, kLinkStore = 2 };

template <typename T>
struct LinkArgs {
    const T* ex;            // V-cycle correction (FP32 or FP64)
    const T* ey;
    Vec3 zold;              // previous z (ignored at the first step)
    int acc;                // 0 at the first step
    const double* srcp;     // pressure part of the step's source
    int src_scaled;         // source energy-scaled (first step inside FGMRES)
    double alpha;
    Vec3 zout;
    Vec3 r;                 // preconditioner input (for kLinkNext)
    int r_scaled;
    T* rx;                  // kLinkNext: next right-hand side
    T* ry;
    double* tp;
    Vec3 wout;              // kLinkApply
    int w_scaled;           // kLinkApply: w = W^(1/2) A z (Krylov basis scaling) instead of A z
};

template <typename T>
__device__ __forceinline__ double link_zx(const LinkArgs<T>& a, int c) {
    return (a.acc ? a.zold.vx()[c] : 0.0) + (double)a.ex[c];
}
template <typename T>
__device__ __forceinline__ double link_zy(const LinkArgs<T>& a, int c) {
    return (a.acc ? a.zold.vy()[c] : 0.0) + (double)a.ey[c];
}
template <typename T>
__device__ __forceinline__ double link_zp(const LinkArgs<T>& a, const double* __restrict__ ep, int c, int P,
                                          const LevelC<double>& k) {
    const double div = ((double)a.ex[c] - (double)a.ex[c - 1]) * k.idx + ((double)a.ey[c] - (double)a.ey[c - P]) * k.idy;
    double sp = a.srcp[c];
    if (a.src_scaled) sp *= 1.0 / sqrt(wp_weight(ep[c], k));
    return (a.acc ? a.zold.p()[c] : 0.0) + a.alpha * ep[c] * (sp - div);
}

// Per-cell loads and stores of the link that no neighbour shares: streaming
// (nontemporal) when NT, so that on grids far larger than the last-level
// cache they do not evict the shared 3 x 3 patch rows; ordinary otherwise,
// where the next kernel finds them in that cache.
template <bool NT, typename V>
__device__ __forceinline__ void link_st(V* p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <bool NT>
__device__ __forceinline__ double link_ld(const double* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T, int MODE, bool NT = false>
__device__ __forceinline__ void uzawa_link_cell(const Geom& g, const LinkArgs<T>& a, const double* __restrict__ eb,
                                                const double* __restrict__ ep, int i, int j) {
    if (i > g.ny || j > g.nx) return;
    const LevelC<double> k = level_consts<double>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    // 3 x 3 patches of z_new velocities and of the viscosities around (i, j)
    double zx[9], zy[9], pb[9], pe[9];
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            const int q = (di + 1) * 3 + (dj + 1), cc = c + di * P + dj;
            zx[q] = link_zx(a, cc);
            zy[q] = link_zy(a, cc);
            pb[q] = eb[cc];
            pe[q] = ep[cc];
        }
    }
    const double zpc = link_zp(a, ep, c, P, k);
    // this cell's z_new (with ghost mirrors of wall-adjacent values)
    if (j < g.nx) {
        link_st<NT>(a.zout.vx() + c, zx[4]);
        if (i == 1) a.zout.vx()[c - P] = (double)g.mir[2] * zx[4];
        if (i == g.ny) a.zout.vx()[c + P] = (double)g.mir[3] * zx[4];
    }
    if (i < g.ny) {
        link_st<NT>(a.zout.vy() + c, zy[4]);
        if (j == 1) a.zout.vy()[c - 1] = (double)g.mir[0] * zy[4];
        if (j == g.nx) a.zout.vy()[c + 1] = (double)g.mir[1] * zy[4];
    }
    link_st<NT>(a.zout.p() + c, zpc);
    if (MODE == kLinkStore) return;
    const double* X = zx + 4;
    const double* Y = zy + 4;
    const double* B = pb + 4;
    const double* E = pe + 4;
    if (j < g.nx) {
        const double av = lx_row(X, Y, B, E, 0, 3, k.idx, k.idy) - (link_zp(a, ep, c + 1, P, k) - zpc) * k.idx;
        const double sq = sqrt(-lx_diag(B, E, 0, 3, i, g.ny, k));
        if (MODE == kLinkNext) {
            double rv = link_ld<NT>(a.r.vx() + c);
            if (a.r_scaled) rv *= sq;
            link_st<NT>(a.rx + c, (T)(rv - av));
        } else {
            link_st<NT>(a.wout.vx() + c, a.w_scaled ? av / sq : av);
        }
    }
    if (i < g.ny) {
        const double av = ly_row(X, Y, B, E, 0, 3, k.idx, k.idy) - (link_zp(a, ep, c + P, P, k) - zpc) * k.idy;
        const double sq = sqrt(-ly_diag(B, E, 0, 3, j, g.nx, k));
        if (MODE == kLinkNext) {
            double rv = link_ld<NT>(a.r.vy() + c);
            if (a.r_scaled) rv *= sq;
            link_st<NT>(a.ry + c, (T)(rv - av));
        } else {
            link_st<NT>(a.wout.vy() + c, a.w_scaled ? av / sq : av);
        }
    }
    {
        const double av = (zx[4] - zx[3]) * k.idx + (zy[4] - zy[1]) * k.idy;
        const double sw = sqrt(wp_weight(ep[c], k));
        if (MODE == kLinkNext) {
            double rv = link_ld<NT>(a.r.p() + c);
            if (a.r_scaled) rv /= sw;
            link_st<NT>(a.tp + c, rv - av);
        } else {
            link_st<NT>(a.wout.p() + c, a.w_scaled ? av * sw : av);
        }
    }
}

}  // namespace tph
