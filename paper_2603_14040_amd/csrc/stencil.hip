// Stencil kernels: outer FP64 residual / operator apply, smoothers on L,
// preconditioner entry/exit (Uzawa pressure step), right-hand side,
// coefficient checks and the adjoint coefficient gradient.
//
// Thread mapping: one thread per cell (i, j), i in [1, ny], j in [1, nx];
// blocks of 64 x 4 with the 64 lanes of a wavefront along a row, so every
// field access of a wavefront is one contiguous, 64-element-aligned segment
// (see the layout note in common.h).  A thread owns vx(i, j) (j < nx),
// vy(i, j) (i < ny) and p(i, j) and writes the ghost entry mirrored from an
// owned wall-adjacent value, so solution-type arrays stay ghost-consistent
// without a separate boundary pass.
#include <hip/hip_ext.h>

#include "kernels.h"
#include "reduce.h"
#include "stencil.h"
#include "stencil_dev.h"

namespace tph {
namespace {

constexpr int BX = kCellBX;
constexpr int BY = kCellBY;
static_assert(BX * BY <= 256, "the cell kernels are compiled for blocks of at most 256 threads");

inline dim3 grid_cells(const Geom& g) { return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY); }

__global__ __launch_bounds__(256) void k_outer_residual(Geom g, Vec3 x, Vec3 b, int has_b,
                                                       const double* __restrict__ eb,
                                                       const double* __restrict__ ep, Vec3 out,
                                                       int apply, int energy, double* partial, int bscaled) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    const double acc = outer_residual_cell(g, x, b, has_b, eb, ep, out, apply, energy, bscaled, i, j);
    if (partial) {
        const double s = block_sum(acc);
        if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_residual_magnitude(Geom g, Vec3 x, Vec3 b, const double* __restrict__ eb,
                                                           const double* __restrict__ ep, double* partial) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    const double s = block_sum(residual_magnitude_cell(g, x, b, eb, ep, i, j));
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_bc(Geom g, T* vx, T* vy) {
    // grid over [0, ny+1] x [0, nx+1]
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y * BY + threadIdx.y;
    if (i > g.ny + 1 || j > g.nx + 1) return;
    const int P = g.pitch;
    const int c = i * P + j;
    // vx: walls j = 0, nx (and the unused column nx + 1) are zero; rows 0 and ny+1 mirror
    if (j == 0 || j >= g.nx) {
        vx[c] = (T)0;
    } else if (i == 0) {
        vx[c] = (T)g.mir[2] * vx[c + P];
    } else if (i == g.ny + 1) {
        vx[c] = (T)g.mir[3] * vx[c - P];
    }
    // vy: walls i = 0, ny (and row ny + 1) are zero; columns 0 and nx+1 mirror
    if (i == 0 || i >= g.ny) {
        vy[c] = (T)0;
    } else if (j == 0) {
        vy[c] = (T)g.mir[0] * vy[c + 1];
    } else if (j == g.nx + 1) {
        vy[c] = (T)g.mir[1] * vy[c - 1];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_jacobi(Geom g, const T* __restrict__ exi, const T* __restrict__ eyi,
                                               T* __restrict__ exo, T* __restrict__ eyo,
                                               const T* __restrict__ rx, const T* __restrict__ ry,
                                               const T* __restrict__ eb, const T* __restrict__ ep, T omega,
                                               int zero) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.ny || j > g.nx) return;
    const LevelC<T> k = level_consts<T>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    if (j < g.nx) {
        const T d = lx_diag(eb, ep, c, P, i, g.ny, k);
        T e;
        if (zero) {
            e = omega * rx[c] / d;
        } else {
            const T res = rx[c] - lx_row(exi, eyi, eb, ep, c, P, k.idx, k.idy);
            e = exi[c] + omega * res / d;
        }
        exo[c] = e;
        if (i == 1) exo[c - P] = k.mirS * e;
        if (i == g.ny) exo[c + P] = k.mirN * e;
    }
    if (i < g.ny) {
        const T d = ly_diag(eb, ep, c, P, j, g.nx, k);
        T e;
        if (zero) {
            e = omega * ry[c] / d;
        } else {
            const T res = ry[c] - ly_row(exi, eyi, eb, ep, c, P, k.idx, k.idy);
            e = eyi[c] + omega * res / d;
        }
        eyo[c] = e;
        if (j == 1) eyo[c - 1] = k.mirW * e;
        if (j == g.nx) eyo[c + 1] = k.mirE * e;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gs_half(Geom g, int comp, int col, T* __restrict__ ex,
                                                T* __restrict__ ey, const T* __restrict__ rx,
                                                const T* __restrict__ ry, const T* __restrict__ eb,
                                                const T* __restrict__ ep, T omega, int zero_guess) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.ny || j > g.nx) return;
    const LevelC<T> k = level_consts<T>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    const bool mine = ((i + j) & 1) == col;
    if (zero_guess) {
        // first half-sweep (vx, colour col) from a zero initial guess: every
        // other entry of the correction is zero, written here as well
        if (j < g.nx) {
            const T e = mine ? omega * rx[c] / lx_diag(eb, ep, c, P, i, g.ny, k) : (T)0;
            ex[c] = e;
            if (i == 1) ex[c - P] = k.mirS * e;
            if (i == g.ny) ex[c + P] = k.mirN * e;
        }
        if (i < g.ny) {
            ey[c] = (T)0;
            if (j == 1) ey[c - 1] = (T)0;
            if (j == g.nx) ey[c + 1] = (T)0;
        }
        return;
    }
    if (!mine) return;
    if (comp == 0) {
        if (j >= g.nx) return;
        const T d = lx_diag(eb, ep, c, P, i, g.ny, k);
        const T res = rx[c] - lx_row(ex, ey, eb, ep, c, P, k.idx, k.idy);
        const T e = ex[c] + omega * res / d;
        ex[c] = e;
        if (i == 1) ex[c - P] = k.mirS * e;
        if (i == g.ny) ex[c + P] = k.mirN * e;
    } else {
        if (i >= g.ny) return;
        const T d = ly_diag(eb, ep, c, P, j, g.nx, k);
        const T res = ry[c] - ly_row(ex, ey, eb, ep, c, P, k.idx, k.idy);
        const T e = ey[c] + omega * res / d;
        ey[c] = e;
        if (j == 1) ey[c - 1] = k.mirW * e;
        if (j == g.nx) ey[c + 1] = k.mirE * e;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_vel_residual(Geom g, const T* __restrict__ ex, const T* __restrict__ ey,
                                                     const T* __restrict__ rx, const T* __restrict__ ry,
                                                     const T* __restrict__ eb, const T* __restrict__ ep,
                                                     T* __restrict__ tx, T* __restrict__ ty) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.ny || j > g.nx) return;
    const LevelC<T> k = level_consts<T>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    if (j < g.nx) tx[c] = rx[c] - lx_row(ex, ey, eb, ep, c, P, k.idx, k.idy);
    if (i < g.ny) ty[c] = ry[c] - ly_row(ex, ey, eb, ep, c, P, k.idx, k.idy);
}

template <typename T>
__global__ __launch_bounds__(256) void k_precond_in(Geom g, Vec3 v, const double* __restrict__ eb,
                                                   const double* __restrict__ ep, int energy,
                                                   T* __restrict__ rx, T* __restrict__ ry) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    precond_in_cell<T>(g, v, eb, ep, energy, rx, ry, i, j);
}

template <typename T>
__global__ __launch_bounds__(256) void k_precond_out(Geom g, const T* __restrict__ ex, const T* __restrict__ ey,
                                                    Vec3 v, const double* __restrict__ ep, int energy,
                                                    double alpha, Vec3 z, int acc) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    precond_out_cell<T>(g, ex, ey, v, ep, energy, alpha, z, acc, i, j);
}

template <typename T, int MODE, bool NT>
__global__ __launch_bounds__(256) void k_uzawa_link(Geom g, LinkArgs<T> a, const double* __restrict__ eb,
                                                   const double* __restrict__ ep) {
    // XCD-aware block order: each XCD takes a band of block rows, so the halo
    // rows of the 3 x 3 patches are shared through that XCD's L2
    int bx, by;
    xcd_tile(bx, by);
    const int j = bx * BX + threadIdx.x + 1;
    const int i = by * BY + threadIdx.y + 1;
    uzawa_link_cell<T, MODE, NT>(g, a, eb, ep, i, j);
}

// Lithostatic pressure, one thread per column marching up the rows: the
// hydrostatic balance of each y-momentum row for zero velocity,
// p(i+1, j) - p(i, j) = gy dy (rho_b(i, j-1) + rho_b(i, j)) / 2, p(1, j) = 0.
__global__ __launch_bounds__(256) void k_lithostatic(Geom g, const double* __restrict__ rho, double gy,
                                                    double* __restrict__ p) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j > g.nx) return;
    const int P = g.pitch;
    double acc = 0.0;
    for (int i = 1; i <= g.ny; ++i) {
        p[i * P + j] = acc;
        if (i < g.ny) acc += gy * g.dy * 0.5 * (rho[i * P + j - 1] + rho[i * P + j]);
    }
}

// block minima of eta_b over the basic nodes (0..ny, 0..nx) and of eta_p over the cells
__global__ __launch_bounds__(256) void k_eta_min(Geom g, const double* __restrict__ eb,
                                                const double* __restrict__ ep, double* __restrict__ partial) {
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y * BY + threadIdx.y;
    double v = HUGE_VAL;
    if (i <= g.ny && j <= g.nx) {
        v = eb[i * g.pitch + j];
        if (i >= 1 && j >= 1) v = fmin(v, ep[i * g.pitch + j]);
    }
    const double m = block_min(v);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_min_rows(const double* __restrict__ partial, int n,
                                                 double* __restrict__ out) {
    double v = HUGE_VAL;
    for (int t = threadIdx.x; t < n; t += blockDim.x) v = fmin(v, partial[t]);
    const double m = block_min(v);
    if (threadIdx.x == 0) out[0] = m;
}

// out = (1 - theta) m + theta in over n entries
__global__ __launch_bounds__(256) void k_blend(const double* __restrict__ in, double* __restrict__ out, size_t n,
                                              double theta, double m) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = (1.0 - theta) * m + theta * in[t];
}

__global__ __launch_bounds__(256) void k_rhs(Geom g, const double* __restrict__ rho, double gx, double gy,
                                            const double* __restrict__ fxe, const double* __restrict__ fye,
                                            Vec3 b) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.ny || j > g.nx) return;
    const int P = g.pitch;
    const int c = i * P + j;
    if (j < g.nx) b.vx()[c] = -gx * 0.5 * (rho[c - P] + rho[c]) + (fxe ? fxe[c] : 0.0);
    if (i < g.ny) b.vy()[c] = -gy * 0.5 * (rho[c - 1] + rho[c]) + (fye ? fye[c] : 0.0);
    b.p()[c] = 0.0;
}

__global__ __launch_bounds__(256) void k_check_coeffs(Geom g, const double* __restrict__ eb,
                                                     const double* __restrict__ ep,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ fxe,
                                                     const double* __restrict__ fye, double* partial,
                                                     int nblk) {
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y * BY + threadIdx.y;
    double bad_eta = 0.0, bad_rho = 0.0;
    if (i <= g.ny && j <= g.nx) {
        const int c = i * g.pitch + j;
        const double b = eb[c];
        if (!(b > 0.0) || !isfinite(b)) bad_eta += 1.0;
        if (!isfinite(rho[c])) bad_rho += 1.0;
        if (i >= 1 && j >= 1) {
            const double p = ep[c];
            if (!(p > 0.0) || !isfinite(p)) bad_eta += 1.0;
        }
        if (fxe && i >= 1 && j >= 1 && j < g.nx && !isfinite(fxe[c])) bad_rho += 1.0;
        if (fye && i >= 1 && j >= 1 && i < g.ny && !isfinite(fye[c])) bad_rho += 1.0;
    }
    const double s1 = block_sum(bad_eta);
    const double s2 = block_sum(bad_rho);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        partial[blk] = s1;
        partial[nblk + blk] = s2;
    }
}

__global__ __launch_bounds__(256) void k_coeff_gradient(Geom g, Vec3 x, Vec3 lam, double gx, double gy,
                                                       double* g_eb, double* g_ep, double* g_rho) {
    // grid over basic nodes [0, ny] x [0, nx]; cell-centre outputs at i, j >= 1
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y * BY + threadIdx.y;
    if (i > g.ny || j > g.nx) return;
    const LevelC<double> k = level_consts<double>(g);
    const int P = g.pitch;
    const int c = i * P + j;
    const double *ux = x.vx(), *uy = x.vy(), *lx = lam.vx(), *ly = lam.vy();
    if (g_ep && i >= 1 && j >= 1) {
        const double exx_u = (ux[c] - ux[c - 1]) * k.idx, exx_l = (lx[c] - lx[c - 1]) * k.idx;
        const double eyy_u = (uy[c] - uy[c - P]) * k.idy, eyy_l = (ly[c] - ly[c - P]) * k.idy;
        g_ep[c] = 2.0 * (exx_l * exx_u + eyy_l * eyy_u);
    }
    if (g_eb) {
        const double gam_u = (ux[c + P] - ux[c]) * k.idy + (uy[c + 1] - uy[c]) * k.idx;
        const double gam_l = (lx[c + P] - lx[c]) * k.idy + (ly[c + 1] - ly[c]) * k.idx;
        double w = 1.0;
        if (i == 0 || i == g.ny) w *= 0.5;
        if (j == 0 || j == g.nx) w *= 0.5;
        g_eb[c] = w * gam_l * gam_u;
    }
    if (g_rho) {
        // rho_b(i, j) enters f_x at vx(i, j), vx(i+1, j) and f_y at vy(i, j), vy(i, j+1)
        double s = 0.0;
        const bool colx = (j >= 1 && j <= g.nx - 1);
        if (colx && i >= 1) s += lx[c];
        if (colx && i + 1 <= g.ny) s += lx[c + P];
        double t = 0.0;
        const bool rowy = (i >= 1 && i <= g.ny - 1);
        if (rowy && j >= 1) t += ly[c];
        if (rowy && j + 1 <= g.nx) t += ly[c + 1];
        g_rho[c] = -gx * 0.5 * s - gy * 0.5 * t;
    }
}

// Gradient with respect to the full output arrays of a solve -> right-hand
// side of the adjoint solve: a ghost entry is mirror * its interior owner,
// so its gradient is folded onto the owner; wall entries are fixed zeros.
__global__ __launch_bounds__(256) void k_fold_ghost_grad(Geom g, Vec3 v) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.ny || j > g.nx) return;
    const int P = g.pitch;
    const int c = i * P + j;
    double* gx = v.vx();
    double* gy = v.vy();
    if (j < g.nx) {
        double a = gx[c];
        if (i == 1) a += (double)g.mir[2] * gx[c - P];
        if (i == g.ny) a += (double)g.mir[3] * gx[c + P];
        gx[c] = a;
    }
    if (i < g.ny) {
        double a = gy[c];
        if (j == 1) a += (double)g.mir[0] * gy[c - 1];
        if (j == g.nx) a += (double)g.mir[1] * gy[c + 1];
        gy[c] = a;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_vel(Geom g, T* __restrict__ ex, T* __restrict__ ey) {
    // grid over [0, ny+1] x [0, nx+1]: every entry of both arrays
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y * BY + threadIdx.y;
    if (i > g.ny + 1 || j > g.nx + 1) return;
    ex[i * g.pitch + j] = (T)0;
    ey[i * g.pitch + j] = (T)0;
}

// FP64 -> FP32 copies of whole arrays, one array of the list per blockIdx.y
__global__ void k_cast_list(CastList c) {
    const double* __restrict__ s = c.src[blockIdx.y];
    float* __restrict__ d = c.dst[blockIdx.y];
    const size_t n = c.n[blockIdx.y];
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        d[t] = (float)s[t];
}

}  // namespace

hipError_t launch_outer_residual(const Geom& g, Vec3 x, const Vec3* b, const double* eb, const double* ep,
                                 Vec3 out, ResMode mode, bool energy, double* partial, int* nblk_out,
                                 hipStream_t st, bool b_scaled) {
    const dim3 grid = grid_cells(g);
    if (nblk_out) *nblk_out = (int)(grid.x * grid.y);
    Vec3 bb = b ? *b : Vec3{nullptr, 0};
    hipLaunchKernelGGL(k_outer_residual, grid, dim3(BX, BY), 0, st, g, x, bb, b ? 1 : 0, eb, ep, out,
                       mode == ResMode::kApply ? 1 : 0, energy ? 1 : 0, partial, b_scaled ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_residual_magnitude(const Geom& g, Vec3 x, Vec3 b, const double* eb, const double* ep,
                                    double* partial, int* nblk_out, hipStream_t st) {
    const dim3 grid = grid_cells(g);
    *nblk_out = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_residual_magnitude, grid, dim3(BX, BY), 0, st, g, x, b, eb, ep, partial);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_bc(const Geom& g, T* vx, T* vy, hipStream_t st) {
    const dim3 grid((g.nx + 2 + BX - 1) / BX, (g.ny + 2 + BY - 1) / BY);
    hipLaunchKernelGGL(k_fill_bc<T>, grid, dim3(BX, BY), 0, st, g, vx, vy);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zero_vel(const Geom& g, T* ex, T* ey, hipStream_t st) {
    const dim3 grid((g.nx + 2 + BX - 1) / BX, (g.ny + 2 + BY - 1) / BY);
    hipLaunchKernelGGL(k_zero_vel<T>, grid, dim3(BX, BY), 0, st, g, ex, ey);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi(const Geom& g, const T* ex_in, const T* ey_in, T* ex_out, T* ey_out, const T* rx,
                         const T* ry, const T* eb, const T* ep, T omega, hipStream_t st) {
    hipLaunchKernelGGL(k_jacobi<T>, grid_cells(g), dim3(BX, BY), 0, st, g, ex_in, ey_in, ex_out, ey_out, rx,
                       ry, eb, ep, omega, ex_in ? 0 : 1);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_half(const Geom& g, int comp, int col, T* ex, T* ey, const T* rx, const T* ry,
                          const T* eb, const T* ep, T omega, bool zero_guess, hipStream_t st) {
    hipLaunchKernelGGL(k_gs_half<T>, grid_cells(g), dim3(BX, BY), 0, st, g, comp, col, ex, ey, rx, ry, eb, ep,
                       omega, zero_guess ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vel_residual(const Geom& g, const T* ex, const T* ey, const T* rx, const T* ry,
                               const T* eb, const T* ep, T* tx, T* ty, hipStream_t st) {
    hipLaunchKernelGGL(k_vel_residual<T>, grid_cells(g), dim3(BX, BY), 0, st, g, ex, ey, rx, ry, eb, ep, tx, ty);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_precond_in(const Geom& g, Vec3 v, const double* eb, const double* ep, bool energy, T* rx,
                             T* ry, hipStream_t st) {
    hipLaunchKernelGGL(k_precond_in<T>, grid_cells(g), dim3(BX, BY), 0, st, g, v, eb, ep, energy ? 1 : 0, rx, ry);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_precond_out(const Geom& g, const T* ex, const T* ey, Vec3 v, const double* ep, bool energy,
                              double alpha, Vec3 z, hipStream_t st, bool accumulate) {
    hipLaunchKernelGGL(k_precond_out<T>, grid_cells(g), dim3(BX, BY), 0, st, g, ex, ey, v, ep, energy ? 1 : 0,
                       alpha, z, accumulate ? 1 : 0);
    return hipGetLastError();
}

template <typename T, int MODE, bool NT>
void launch_link_nt(const Geom& g, const LinkArgs<T>& a, const double* eb, const double* ep, hipStream_t st,
                    hipEvent_t t0, hipEvent_t t1) {
    const dim3 grid = grid_cells(g);
    if (t0)
        hipExtLaunchKernelGGL((k_uzawa_link<T, MODE, NT>), grid, dim3(BX, BY), 0, st, t0, t1, 0, g, a, eb, ep);
    else
        hipLaunchKernelGGL((k_uzawa_link<T, MODE, NT>), grid, dim3(BX, BY), 0, st, g, a, eb, ep);
}

// Streaming per-cell accesses once one FP64 vector of the grid (three
// fields) outgrows the 256 MB last-level cache (4096^2: 2.5 % faster links);
// below that the next kernel reads the link's outputs from that cache, and
// streaming them costs 3 % of a 1024^2 solve.
constexpr double kLinkStreamBytes = 256.0 * 1024 * 1024;

template <typename T, int MODE>
void launch_link_mode(const Geom& g, const LinkArgs<T>& a, const double* eb, const double* ep, hipStream_t st,
                      hipEvent_t t0, hipEvent_t t1) {
    if (3.0 * sizeof(double) * (double)g.elems() > kLinkStreamBytes)
        launch_link_nt<T, MODE, true>(g, a, eb, ep, st, t0, t1);
    else
        launch_link_nt<T, MODE, false>(g, a, eb, ep, st, t0, t1);
}

template <typename T>
hipError_t launch_uzawa_link(const Geom& g, const LinkArgs<T>& a, int mode, const double* eb, const double* ep,
                             hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    if (mode == kLinkApply)
        launch_link_mode<T, kLinkApply>(g, a, eb, ep, st, t0, t1);
    else if (mode == kLinkStore)
        launch_link_mode<T, kLinkStore>(g, a, eb, ep, st, t0, t1);
    else if (mode == kLinkNext)
        launch_link_mode<T, kLinkNext>(g, a, eb, ep, st, t0, t1);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lithostatic(const Geom& g, const double* rho, double gy, double* p, hipStream_t st) {
    hipLaunchKernelGGL(k_lithostatic, dim3((g.nx + 255) / 256), dim3(256), 0, st, g, rho, gy, p);
    return hipGetLastError();
}

hipError_t launch_eta_min(const Geom& g, const double* eb, const double* ep, double* partial, double* out,
                          hipStream_t st) {
    const dim3 grid((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY);
    hipLaunchKernelGGL(k_eta_min, grid, dim3(BX, BY), 0, st, g, eb, ep, partial);
    hipLaunchKernelGGL(k_min_rows, dim3(1), dim3(256), 0, st, partial, (int)(grid.x * grid.y), out);
    return hipGetLastError();
}

hipError_t launch_blend(const double* in, double* out, size_t n, double theta, double m, hipStream_t st) {
    size_t b = (n + 2047) / 2048;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_blend, dim3((unsigned)b), dim3(256), 0, st, in, out, n, theta, m);
    return hipGetLastError();
}

hipError_t launch_rhs(const Geom& g, const double* rho, double gx, double gy, const double* fxe,
                      const double* fye, Vec3 b, hipStream_t st) {
    hipLaunchKernelGGL(k_rhs, grid_cells(g), dim3(BX, BY), 0, st, g, rho, gx, gy, fxe, fye, b);
    return hipGetLastError();
}

hipError_t launch_check_coeffs(const Geom& g, const double* eb, const double* ep, const double* rho,
                               const double* fxe, const double* fye, double* partial, int* nblk_out,
                               hipStream_t st) {
    const dim3 grid((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY);
    const int nblk = (int)(grid.x * grid.y);
    if (nblk_out) *nblk_out = nblk;
    hipLaunchKernelGGL(k_check_coeffs, grid, dim3(BX, BY), 0, st, g, eb, ep, rho, fxe, fye, partial, nblk);
    return hipGetLastError();
}

hipError_t launch_coeff_gradient(const Geom& g, Vec3 x, Vec3 lam, double gx, double gy, double* g_eb,
                                 double* g_ep, double* g_rho, hipStream_t st) {
    const dim3 grid((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY);
    hipLaunchKernelGGL(k_coeff_gradient, grid, dim3(BX, BY), 0, st, g, x, lam, gx, gy, g_eb, g_ep, g_rho);
    return hipGetLastError();
}

hipError_t launch_fold_ghost_grad(const Geom& g, Vec3 v, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_ghost_grad, grid_cells(g), dim3(BX, BY), 0, st, g, v);
    return hipGetLastError();
}

hipError_t launch_cast_list(const CastList& c, hipStream_t st) {
    if (c.count < 1 || c.count > 2 * kMaxLevels) return hipErrorInvalidValue;
    size_t nmax = 0;
    for (int k = 0; k < c.count; ++k) nmax = c.n[k] > nmax ? c.n[k] : nmax;
    const int nb = (int)((nmax + 255) / 256 < 4096 ? (nmax + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_cast_list, dim3(nb > 0 ? nb : 1, c.count), dim3(256), 0, st, c);
    return hipGetLastError();
}

#define TPH_INST(T)                                                                                          \
    template hipError_t launch_fill_bc<T>(const Geom&, T*, T*, hipStream_t);                                 \
    template hipError_t launch_zero_vel<T>(const Geom&, T*, T*, hipStream_t);                                \
    template hipError_t launch_jacobi<T>(const Geom&, const T*, const T*, T*, T*, const T*, const T*,        \
                                         const T*, const T*, T, hipStream_t);                                \
    template hipError_t launch_gs_half<T>(const Geom&, int, int, T*, T*, const T*, const T*, const T*,       \
                                          const T*, T, bool, hipStream_t);                                   \
    template hipError_t launch_vel_residual<T>(const Geom&, const T*, const T*, const T*, const T*,          \
                                               const T*, const T*, T*, T*, hipStream_t);                     \
    template hipError_t launch_precond_in<T>(const Geom&, Vec3, const double*, const double*, bool, T*, T*,  \
                                             hipStream_t);                                                   \
    template hipError_t launch_precond_out<T>(const Geom&, const T*, const T*, Vec3, const double*, bool,    \
                                              double, Vec3, hipStream_t, bool);                              \
    template hipError_t launch_uzawa_link<T>(const Geom&, const LinkArgs<T>&, int, const double*,           \
                                             const double*, hipStream_t, hipEvent_t, hipEvent_t);
TPH_INST(float)
TPH_INST(double)
#undef TPH_INST

}  // namespace tph
