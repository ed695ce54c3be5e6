// Inter-level transfers (Ch. 4 "Restriction and Prolongation Operators"):
// dedicated factor-2 kernels, and coordinate-based ones for any other factor.
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

// ---------------------------------------------------------------------------
// Any coarsening factor (the coarse nodes fall between fine nodes).  The
// same normalised bilinear weighting, computed from node coordinates: along
// one axis the nodes of a kind sit at x(j) = (j + off) h with off = 0 on
// basic-node lines and -1/2 on cell-centre lines, and the nodes inside the
// physical domain are j in [lo, hi] (basic lines [0, n], cell lines
// [1, n]).  A coarse node X gathers the fine nodes with |x - X| < H, found
// with the index search of Alg. "Bisect Bound" over the implicit fine
// coordinates, weighted by the hat 1 - |x - X| / H; prolongation weights the
// two coarse nodes that bracket a fine node by the same hat.
// ---------------------------------------------------------------------------
struct Axis {
    double h, off;     // spacing and node offset in spacings
    int lo, hi;        // nodes inside the domain
};

__device__ __forceinline__ Axis axis_of(int n, double h, bool cell_line) {
    return cell_line ? Axis{h, -0.5, 1, n} : Axis{h, 0.0, 0, n};
}

__device__ __forceinline__ double coord(const Axis& a, int j) { return (j + a.off) * a.h; }

// smallest j in [a.lo, a.hi] with coord(j) >= t (a.hi when there is none)
__device__ __forceinline__ int bisect_bound(const Axis& a, double t) {
    int l = a.lo, r = a.hi;
    while (l < r) {
        const int m = (l + r) >> 1;
        if (coord(a, m) < t) l = m + 1;
        else r = m;
    }
    return l;
}

__device__ __forceinline__ double hat(double t) { return fmax(0.0, 1.0 - fabs(t)); }

// sum of w * u and of w over the fine nodes around coarse node (I, J);
// value(i, j) gives the fine entry (zero where the field has no equation)
template <typename F>
__device__ __forceinline__ double gather(const Axis& fy, const Axis& fx, const Axis& cy, const Axis& cx, int I, int J,
                                         F value) {
    const double Y = coord(cy, I), X = coord(cx, J);
    const int i0 = bisect_bound(fy, Y - cy.h), i1 = bisect_bound(fy, Y + cy.h);
    const int j0 = bisect_bound(fx, X - cx.h), j1 = bisect_bound(fx, X + cx.h);
    double num = 0.0, wys = 0.0, wxs = 0.0;
    for (int j = j0; j <= j1; ++j) wxs += hat((coord(fx, j) - X) / cx.h);
    for (int i = i0; i <= i1; ++i) {
        const double wy = hat((coord(fy, i) - Y) / cy.h);
        if (wy == 0.0) continue;
        wys += wy;
        double row = 0.0;
        for (int j = j0; j <= j1; ++j) row += hat((coord(fx, j) - X) / cx.h) * value(i, j);
        num += wy * row;
    }
    const double den = wys * wxs;
    return den > 0.0 ? num / den : 0.0;
}

__global__ __launch_bounds__(256) void k_restrict_eta_gen(Geom gf, Geom gc, const double* __restrict__ ebf,
                                                         const double* __restrict__ epf, double* __restrict__ ebc,
                                                         double* __restrict__ epc, int geometric) {
    const int J = blockIdx.x * BX + threadIdx.x;
    const int I = blockIdx.y * BY + threadIdx.y;
    if (I > gc.ny || J > gc.nx) return;
    const int Pf = gf.pitch;
    {   // basic grid: nodes [0, n] in both directions
        const Axis fy = axis_of(gf.ny, gf.dy, false), fx = axis_of(gf.nx, gf.dx, false);
        const Axis cy = axis_of(gc.ny, gc.dy, false), cx = axis_of(gc.nx, gc.dx, false);
        const double m = gather(fy, fx, cy, cx, I, J, [&](int i, int j) {
            const double v = ebf[i * Pf + j];
            return geometric ? log(v) : v;
        });
        ebc[I * gc.pitch + J] = geometric ? exp(m) : m;
    }
    if (I >= 1 && J >= 1) {   // cell centres: [1, n] in both directions
        const Axis fy = axis_of(gf.ny, gf.dy, true), fx = axis_of(gf.nx, gf.dx, true);
        const Axis cy = axis_of(gc.ny, gc.dy, true), cx = axis_of(gc.nx, gc.dx, true);
        const double m = gather(fy, fx, cy, cx, I, J, [&](int i, int j) {
            const double v = epf[i * Pf + j];
            return geometric ? log(v) : v;
        });
        epc[I * gc.pitch + J] = geometric ? exp(m) : m;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict_res_gen(Geom gf, Geom gc, const T* __restrict__ tx,
                                                         const T* __restrict__ ty, T* __restrict__ rx,
                                                         T* __restrict__ ry) {
    const int J = blockIdx.x * BX + threadIdx.x + 1;
    const int I = blockIdx.y * BY + threadIdx.y + 1;
    if (I > gc.ny || J > gc.nx) return;
    const int Pf = gf.pitch;
    const int C = I * gc.pitch + J;
    if (J < gc.nx) {
        // vx: basic lines in x (walls inside, holding zero), cell lines in y
        const Axis fy = axis_of(gf.ny, gf.dy, true), fx = axis_of(gf.nx, gf.dx, false);
        const Axis cy = axis_of(gc.ny, gc.dy, true), cx = axis_of(gc.nx, gc.dx, false);
        rx[C] = (T)gather(fy, fx, cy, cx, I, J, [&](int i, int j) {
            return (j >= 1 && j < gf.nx) ? (double)tx[i * Pf + j] : 0.0;
        });
    }
    if (I < gc.ny) {
        // vy: cell lines in x, basic lines in y (walls inside, holding zero)
        const Axis fy = axis_of(gf.ny, gf.dy, false), fx = axis_of(gf.nx, gf.dx, true);
        const Axis cy = axis_of(gc.ny, gc.dy, false), cx = axis_of(gc.nx, gc.dx, true);
        ry[C] = (T)gather(fy, fx, cy, cx, I, J, [&](int i, int j) {
            return (i >= 1 && i < gf.ny) ? (double)ty[i * Pf + j] : 0.0;
        });
    }
}

// bilinear value at fine coordinate (y, x) from the coarse nodes that bracket
// it; coarse entries [0, n + 1] (ghosts hold the mirrored values)
template <typename T>
__device__ __forceinline__ double interp_coarse(const T* __restrict__ ec, int Pc, const Axis& cy, const Axis& cx,
                                                int ny1, int nx1, double y, double x) {
    int I = (int)floor(y / cy.h - cy.off), J = (int)floor(x / cx.h - cx.off);
    I = I < 0 ? 0 : (I > ny1 - 1 ? ny1 - 1 : I);
    J = J < 0 ? 0 : (J > nx1 - 1 ? nx1 - 1 : J);
    double v = 0.0;
    for (int a = 0; a < 2; ++a) {
        const double wy = hat((y - coord(cy, I + a)) / cy.h);
        for (int b = 0; b < 2; ++b) v += wy * hat((x - coord(cx, J + b)) / cx.h) * (double)ec[(I + a) * Pc + J + b];
    }
    return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add_gen(Geom gf, Geom gc, const T* __restrict__ ecx,
                                                        const T* __restrict__ ecy, T* __restrict__ ex,
                                                        T* __restrict__ ey) {
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y * BY + threadIdx.y + 1;
    if (i > gf.ny || j > gf.nx) return;
    const int P = gf.pitch;
    const int c = i * P + j;
    if (j < gf.nx) {
        const Axis cy = axis_of(gc.ny, gc.dy, true), cx = axis_of(gc.nx, gc.dx, false);
        const double v = interp_coarse(ecx, gc.pitch, cy, cx, gc.ny + 1, gc.nx + 1, (i - 0.5) * gf.dy, j * gf.dx);
        const T e = ex[c] + (T)v;
        ex[c] = e;
        if (i == 1) ex[c - P] = (T)gf.mir[2] * e;
        if (i == gf.ny) ex[c + P] = (T)gf.mir[3] * e;
    }
    if (i < gf.ny) {
        const Axis cy = axis_of(gc.ny, gc.dy, false), cx = axis_of(gc.nx, gc.dx, true);
        const double v = interp_coarse(ecy, gc.pitch, cy, cx, gc.ny + 1, gc.nx + 1, i * gf.dy, (j - 0.5) * gf.dx);
        const T e = ey[c] + (T)v;
        ey[c] = e;
        if (j == 1) ey[c - 1] = (T)gf.mir[0] * e;
        if (j == gf.nx) ey[c + 1] = (T)gf.mir[1] * e;
    }
}

}  // namespace

// factor 2 when each fine side is twice the coarse one, else the general form
inline bool halving(const Geom& gf, const Geom& gc) { return gf.nx == 2 * gc.nx && gf.ny == 2 * gc.ny; }

hipError_t launch_restrict_eta(const Geom& gf, const Geom& gc, const double* ebf, const double* epf,
                               double* ebc, double* epc, bool geometric, hipStream_t st) {
    const dim3 grid((gc.nx + 1 + BX - 1) / BX, (gc.ny + 1 + BY - 1) / BY);
    if (halving(gf, gc))
        hipLaunchKernelGGL(k_restrict_eta, grid, dim3(BX, BY), 0, st, gf, gc, ebf, epf, ebc, epc, geometric ? 1 : 0);
    else
        hipLaunchKernelGGL(k_restrict_eta_gen, grid, dim3(BX, BY), 0, st, gf, gc, ebf, epf, ebc, epc,
                           geometric ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_res(const Geom& gf, const Geom& gc, const T* tx, const T* ty, T* rx, T* ry,
                               hipStream_t st) {
    const dim3 grid((gc.nx + BX - 1) / BX, (gc.ny + BY - 1) / BY);
    if (halving(gf, gc))
        hipLaunchKernelGGL(k_restrict_res<T>, grid, dim3(BX, BY), 0, st, gf, gc, tx, ty, rx, ry);
    else
        hipLaunchKernelGGL(k_restrict_res_gen<T>, grid, dim3(BX, BY), 0, st, gf, gc, tx, ty, rx, ry);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const Geom& gf, const Geom& gc, const T* ecx, const T* ecy, T* ex, T* ey,
                              hipStream_t st) {
    const dim3 grid((gf.nx + BX - 1) / BX, (gf.ny + BY - 1) / BY);
    if (halving(gf, gc))
        hipLaunchKernelGGL(k_prolong_add<T>, grid, dim3(BX, BY), 0, st, gf, gc, ecx, ecy, ex, ey);
    else
        hipLaunchKernelGGL(k_prolong_add_gen<T>, grid, dim3(BX, BY), 0, st, gf, gc, ecx, ecy, ex, ey);
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
