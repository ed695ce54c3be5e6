// Point-wise stencils of the stress-conservative staggered discretisation
// (Ch. 4 "Stress-Conservative Finite Differences"; the x-momentum operator
// of the Ch. 6 listing, written here in flux form, and its y mirror).
//
// All functions take the flat index c = i * pitch + j of node (i, j) of a
// field in the device layout of common.h and read the eight neighbours of
// the velocity stencils directly; ghost rows/columns must hold the mirrored
// values and walls zero (free slip: mirror +1 makes the wall shear vanish;
// no slip: mirror -1 doubles it).
#pragma once
#include "common.h"

namespace tph {

template <typename T>
struct LevelC {             // level constants in the arithmetic type
    T idx, idy, idx2, idy2;
    T mirW, mirE, mirS, mirN;
};

template <typename T>
__host__ __device__ inline LevelC<T> level_consts(const Geom& g) {
    LevelC<T> k;
    k.idx = (T)(1.0 / g.dx);
    k.idy = (T)(1.0 / g.dy);
    k.idx2 = (T)(1.0 / (g.dx * g.dx));
    k.idy2 = (T)(1.0 / (g.dy * g.dy));
    k.mirW = (T)g.mir[0];
    k.mirE = (T)g.mir[1];
    k.mirS = (T)g.mir[2];
    k.mirN = (T)g.mir[3];
    return k;
}

// (L v)_x at vx(i, j): d(sxx)/dx + d(sxy)/dy, sxx = 2 eta_p dvx/dx at cell
// centres, sxy = eta_b (dvx/dy + dvy/dx) at basic nodes.
template <typename T>
__device__ __forceinline__ T lx_row(const T* __restrict__ vx, const T* __restrict__ vy,
                                    const T* __restrict__ eb, const T* __restrict__ ep,
                                    int c, int P, T idx, T idy) {
    const T v = vx[c];
    const T sxx_r = (T)2 * ep[c + 1] * ((vx[c + 1] - v) * idx);
    const T sxx_l = (T)2 * ep[c] * ((v - vx[c - 1]) * idx);
    const T sxy_t = eb[c] * ((vx[c + P] - v) * idy + (vy[c + 1] - vy[c]) * idx);
    const T sxy_b = eb[c - P] * ((v - vx[c - P]) * idy + (vy[c - P + 1] - vy[c - P]) * idx);
    return (sxx_r - sxx_l) * idx + (sxy_t - sxy_b) * idy;
}

// lx_row where every vy the stencil reads is zero (the vy differences drop
// out; equal to lx_row up to how the fused multiply-adds round)
template <typename T>
__device__ __forceinline__ T lx_row_novy(const T* __restrict__ vx, const T* __restrict__ eb,
                                         const T* __restrict__ ep, int c, int P, T idx, T idy) {
    const T v = vx[c];
    const T sxx_r = (T)2 * ep[c + 1] * ((vx[c + 1] - v) * idx);
    const T sxx_l = (T)2 * ep[c] * ((v - vx[c - 1]) * idx);
    const T sxy_t = eb[c] * ((vx[c + P] - v) * idy);
    const T sxy_b = eb[c - P] * ((v - vx[c - P]) * idy);
    return (sxx_r - sxx_l) * idx + (sxy_t - sxy_b) * idy;
}

// (L v)_y at vy(i, j): d(syx)/dx + d(syy)/dy.
template <typename T>
__device__ __forceinline__ T ly_row(const T* __restrict__ vx, const T* __restrict__ vy,
                                    const T* __restrict__ eb, const T* __restrict__ ep,
                                    int c, int P, T idx, T idy) {
    const T v = vy[c];
    const T syy_t = (T)2 * ep[c + P] * ((vy[c + P] - v) * idy);
    const T syy_b = (T)2 * ep[c] * ((v - vy[c - P]) * idy);
    const T syx_r = eb[c] * ((vx[c + P] - vx[c]) * idy + (vy[c + 1] - v) * idx);
    const T syx_l = eb[c - 1] * ((vx[c + P - 1] - vx[c - 1]) * idy + (v - vy[c - 1]) * idx);
    return (syy_t - syy_b) * idy + (syx_r - syx_l) * idx;
}

// ly_row where every vy the stencil reads is zero (syy vanishes, syx keeps its
// vx differences)
template <typename T>
__device__ __forceinline__ T ly_row_novy(const T* __restrict__ vx, const T* __restrict__ eb, int c, int P, T idx,
                                         T idy) {
    const T syx_r = eb[c] * ((vx[c + P] - vx[c]) * idy);
    const T syx_l = eb[c - 1] * ((vx[c + P - 1] - vx[c - 1]) * idy);
    return (syx_r - syx_l) * idx;
}

// Magnitudes of the terms of lx_row / ly_row, each flux product taken in
// absolute value: the scale of the rounding error of a residual row.
template <typename T>
__device__ __forceinline__ T lx_row_abs(const T* __restrict__ vx, const T* __restrict__ vy,
                                        const T* __restrict__ eb, const T* __restrict__ ep,
                                        int c, int P, T idx, T idy) {
    const T v = vx[c];
    const T sxx_r = (T)2 * ep[c + 1] * (fabs(vx[c + 1]) + fabs(v)) * idx;
    const T sxx_l = (T)2 * ep[c] * (fabs(v) + fabs(vx[c - 1])) * idx;
    const T sxy_t = eb[c] * ((fabs(vx[c + P]) + fabs(v)) * idy + (fabs(vy[c + 1]) + fabs(vy[c])) * idx);
    const T sxy_b = eb[c - P] * ((fabs(v) + fabs(vx[c - P])) * idy + (fabs(vy[c - P + 1]) + fabs(vy[c - P])) * idx);
    return (sxx_r + sxx_l) * idx + (sxy_t + sxy_b) * idy;
}

template <typename T>
__device__ __forceinline__ T ly_row_abs(const T* __restrict__ vx, const T* __restrict__ vy,
                                        const T* __restrict__ eb, const T* __restrict__ ep,
                                        int c, int P, T idx, T idy) {
    const T v = vy[c];
    const T syy_t = (T)2 * ep[c + P] * (fabs(vy[c + P]) + fabs(v)) * idy;
    const T syy_b = (T)2 * ep[c] * (fabs(v) + fabs(vy[c - P])) * idy;
    const T syx_r = eb[c] * ((fabs(vx[c + P]) + fabs(vx[c])) * idy + (fabs(vy[c + 1]) + fabs(v)) * idx);
    const T syx_l = eb[c - 1] * ((fabs(vx[c + P - 1]) + fabs(vx[c - 1])) * idy + (fabs(v) + fabs(vy[c - 1])) * idx);
    return (syy_t + syy_b) * idy + (syx_r + syx_l) * idx;
}

// diag(L) at vx(i, j) and vy(i, j).  At a wall-adjacent node the shear term
// of the boundary basic node enters with weight (1 - mirror): 0 for free
// slip, 2 for no slip.
template <typename T>
__device__ __forceinline__ T lx_diag(const T* __restrict__ eb, const T* __restrict__ ep, int c, int P,
                                     int i, int ny, const LevelC<T>& k) {
    const T ct = (i == ny) ? ((T)1 - k.mirN) : (T)1;
    const T cb = (i == 1) ? ((T)1 - k.mirS) : (T)1;
    return -(T)2 * (ep[c + 1] + ep[c]) * k.idx2 - (eb[c] * ct + eb[c - P] * cb) * k.idy2;
}

template <typename T>
__device__ __forceinline__ T ly_diag(const T* __restrict__ eb, const T* __restrict__ ep, int c, int P,
                                     int j, int nx, const LevelC<T>& k) {
    const T cr = (j == nx) ? ((T)1 - k.mirE) : (T)1;
    const T cl = (j == 1) ? ((T)1 - k.mirW) : (T)1;
    return -(T)2 * (ep[c + P] + ep[c]) * k.idy2 - (eb[c] * cr + eb[c - 1] * cl) * k.idx2;
}

// diag(L) at a node with no wall-adjacent shear term (1 < i < ny, resp.
// 1 < j < nx): the general formulas with both boundary factors equal to 1
template <typename T>
__device__ __forceinline__ T lx_diag_inner(const T* __restrict__ eb, const T* __restrict__ ep, int c, int P,
                                           const LevelC<T>& k) {
    return -(T)2 * (ep[c + 1] + ep[c]) * k.idx2 - (eb[c] + eb[c - P]) * k.idy2;
}

template <typename T>
__device__ __forceinline__ T ly_diag_inner(const T* __restrict__ eb, const T* __restrict__ ep, int c, int P,
                                           const LevelC<T>& k) {
    return -(T)2 * (ep[c + P] + ep[c]) * k.idy2 - (eb[c] + eb[c - 1]) * k.idx2;
}

// damped point update e + omega (r - (L e)) / diag.  FP32 (inside the
// mixed-precision V-cycle) multiplies by the hardware reciprocal of the
// diagonal (1 ulp) instead of the correctly rounded division; FP64 divides.
__device__ __forceinline__ float relax(float e, float omega, float res, float d) {
    return e + omega * res * __builtin_amdgcn_rcpf(d);
}
__device__ __forceinline__ double relax(double e, double omega, double res, double d) {
    return e + omega * res / d;
}

// Energy weight of a continuity row: eta_p / (2/dx^2 + 2/dy^2)
// (Sec. "Residual Norms", diagonal Schur surrogate).
template <typename T>
__device__ __forceinline__ T wp_weight(T etap, const LevelC<T>& k) {
    return etap / ((T)2 * k.idx2 + (T)2 * k.idy2);
}

}  // namespace tph
