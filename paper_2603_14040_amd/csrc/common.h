// Internal definitions shared by the HIP kernels and the host solver.
//
// Device layout: every field of a level is a row-major array of (ny + 2)
// rows with a padded row pitch (a multiple of 64 elements).  The base
// pointer addresses entry (0, 0) and is offset by 63 elements inside its
// allocation, so entry (i, 1) - the first interior column - starts on a
// 64-element boundary in every row: a wavefront of 64 lanes reading columns
// 1..64 touches whole 256 B (FP32) / 512 B (FP64) segments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tph {

constexpr int kAlign = 64;          // pitch granularity and (i, 1) alignment (elements)
constexpr int kMaxLevels = 16;
constexpr int kMaxRestart = 64;

// One multigrid level.
struct Geom {
    int nx, ny;          // cells
    int pitch;           // elements per row
    double dx, dy;
    float mir[4];        // ghost = mir * interior at walls W, E, S, N (+1 free slip, -1 no slip)
    __host__ __device__ size_t elems() const { return (size_t)(ny + 2) * pitch; }
    __host__ __device__ size_t idx(int i, int j) const { return (size_t)i * pitch + j; }
};

inline int pitch_for(int nx) { return ((nx + 2 + kAlign - 1) / kAlign) * kAlign; }
// allocation size (elements) of one field including the alignment offset
inline size_t field_alloc(const Geom& g) { return g.elems() + kAlign; }

// Three-field vector (vx | vy | p) stored contiguously with a common stride,
// so Krylov kernels can treat it as one flat array.
struct Vec3 {
    double* base;        // entry (0, 0) of vx; vy at base + stride, p at base + 2 stride
    size_t stride;       // elements between fields
    __host__ __device__ double* vx() const { return base; }
    __host__ __device__ double* vy() const { return base + stride; }
    __host__ __device__ double* p() const { return base + 2 * stride; }
};

// Workgroups are dispatched to the 8 XCDs round-robin by flat id.  Map the
// flat id so that XCD x gets a contiguous run of tiles (a band of tile rows):
// halo re-reads and the next kernel's reads of this band then hit that
// XCD's own L2.  Bijective for any tile count.
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
    const int nbx = gridDim.x;
    const int n = nbx * gridDim.y;
    const int b = blockIdx.y * nbx + blockIdx.x;
    const int x = b & 7, k = b >> 3;
    const int q = n >> 3, r = n & 7;
    const int t = x * q + (x < r ? x : r) + k;
    by = t / nbx;
    bx = t - by * nbx;
}

}  // namespace tph
