// Single-problem launchers of the fused multigrid kernels (device bodies in
// fused_dev.h): LDS-tiled smoothing sweep, fused residual + restriction,
// single-workgroup coarse tail.
#include <hip/hip_ext.h>

#include "fused_dev.h"

namespace tph {
namespace {

using namespace dev;

template <typename T, int TW, int TH, int SM, int MODE>
__global__ __launch_bounds__(kTileThreads) void k_smooth_tile(Geom g, Geom gc, const T* __restrict__ exi,
                                                    const T* __restrict__ eyi, T* __restrict__ exo,
                                                    T* __restrict__ eyo, const T* __restrict__ rx,
                                                    const T* __restrict__ ry, const T* __restrict__ eb,
                                                    const T* __restrict__ ep, const T* __restrict__ ecx,
                                                    const T* __restrict__ ecy, T omega) {
    int tbx, tby;
    xcd_tile(tbx, tby);
    smooth_tile_body<T, TW, TH, SM, MODE>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, omega, tbx, tby);
}

template <typename T, int CTW, int CTH>
__global__ __launch_bounds__(CTW * CTH) void k_res_restrict(Geom g, Geom gc, const T* __restrict__ ex,
                                                           const T* __restrict__ ey, const T* __restrict__ rx,
                                                           const T* __restrict__ ry, const T* __restrict__ eb,
                                                           const T* __restrict__ ep, T* __restrict__ rcx,
                                                           T* __restrict__ rcy) {
    int tbx, tby;
    xcd_tile(tbx, tby);
    res_restrict_body<T, CTW, CTH>(g, gc, ex, ey, rx, ry, eb, ep, rcx, rcy, tbx, tby);
}

template <typename T>
__global__ __launch_bounds__(coarse_threads<T>()) void k_coarse_cycle(CoarseArgs<T> A) {
    coarse_cycle_body<T>(A);
}

}  // namespace


template <typename T>
size_t coarse_cycle_lds_bytes(const Geom* g, int nl, int nc) {
    size_t n = 0;
    for (int l = 0; l < nl; ++l) n += 6 * (size_t)(g[l].ny + 2) * (g[l].nx + 2);
    n += 2 * (size_t)(g[0].ny + 2) * (g[0].nx + 2);
    size_t bytes = n * sizeof(T);
    bytes = (bytes + 7) / 8 * 8 + (size_t)nc * sizeof(double);
    return bytes;
}

template <typename T>
hipError_t launch_smooth_tile(const Geom& g, const Geom* gc, int smoother, int mode, const T* exi, const T* eyi,
                              T* exo, T* eyo, const T* rx, const T* ry, const T* eb, const T* ep, const T* ecx,
                              const T* ecy, T omega, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    constexpr int TW = kTileW, TH = tile_h<T>();
    const dim3 grid((g.nx + TW - 1) / TW, (g.ny + TH - 1) / TH);
    const Geom gcc = gc ? *gc : g;
#define TPH_SMT(SM, MODE)                                                                                        \
    do {                                                                                                          \
        if (t0)                                                                                                   \
            hipExtLaunchKernelGGL((k_smooth_tile<T, TW, TH, SM, MODE>), grid, dim3(kTileThreads), 0, st, t0, t1, \
                                  0, g, gcc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, omega);              \
        else                                                                                                      \
            hipLaunchKernelGGL((k_smooth_tile<T, TW, TH, SM, MODE>), grid, dim3(kTileThreads), 0, st, g, gcc, exi, \
                               eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, omega);                                   \
    } while (0)
    if (smoother == kSmGS) {
        if (mode == kModeZero) TPH_SMT(kSmGS, kModeZero);
        else if (mode == kModeProlong) TPH_SMT(kSmGS, kModeProlong);
        else TPH_SMT(kSmGS, kModePlain);
    } else {
        if (mode == kModeZero) TPH_SMT(kSmJacobi, kModeZero);
        else if (mode == kModeProlong) TPH_SMT(kSmJacobi, kModeProlong);
        else TPH_SMT(kSmJacobi, kModePlain);
    }
#undef TPH_SMT
    return hipGetLastError();
}

template <typename T>
hipError_t launch_res_restrict(const Geom& gf, const Geom& gc, const T* ex, const T* ey, const T* rx, const T* ry,
                               const T* eb, const T* ep, T* rcx, T* rcy, hipStream_t st) {
    constexpr int CTW = kRRTileW, CTH = rr_tile_h<T>();
    const dim3 grid((gc.nx + CTW - 1) / CTW, (gc.ny + CTH - 1) / CTH);
    hipLaunchKernelGGL((k_res_restrict<T, CTW, CTH>), grid, dim3(CTW * CTH), 0, st, gf, gc, ex, ey, rx, ry, eb, ep,
                       rcx, rcy);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_cycle(const CoarseArgs<T>& a, size_t lds_bytes, int max_lds, hipStream_t st) {
    // raise the kernel's dynamic LDS limit when a launch needs more than 64 KB;
    // the attribute is per function (and device), so it is set only when a
    // launch needs more than any earlier one on this device
    (void)max_lds;
    static thread_local int dev_cached = -1;
    static thread_local size_t granted = 64 * 1024;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
    if (dev != dev_cached) {
        dev_cached = dev;
        granted = 64 * 1024;
    }
    if (lds_bytes > granted) {
        hipError_t e = hipFuncSetAttribute((const void*)k_coarse_cycle<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();   // do not leave the error pending for unrelated later launches
            return e;
        }
        granted = lds_bytes;
    }
    hipLaunchKernelGGL(k_coarse_cycle<T>, dim3(1), dim3(coarse_threads<T>()), lds_bytes, st, a);
    return hipGetLastError();
}

#define TPH_INST(T)                                                                                                \
    template size_t coarse_cycle_lds_bytes<T>(const Geom*, int, int);                                             \
    template hipError_t launch_smooth_tile<T>(const Geom&, const Geom*, int, int, const T*, const T*, T*, T*,       \
                                              const T*, const T*, const T*, const T*, const T*, const T*, T,         \
                                              hipStream_t, hipEvent_t, hipEvent_t);                                 \
    template hipError_t launch_res_restrict<T>(const Geom&, const Geom&, const T*, const T*, const T*, const T*,    \
                                               const T*, const T*, T*, T*, hipStream_t);                            \
    template hipError_t launch_coarse_cycle<T>(const CoarseArgs<T>&, size_t, int, hipStream_t);
TPH_INST(float)
TPH_INST(double)
#undef TPH_INST

}  // namespace tph
