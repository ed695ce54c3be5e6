// Multi-sweep Gauss-Seidel tile kernels (device body gs_tile_body in
// fused_dev.h) and their launcher, instantiated per arithmetic type in
// msweep_f32.hip / msweep_f64.hip.
//
// Tile shapes (fine nodes, TW x TH; kTileThreads threads per tile):
//   shape 0, FP32: 64 x 16 for one or two sweeps per pass
//   shape 0, FP64: 64 x 8 for one sweep, 32 x 8 for two (64 KB of LDS)
//   shape 1: 32 x 8 (FP32) / 32 x 4 (FP64): four times the tiles, for
//            levels too small to fill the chip with shape 0
#pragma once
#include <hip/hip_ext.h>

#include "fused_dev.h"

namespace tph {
namespace msw {

using namespace dev;

template <typename T, int NS, int SHAPE>
struct TileShape {
    static constexpr int TW = SHAPE == 0 ? (sizeof(T) == 4 || NS == 1 ? 64 : 32) : 32;
    static constexpr int TH = SHAPE == 0 ? (sizeof(T) == 4 ? 16 : 8) : (sizeof(T) == 4 ? 8 : 4);
};

template <typename T, int TW, int TH, int NS, int MODE, int RR>
__global__ __launch_bounds__(kTileThreads) void k_gs_tile(Geom g, Geom gc, const T* __restrict__ exi,
                                                         const T* __restrict__ eyi, T* __restrict__ exo,
                                                         T* __restrict__ eyo, const T* __restrict__ rx,
                                                         const T* __restrict__ ry, const T* __restrict__ eb,
                                                         const T* __restrict__ ep, const T* __restrict__ ecx,
                                                         const T* __restrict__ ecy, T* __restrict__ rcx,
                                                         T* __restrict__ rcy, T omega) {
    int tbx, tby;
    xcd_tile(tbx, tby);
    gs_tile_body<T, TW, TH, NS, MODE, RR>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega, tbx,
                                          tby);
}

template <typename T, int NS, int MODE, int RR, int SHAPE>
hipError_t launch_one(const Geom& g, const Geom& gc, const T* exi, const T* eyi, T* exo, T* eyo, const T* rx,
                      const T* ry, const T* eb, const T* ep, const T* ecx, const T* ecy, T* rcx, T* rcy, T omega,
                      hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    constexpr int TW = TileShape<T, NS, SHAPE>::TW, TH = TileShape<T, NS, SHAPE>::TH;
    const dim3 grid((g.nx + TW - 1) / TW, (g.ny + TH - 1) / TH);
    if (t0)
        hipExtLaunchKernelGGL((k_gs_tile<T, TW, TH, NS, MODE, RR>), grid, dim3(kTileThreads), 0, st, t0, t1, 0, g,
                              gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega);
    else
        hipLaunchKernelGGL((k_gs_tile<T, TW, TH, NS, MODE, RR>), grid, dim3(kTileThreads), 0, st, g, gc, exi, eyi,
                           exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega);
    return hipGetLastError();
}

template <typename T, int NS, int MODE, int RR>
hipError_t launch_shape(int shape, const Geom& g, const Geom& gc, const T* exi, const T* eyi, T* exo, T* eyo,
                        const T* rx, const T* ry, const T* eb, const T* ep, const T* ecx, const T* ecy, T* rcx, T* rcy,
                        T omega, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    if (shape == 0)
        return launch_one<T, NS, MODE, RR, 0>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega, st,
                                              t0, t1);
    return launch_one<T, NS, MODE, RR, 1>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega, st,
                                          t0, t1);
}

template <typename T, int NS>
hipError_t launch_ns(int mode, int rr, int shape, const Geom& g, const Geom& gc, const T* exi, const T* eyi, T* exo,
                     T* eyo, const T* rx, const T* ry, const T* eb, const T* ep, const T* ecx, const T* ecy, T* rcx,
                     T* rcy, T omega, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
#define TPH_MSW(MODE, RR)                                                                                             \
    launch_shape<T, NS, MODE, RR>(shape, g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega, st, t0, \
                                  t1)
    if (mode == kModeProlong) return TPH_MSW(kModeProlong, 0);
    if (mode == kModeZero) return rr ? TPH_MSW(kModeZero, 1) : TPH_MSW(kModeZero, 0);
    return rr ? TPH_MSW(kModePlain, 1) : TPH_MSW(kModePlain, 0);
#undef TPH_MSW
}

}  // namespace msw

template <typename T>
hipError_t launch_gs_tile(const Geom& g, const Geom& gc, int ns, int mode, int rr, int shape, const T* exi,
                          const T* eyi, T* exo, T* eyo, const T* rx, const T* ry, const T* eb, const T* ep,
                          const T* ecx, const T* ecy, T* rcx, T* rcy, T omega, hipStream_t st, hipEvent_t t0,
                          hipEvent_t t1) {
    if (ns < 1 || ns > 2 || mode < 0 || mode > 2 || rr < 0 || rr > 1 || shape < 0 || shape > 1 ||
        (rr && mode == kTileProlong))
        return hipErrorInvalidValue;
    if (rr && (g.nx != 2 * gc.nx || g.ny != 2 * gc.ny)) return hipErrorInvalidValue;
    if (mode == kTileProlong && (g.nx != 2 * gc.nx || g.ny != 2 * gc.ny)) return hipErrorInvalidValue;
    if (ns == 1)
        return msw::launch_ns<T, 1>(mode, rr, shape, g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy,
                                    omega, st, t0, t1);
    return msw::launch_ns<T, 2>(mode, rr, shape, g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy, omega,
                                st, t0, t1);
}

}  // namespace tph
