// Device bodies of the fused multigrid kernels, shared by the single-problem
// kernels (fused.hip) and the batched kernels (batch.hip).
//
// smooth_tile_body: one full smoothing sweep on an LDS tile.
//   Gauss-Seidel: the four colour half-sweeps (vx red, vx black, vy red,
//   vy black) run inside the tile; each half-sweep needs the result of the
//   previous one one node further out, so the tile loads a halo of 4 nodes
//   and updates shrinking regions (halo 3, 2, 1, 0).  The sweep reads the
//   old iterate from one buffer and writes the interior of the tile to the
//   other, so overlapping tiles never see each other's new values and the
//   result equals the four separate half-sweeps exactly.
//   Jacobi: one stage, halo 1.
//   Modes: plain, zero initial guess (no load of the iterate), and
//   prolongation + correction fused into the load (bilinear coarse-to-fine
//   interpolation from an LDS window of the coarse correction, ghosts
//   re-mirrored).
// res_restrict_body: residual r - L e on the fine footprint of a tile of
//   coarse cells, kept in LDS, then the normalised restriction (gather form
//   of Alg. "4-Color Parallel Restriction"); the fine residual never goes
//   to memory.
// coarse_cycle_body: the V-cycle on every level from a small level down to
//   the coarsest in one workgroup, all fields resident in LDS, ending in the
//   FP64 dense solve.
#pragma once
#include "kernels.h"
#include "reduce.h"
#include "stencil.h"

namespace tph {
namespace dev {


enum { kModePlain = kTilePlain, kModeZero = kTileZero, kModeProlong = kTileProlong };
enum { kSmJacobi = 0, kSmGS = 1 };

// bilinear prolongation of the coarse vx / vy correction to fine node (i, j)
// (same weights as k_prolong_add; coarse ghosts hold mirrored values)
template <typename T>
__device__ __forceinline__ T prolong_vx(const T* __restrict__ ec, int Pc, int i, int j) {
    const int I0 = (i + 1) >> 1;
    const int I1 = (i & 1) ? I0 - 1 : I0 + 1;
    const int J = j >> 1;
    if ((j & 1) == 0) return (T)0.75 * ec[I0 * Pc + J] + (T)0.25 * ec[I1 * Pc + J];
    return (T)0.375 * (ec[I0 * Pc + J] + ec[I0 * Pc + J + 1]) + (T)0.125 * (ec[I1 * Pc + J] + ec[I1 * Pc + J + 1]);
}

template <typename T>
__device__ __forceinline__ T prolong_vy(const T* __restrict__ ec, int Pc, int i, int j) {
    const int J0 = (j + 1) >> 1;
    const int J1 = (j & 1) ? J0 - 1 : J0 + 1;
    const int I = i >> 1;
    if ((i & 1) == 0) return (T)0.75 * ec[I * Pc + J0] + (T)0.25 * ec[I * Pc + J1];
    return (T)0.375 * (ec[I * Pc + J0] + ec[(I + 1) * Pc + J0]) + (T)0.125 * (ec[I * Pc + J1] + ec[(I + 1) * Pc + J1]);
}

__device__ __forceinline__ bool is_vx(const Geom& g, int i, int j) { return i >= 1 && i <= g.ny && j >= 1 && j < g.nx; }
__device__ __forceinline__ bool is_vy(const Geom& g, int i, int j) { return i >= 1 && i < g.ny && j >= 1 && j <= g.nx; }

// Node predicates inside an LDS tile.  IN marks an interior tile: the tile
// and its whole halo lie in rows 1..ny-1 and columns 1..nx-1, so every node
// is an unknown of both components, no node is wall-adjacent and no ghost
// or wall is touched; the checks then vanish at compile time.
template <bool IN>
__device__ __forceinline__ bool ux_at(const Geom& g, int i, int j) { return IN || is_vx(g, i, j); }
template <bool IN>
__device__ __forceinline__ bool uy_at(const Geom& g, int i, int j) { return IN || is_vy(g, i, j); }

template <bool IN, typename T>
__device__ __forceinline__ T dx_at(const T* sb, const T* sp, int c, int RW, int gi, const Geom& g,
                                   const LevelC<T>& k) {
    return IN ? lx_diag_inner(sb, sp, c, RW, k) : lx_diag(sb, sp, c, RW, gi, g.ny, k);
}
template <bool IN, typename T>
__device__ __forceinline__ T dy_at(const T* sb, const T* sp, int c, int RW, int gj, const Geom& g,
                                   const LevelC<T>& k) {
    return IN ? ly_diag_inner(sb, sp, c, RW, k) : ly_diag(sb, sp, c, RW, gj, g.nx, k);
}

// tile origin (gi0, gj0) and region RW x RH: is it an interior tile?
template <int RW, int RH>
__device__ __forceinline__ bool interior_tile(const Geom& g, int gi0, int gj0) {
    return gi0 >= 1 && gj0 >= 1 && gi0 + RH <= g.ny && gj0 + RW <= g.nx;
}

// ---------------------------------------------------------------------------
// LDS tiles.  A tile of TW x TH nodes (origin (i0, j0) = (1 + tby TH,
// 1 + tbx TW)) is held with a halo of H nodes: the iterate (sx, sy) and the
// viscosities (sb, sp).  The right-hand side r is only ever needed at the
// node being updated, so it is read from memory there and takes no LDS.
// ---------------------------------------------------------------------------
template <int RH>
constexpr int prolong_rows() { return RH / 2 + 4; }

// Every Gauss-Seidel / Jacobi LDS tile kernel runs kTileThreads threads.
// Loops over a tile region have a compile-time trip count and are unrolled
// with all global loads of a phase issued into registers before the first
// one is used: a tile is latency-bound (few waves per CU at the finest
// level, a handful of tiles on the small ones), and a load loop that waited
// for each load before issuing the next would serialise one memory latency
// per iteration.  512 threads: each colour stage of a small-level tile is
// then one node per thread, which shortens the dependent chain of a launch;
// the 1024^2 solve ran 5 % faster than with 256 threads (1024 threads were
// slower again), with bitwise the same results, since nodes of one stage
// are independent of each other.
constexpr int kTileThreads = 512;

template <int N>
constexpr int tile_iters() { return (N + kTileThreads - 1) / kTileThreads; }

// load the iterate (zero / from memory / from memory + prolongated coarse
// correction) and the viscosities of the region starting at (gi0, gj0)
template <typename T, int RW, int RH, int MODE, bool IN>
__device__ __forceinline__ void tile_load(const Geom& g, const Geom& gc, int gi0, int gj0, const T* __restrict__ exi,
                                          const T* __restrict__ eyi, const T* __restrict__ eb,
                                          const T* __restrict__ ep, const T* __restrict__ ecx,
                                          const T* __restrict__ ecy, T* sx, T* sy, T* sb, T* sp, T* scx, T* scy,
                                          const LevelC<T>& k) {
    constexpr int RN = RW * RH, IT = tile_iters<RN>();
    constexpr int CR = prolong_rows<RH>(), CC = prolong_rows<RW>(), ITC = tile_iters<CR * CC>();
    constexpr bool kIter = MODE != kModeZero;
    const int tid = threadIdx.x;
    const int P = g.pitch;
    T vb[IT], vp[IT], vx[kIter ? IT : 1], vy[kIter ? IT : 1];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int q = tid + it * kTileThreads;
        const int a = q / RW, b = q - (q / RW) * RW;
        const int gi = gi0 + a, gj = gj0 + b;
        const bool in = q < RN && (IN || (gi >= 0 && gi <= g.ny + 1 && gj >= 0 && gj <= g.nx + 1));
        const int c = in ? gi * P + gj : 0;
        vb[it] = in ? eb[c] : (T)0;
        vp[it] = in ? ep[c] : (T)0;
        if (kIter) {
            vx[it] = in ? exi[c] : (T)0;
            vy[it] = in ? eyi[c] : (T)0;
        }
    }
    // first coarse row / column of the prolongation window: floor(gi0 / 2) - 1
    // (gi0 may be negative; the +64 keeps the shift on a non-negative value)
    const int ci0 = ((gi0 + 64) >> 1) - 32 - 1;
    const int cj0 = ((gj0 + 64) >> 1) - 32 - 1;
    if (MODE == kModeProlong) {
        T wx[ITC], wy[ITC];
#pragma unroll
        for (int it = 0; it < ITC; ++it) {
            const int q = tid + it * kTileThreads;
            const int a = q / CC, b = q - (q / CC) * CC;
            const int I = ci0 + a, J = cj0 + b;
            const bool in = q < CR * CC && I >= 0 && I <= gc.ny + 1 && J >= 0 && J <= gc.nx + 1;
            const int c = in ? I * gc.pitch + J : 0;
            wx[it] = in ? ecx[c] : (T)0;
            wy[it] = in ? ecy[c] : (T)0;
        }
#pragma unroll
        for (int it = 0; it < ITC; ++it) {
            const int q = tid + it * kTileThreads;
            if (q < CR * CC) {
                scx[q] = wx[it];
                scy[q] = wy[it];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int q = tid + it * kTileThreads;
        if (q >= RN) continue;
        sb[q] = vb[it];
        sp[q] = vp[it];
        if (MODE == kModeZero) {
            sx[q] = (T)0;
            sy[q] = (T)0;
        } else {
            T ux = vx[it], uy = vy[it];
            if (MODE == kModeProlong) {
                // coarse indices are taken relative to the LDS window
                const int a = q / RW, b = q - (q / RW) * RW;
                const int gi = gi0 + a, gj = gj0 + b;
                if (ux_at<IN>(g, gi, gj)) ux += prolong_vx(scx - ci0 * CC - cj0, CC, gi, gj);
                if (uy_at<IN>(g, gi, gj)) uy += prolong_vy(scy - ci0 * CC - cj0, CC, gi, gj);
            }
            sx[q] = ux;
            sy[q] = uy;
        }
    }
    __syncthreads();
    if (MODE == kModeProlong && !IN) {
        // ghosts mirror the corrected interior values
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int q = tid + it * kTileThreads;
            if (q >= RN) continue;
            const int a = q / RW, b = q - (q / RW) * RW;
            const int gi = gi0 + a, gj = gj0 + b;
            if (gj >= 1 && gj < g.nx) {
                if (gi == 0 && a + 1 < RH) sx[q] = k.mirS * sx[q + RW];
                if (gi == g.ny + 1 && a >= 1) sx[q] = k.mirN * sx[q - RW];
            }
            if (gi >= 1 && gi < g.ny) {
                if (gj == 0 && b + 1 < RW) sy[q] = k.mirW * sy[q + 1];
                if (gj == g.nx + 1 && b >= 1) sy[q] = k.mirE * sy[q - 1];
            }
        }
        __syncthreads();
    }
}

// Shape of the colour stages of a tile: stage s (component (s >> 1) & 1,
// colour s & 1, i.e. vx red, vx black, vy red, vy black, repeated) updates
// the nodes within h = H - 1 - s of the tile; thread t takes the nodes
// t, t + kTileThreads, ... of the stage's list (rows x half, one colour per row).
template <int TW, int TH, int H, int NSTAGE>
struct Stages {
    static constexpr int rows(int s) { return TH + 2 * (H - 1 - s); }
    static constexpr int half(int s) { return (TW + 2 * (H - 1 - s)) / 2; }
    static constexpr int iters(int s) { return (rows(s) * half(s) + kTileThreads - 1) / kTileThreads; }
    static constexpr int offset(int s) {
        int o = 0;
        for (int q = 0; q < s; ++q) o += iters(q);
        return o;
    }
    static constexpr int total() { return offset(NSTAGE); }
};

// LDS coordinates (a, b) of item q of stage s
template <int TW, int TH, int H>
__device__ __forceinline__ void stage_node(int s, int q, int gi0, int gj0, int& a, int& b) {
    const int h = H - 1 - s, col = s & 1;
    const int half = (TW + 2 * h) / 2;
    const int ar = q / half, bb = q - (q / half) * half;
    const int a0 = H - h, b0 = H - h;
    a = a0 + ar;
    const int p0 = (gi0 + a + gj0 + b0) & 1;
    b = b0 + 2 * bb + (col ^ p0);
}

// right-hand side of every node this thread updates, in stage order
template <typename T, int TW, int TH, int H, int NSTAGE, bool IN>
__device__ __forceinline__ void stage_rhs(const Geom& g, int gi0, int gj0, const T* __restrict__ rx,
                                          const T* __restrict__ ry, T* rr) {
    using S = Stages<TW, TH, H, NSTAGE>;
    const int tid = threadIdx.x;
    const int P = g.pitch;
#pragma unroll
    for (int s = 0; s < NSTAGE; ++s) {
        const int comp = (s >> 1) & 1;
#pragma unroll
        for (int it = 0; it < S::iters(s); ++it) {
            const int q = tid + it * kTileThreads;
            int a, b;
            stage_node<TW, TH, H>(s, q, gi0, gj0, a, b);
            const int gi = gi0 + a, gj = gj0 + b;
            const bool ok = q < S::rows(s) * S::half(s) && (comp == 0 ? ux_at<IN>(g, gi, gj) : uy_at<IN>(g, gi, gj));
            const int c = ok ? gi * P + gj : 0;
            rr[S::offset(s) + it] = ok ? (comp == 0 ? rx[c] : ry[c]) : (T)0;
        }
    }
}

// NSTAGE colour half-sweeps.  Each stage needs the previous one's values
// one node further out, hence the shrinking regions.  With GHOSTS a
// wall-adjacent node refreshes its own ghost right away; only that node
// reads the ghost, so a later sweep (or the residual) in the same pass sees
// the mirror of the latest value, as a sweep over the whole grid with
// ghosts refilled between sweeps does.  A single sweep without residual
// never re-reads a ghost, and the store writes the ghosts.  With ZERO the
// pass starts from a zero iterate, so in the first sweep the vx-red stage
// reads only zeros (L e = 0) and the vx-black and vy-red stages read no
// non-zero vy: their stencils skip those terms (fewer loads; the same values
// up to rounding).
template <typename T, int TW, int TH, int H, int NSTAGE, bool IN, bool GHOSTS, bool ZERO>
__device__ __forceinline__ void gs_stages(const Geom& g, int gi0, int gj0, T* sx, T* sy, const T* sb, const T* sp,
                                          const T* rr, T omega, const LevelC<T>& k) {
    using S = Stages<TW, TH, H, NSTAGE>;
    constexpr int RW = TW + 2 * H, RH = TH + 2 * H;
    const int tid = threadIdx.x;
#pragma unroll
    for (int s = 0; s < NSTAGE; ++s) {
        const int comp = (s >> 1) & 1;
#pragma unroll
        for (int it = 0; it < S::iters(s); ++it) {
            const int q = tid + it * kTileThreads;
            if (q >= S::rows(s) * S::half(s)) continue;
            int a, b;
            stage_node<TW, TH, H>(s, q, gi0, gj0, a, b);
            const int gi = gi0 + a, gj = gj0 + b;
            const int c = a * RW + b;
            const T r = rr[S::offset(s) + it];
            if (comp == 0) {
                if (!ux_at<IN>(g, gi, gj)) continue;
                const T d = dx_at<IN>(sb, sp, c, RW, gi, g, k);
                T e;
                if (ZERO && s == 0) e = relax((T)0, omega, r, d);
                else if (ZERO && s == 1) e = relax(sx[c], omega, r - lx_row_novy(sx, sb, sp, c, RW, k.idx, k.idy), d);
                else e = relax(sx[c], omega, r - lx_row(sx, sy, sb, sp, c, RW, k.idx, k.idy), d);
                sx[c] = e;
                if (GHOSTS && !IN) {
                    if (gi == 1 && a >= 1) sx[c - RW] = k.mirS * e;
                    if (gi == g.ny && a + 1 < RH) sx[c + RW] = k.mirN * e;
                }
            } else {
                if (!uy_at<IN>(g, gi, gj)) continue;
                const T d = dy_at<IN>(sb, sp, c, RW, gj, g, k);
                const T e = (ZERO && s == 2) ? relax((T)0, omega, r - ly_row_novy(sx, sb, c, RW, k.idx, k.idy), d)
                                             : relax(sy[c], omega, r - ly_row(sx, sy, sb, sp, c, RW, k.idx, k.idy), d);
                sy[c] = e;
                if (GHOSTS && !IN) {
                    if (gj == 1 && b >= 1) sy[c - 1] = k.mirW * e;
                    if (gj == g.nx && b + 1 < RW) sy[c + 1] = k.mirE * e;
                }
            }
        }
        __syncthreads();
    }
}

// write the tile's own nodes (and the ghosts they own) to memory
template <typename T, int TW, int TH, int H, bool IN>
__device__ __forceinline__ void tile_store(const Geom& g, int gi0, int gj0, const T* sx, const T* sy,
                                           T* __restrict__ exo, T* __restrict__ eyo, const LevelC<T>& k) {
    constexpr int RW = TW + 2 * H;
    const int P = g.pitch;
#pragma unroll
    for (int it = 0; it < tile_iters<TW * TH>(); ++it) {
        const int q = threadIdx.x + it * kTileThreads;
        if (q >= TW * TH) continue;
        const int a = H + q / TW, b = H + (q - (q / TW) * TW);
        const int gi = gi0 + a, gj = gj0 + b;
        const int c = a * RW + b;
        const int cg = gi * P + gj;
        if (ux_at<IN>(g, gi, gj)) {
            const T e = sx[c];
            exo[cg] = e;
            if (!IN && gi == 1) exo[cg - P] = k.mirS * e;
            if (!IN && gi == g.ny) exo[cg + P] = k.mirN * e;
        }
        if (uy_at<IN>(g, gi, gj)) {
            const T e = sy[c];
            eyo[cg] = e;
            if (!IN && gj == 1) eyo[cg - 1] = k.mirW * e;
            if (!IN && gj == g.nx) eyo[cg + 1] = k.mirE * e;
        }
    }
}

// normalised restriction of the fine residual held in LDS (stx, sty of
// row length RC, first row / column fi0, fj0) to coarse cell (I, J)
// (gather form of Alg. "4-Color Parallel Restriction", factor 2)
template <typename T, int RC>
__device__ __forceinline__ void restrict_cell(const Geom& g, const Geom& gc, const T* stx, const T* sty, int fi0,
                                              int fj0, int I, int J, T* __restrict__ rcx, T* __restrict__ rcy) {
    const int C = I * gc.pitch + J;
    if (J < gc.nx) {
        T s = (T)0, wy = (T)0;
        for (int a4 = 0; a4 < 4; ++a4) {
            const int i = 2 * I - 2 + a4;
            if (i < 1 || i > g.ny) continue;
            const T w = (a4 == 1 || a4 == 2) ? (T)0.75 : (T)0.25;
            const int c = (i - fi0) * RC + (2 * J - fj0);
            s += w * ((T)0.5 * stx[c - 1] + stx[c] + (T)0.5 * stx[c + 1]);
            wy += w;
        }
        rcx[C] = s / ((T)2 * wy);
    }
    if (I < gc.ny) {
        T s = (T)0, wx = (T)0;
        for (int b4 = 0; b4 < 4; ++b4) {
            const int j = 2 * J - 2 + b4;
            if (j < 1 || j > g.nx) continue;
            const T w = (b4 == 1 || b4 == 2) ? (T)0.75 : (T)0.25;
            const int c = (2 * I - fi0) * RC + (j - fj0);
            s += w * ((T)0.5 * sty[c - RC] + sty[c] + (T)0.5 * sty[c + RC]);
            wx += w;
        }
        rcy[C] = s / ((T)2 * wx);
    }
}

// Gauss-Seidel on an LDS tile: NS full sweeps in one pass (halo 4 NS), the
// first from zero, from the iterate in memory, or from the iterate plus the
// prolongated coarse correction (MODE).  The tile reads the old iterate and
// writes its own nodes to the other buffer, so overlapping tiles never see
// each other's new values and the result equals NS sweeps over the whole
// grid exactly.  With RR the pass continues (halo 4 NS + 2) with the
// residual r - L e on the tile grown by one node and the restriction of the
// coarse cells the tile covers (TW x TH fine = TW/2 x TH/2 coarse): the
// down leg of a V-cycle level in one launch, the fine residual never going
// to memory.
template <typename T, int TW, int TH, int NS, int MODE, int RR, bool IN>
__device__ __forceinline__ void gs_tile_run(const Geom& g, const Geom& gc, const T* __restrict__ exi,
                                            const T* __restrict__ eyi, T* __restrict__ exo, T* __restrict__ eyo,
                                            const T* __restrict__ rx, const T* __restrict__ ry,
                                            const T* __restrict__ eb, const T* __restrict__ ep,
                                            const T* __restrict__ ecx, const T* __restrict__ ecy,
                                            T* __restrict__ rcx, T* __restrict__ rcy, T omega, int tbx, int tby,
                                            T* sx, T* sy, T* sb, T* sp, T* scx, T* scy, T* stx, T* sty) {
    constexpr int H = 4 * NS + (RR ? 2 : 0);
    constexpr int RW = TW + 2 * H, RH = TH + 2 * H;
    constexpr int TRW = RR ? TW + 2 : 1, TRH = RR ? TH + 2 : 1;
    constexpr int NR = Stages<TW, TH, H, 4 * NS>::total();
    constexpr int ITR = RR ? tile_iters<TRW * TRH>() : 1;
    const int i0 = 1 + tby * TH, j0 = 1 + tbx * TW;
    const int gi0 = i0 - H, gj0 = j0 - H;
    const int P = g.pitch;
    const LevelC<T> k = level_consts<T>(g);
    // right-hand sides first: they are in flight while the tile loads
    T rr[NR];
    stage_rhs<T, TW, TH, H, 4 * NS, IN>(g, gi0, gj0, rx, ry, rr);
    T rrx[ITR], rry[ITR];
    if (RR) {
#pragma unroll
        for (int it = 0; it < ITR; ++it) {
            const int q = threadIdx.x + it * kTileThreads;
            const int a = q / TRW, b = q - (q / TRW) * TRW;
            const int gi = i0 - 1 + a, gj = j0 - 1 + b;
            const bool okx = q < TRW * TRH && ux_at<IN>(g, gi, gj), oky = q < TRW * TRH && uy_at<IN>(g, gi, gj);
            rrx[it] = okx ? rx[gi * P + gj] : (T)0;
            rry[it] = oky ? ry[gi * P + gj] : (T)0;
        }
    }
    tile_load<T, RW, RH, MODE, IN>(g, gc, gi0, gj0, exi, eyi, eb, ep, ecx, ecy, sx, sy, sb, sp, scx, scy, k);
    gs_stages<T, TW, TH, H, 4 * NS, IN, (NS > 1 || RR), MODE == kModeZero>(g, gi0, gj0, sx, sy, sb, sp, rr, omega,
                                                                          k);
    tile_store<T, TW, TH, H, IN>(g, gi0, gj0, sx, sy, exo, eyo, k);
    if (RR) {
#pragma unroll
        for (int it = 0; it < ITR; ++it) {
            const int q = threadIdx.x + it * kTileThreads;
            if (q >= TRW * TRH) continue;
            const int a = q / TRW, b = q - (q / TRW) * TRW;
            const int gi = i0 - 1 + a, gj = j0 - 1 + b;
            const int c = (a + H - 1) * RW + (b + H - 1);
            stx[q] = ux_at<IN>(g, gi, gj) ? rrx[it] - lx_row(sx, sy, sb, sp, c, RW, k.idx, k.idy) : (T)0;
            sty[q] = uy_at<IN>(g, gi, gj) ? rry[it] - ly_row(sx, sy, sb, sp, c, RW, k.idx, k.idy) : (T)0;
        }
        __syncthreads();
        const int I0 = 1 + tby * (TH / 2), J0 = 1 + tbx * (TW / 2);
#pragma unroll
        for (int it = 0; it < tile_iters<(TH / 2) * (TW / 2)>(); ++it) {
            const int q = threadIdx.x + it * kTileThreads;
            if (q >= (TH / 2) * (TW / 2)) continue;
            const int I = I0 + q / (TW / 2), J = J0 + (q - (q / (TW / 2)) * (TW / 2));
            if (I > gc.ny || J > gc.nx) continue;
            restrict_cell<T, TRW>(g, gc, stx, sty, i0 - 1, j0 - 1, I, J, rcx, rcy);
        }
    }
}

template <typename T, int TW, int TH, int NS, int MODE, int RR>
__device__ __forceinline__ void gs_tile_body(const Geom& g, const Geom& gc, const T* __restrict__ exi,
                                             const T* __restrict__ eyi, T* __restrict__ exo, T* __restrict__ eyo,
                                             const T* __restrict__ rx, const T* __restrict__ ry,
                                             const T* __restrict__ eb, const T* __restrict__ ep,
                                             const T* __restrict__ ecx, const T* __restrict__ ecy,
                                             T* __restrict__ rcx, T* __restrict__ rcy, T omega, int tbx, int tby) {
    static_assert(TW % 2 == 0 && TH % 2 == 0, "tiles cover whole coarse cells");
    static_assert(!(RR && MODE == kModeProlong), "the down leg starts from zero or an iterate");
    constexpr int H = 4 * NS + (RR ? 2 : 0);
    constexpr int RW = TW + 2 * H, RH = TH + 2 * H, RN = RW * RH;
    constexpr int CN = MODE == kModeProlong ? prolong_rows<RH>() * prolong_rows<RW>() : 1;
    constexpr int TRW = RR ? TW + 2 : 1, TRH = RR ? TH + 2 : 1;
    static_assert((4 * RN + 2 * CN + 2 * TRW * TRH) * sizeof(T) <= 65536, "tile exceeds 64 KB of LDS");
    __shared__ T sx[RN], sy[RN], sb[RN], sp[RN];
    __shared__ T scx[CN], scy[CN];
    __shared__ T stx[TRW * TRH], sty[TRW * TRH];
    // uniform per tile: interior tiles take the check-free path
    if (interior_tile<RW, RH>(g, 1 + tby * TH - H, 1 + tbx * TW - H))
        gs_tile_run<T, TW, TH, NS, MODE, RR, true>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy,
                                                   omega, tbx, tby, sx, sy, sb, sp, scx, scy, stx, sty);
    else
        gs_tile_run<T, TW, TH, NS, MODE, RR, false>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, rcx, rcy,
                                                    omega, tbx, tby, sx, sy, sb, sp, scx, scy, stx, sty);
}

// one damped Jacobi sweep on an LDS tile (halo 1)
template <typename T, int TW, int TH, int MODE>
__device__ __forceinline__ void jacobi_tile_body(const Geom& g, const Geom& gc, const T* __restrict__ exi,
                                                 const T* __restrict__ eyi, T* __restrict__ exo,
                                                 T* __restrict__ eyo, const T* __restrict__ rx,
                                                 const T* __restrict__ ry, const T* __restrict__ eb,
                                                 const T* __restrict__ ep, const T* __restrict__ ecx,
                                                 const T* __restrict__ ecy, T omega, int tbx, int tby) {
    constexpr int H = 1;
    constexpr int RW = TW + 2 * H, RH = TH + 2 * H, RN = RW * RH;
    constexpr int CN = MODE == kModeProlong ? prolong_rows<RH>() * prolong_rows<RW>() : 1;
    __shared__ T sx[RN], sy[RN], sb[RN], sp[RN];
    __shared__ T scx[CN], scy[CN];
    constexpr int IT = tile_iters<TW * TH>();
    const int i0 = 1 + tby * TH, j0 = 1 + tbx * TW;
    const int gi0 = i0 - H, gj0 = j0 - H;
    const int P = g.pitch;
    const LevelC<T> k = level_consts<T>(g);
    T rrx[IT], rry[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int q = threadIdx.x + it * kTileThreads;
        const int a = H + q / TW, b = H + (q - (q / TW) * TW);
        const int gi = gi0 + a, gj = gj0 + b;
        rrx[it] = q < TW * TH && is_vx(g, gi, gj) ? rx[gi * P + gj] : (T)0;
        rry[it] = q < TW * TH && is_vy(g, gi, gj) ? ry[gi * P + gj] : (T)0;
    }
    tile_load<T, RW, RH, MODE, false>(g, gc, gi0, gj0, exi, eyi, eb, ep, ecx, ecy, sx, sy, sb, sp, scx, scy, k);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int q = threadIdx.x + it * kTileThreads;
        if (q >= TW * TH) continue;
        const int a = H + q / TW, b = H + (q - (q / TW) * TW);
        const int gi = gi0 + a, gj = gj0 + b;
        const int c = a * RW + b;
        const int cg = gi * P + gj;
        if (is_vx(g, gi, gj)) {
            const T d = lx_diag(sb, sp, c, RW, gi, g.ny, k);
            const T e = relax(sx[c], omega, rrx[it] - lx_row(sx, sy, sb, sp, c, RW, k.idx, k.idy), d);
            exo[cg] = e;
            if (gi == 1) exo[cg - P] = k.mirS * e;
            if (gi == g.ny) exo[cg + P] = k.mirN * e;
        }
        if (is_vy(g, gi, gj)) {
            const T d = ly_diag(sb, sp, c, RW, gj, g.nx, k);
            const T e = relax(sy[c], omega, rry[it] - ly_row(sx, sy, sb, sp, c, RW, k.idx, k.idy), d);
            eyo[cg] = e;
            if (gj == 1) eyo[cg - 1] = k.mirW * e;
            if (gj == g.nx) eyo[cg + 1] = k.mirE * e;
        }
    }
}

// one smoothing sweep on an LDS tile (either smoother)
template <typename T, int TW, int TH, int SM, int MODE>
__device__ __forceinline__ void smooth_tile_body(const Geom& g, const Geom& gc, const T* __restrict__ exi,
                                                 const T* __restrict__ eyi, T* __restrict__ exo,
                                                 T* __restrict__ eyo, const T* __restrict__ rx,
                                                 const T* __restrict__ ry, const T* __restrict__ eb,
                                                 const T* __restrict__ ep, const T* __restrict__ ecx,
                                                 const T* __restrict__ ecy, T omega, int tbx, int tby) {
    if (SM == kSmGS)
        gs_tile_body<T, TW, TH, 1, MODE, 0>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, nullptr, nullptr,
                                            omega, tbx, tby);
    else
        jacobi_tile_body<T, TW, TH, MODE>(g, gc, exi, eyi, exo, eyo, rx, ry, eb, ep, ecx, ecy, omega, tbx, tby);
}

// ---------------------------------------------------------------------------
// fused residual + restriction
// ---------------------------------------------------------------------------
template <typename T, int CTW, int CTH>
__device__ __forceinline__ void res_restrict_body(const Geom& g, const Geom& gc, const T* __restrict__ ex,
                                                  const T* __restrict__ ey, const T* __restrict__ rx,
                                                  const T* __restrict__ ry, const T* __restrict__ eb,
                                                  const T* __restrict__ ep, T* __restrict__ rcx,
                                                  T* __restrict__ rcy, int tbx, int tby) {
    constexpr int NT = CTW * CTH;
    constexpr int RR = 2 * CTH + 2, RC = 2 * CTW + 2;   // fine residual footprint
    constexpr int LR = RR + 2, LC = RC + 2;             // loaded region
    constexpr int LN = LR * LC, RN = RR * RC;
    __shared__ T sx[LN], sy[LN], sb[LN], sp[LN], stx[RN], sty[RN];
    const int tid = threadIdx.x;
    const int I0 = 1 + tby * CTH, J0 = 1 + tbx * CTW;
    const int fi0 = 2 * I0 - 2, fj0 = 2 * J0 - 2;       // first residual row / column
    const int li0 = fi0 - 1, lj0 = fj0 - 1;             // first loaded row / column
    const int P = g.pitch;
    const LevelC<T> k = level_consts<T>(g);
    constexpr int ITL = (LN + NT - 1) / NT, ITR = (RN + NT - 1) / NT;
    // every load of the tile in flight before the first use (see kTileThreads)
    T vx[ITL], vy[ITL], vb[ITL], vp[ITL], rrx[ITR], rry[ITR];
#pragma unroll
    for (int it = 0; it < ITR; ++it) {
        const int q = tid + it * NT;
        const int a = q / RC, b = q - (q / RC) * RC;
        const int gi = fi0 + a, gj = fj0 + b;
        rrx[it] = q < RN && is_vx(g, gi, gj) ? rx[gi * P + gj] : (T)0;
        rry[it] = q < RN && is_vy(g, gi, gj) ? ry[gi * P + gj] : (T)0;
    }
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
        const int q = tid + it * NT;
        const int a = q / LC, b = q - (q / LC) * LC;
        const int gi = li0 + a, gj = lj0 + b;
        const bool in = q < LN && gi >= 0 && gi <= g.ny + 1 && gj >= 0 && gj <= g.nx + 1;
        const int c = in ? gi * P + gj : 0;
        vx[it] = in ? ex[c] : (T)0;
        vy[it] = in ? ey[c] : (T)0;
        vb[it] = in ? eb[c] : (T)0;
        vp[it] = in ? ep[c] : (T)0;
    }
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
        const int q = tid + it * NT;
        if (q >= LN) continue;
        sx[q] = vx[it];
        sy[q] = vy[it];
        sb[q] = vb[it];
        sp[q] = vp[it];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITR; ++it) {
        const int q = tid + it * NT;
        if (q >= RN) continue;
        const int a = q / RC, b = q - (q / RC) * RC;
        const int gi = fi0 + a, gj = fj0 + b;
        const int cl = (a + 1) * LC + (b + 1);
        stx[q] = is_vx(g, gi, gj) ? rrx[it] - lx_row(sx, sy, sb, sp, cl, LC, k.idx, k.idy) : (T)0;
        sty[q] = is_vy(g, gi, gj) ? rry[it] - ly_row(sx, sy, sb, sp, cl, LC, k.idx, k.idy) : (T)0;
    }
    __syncthreads();
    const int I = I0 + tid / CTW, J = J0 + (tid - (tid / CTW) * CTW);
    if (I > gc.ny || J > gc.nx) return;
    restrict_cell<T, RC>(g, gc, stx, sty, fi0, fj0, I, J, rcx, rcy);
}

// ---------------------------------------------------------------------------
// coarse tail of the V-cycle in one workgroup
// ---------------------------------------------------------------------------
template <typename T>
struct LGeo {            // a level inside LDS: tight pitch nx + 2
    int nx, ny, P;
    T idx, idy, idx2, idy2;
};

// Loops of the coarse tail map threads to rows: 2^s consecutive threads
// share a row, with 2^s the smallest power of two covering the row (at most
// 64), so every lane of a wave has work on small levels and node indices come
// from shifts instead of divisions by a runtime width.
__device__ __forceinline__ int lanes_log2(int width) {
    const int s = width <= 1 ? 0 : 32 - __clz(width - 1);
    return s < 6 ? s : 6;
}

// one Gauss-Seidel colour half-sweep of component comp, in place
template <typename T>
__device__ void cc_gs_half(const LGeo<T>& L, const LevelC<T>& k, int comp, int col, T* ex, T* ey, const T* rx,
                           const T* ry, const T* eb, const T* ep, T omega) {
    const int ncol = comp == 0 ? L.nx - 1 : L.nx;
    const int nrow = comp == 0 ? L.ny : L.ny - 1;
    const int tid = threadIdx.x;
    const int ls = lanes_log2((ncol + 1) >> 1);          // lanes per row: one node of the colour each
    const int lm = (1 << ls) - 1;
    for (int i = 1 + (tid >> ls); i <= nrow; i += blockDim.x >> ls) {
        // first column of colour col in row i: (i + j) & 1 == col
        const int j0 = 1 + (((i + 1) & 1) != col ? 1 : 0);
        for (int j = j0 + 2 * (tid & lm); j <= ncol; j += 2 << ls) {
            const int c = i * L.P + j;
            if (comp == 0) {
                const T d = lx_diag(eb, ep, c, L.P, i, L.ny, k);
                const T e = relax(ex[c], omega, rx[c] - lx_row(ex, ey, eb, ep, c, L.P, k.idx, k.idy), d);
                ex[c] = e;
                if (i == 1) ex[c - L.P] = k.mirS * e;
                if (i == L.ny) ex[c + L.P] = k.mirN * e;
            } else {
                const T d = ly_diag(eb, ep, c, L.P, j, L.nx, k);
                const T e = relax(ey[c], omega, ry[c] - ly_row(ex, ey, eb, ep, c, L.P, k.idx, k.idy), d);
                ey[c] = e;
                if (j == 1) ey[c - 1] = k.mirW * e;
                if (j == L.nx) ey[c + 1] = k.mirE * e;
            }
        }
    }
}

// Jacobi sweep in place: new values held in registers across a barrier.
// Flat mapping over the level's nx * ny nodes: the coarse tail holds at most
// 64 x 64 cells, so a thread owns at most 4096 / blockDim.x <= KMAX nodes.
template <typename T>
__device__ void cc_jacobi(const LGeo<T>& L, const LevelC<T>& k, T* ex, T* ey, const T* rx, const T* ry,
                          const T* eb, const T* ep, T omega) {
    constexpr int KMAX = 8;
    T nvx[KMAX], nvy[KMAX];
    const int n = L.ny * L.nx;
    int t = 0;
    for (int q = threadIdx.x; q < n && t < KMAX; q += blockDim.x, ++t) {
        const int i = 1 + q / L.nx, j = 1 + (q - (q / L.nx) * L.nx);
        const int c = i * L.P + j;
        nvx[t] = (j < L.nx) ? relax(ex[c], omega, rx[c] - lx_row(ex, ey, eb, ep, c, L.P, k.idx, k.idy),
                                    lx_diag(eb, ep, c, L.P, i, L.ny, k))
                            : (T)0;
        nvy[t] = (i < L.ny) ? relax(ey[c], omega, ry[c] - ly_row(ex, ey, eb, ep, c, L.P, k.idx, k.idy),
                                    ly_diag(eb, ep, c, L.P, j, L.nx, k))
                            : (T)0;
    }
    __syncthreads();
    t = 0;
    for (int q = threadIdx.x; q < n && t < KMAX; q += blockDim.x, ++t) {
        const int i = 1 + q / L.nx, j = 1 + (q - (q / L.nx) * L.nx);
        const int c = i * L.P + j;
        if (j < L.nx) {
            ex[c] = nvx[t];
            if (i == 1) ex[c - L.P] = k.mirS * nvx[t];
            if (i == L.ny) ex[c + L.P] = k.mirN * nvx[t];
        }
        if (i < L.ny) {
            ey[c] = nvy[t];
            if (j == 1) ey[c - 1] = k.mirW * nvy[t];
            if (j == L.nx) ey[c + 1] = k.mirE * nvy[t];
        }
    }
    __syncthreads();
}

template <typename T>
constexpr int coarse_threads() { return sizeof(T) == 4 ? 1024 : 512; }

template <typename T>
__device__ __forceinline__ void coarse_cycle_body(const CoarseArgs<T>& A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = (T*)smem_raw;
    const int nl = A.nl;
    // per-level tables live in LDS (not in per-lane arrays, which would go
    // to scratch when indexed by the level number)
    __shared__ LGeo<T> L[kMaxLevels];
    __shared__ LevelC<T> K[kMaxLevels];
    __shared__ int foff[kMaxLevels];
    __shared__ int s_top_off;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // row-parallel mapping for a row of `w` entries: (row, column, row stride, column stride)
    auto rowmap = [&](int w, int& r0, int& rstep, int& c0, int& cstep) {
        const int ls = lanes_log2(w);
        r0 = tid >> ls;
        rstep = nthr >> ls;
        c0 = tid & ((1 << ls) - 1);
        cstep = 1 << ls;
    };
    // Small coarsest systems (at most 128 unknowns, RM rows per 16-lane
    // group): each lane's entries of the inverse are loaded into registers
    // first, so their memory latency hides behind the load phase below
    // instead of stalling the coarsest solve.  Same products and sums in the
    // same order as the loop over memory.
    constexpr int KM = 8, RM = sizeof(T) == 4 ? 2 : 4;
    const int sub = tid & 15, grp = tid >> 4, ngrp = nthr >> 4;
    const bool minv_regs = A.nc <= 16 * KM && A.nc <= RM * ngrp;
    double mv[RM][KM];
    if (minv_regs) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            const int m = grp + r * ngrp;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int q = sub + 16 * k;
                mv[r][k] = (m < A.nc && q < A.nc) ? A.Minv[(size_t)m * A.nc + q] : 0.0;
            }
        }
    }
    if (tid == 0) {
        int off = 0;
        for (int l = 0; l < nl; ++l) {
            L[l].nx = A.g[l].nx;
            L[l].ny = A.g[l].ny;
            L[l].P = A.g[l].nx + 2;
            K[l] = level_consts<T>(A.g[l]);
            foff[l] = off;
            off += 6 * (L[l].ny + 2) * L[l].P;
        }
        s_top_off = off;
    }
    __syncthreads();
    // field q of level l: ex, ey, rx, ry, eb, ep
    auto F = [&](int l, int q) -> T* { return sm + foff[l] + q * (L[l].ny + 2) * L[l].P; };
    const int ntop = (L[0].ny + 2) * L[0].P;
    T* tx = sm + s_top_off;
    T* ty = tx + ntop;
    const size_t off_end = (size_t)s_top_off + 2 * (size_t)ntop;
    double* rs = (double*)(sm + ((off_end * sizeof(T) + 7) / 8) * 8 / sizeof(T));

    // load viscosities of every level and the right-hand side of the top level; zero the rest.
    // One flat index over all levels; the first KL entries of every thread are
    // loaded into registers together (all loads in flight) before any store.
    __shared__ int qoff[kMaxLevels + 1];
    if (tid == 0) {
        int q = 0;
        for (int l = 0; l < nl; ++l) {
            qoff[l] = q;
            q += (L[l].ny + 2) * L[l].P;
        }
        qoff[nl] = q;
    }
    __syncthreads();
    {
        constexpr int KL = sizeof(T) == 4 ? 8 : 16;
        const int ntot = qoff[nl];
        auto locate = [&](int q, int& l, int& i, int& j) {
            l = 0;
            while (q >= qoff[l + 1]) ++l;
            const int r = q - qoff[l];
            i = r / L[l].P;
            j = r - i * L[l].P;
        };
        T vb[KL], vp[KL], vx[KL], vy[KL];
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int q = tid + k * nthr;
            vb[k] = vp[k] = vx[k] = vy[k] = (T)0;
            if (q < ntot) {
                int l, i, j;
                locate(q, l, i, j);
                const int cg = i * A.g[l].pitch + j;
                vb[k] = A.eb[l][cg];
                vp[k] = A.ep[l][cg];
                if (l == 0) {
                    vx[k] = A.rx[cg];
                    vy[k] = A.ry[cg];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int q = tid + k * nthr;
            if (q < ntot) {
                int l, i, j;
                locate(q, l, i, j);
                const int r = i * L[l].P + j;
                F(l, 0)[r] = (T)0;
                F(l, 1)[r] = (T)0;
                F(l, 2)[r] = vx[k];
                F(l, 3)[r] = vy[k];
                F(l, 4)[r] = vb[k];
                F(l, 5)[r] = vp[k];
            }
        }
        // remaining entries (only for very elongated tails)
        for (int q = tid + KL * nthr; q < ntot; q += nthr) {
            int l, i, j;
            locate(q, l, i, j);
            const int r = i * L[l].P + j, cg = i * A.g[l].pitch + j;
            F(l, 0)[r] = (T)0;
            F(l, 1)[r] = (T)0;
            F(l, 2)[r] = l == 0 ? A.rx[cg] : (T)0;
            F(l, 3)[r] = l == 0 ? A.ry[cg] : (T)0;
            F(l, 4)[r] = A.eb[l][cg];
            F(l, 5)[r] = A.ep[l][cg];
        }
    }
    __syncthreads();

    // The level tables are read from LDS once per level and phase group into
    // registers (the colour phases then start without an LDS round trip).
    auto smooth = [&](int l, int nu) {
        T *ex = F(l, 0), *ey = F(l, 1), *rx = F(l, 2), *ry = F(l, 3), *eb = F(l, 4), *ep = F(l, 5);
        const LGeo<T> Lg = L[l];
        const LevelC<T> Kg = K[l];
        for (int s = 0; s < nu; ++s) {
            if (A.smoother == kSmGS) {
                for (int h = 0; h < 4; ++h) {
                    cc_gs_half(Lg, Kg, h >> 1, h & 1, ex, ey, rx, ry, eb, ep, A.omega);
                    __syncthreads();
                }
            } else {
                cc_jacobi(Lg, Kg, ex, ey, rx, ry, eb, ep, A.omega);
            }
        }
    };

    // ---- down: smooth, residual, restrict
    for (int l = 0; l < nl - 1; ++l) {
        smooth(l, A.nu_pre[l]);
        const LGeo<T> G = L[l];
        const LevelC<T> Kl = K[l];
        T *ex = F(l, 0), *ey = F(l, 1), *rx = F(l, 2), *ry = F(l, 3), *eb = F(l, 4), *ep = F(l, 5);
        int rt, rs_, ct, cs_;
        rowmap(G.P, rt, rs_, ct, cs_);
        for (int i = rt; i < G.ny + 2; i += rs_) {
            for (int j = ct; j < G.P; j += cs_) {
                const int q = i * G.P + j;
                const bool vx = i >= 1 && i <= G.ny && j >= 1 && j < G.nx;
                const bool vy = i >= 1 && i < G.ny && j >= 1 && j <= G.nx;
                tx[q] = vx ? rx[q] - lx_row(ex, ey, eb, ep, q, G.P, Kl.idx, Kl.idy) : (T)0;
                ty[q] = vy ? ry[q] - ly_row(ex, ey, eb, ep, q, G.P, Kl.idx, Kl.idy) : (T)0;
            }
        }
        __syncthreads();
        const LGeo<T> C = L[l + 1];
        T *rcx = F(l + 1, 2), *rcy = F(l + 1, 3);
        rowmap(C.nx, rt, rs_, ct, cs_);
        for (int I = 1 + rt; I <= C.ny; I += rs_) {
            for (int J = 1 + ct; J <= C.nx; J += cs_) {
                const int Cc = I * C.P + J;
                if (J < C.nx) {
                    T s = (T)0, wy = (T)0;
                    for (int a4 = 0; a4 < 4; ++a4) {
                        const int i = 2 * I - 2 + a4;
                        if (i < 1 || i > G.ny) continue;
                        const T w = (a4 == 1 || a4 == 2) ? (T)0.75 : (T)0.25;
                        const int c = i * G.P + 2 * J;
                        s += w * ((T)0.5 * tx[c - 1] + tx[c] + (T)0.5 * tx[c + 1]);
                        wy += w;
                    }
                    rcx[Cc] = s / ((T)2 * wy);
                }
                if (I < C.ny) {
                    T s = (T)0, wx = (T)0;
                    for (int b4 = 0; b4 < 4; ++b4) {
                        const int j = 2 * J - 2 + b4;
                        if (j < 1 || j > G.nx) continue;
                        const T w = (b4 == 1 || b4 == 2) ? (T)0.75 : (T)0.25;
                        const int c = 2 * I * G.P + j;
                        s += w * ((T)0.5 * ty[c - G.P] + ty[c] + (T)0.5 * ty[c + G.P]);
                        wx += w;
                    }
                    rcy[Cc] = s / ((T)2 * wx);
                }
            }
        }
        __syncthreads();
    }

    // ---- coarsest: e = -(-L)^{-1} r in FP64.  16 threads per row of the
    // inverse, each summing every 16th entry (loads unrolled so that they are
    // in flight together), then a 16-lane shuffle reduction.
    {
        const int l = nl - 1;
        const LGeo<T>& G = L[l];
        T *ex = F(l, 0), *ey = F(l, 1), *rx = F(l, 2), *ry = F(l, 3);
        const int nvx = G.ny * (G.nx - 1);
        const int n = A.nc;
        for (int m = tid; m < n; m += nthr) {
            int i, j;
            if (m < nvx) { i = 1 + m / (G.nx - 1); j = 1 + m % (G.nx - 1); rs[m] = (double)rx[i * G.P + j]; }
            else { const int mm = m - nvx; i = 1 + mm / G.nx; j = 1 + mm % G.nx; rs[m] = (double)ry[i * G.P + j]; }
        }
        __syncthreads();
        auto put = [&](int m, double sv) {
            const T e = (T)(-sv);
            if (m < nvx) {
                const int i = 1 + m / (G.nx - 1), j = 1 + m % (G.nx - 1);
                const int c = i * G.P + j;
                ex[c] = e;
                if (i == 1) ex[c - G.P] = K[l].mirS * e;
                if (i == G.ny) ex[c + G.P] = K[l].mirN * e;
            } else {
                const int mm = m - nvx;
                const int i = 1 + mm / G.nx, j = 1 + mm % G.nx;
                const int c = i * G.P + j;
                ey[c] = e;
                if (j == 1) ey[c - 1] = K[l].mirW * e;
                if (j == G.nx) ey[c + 1] = K[l].mirE * e;
            }
        };
        if (minv_regs) {
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const int m = grp + r * ngrp;
                double sv = 0.0;
#pragma unroll
                for (int k = 0; k < KM; ++k) {
                    const int q = sub + 16 * k;
                    if (q < n) sv += mv[r][k] * rs[q];
                }
                for (int o = 8; o > 0; o >>= 1) sv += __shfl_xor(sv, o, 16);
                if (sub == 0 && m < n) put(m, sv);
            }
        }
        // otherwise two rows per 16-lane group at a time, column loop unrolled:
        // the loads of both rows are in flight together
        for (int m0 = minv_regs ? n : grp; m0 < n; m0 += 2 * ngrp) {
            const int m1 = m0 + ngrp;
            const double* row0 = A.Minv + (size_t)m0 * n;
            const double* row1 = A.Minv + (size_t)(m1 < n ? m1 : m0) * n;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll 8
            for (int q = sub; q < n; q += 16) {
                const double x = rs[q];
                s0 += row0[q] * x;
                s1 += row1[q] * x;
            }
            for (int o = 8; o > 0; o >>= 1) {
                s0 += __shfl_xor(s0, o, 16);
                s1 += __shfl_xor(s1, o, 16);
            }
            if (sub == 0) {
                put(m0, s0);
                if (m1 < n) put(m1, s1);
            }
        }
        __syncthreads();
    }

    // ---- up: prolong + correct, post-smooth
    for (int l = nl - 2; l >= 0; --l) {
        const LGeo<T> G = L[l];
        const LGeo<T> C = L[l + 1];
        const LevelC<T> Kl = K[l];
        T *ex = F(l, 0), *ey = F(l, 1);
        const T *ecx = F(l + 1, 0), *ecy = F(l + 1, 1);
        int rt, rs_, ct, cs_;
        rowmap(G.nx, rt, rs_, ct, cs_);
        for (int i = 1 + rt; i <= G.ny; i += rs_) {
            for (int j = 1 + ct; j <= G.nx; j += cs_) {
                const int c = i * G.P + j;
                if (j < G.nx) {
                    const T e = ex[c] + prolong_vx(ecx, C.P, i, j);
                    ex[c] = e;
                    if (i == 1) ex[c - G.P] = Kl.mirS * e;
                    if (i == G.ny) ex[c + G.P] = Kl.mirN * e;
                }
                if (i < G.ny) {
                    const T e = ey[c] + prolong_vy(ecy, C.P, i, j);
                    ey[c] = e;
                    if (j == 1) ey[c - 1] = Kl.mirW * e;
                    if (j == G.nx) ey[c + 1] = Kl.mirE * e;
                }
            }
        }
        __syncthreads();
        smooth(l, A.nu_post[l]);
    }

    // ---- write the top-level correction (every entry: walls zero, ghosts mirrored)
    {
        const int P = L[0].P;
        const int Pg = A.g[0].pitch;
        const T* sx = F(0, 0);
        const T* sy = F(0, 1);
        int rt, rs_, ct, cs_;
        rowmap(P, rt, rs_, ct, cs_);
        for (int i = rt; i < L[0].ny + 2; i += rs_) {
            for (int j = ct; j < P; j += cs_) {
                A.ex[i * Pg + j] = sx[i * P + j];
                A.ey[i * Pg + j] = sy[i * P + j];
            }
        }
    }
}

template <typename T>
constexpr int tile_h() { return sizeof(T) == 4 ? 16 : 8; }
// coarse cells per fused residual + restriction tile: kRRTileW x rr_tile_h
// (one thread each; 32 x 8 for either type: taller FP32 tiles gained nothing,
// 32 x 4 FP64 tiles were 2 % slower per solve)
template <typename T>
constexpr int rr_tile_h() { return 8; }
constexpr int kTileW = 64;
constexpr int kRRTileW = 32;

}  // namespace dev
}  // namespace tph
