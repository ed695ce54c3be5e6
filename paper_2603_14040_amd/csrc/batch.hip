// Batched solve: many independent Stokes problems of uneven sizes advanced
// in lockstep, one launch per V-cycle phase for the whole batch.
//
// Every problem keeps its own hierarchy and Krylov workspace (a tph_solver
// each).  Kernels take device tables (per problem, per level) and work lists
// of (problem, tile) items, so one launch covers the tiles of every problem
// at one depth of its V-cycle; the coarse tails run as one workgroup per
// problem.  Converged problems are masked by a device flag.  The FGMRES
// iteration index is read from device memory, so the device work of one
// iteration (Uzawa/V-cycle preconditioner, each step closed by one link pass
// that also forms the next step's right-hand side or, after the last step,
// the operator apply; classical Gram-Schmidt, normalisation, read-back of
// the Hessenberg columns) is captured once as a hipGraph and replayed for
// every iteration while every problem iterates; once some have converged the
// iteration is launched directly over work lists compacted to the others,
// so the launches no longer dispatch the converged problems' items.  The
// host only runs the Givens updates of each problem between iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tephra.h"
#include "devmem.h"
#include "fused_dev.h"
#include "solver_internal.h"
#include "stencil_dev.h"

namespace tph {
namespace {

using namespace dev;

constexpr int kChunk = 8192;      // flat elements per Krylov work item

// slots of a problem's device scalar block (same layout as the single solver's)
constexpr int kSlotH1 = 0;
constexpr int kSlotH2 = kSlotH1 + tph::kMaxRestart + 1;
constexpr int kSlotNrm = kSlotH2 + tph::kMaxRestart + 1;
constexpr int kSlotY = kSlotNrm + 1;
constexpr int kSlotMisc = kSlotY + tph::kMaxRestart;
constexpr int kScal = kSlotMisc + 8;

template <typename T>
struct BLevel {
    Geom g;
    const T* eb;
    const T* ep;
    T* ex[2];
    T* ey[2];
    T* rx;
    T* ry;
};

struct BProb {
    Geom g;                        // finest level
    const double* eb64;
    const double* ep64;
    double* x;                     // raw vector allocations (entry 0 of the allocation)
    double* b;
    double* V;
    double* Z;
    double* t1;                    // second z of the Uzawa link
    double* t2;                    // pressure residuals of the Uzawa link (t2, t3)
    double* t3;
    size_t F, n3;
    int nchunk;                    // Krylov work items per vector
    int ncell;                     // kCellBX x kCellBY cell blocks of the finest level
    int nbx;                       // cell blocks per row
    int lc;                        // level of the coarse-tail kernel
    double alpha;
    double* part;                  // reduction partials, rows of max(nchunk, ncell)
    int prow;                      // row length of part
    double* scal;                  // per-problem scalars (same slots as the single solver)
};

__device__ __forceinline__ Vec3 bvec(const BProb& P, double* raw) { return Vec3{raw + (kAlign - 1), P.F}; }

// flat logical item of this block (XCD-aware over the 1D grid)
__device__ __forceinline__ int item_index() {
    int bx, by;
    xcd_tile(bx, by);
    return by * gridDim.x + bx;
}

// ------------------------------------------------------------------ V-cycle
template <typename T, int SM, int MODE>
__global__ __launch_bounds__(kTileThreads) void kb_smooth_tile(const BLevel<T>* __restrict__ lev,
                                                     const BProb* __restrict__ prob, const int2* __restrict__ items,
                                                     const int* __restrict__ active, int depth, int src, int dst,
                                                     int ccur_post, T omega) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BLevel<T>& L = lev[p * kMaxLevels + depth];
    const BLevel<T>& C = lev[p * kMaxLevels + (MODE == kModeProlong ? depth + 1 : depth)];
    const int cc = (MODE == kModeProlong && depth + 1 != prob[p].lc) ? ccur_post : 0;
    smooth_tile_body<T, kTileW, tile_h<T>(), SM, MODE>(
        L.g, C.g, MODE == kModeZero ? nullptr : L.ex[src], MODE == kModeZero ? nullptr : L.ey[src], L.ex[dst],
        L.ey[dst], L.rx, L.ry, L.eb, L.ep, C.ex[cc], C.ey[cc], omega, it.y & 0xffff, it.y >> 16);
}

// Multi-sweep pass over the tiles of one depth (the single solver's
// gs_tile_body on the batch tables): NS Gauss-Seidel sweeps from zero, from
// the iterate in buffer src, or from it plus the prolongated correction of
// the next depth (buffer ccur there, 0 where that depth is the coarse
// tail); with RR the pass ends with the residual restricted to the next
// depth's right-hand side.  The tiles are the depth's one-sweep tiles
// (kTileW x tile_h), which are the multi-sweep tiles for FP32 passes of one
// or two sweeps and FP64 passes of one.
template <typename T, int NS, int MODE, int RR>
__global__ __launch_bounds__(kTileThreads) void kb_gs_tile(const BLevel<T>* __restrict__ lev,
                                                          const BProb* __restrict__ prob,
                                                          const int2* __restrict__ items,
                                                          const int* __restrict__ active, int depth, int src, int dst,
                                                          int ccur, T omega) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BLevel<T>& L = lev[p * kMaxLevels + depth];
    const BLevel<T>& C = lev[p * kMaxLevels + depth + 1];
    const int cc = (MODE == kModeProlong && depth + 1 != prob[p].lc) ? ccur : 0;
    gs_tile_body<T, kTileW, tile_h<T>(), NS, MODE, RR>(
        L.g, C.g, MODE == kModeZero ? nullptr : L.ex[src], MODE == kModeZero ? nullptr : L.ey[src], L.ex[dst],
        L.ey[dst], L.rx, L.ry, L.eb, L.ep, MODE == kModeProlong ? C.ex[cc] : nullptr,
        MODE == kModeProlong ? C.ey[cc] : nullptr, RR ? C.rx : nullptr, RR ? C.ry : nullptr, omega, it.y & 0xffff,
        it.y >> 16);
}

template <typename T>
__global__ __launch_bounds__(kRRTileW * rr_tile_h<T>()) void kb_res_restrict(const BLevel<T>* __restrict__ lev,
                                                                             const int2* __restrict__ items,
                                                                             const int* __restrict__ active,
                                                                             int depth, int cur) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BLevel<T>& L = lev[p * kMaxLevels + depth];
    const BLevel<T>& C = lev[p * kMaxLevels + depth + 1];
    res_restrict_body<T, kRRTileW, rr_tile_h<T>()>(L.g, C.g, L.ex[cur], L.ey[cur], L.rx, L.ry, L.eb, L.ep, C.rx, C.ry,
                                                   it.y & 0xffff, it.y >> 16);
}

template <typename T>
__global__ __launch_bounds__(coarse_threads<T>()) void kb_coarse(const CoarseArgs<T>* __restrict__ args,
                                                                const int* __restrict__ active) {
    if (!active[blockIdx.x]) return;
    coarse_cycle_body<T>(args[blockIdx.x]);
}

// ---------------------------------------------------- finest-level cell kernels
// Entry of the preconditioner: the level-0 right-hand side from the Krylov
// basis vector V_j (energy-scaled).
template <typename T>
__global__ __launch_bounds__(kCellBX * kCellBY) void kb_precond_in(const BLevel<T>* __restrict__ lev,
                                                                   const BProb* __restrict__ prob,
                                                                   const int2* __restrict__ items,
                                                                   const int* __restrict__ active,
                                                                   const int* __restrict__ dj) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BProb& P = prob[p];
    const Vec3 v = bvec(P, P.V + (size_t)(*dj) * P.n3);
    const int j = (it.y & 0xffff) * kCellBX + threadIdx.x + 1;
    const int i = (it.y >> 16) * kCellBY + threadIdx.y + 1;
    precond_in_cell<T>(P.g, v, P.eb64, P.ep64, 1, lev[p * kMaxLevels].rx, lev[p * kMaxLevels].ry, i, j);
}

// Exit of Uzawa step q of S (the single solver's link pass, uzawa_link_cell):
// z = z_old + e with the pressure update, then the next step's right-hand
// side (kLinkNext) or, after the last step, the Krylov apply
// V_{j+1} = W^(1/2) A Z_j (kLinkApply).  z alternates between t1 and Z_j so
// that the last step writes Z_j; the pressure residual between t3 and t2.
template <typename T, int MODE>
__global__ __launch_bounds__(kCellBX * kCellBY) void kb_uzawa_link(const BLevel<T>* __restrict__ lev,
                                                                   const BProb* __restrict__ prob,
                                                                   const int2* __restrict__ items,
                                                                   const int* __restrict__ active,
                                                                   const int* __restrict__ dj, int q, int S, int cur) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BProb& P = prob[p];
    const int jj = *dj;
    const BLevel<T>& L = lev[p * kMaxLevels];
    // the coarse-tail kernel leaves the correction in buffer 0 when it owns the finest level
    const int c = P.lc == 0 ? 0 : cur;
    const Vec3 v = bvec(P, P.V + (size_t)jj * P.n3);
    const Vec3 zj = bvec(P, P.Z + (size_t)jj * P.n3), z1 = bvec(P, P.t1);
    double* const tp0 = bvec(P, P.t3).p();
    double* const tp1 = bvec(P, P.t2).p();
    LinkArgs<T> a{};
    a.ex = L.ex[c];
    a.ey = L.ey[c];
    a.zold = ((S - q) & 1) ? z1 : zj;
    a.acc = q > 0 ? 1 : 0;
    a.srcp = q == 0 ? v.p() : (((q - 1) & 1) ? tp1 : tp0);
    a.src_scaled = q == 0 ? 1 : 0;
    a.alpha = P.alpha;
    a.zout = ((S - 1 - q) & 1) ? z1 : zj;
    a.r = v;
    a.r_scaled = 1;
    a.rx = L.rx;
    a.ry = L.ry;
    a.tp = (q & 1) ? tp1 : tp0;
    a.wout = bvec(P, P.V + (size_t)(jj + 1) * P.n3);
    a.w_scaled = 1;
    const int j = (it.y & 0xffff) * kCellBX + threadIdx.x + 1;
    const int i = (it.y >> 16) * kCellBY + threadIdx.y + 1;
    uzawa_link_cell<T, MODE>(P.g, a, P.eb64, P.ep64, i, j);
}

enum { kResRestart = 0, kResBnorm = 1 };

// FP64 residual at a restart: V_0 = W^(1/2) (b - A x), or of x = 0 (the
// zeroed scratch vector t3) for |W^(1/2) b|; block sums of squares to part
__global__ __launch_bounds__(kCellBX * kCellBY) void kb_outer(const BProb* __restrict__ prob,
                                                              const int2* __restrict__ items,
                                                              const int* __restrict__ active, int mode) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BProb& P = prob[p];
    const int bx = it.y & 0xffff, by = it.y >> 16;
    const int j = bx * kCellBX + threadIdx.x + 1;
    const int i = by * kCellBY + threadIdx.y + 1;
    const Vec3 x = mode == kResRestart ? bvec(P, P.x) : bvec(P, P.t3);
    const double acc = outer_residual_cell(P.g, x, bvec(P, P.b), 1, P.eb64, P.ep64, bvec(P, P.V), 0, 1, 0, i, j);
    const double s = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) P.part[by * P.nbx + bx] = s;
}

// ---------------------------------------------------------------- Krylov
// items: (problem, chunk); a chunk is kChunk consecutive entries of the flat vector
__device__ __forceinline__ void chunk_range(const BProb& P, int c, size_t& lo, size_t& hi) {
    lo = (size_t)c * kChunk;
    hi = lo + kChunk < P.n3 ? lo + kChunk : P.n3;
}

// Classical Gram-Schmidt of w = V_{j+1} against V_0..V_j, with a second pass
// only for the problems where the first one cancels badly: after the
// explicit first projection the norm |w_perp| is exact and the projected
// vector is off orthogonality by about eps |w| / |w_perp|, which stays near
// 1e-13 while |w_perp|^2 >= kCgsTrust |w|^2 (kb_decide sets the per-problem
// flag the second-pass kernels read).
constexpr double kCgsTrust = 1e-6;

// partial rows: v < j+1 dots of V_v with w = V_{j+1}; row j+1: w.w.  With a
// gate, only the problems whose gate flag is set take part.
__global__ __launch_bounds__(256) void kb_multidot(const BProb* __restrict__ prob, const int2* __restrict__ items,
                                                  const int* __restrict__ active, const int* __restrict__ dj,
                                                  const int* __restrict__ gate) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p] || (gate && !gate[p])) return;
    const BProb& P = prob[p];
    const int nv = *dj + 1;
    size_t lo, hi;
    chunk_range(P, it.y, lo, hi);
    const double* w = P.V + (size_t)nv * P.n3;
    double ww = 0.0;
    for (int v0 = 0; v0 < nv; v0 += 8) {
        double acc[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[v] = 0.0;
        for (size_t t = lo + threadIdx.x; t < hi; t += 256) {
            const double wv = w[t];
            if (v0 == 0) ww += wv * wv;
#pragma unroll
            for (int v = 0; v < 8; ++v)
                if (v0 + v < nv) acc[v] += P.V[(size_t)(v0 + v) * P.n3 + t] * wv;
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            if (v0 + v < nv) {
                const double s = block_sum(acc[v]);
                if (threadIdx.x == 0) P.part[(size_t)(v0 + v) * P.prow + it.y] = s;
            }
        }
    }
    const double s = block_sum(ww);
    if (threadIdx.x == 0) P.part[(size_t)nv * P.prow + it.y] = s;
}

// w -= sum_v h[v] V_v and the partial norms of the new w (row 0); gated like kb_multidot
__global__ __launch_bounds__(256) void kb_axpy(const BProb* __restrict__ prob, const int2* __restrict__ items,
                                              const int* __restrict__ active, const int* __restrict__ dj, int hslot,
                                              const int* __restrict__ gate) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p] || (gate && !gate[p])) return;
    const BProb& P = prob[p];
    const int nv = *dj + 1;
    size_t lo, hi;
    chunk_range(P, it.y, lo, hi);
    double* w = P.V + (size_t)nv * P.n3;
    const double* h = P.scal + hslot;
    double acc = 0.0;
    for (size_t t = lo + threadIdx.x; t < hi; t += 256) {
        double x = w[t];
        for (int v = 0; v < nv; ++v) x -= h[v] * P.V[(size_t)v * P.n3 + t];
        w[t] = x;
        acc += x * x;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) P.part[it.y] = s;
}

// per problem: second Gram-Schmidt pass wanted when |w_perp|^2 < kCgsTrust |w|^2;
// otherwise the second-pass coefficients are zero
__global__ __launch_bounds__(64) void kb_decide(const BProb* __restrict__ prob, const int* __restrict__ active,
                                               const int* __restrict__ dj, int* __restrict__ reorth) {
    const int p = blockIdx.x;
    if (!active[p]) return;
    const BProb& P = prob[p];
    const int nv = *dj + 1;
    const double w2 = P.scal[kSlotH1 + nv], n2 = P.scal[kSlotNrm];
    const int r = !(n2 >= kCgsTrust * w2);
    if (threadIdx.x == 0) reorth[p] = r;
    if (!r)
        for (int v = threadIdx.x; v < nv; v += 64) P.scal[kSlotH2 + v] = 0.0;
}

// out[slot + r] = sum over the problem's partial row r
__global__ __launch_bounds__(256) void kb_reduce(const BProb* __restrict__ prob, const int* __restrict__ active,
                                                const int* __restrict__ dj, int rows_plus, int fixed_rows, int ncols_kind,
                                                int slot, const int* __restrict__ gate) {
    const int p = blockIdx.x;
    if (!active[p] || (gate && !gate[p])) return;
    const BProb& P = prob[p];
    const int rows = fixed_rows > 0 ? fixed_rows : *dj + rows_plus;
    const int r = blockIdx.y;
    if (r >= rows) return;
    const int n = ncols_kind == 0 ? P.nchunk : P.ncell;
    double s = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) s += P.part[(size_t)r * P.prow + c];
    s = block_sum(s);
    if (threadIdx.x == 0) P.scal[slot + r] = s;
}

// target = V_{j+1} (which = 0) or V_0 (which = 1): scale by 1 / sqrt(scal[slot])
__global__ __launch_bounds__(256) void kb_scale(const BProb* __restrict__ prob, const int2* __restrict__ items,
                                               const int* __restrict__ active, const int* __restrict__ dj, int which,
                                               int slot) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BProb& P = prob[p];
    double* w = which == 0 ? P.V + (size_t)(*dj + 1) * P.n3 : P.V;
    const double r = 1.0 / sqrt(P.scal[slot]);
    size_t lo, hi;
    chunk_range(P, it.y, lo, hi);
    for (size_t t = lo + threadIdx.x; t < hi; t += 256) w[t] *= r;
}

// x += sum_{v < k_p} y_p[v] Z_v
__global__ __launch_bounds__(256) void kb_update_x(const BProb* __restrict__ prob, const int2* __restrict__ items,
                                                  const int* __restrict__ active, const int* __restrict__ kcount,
                                                  int yslot) {
    const int2 it = items[item_index()];
    const int p = it.x;
    if (!active[p]) return;
    const BProb& P = prob[p];
    const int k = kcount[p];
    size_t lo, hi;
    chunk_range(P, it.y, lo, hi);
    for (size_t t = lo + threadIdx.x; t < hi; t += 256) {
        double s = P.x[t];
        for (int v = 0; v < k; ++v) s += P.scal[yslot + v] * P.Z[(size_t)v * P.n3 + t];
        P.x[t] = s;
    }
}

template <typename T>
inline T* as_t(void* p) { return (T*)p; }

}  // namespace
}  // namespace tph

using namespace tph;

struct tph_batch {
    int count = 0;
    hipStream_t st = nullptr;                      // own stream (graph capture needs a non-null stream)
    hipStream_t user_st = nullptr;                 // caller's stream
    hipEvent_t ev = nullptr;
    // per-problem work (set-ups, copies in and out, residual checks: a few
    // small launches per problem) runs on streams of its own, problem p on
    // ps[p % size], forked from and joined back to st by events
    std::vector<hipStream_t> ps;
    std::vector<hipEvent_t> pev;
    tph_desc d{};                                  // shared settings (first problem's)
    std::vector<tph_solver*> s;
    int maxdepth = 0;                              // fine depths driven by tile kernels
    unsigned msw_mask = 0;                         // depths smoothed in multi-sweep passes (bit d)
    // device tables
    void* d_lev = nullptr;                         // BLevel<T>[count * kMaxLevels]
    BProb* d_prob = nullptr;
    void* d_cargs = nullptr;                       // CoarseArgs<T>[count]
    size_t coarse_lds = 0;
    int* d_active = nullptr;                       // iteration mask
    int* d_reorth = nullptr;                       // per problem: second Gram-Schmidt pass this iteration
    int* d_unfinished = nullptr;                   // restart / update mask
    int* d_j = nullptr;
    int* d_k = nullptr;                            // per problem, basis vectors in this cycle
    double* d_scal = nullptr;                      // count * kScalars
    double* h_scal = nullptr;                      // pinned mirror
    int* h_j = nullptr;                            // pinned
    int* h_int = nullptr;                          // pinned staging: masks and counts (3 * count)
    double* d_part = nullptr;
    // work lists
    std::vector<int2*> d_tiles, d_rr;              // per depth
    std::vector<int> n_tiles, n_rr;
    int2* d_cells = nullptr;
    int n_cells = 0;
    int2* d_chunks = nullptr;
    int n_chunks = 0;
    // Work lists of the lockstep iterations: the full lists above, or only the
    // items of the problems still iterating (same order).  The captured graph
    // holds the full counts, so it runs only while the lists are full; with
    // compacted lists the iteration is launched directly.
    std::vector<std::vector<int2>> h_tiles, h_rr;  // full lists (host)
    std::vector<int2> h_cells, h_chunks;
    std::vector<int2*> it_tiles, it_rr;            // device, capacity of the full lists
    int2* it_cells = nullptr;
    int2* it_chunks = nullptr;
    std::vector<int> itn_tiles, itn_rr;
    int itn_cells = 0, itn_chunks = 0;
    int2* h_stage = nullptr;                       // pinned staging of list uploads
    bool it_full = true;
    hipGraphExec_t iter_exec = nullptr;
    hipGraph_t iter_graph = nullptr;
    // batched coarsest factorisation: one workgroup per problem (null: some problem too large)
    double** d_gj_mats = nullptr;
    int* d_gj_n = nullptr;
    int gj_nmax = 0;
    tph::DeviceArena mem;        // device workspace (through the allocator current at creation)
    bool ready = false;
    bool mixed() const { return d.precision == TPH_MIXED; }
};

namespace {


tph_status b_alloc(tph_batch* b, void** p, size_t bytes) {
    std::string what;
    const hipError_t e = b->mem.alloc(p, bytes, &what);
    if (e != hipSuccess) {
        tph_internal_set_error("batch workspace: " + what);
        return e == hipErrorOutOfMemory ? TPH_ERR_OOM : TPH_ERR_HIP;
    }
    return TPH_OK;
}

#define B_HIP(call)                                                                                     \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) {                                                                         \
            tph_internal_set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
            return TPH_ERR_HIP;                                                                         \
        }                                                                                               \
    } while (0)
#define B_TRY(expr)                    \
    do {                               \
        tph_status s_ = (expr);        \
        if (s_ != TPH_OK) return s_;   \
    } while (0)

constexpr int kProblemStreams = 4;

hipStream_t problem_stream(const tph_batch* b, int p) { return b->ps[(size_t)p % b->ps.size()]; }

// the per-problem streams wait for the work enqueued so far on the batch stream
tph_status fork_problems(tph_batch* b) {
    B_HIP(hipEventRecord(b->ev, b->st));
    for (hipStream_t q : b->ps) B_HIP(hipStreamWaitEvent(q, b->ev, 0));
    return TPH_OK;
}

// the batch stream waits for the work enqueued so far on the per-problem streams
tph_status join_problems(tph_batch* b) {
    for (size_t k = 0; k < b->ps.size(); ++k) {
        B_HIP(hipEventRecord(b->pev[k], b->ps[k]));
        B_HIP(hipStreamWaitEvent(b->st, b->pev[k], 0));
    }
    return TPH_OK;
}

template <typename T>
tph_status build_tables_t(tph_batch* b) {
    const int P = b->count;
    std::vector<BLevel<T>> lev((size_t)P * kMaxLevels);
    std::vector<CoarseArgs<T>> ca(P);
    size_t lds = 0;
    for (int p = 0; p < P; ++p) {
        const TphSolverView v = tph_internal_view(b->s[p]);
        for (int l = 0; l < v.nlev; ++l) {
            BLevel<T>& L = lev[(size_t)p * kMaxLevels + l];
            L.g = v.g[l];
            L.eb = (const T*)v.eb[l];
            L.ep = (const T*)v.ep[l];
            for (int k = 0; k < 2; ++k) {
                L.ex[k] = (T*)v.ex[l][k];
                L.ey[k] = (T*)v.ey[l][k];
            }
            L.rx = (T*)v.rx[l];
            L.ry = (T*)v.ry[l];
        }
        CoarseArgs<T>& a = ca[p];
        std::memset(&a, 0, sizeof(a));
        a.nl = v.nlev - v.lc;
        a.nc = v.ncoarse;
        a.smoother = b->d.smoother;
        a.omega = (T)b->d.omega;
        for (int q = 0; q < a.nl; ++q) {
            a.g[q] = v.g[v.lc + q];
            a.eb[q] = (const T*)v.eb[v.lc + q];
            a.ep[q] = (const T*)v.ep[v.lc + q];
            a.nu_pre[q] = v.nu_pre[v.lc + q];
            a.nu_post[q] = v.nu_post[v.lc + q];
        }
        a.rx = (const T*)v.rx[v.lc];
        a.ry = (const T*)v.ry[v.lc];
        a.ex = (T*)v.ex[v.lc][0];
        a.ey = (T*)v.ey[v.lc][0];
        a.Minv = v.Minv;
        lds = std::max(lds, v.lc_lds);
    }
    B_TRY(b_alloc(b, &b->d_lev, lev.size() * sizeof(BLevel<T>)));
    B_HIP(hipMemcpy(b->d_lev, lev.data(), lev.size() * sizeof(BLevel<T>), hipMemcpyHostToDevice));
    B_TRY(b_alloc(b, &b->d_cargs, ca.size() * sizeof(CoarseArgs<T>)));
    B_HIP(hipMemcpy(b->d_cargs, ca.data(), ca.size() * sizeof(CoarseArgs<T>), hipMemcpyHostToDevice));
    b->coarse_lds = lds;
    if (lds > 64 * 1024)
        B_HIP(hipFuncSetAttribute((const void*)kb_coarse<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return TPH_OK;
}

// device work of one FGMRES iteration (index read from d_j)
template <typename T>
tph_status enqueue_iteration_t(tph_batch* b) {
    hipStream_t st = b->st;
    const BLevel<T>* lev = (const BLevel<T>*)b->d_lev;
    const T om = (T)b->d.omega;
    const int sm = b->d.smoother;
    const int nu_pre = b->d.nu_pre, nu_post = b->d.nu_post;
    const int* act = b->d_active;
    auto tile_launch = [&](int d, int mode, int src, int dst, int ccur) {
        const dim3 grid(b->itn_tiles[d]);
#define KB(SM_, MODE_)                                                                                          \
    hipLaunchKernelGGL((kb_smooth_tile<T, SM_, MODE_>), grid, dim3(kTileThreads), 0, st, lev, b->d_prob,            \
                       b->it_tiles[d], act, d, src, dst, ccur, om)
        if (sm == TPH_SMOOTH_GS) {
            if (mode == kModeZero) KB(kSmGS, kModeZero);
            else if (mode == kModeProlong) KB(kSmGS, kModeProlong);
            else KB(kSmGS, kModePlain);
        } else {
            if (mode == kModeZero) KB(kSmJacobi, kModeZero);
            else if (mode == kModeProlong) KB(kSmJacobi, kModeProlong);
            else KB(kSmJacobi, kModePlain);
        }
#undef KB
    };
    // Multi-sweep passes of a depth: passes of up to two sweeps (FP32) or of
    // one (FP64), the last pre-smoothing pass with the residual restriction,
    // the first post-smoothing pass with the prolongation.
    auto msw_launch = [&](int d, int ns, int mode, int rr, int src, int dst, int ccur) {
        const dim3 grid(b->itn_tiles[d]);
#define KG(NS_, MODE_, RR_)                                                                                    \
    hipLaunchKernelGGL((kb_gs_tile<T, NS_, MODE_, RR_>), grid, dim3(kTileThreads), 0, st, lev, b->d_prob,       \
                       b->it_tiles[d], act, d, src, dst, ccur, om)
#define KG_NS(NS_)                                                                                             \
    do {                                                                                                       \
        if (mode == kModeProlong) KG(NS_, kModeProlong, 0);                                                    \
        else if (mode == kModeZero) { if (rr) KG(NS_, kModeZero, 1); else KG(NS_, kModeZero, 0); }           \
        else { if (rr) KG(NS_, kModePlain, 1); else KG(NS_, kModePlain, 0); }                                 \
    } while (0)
        if constexpr (sizeof(T) == 4) {
            if (ns == 2) KG_NS(2);
            else KG_NS(1);
        } else {
            KG_NS(1);
        }
#undef KG_NS
#undef KG
    };
    const int max_ns = sizeof(T) == 4 ? 2 : 1;
    auto msw = [&](int d) { return ((b->msw_mask >> d) & 1u) != 0; };
    // buffer of the iterate after pre-smoothing and after post-smoothing, per
    // depth (the same for every problem at that depth)
    std::vector<int> cur_pre(b->maxdepth + 1, 0), fin(b->maxdepth + 1, 0);
    for (int d = 0; d < b->maxdepth; ++d) {
        if (msw(d)) {
            const int np = (nu_pre + max_ns - 1) / max_ns, nq = (nu_post + max_ns - 1) / max_ns;
            cur_pre[d] = (np - 1) & 1;
            fin[d] = (cur_pre[d] + nq) & 1;
        } else {
            cur_pre[d] = (nu_pre - 1) & 1;
            fin[d] = (cur_pre[d] + nu_post) & 1;
        }
    }
    const dim3 cells(b->itn_cells);
    const int S = b->d.uzawa_steps;
    hipLaunchKernelGGL(kb_precond_in<T>, cells, dim3(kCellBX, kCellBY), 0, st, lev, b->d_prob, b->it_cells, act, b->d_j);
    for (int step = 0; step < S; ++step) {
        for (int d = 0; d < b->maxdepth; ++d) {
            if (b->itn_tiles[d] == 0) continue;
            if (msw(d)) {
                int cur = 0;
                bool zero = true;
                for (int left = nu_pre; left > 0;) {
                    const int ns = left >= max_ns ? max_ns : 1;
                    const int dst = zero ? 0 : 1 - cur;
                    msw_launch(d, ns, zero ? kModeZero : kModePlain, left == ns ? 1 : 0, cur, dst, 0);
                    cur = dst;
                    zero = false;
                    left -= ns;
                }
                continue;
            }
            tile_launch(d, kModeZero, 0, 0, 0);
            int cur = 0;
            for (int k = 1; k < nu_pre; ++k) {
                tile_launch(d, kModePlain, cur, 1 - cur, 0);
                cur = 1 - cur;
            }
            hipLaunchKernelGGL(kb_res_restrict<T>, dim3(b->itn_rr[d]), dim3(kRRTileW * rr_tile_h<T>()), 0, st, lev,
                               b->it_rr[d], act, d, cur);
        }
        hipLaunchKernelGGL(kb_coarse<T>, dim3(b->count), dim3(coarse_threads<T>()), b->coarse_lds, st,
                           (const CoarseArgs<T>*)b->d_cargs, act);
        for (int d = b->maxdepth - 1; d >= 0; --d) {
            if (b->itn_tiles[d] == 0) continue;
            int cur = cur_pre[d];
            if (msw(d)) {
                bool pro = true;
                for (int left = nu_post; left > 0;) {
                    const int ns = left >= max_ns ? max_ns : 1;
                    msw_launch(d, ns, pro ? kModeProlong : kModePlain, 0, cur, 1 - cur, fin[d + 1]);
                    cur = 1 - cur;
                    pro = false;
                    left -= ns;
                }
                continue;
            }
            tile_launch(d, kModeProlong, cur, 1 - cur, fin[d + 1]);
            cur = 1 - cur;
            for (int k = 1; k < nu_post; ++k) {
                tile_launch(d, kModePlain, cur, 1 - cur, 0);
                cur = 1 - cur;
            }
        }
        if (step < S - 1)
            hipLaunchKernelGGL((kb_uzawa_link<T, kLinkNext>), cells, dim3(kCellBX, kCellBY), 0, st, lev, b->d_prob, b->it_cells,
                               act, b->d_j, step, S, fin[0]);
        else
            hipLaunchKernelGGL((kb_uzawa_link<T, kLinkApply>), cells, dim3(kCellBX, kCellBY), 0, st, lev, b->d_prob, b->it_cells,
                               act, b->d_j, step, S, fin[0]);
    }
    const dim3 chunks(b->itn_chunks);
    const int2* ck = b->it_chunks;
    const dim3 rgrid(b->count, tph::kMaxRestart + 2);
    // classical Gram-Schmidt (dots and |w|^2, projection with the exact new
    // norm), then a second pass only where the first cancelled (kb_decide)
    const dim3 ngrid(b->count, 1);
    const int* ro = b->d_reorth;
    hipLaunchKernelGGL(kb_multidot, chunks, dim3(256), 0, st, b->d_prob, ck, act, b->d_j, nullptr);
    hipLaunchKernelGGL(kb_reduce, rgrid, dim3(256), 0, st, b->d_prob, act, b->d_j, 2, 0, 0, kSlotH1, nullptr);
    hipLaunchKernelGGL(kb_axpy, chunks, dim3(256), 0, st, b->d_prob, ck, act, b->d_j, kSlotH1, nullptr);
    hipLaunchKernelGGL(kb_reduce, ngrid, dim3(256), 0, st, b->d_prob, act, b->d_j, 0, 1, 0, kSlotNrm, nullptr);
    hipLaunchKernelGGL(kb_decide, dim3(b->count), dim3(64), 0, st, b->d_prob, act, b->d_j, b->d_reorth);
    hipLaunchKernelGGL(kb_multidot, chunks, dim3(256), 0, st, b->d_prob, ck, act, b->d_j, ro);
    hipLaunchKernelGGL(kb_reduce, rgrid, dim3(256), 0, st, b->d_prob, act, b->d_j, 1, 0, 0, kSlotH2, ro);
    hipLaunchKernelGGL(kb_axpy, chunks, dim3(256), 0, st, b->d_prob, ck, act, b->d_j, kSlotH2, ro);
    hipLaunchKernelGGL(kb_reduce, ngrid, dim3(256), 0, st, b->d_prob, act, b->d_j, 0, 1, 0, kSlotNrm, ro);
    hipLaunchKernelGGL(kb_scale, chunks, dim3(256), 0, st, b->d_prob, ck, act, b->d_j, 0, kSlotNrm);
    B_HIP(hipMemcpyAsync(b->h_scal, b->d_scal, (size_t)b->count * kScal * sizeof(double), hipMemcpyDeviceToHost, st));
    return TPH_OK;
}

tph_status enqueue_iteration(tph_batch* b) {
    return b->mixed() ? enqueue_iteration_t<float>(b) : enqueue_iteration_t<double>(b);
}

tph_status build_graph(tph_batch* b) {
    B_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeRelaxed));
    const tph_status s = enqueue_iteration(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->st, &g);
    if (s != TPH_OK) return s;
    B_HIP(e);
    b->iter_graph = g;
    B_HIP(hipGraphInstantiate(&b->iter_exec, g, nullptr, nullptr, 0));
    return TPH_OK;
}

tph_status batch_create_impl(tph_batch* b, int count, const tph_desc* descs) {
    b->count = count;
    b->d = descs[0];
    for (int p = 0; p < count; ++p) {
        const tph_desc& q = descs[p];
        const tph_desc& r = descs[0];
        if (q.precision != r.precision || q.smoother != r.smoother || q.nu_pre != r.nu_pre || q.nu_post != r.nu_post ||
            q.nu_growth != r.nu_growth || q.omega != r.omega || q.alpha != r.alpha || q.restart != r.restart ||
            q.max_iters != r.max_iters || q.uzawa_steps != r.uzawa_steps || q.rtol != r.rtol || q.fused != 1 ||
            q.nu_pre < 1 || q.nu_post < 1 || q.nu_growth != 1.0 || q.msweep != r.msweep) {
            tph_internal_set_error("batched problems must share precision, smoother, sweeps (>= 1, no growth), "
                                   "omega, alpha, restart, max_iters, uzawa_steps, rtol and msweep, with fused "
                                   "kernels");
            return TPH_ERR_INVALID;
        }
        if (q.smoother != TPH_SMOOTH_JACOBI && q.smoother != TPH_SMOOTH_GS) {
            tph_internal_set_error("the batched solver smooths with Jacobi or Gauss-Seidel only");
            return TPH_ERR_UNSUPPORTED;
        }
        if (q.accel != TPH_ACCEL_FGMRES) {
            tph_internal_set_error("the batched solver runs flexible GMRES only (accel = TPH_ACCEL_FGMRES)");
            return TPH_ERR_UNSUPPORTED;
        }
        if (q.eta_mean != r.eta_mean) {
            tph_internal_set_error("batched problems must share eta_mean");
            return TPH_ERR_INVALID;
        }
    }
    b->s.assign(count, nullptr);
    for (int p = 0; p < count; ++p) {
        B_TRY(tph_create(&descs[p], problem_stream(b, p), &b->s[p]));
        const TphSolverView v = tph_internal_view(b->s[p]);
        if (v.lc < 0) {
            tph_internal_set_error("problem " + std::to_string(p) + " has no single-workgroup coarse tail");
            return TPH_ERR_UNSUPPORTED;
        }
        b->maxdepth = std::max(b->maxdepth, v.lc);
    }
    // depths smoothed in multi-sweep passes (desc.msweep: bit d = depth d;
    // -1, the default, = none: with many problems in flight the one-sweep
    // launches are wide enough that the halo recomputation of the passes
    // costs more than the launches they save; Gauss-Seidel only)
    if (b->d.smoother == TPH_SMOOTH_GS && b->maxdepth > 0 && b->d.msweep > 0) {
        const unsigned all = b->maxdepth >= 32 ? ~0u : ((1u << b->maxdepth) - 1u);
        b->msw_mask = (unsigned)b->d.msweep & all;
    }
    {
        std::vector<double*> mats(count);
        std::vector<int> ns(count);
        bool small = true;
        for (int p = 0; p < count; ++p) {
            const TphSolverView v = tph_internal_view(b->s[p]);
            mats[p] = const_cast<double*>(v.Minv);
            ns[p] = v.ncoarse;
            small = small && v.ncoarse <= kGJLds;
            b->gj_nmax = std::max(b->gj_nmax, v.ncoarse);
        }
        if (small) {
            B_TRY(b_alloc(b, (void**)&b->d_gj_mats, count * sizeof(double*)));
            B_TRY(b_alloc(b, (void**)&b->d_gj_n, count * sizeof(int)));
            B_HIP(hipMemcpyAsync(b->d_gj_mats, mats.data(), count * sizeof(double*), hipMemcpyHostToDevice, b->st));
            B_HIP(hipMemcpyAsync(b->d_gj_n, ns.data(), count * sizeof(int), hipMemcpyHostToDevice, b->st));
            B_HIP(hipStreamSynchronize(b->st));
        }
    }
    // per-problem tables and work lists
    std::vector<BProb> pr(count);
    std::vector<std::vector<int2>> tiles(b->maxdepth), rr(b->maxdepth);
    std::vector<int2> cells, chunks;
    size_t prow_total = 0;
    std::vector<size_t> prow_off(count);
    for (int p = 0; p < count; ++p) {
        const TphSolverView v = tph_internal_view(b->s[p]);
        BProb& P = pr[p];
        P.g = v.g[0];
        P.eb64 = v.eb64;
        P.ep64 = v.ep64;
        P.x = v.x;
        P.b = v.b;
        P.V = v.V;
        P.Z = v.Z;
        P.t1 = v.t1;
        P.t2 = v.t2;
        P.t3 = v.t3;
        P.F = v.F;
        P.n3 = v.n3;
        P.nchunk = (int)((v.n3 + kChunk - 1) / kChunk);
        P.nbx = (P.g.nx + kCellBX - 1) / kCellBX;
        P.ncell = P.nbx * ((P.g.ny + kCellBY - 1) / kCellBY);
        P.lc = v.lc;
        P.alpha = descs[p].alpha;
        P.prow = std::max(P.nchunk, P.ncell);
        prow_off[p] = prow_total;
        prow_total += (size_t)P.prow * (tph::kMaxRestart + 2);
    }
    // work lists in longest-processing-time order: problems by decreasing cell
    // count (ties by index), so every launch starts the items of the largest
    // problems first and the small ones fill in behind them
    std::vector<int> lpt(count);
    for (int p = 0; p < count; ++p) lpt[p] = p;
    std::stable_sort(lpt.begin(), lpt.end(), [&](int a, int c) {
        return (long long)pr[a].g.nx * pr[a].g.ny > (long long)pr[c].g.nx * pr[c].g.ny;
    });
    for (const int p : lpt) {
        const TphSolverView v = tph_internal_view(b->s[p]);
        const BProb& P = pr[p];
        for (int d = 0; d < v.lc; ++d) {
            const Geom& g = v.g[d];
            const int th = b->mixed() ? tile_h<float>() : tile_h<double>();
            const int nbx = (g.nx + kTileW - 1) / kTileW, nby = (g.ny + th - 1) / th;
            for (int y = 0; y < nby; ++y)
                for (int x = 0; x < nbx; ++x) tiles[d].push_back(make_int2(p, x | (y << 16)));
            const Geom& gc = v.g[d + 1];
            const int rh = b->mixed() ? rr_tile_h<float>() : rr_tile_h<double>();
            const int cbx = (gc.nx + kRRTileW - 1) / kRRTileW, cby = (gc.ny + rh - 1) / rh;
            for (int y = 0; y < cby; ++y)
                for (int x = 0; x < cbx; ++x) rr[d].push_back(make_int2(p, x | (y << 16)));
        }
        for (int y = 0; y < (P.g.ny + kCellBY - 1) / kCellBY; ++y)
            for (int x = 0; x < P.nbx; ++x) cells.push_back(make_int2(p, x | (y << 16)));
        for (int c = 0; c < P.nchunk; ++c) chunks.push_back(make_int2(p, c));
    }
    B_TRY(b_alloc(b, (void**)&b->d_part, prow_total * sizeof(double)));
    B_TRY(b_alloc(b, (void**)&b->d_scal, (size_t)count * kScal * sizeof(double)));
    B_HIP(hipMemset(b->d_scal, 0, (size_t)count * kScal * sizeof(double)));
    for (int p = 0; p < count; ++p) {
        pr[p].part = b->d_part + prow_off[p];
        pr[p].scal = b->d_scal + (size_t)p * kScal;
    }
    B_TRY(b_alloc(b, (void**)&b->d_prob, pr.size() * sizeof(BProb)));
    B_HIP(hipMemcpy(b->d_prob, pr.data(), pr.size() * sizeof(BProb), hipMemcpyHostToDevice));
    auto upload = [&](const std::vector<int2>& v, int2** dst) -> tph_status {
        if (v.empty()) { *dst = nullptr; return TPH_OK; }
        B_TRY(b_alloc(b, (void**)dst, v.size() * sizeof(int2)));
        B_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice));
        return TPH_OK;
    };
    b->d_tiles.assign(b->maxdepth, nullptr);
    b->d_rr.assign(b->maxdepth, nullptr);
    b->n_tiles.assign(b->maxdepth, 0);
    b->n_rr.assign(b->maxdepth, 0);
    for (int d = 0; d < b->maxdepth; ++d) {
        B_TRY(upload(tiles[d], &b->d_tiles[d]));
        B_TRY(upload(rr[d], &b->d_rr[d]));
        b->n_tiles[d] = (int)tiles[d].size();
        b->n_rr[d] = (int)rr[d].size();
    }
    B_TRY(upload(cells, &b->d_cells));
    B_TRY(upload(chunks, &b->d_chunks));
    b->n_cells = (int)cells.size();
    b->n_chunks = (int)chunks.size();
    // the iteration lists start full; the host keeps the full lists to compact from
    b->it_tiles.assign(b->maxdepth, nullptr);
    b->it_rr.assign(b->maxdepth, nullptr);
    size_t stage = cells.size() + chunks.size();
    for (int d = 0; d < b->maxdepth; ++d) {
        B_TRY(upload(tiles[d], &b->it_tiles[d]));
        B_TRY(upload(rr[d], &b->it_rr[d]));
        stage += tiles[d].size() + rr[d].size();
    }
    B_TRY(upload(cells, &b->it_cells));
    B_TRY(upload(chunks, &b->it_chunks));
    b->itn_tiles = b->n_tiles;
    b->itn_rr = b->n_rr;
    b->itn_cells = b->n_cells;
    b->itn_chunks = b->n_chunks;
    b->h_tiles = std::move(tiles);
    b->h_rr = std::move(rr);
    b->h_cells = std::move(cells);
    b->h_chunks = std::move(chunks);
    b->it_full = true;
    B_HIP(hipHostMalloc((void**)&b->h_stage, std::max<size_t>(stage, 1) * sizeof(int2), hipHostMallocDefault));
    B_TRY(b_alloc(b, (void**)&b->d_active, count * sizeof(int)));
    B_TRY(b_alloc(b, (void**)&b->d_reorth, count * sizeof(int)));
    B_TRY(b_alloc(b, (void**)&b->d_unfinished, count * sizeof(int)));
    B_TRY(b_alloc(b, (void**)&b->d_k, count * sizeof(int)));
    B_TRY(b_alloc(b, (void**)&b->d_j, sizeof(int)));
    B_HIP(hipMemset(b->d_j, 0, sizeof(int)));
    B_HIP(hipHostMalloc((void**)&b->h_scal, (size_t)count * kScal * sizeof(double), hipHostMallocDefault));
    B_HIP(hipHostMalloc((void**)&b->h_j, 64 * sizeof(int), hipHostMallocDefault));
    B_HIP(hipHostMalloc((void**)&b->h_int, 3 * (size_t)count * sizeof(int), hipHostMallocDefault));
    if (b->mixed()) B_TRY(build_tables_t<float>(b));
    else B_TRY(build_tables_t<double>(b));
    B_HIP(hipDeviceSynchronize());
    B_TRY(build_graph(b));
    return TPH_OK;
}

// Iteration work lists of the problems with mask[p] set (all set: the full
// lists, which the captured graph expects).  The stream is idle on entry (the
// solve loop has just synchronised it), so the staging buffer is free.
tph_status set_iteration_lists(tph_batch* b, const std::vector<int>& mask) {
    bool all = true;
    for (int p = 0; p < b->count; ++p) all = all && mask[p] != 0;
    if (all && b->it_full) return TPH_OK;
    B_HIP(hipStreamSynchronize(b->st));
    b->it_full = false;    // until every list is written (a failed upload leaves them to be rewritten)
    size_t off = 0;
    auto put = [&](const std::vector<int2>& full, int2* dst, int* n) -> tph_status {
        int2* out = b->h_stage + off;
        int k = 0;
        for (const int2& it : full)
            if (all || mask[it.x]) out[k++] = it;
        *n = k;
        if (k > 0) B_HIP(hipMemcpyAsync(dst, out, (size_t)k * sizeof(int2), hipMemcpyHostToDevice, b->st));
        off += (size_t)k;
        return TPH_OK;
    };
    for (int d = 0; d < b->maxdepth; ++d) {
        B_TRY(put(b->h_tiles[d], b->it_tiles[d], &b->itn_tiles[d]));
        B_TRY(put(b->h_rr[d], b->it_rr[d], &b->itn_rr[d]));
    }
    B_TRY(put(b->h_cells, b->it_cells, &b->itn_cells));
    B_TRY(put(b->h_chunks, b->it_chunks, &b->itn_chunks));
    b->it_full = all;
    return TPH_OK;
}

// lockstep FGMRES over the batch
tph_status batch_solve_impl(tph_batch* b, tph_info* infos) {
    const int P = b->count, m = b->d.restart;
    hipStream_t st = b->st;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<int> h_act(P, 1), h_unf(P, 1), its(P, 0), restarts(P, 0), jdone(P, 0), status(P, TPH_NOT_CONVERGED);
    std::vector<double> bnorm(P), true_res(P, 0.0), est(P, 0.0), best(P, HUGE_VAL);
    std::vector<int> stall(P, 0);
    std::vector<std::vector<double>> H(P, std::vector<double>((size_t)(m + 1) * m)), cs(P, std::vector<double>(m)),
        sn(P, std::vector<double>(m)), gv(P, std::vector<double>(m + 1));
    const dim3 cells(b->n_cells), chunks(b->n_chunks);
    // masks and counts go through pinned staging (one slot per kind, so a
    // pending copy never reads a buffer the host is already overwriting)
    int* h_unf_pin = b->h_int;
    int* h_act_pin = b->h_int + P;
    int* h_k_pin = b->h_int + 2 * P;
    auto set_mask = [&](int* dmask, const std::vector<int>& h) -> tph_status {
        int* pin = dmask == b->d_active ? h_act_pin : h_unf_pin;
        B_HIP(hipStreamSynchronize(st));
        std::memcpy(pin, h.data(), P * sizeof(int));
        B_HIP(hipMemcpyAsync(dmask, pin, P * sizeof(int), hipMemcpyHostToDevice, st));
        return TPH_OK;
    };
    // |W^(1/2) b| per problem
    B_TRY(set_mask(b->d_unfinished, h_unf));
    B_TRY(fork_problems(b));
    for (int p = 0; p < P; ++p) {
        const TphSolverView v = tph_internal_view(b->s[p]);
        B_HIP(hipMemsetAsync(v.t3, 0, v.n3 * sizeof(double), problem_stream(b, p)));
    }
    B_TRY(join_problems(b));
    hipLaunchKernelGGL(kb_outer, cells, dim3(kCellBX, kCellBY), 0, st, b->d_prob, b->d_cells, b->d_unfinished, (int)kResBnorm);
    hipLaunchKernelGGL(kb_reduce, dim3(P, 1), dim3(256), 0, st, b->d_prob, b->d_unfinished, b->d_j, 0, 1, 1,
                       kSlotMisc, nullptr);
    B_HIP(hipMemcpyAsync(b->h_scal, b->d_scal, (size_t)P * kScal * sizeof(double), hipMemcpyDeviceToHost, st));
    B_HIP(hipStreamSynchronize(st));
    for (int p = 0; p < P; ++p) bnorm[p] = std::sqrt(b->h_scal[(size_t)p * kScal + kSlotMisc]);
    while (true) {
        // true residual of every unfinished problem into V_0
        B_TRY(set_mask(b->d_unfinished, h_unf));
        hipLaunchKernelGGL(kb_outer, cells, dim3(kCellBX, kCellBY), 0, st, b->d_prob, b->d_cells, b->d_unfinished,
                           (int)kResRestart);
        hipLaunchKernelGGL(kb_reduce, dim3(P, 1), dim3(256), 0, st, b->d_prob, b->d_unfinished, b->d_j, 0, 1, 1,
                           kSlotMisc, nullptr);
        B_HIP(hipMemcpyAsync(b->h_scal, b->d_scal, (size_t)P * kScal * sizeof(double), hipMemcpyDeviceToHost, st));
        B_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int p = 0; p < P; ++p) {
            if (!h_unf[p]) continue;
            const double beta = std::sqrt(b->h_scal[(size_t)p * kScal + kSlotMisc]);
            if (!std::isfinite(beta)) {
                tph_internal_set_error("non-finite residual in batched problem " + std::to_string(p));
                return TPH_ERR_NONFINITE;
            }
            true_res[p] = bnorm[p] > 0 ? beta / bnorm[p] : beta;
            if (bnorm[p] == 0.0 || true_res[p] <= b->d.rtol) { h_unf[p] = 0; status[p] = TPH_OK; continue; }
            if (its[p] >= b->d.max_iters) { h_unf[p] = 0; continue; }
            if (true_res[p] > 0.9 * best[p]) {
                if (++stall[p] >= 3) {
                    // stagnation only near the rounding floor (see the single solver); the
                    // problem's x and b live in its solver, the stream is idle here
                    double floor_ = 0.0;
                    B_TRY(tph_internal_rounding_floor(b->s[p], bnorm[p], &floor_));
                    if (true_res[p] <= 100.0 * floor_) { h_unf[p] = 0; continue; }
                    stall[p] = 0;
                }
            } else {
                stall[p] = 0;
            }
            best[p] = std::min(best[p], true_res[p]);
            std::fill(gv[p].begin(), gv[p].end(), 0.0);
            gv[p][0] = beta;
            restarts[p]++;
            any = true;
        }
        if (!any) break;
        h_act = h_unf;
        B_TRY(set_mask(b->d_unfinished, h_unf));
        B_TRY(set_mask(b->d_active, h_act));
        B_TRY(set_iteration_lists(b, h_act));
        hipLaunchKernelGGL(kb_scale, chunks, dim3(256), 0, st, b->d_prob, b->d_chunks, b->d_active, b->d_j, 1,
                           kSlotMisc);
        std::fill(jdone.begin(), jdone.end(), 0);
        for (int j = 0; j < m; ++j) {
            b->h_j[0] = j;
            B_HIP(hipMemcpyAsync(b->d_j, b->h_j, sizeof(int), hipMemcpyHostToDevice, st));
            if (b->it_full) B_HIP(hipGraphLaunch(b->iter_exec, st));
            else B_TRY(enqueue_iteration(b));
            B_HIP(hipStreamSynchronize(st));
            bool changed = false, left = false;
            for (int p = 0; p < P; ++p) {
                if (!h_act[p]) continue;
                const double* sc = b->h_scal + (size_t)p * kScal;
                double* col = &H[p][(size_t)j * (m + 1)];
                for (int i = 0; i <= j; ++i) col[i] = sc[kSlotH1 + i] + sc[kSlotH2 + i];
                const double hn = std::sqrt(sc[kSlotNrm]);
                col[j + 1] = hn;
                if (!std::isfinite(hn)) {
                    tph_internal_set_error("non-finite Krylov basis in batched problem " + std::to_string(p));
                    return TPH_ERR_NONFINITE;
                }
                for (int i = 0; i < j; ++i) {
                    const double a = cs[p][i] * col[i] + sn[p][i] * col[i + 1];
                    col[i + 1] = -sn[p][i] * col[i] + cs[p][i] * col[i + 1];
                    col[i] = a;
                }
                const double rr = std::hypot(col[j], col[j + 1]);
                cs[p][j] = rr > 0 ? col[j] / rr : 1.0;
                sn[p][j] = rr > 0 ? col[j + 1] / rr : 0.0;
                col[j] = rr;
                col[j + 1] = 0.0;
                gv[p][j + 1] = -sn[p][j] * gv[p][j];
                gv[p][j] = cs[p][j] * gv[p][j];
                est[p] = std::fabs(gv[p][j + 1]) / bnorm[p];
                its[p]++;
                jdone[p] = j + 1;
                if (est[p] <= b->d.rtol || its[p] >= b->d.max_iters || hn == 0.0) {
                    h_act[p] = 0;
                    changed = true;
                } else {
                    left = true;
                }
            }
            if (!left) break;
            if (changed) {
                B_TRY(set_mask(b->d_active, h_act));
                B_TRY(set_iteration_lists(b, h_act));
            }
        }
        // y_p = R^{-1} g, x_p += Z y_p
        for (int p = 0; p < P; ++p) {
            double* y = b->h_scal + (size_t)p * kScal + kSlotY;
            const int k = h_unf[p] ? jdone[p] : 0;
            for (int i = k - 1; i >= 0; --i) {
                double t = gv[p][i];
                for (int q = i + 1; q < k; ++q) t -= H[p][(size_t)q * (m + 1) + i] * y[q];
                y[i] = t / H[p][(size_t)i * (m + 1) + i];
            }
            jdone[p] = k;
        }
        B_HIP(hipMemcpyAsync(b->d_scal, b->h_scal, (size_t)P * kScal * sizeof(double), hipMemcpyHostToDevice, st));
        std::memcpy(h_k_pin, jdone.data(), P * sizeof(int));
        B_HIP(hipMemcpyAsync(b->d_k, h_k_pin, P * sizeof(int), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(kb_update_x, chunks, dim3(256), 0, st, b->d_prob, b->d_chunks, b->d_unfinished, b->d_k,
                           kSlotY);
        B_HIP(hipStreamSynchronize(st));
    }
    const auto t1 = std::chrono::steady_clock::now();
    if (infos) {
        B_TRY(fork_problems(b));
        for (int p = 0; p < P; ++p) B_TRY(tph_internal_plain_residual_enqueue(b->s[p]));
        B_TRY(join_problems(b));
        B_HIP(hipStreamSynchronize(st));
    }
    tph_status worst = TPH_OK;
    for (int p = 0; p < P; ++p) {
        if (infos) {
            infos[p].iters = its[p];
            infos[p].vcycles = its[p] * b->d.uzawa_steps;
            infos[p].res_l2 = tph_internal_plain_residual_read(b->s[p]);
            infos[p].restarts = restarts[p];
            infos[p].res_energy = true_res[p];
            infos[p].res_estimate = its[p] ? est[p] : true_res[p];
            infos[p].t_setup_ms = 0.0;
            infos[p].t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        }
        if (status[p] != TPH_OK) worst = TPH_NOT_CONVERGED;
    }
    if (worst == TPH_NOT_CONVERGED) tph_internal_set_error("some batched problems did not converge");
    return worst;
}

}  // namespace

extern "C" {

tph_status tph_batch_create(int32_t count, const tph_desc* descs, void* hip_stream, tph_batch** out) {
    tph_internal_set_error("");
    if (!out || !descs || count < 1) {
        tph_internal_set_error("count must be >= 1 and descs, out non-NULL");
        return TPH_ERR_INVALID;
    }
    *out = nullptr;
    tph_batch* b = new tph_batch();
    b->mem.a = tph::default_allocator();
    b->user_st = (hipStream_t)hip_stream;
    tph_status s = TPH_OK;
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
        tph_internal_set_error("could not create the batch stream");
        s = TPH_ERR_HIP;
    }
    for (int k = 0; s == TPH_OK && k < std::min<int>(kProblemStreams, count); ++k) {
        hipStream_t q = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
            tph_internal_set_error("could not create the per-problem streams");
            s = TPH_ERR_HIP;
            break;
        }
        b->ps.push_back(q);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            tph_internal_set_error("could not create the per-problem stream events");
            s = TPH_ERR_HIP;
            break;
        }
        b->pev.push_back(e);
    }
    if (s == TPH_OK) s = batch_create_impl(b, count, descs);
    if (s != TPH_OK) {
        const std::string msg = tph_last_error();
        tph_batch_destroy(b);
        tph_internal_set_error(msg);
        return s;
    }
    *out = b;
    return TPH_OK;
}

tph_status tph_batch_set_coefficients(tph_batch* b, const double* const* eta_b, const double* const* eta_p,
                                      const double* const* rho_b, const double* gxy) {
    tph_internal_set_error("");
    if (!b || !eta_b || !eta_p || !rho_b || !gxy) {
        tph_internal_set_error("batch, eta_b, eta_p, rho_b and gxy are required");
        return TPH_ERR_INVALID;
    }
    b->ready = false;
    // order after the caller's stream, where the coefficient arrays were produced
    if (hipEventRecord(b->ev, b->user_st) != hipSuccess || hipStreamWaitEvent(b->st, b->ev, 0) != hipSuccess) {
        tph_internal_set_error("could not order the batch stream after the caller's stream");
        return TPH_ERR_HIP;
    }
    B_TRY(fork_problems(b));
    if (b->d_gj_mats) {
        // every problem's setup enqueued on its stream, one launch on the batch
        // stream factors all coarsest operators
        for (int p = 0; p < b->count; ++p) {
            const tph_status s = tph_internal_setup_enqueue(b->s[p], eta_b[p], eta_p[p], rho_b[p], gxy[2 * p],
                                                            gxy[2 * p + 1]);
            if (s != TPH_OK) {
                tph_internal_set_error("problem " + std::to_string(p) + ": " + tph_last_error());
                return s;
            }
        }
        B_TRY(join_problems(b));
        B_HIP(launch_gauss_jordan_batched(b->d_gj_mats, b->d_gj_n, b->count, b->gj_nmax, b->st));
        for (int p = 0; p < b->count; ++p) {
            const tph_status s = tph_internal_setup_finish(b->s[p]);
            if (s != TPH_OK) {
                tph_internal_set_error("problem " + std::to_string(p) + ": " + tph_last_error());
                return s;
            }
        }
    } else {
        for (int p = 0; p < b->count; ++p) {
            const tph_status s = tph_set_coefficients(b->s[p], eta_b[p], eta_p[p], rho_b[p], gxy[2 * p],
                                                      gxy[2 * p + 1], nullptr, nullptr);
            if (s != TPH_OK) {
                tph_internal_set_error("problem " + std::to_string(p) + ": " + tph_last_error());
                return s;
            }
        }
        B_TRY(join_problems(b));
    }
    b->ready = true;
    return TPH_OK;
}

tph_status tph_batch_solve(tph_batch* b, double* const* vx, double* const* vy, double* const* p, tph_info* infos) {
    tph_internal_set_error("");
    if (!b || !vx || !vy || !p) {
        tph_internal_set_error("batch, vx, vy and p are required");
        return TPH_ERR_INVALID;
    }
    if (!b->ready) {
        tph_internal_set_error("tph_batch_set_coefficients has not succeeded on this batch");
        return TPH_ERR_INVALID;
    }
    if (hipEventRecord(b->ev, b->user_st) != hipSuccess || hipStreamWaitEvent(b->st, b->ev, 0) != hipSuccess) {
        tph_internal_set_error("could not order the batch stream after the caller's stream");
        return TPH_ERR_HIP;
    }
    B_TRY(fork_problems(b));
    for (int q = 0; q < b->count; ++q) {
        const tph_status s = tph_internal_load_solution(b->s[q], vx[q], vy[q], p[q]);
        if (s != TPH_OK) return s;
    }
    B_TRY(join_problems(b));
    const tph_status r = batch_solve_impl(b, infos);
    if (r < 0) return r;
    B_TRY(fork_problems(b));
    for (int q = 0; q < b->count; ++q) {
        const tph_status s = tph_internal_finish_solution(b->s[q], vx[q], vy[q], p[q]);
        if (s != TPH_OK) return s;
    }
    B_TRY(join_problems(b));
    const hipError_t e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        tph_internal_set_error(std::string("HIP error: ") + hipGetErrorString(e));
        return TPH_ERR_HIP;
    }
    return r;
}

void tph_batch_destroy(tph_batch* b) {
    if (!b) return;
    if (b->st) (void)hipStreamSynchronize(b->st);
    for (hipStream_t q : b->ps) (void)hipStreamSynchronize(q);
    if (b->iter_exec) (void)hipGraphExecDestroy(b->iter_exec);
    if (b->iter_graph) (void)hipGraphDestroy(b->iter_graph);
    for (tph_solver* s : b->s) tph_destroy(s);
    b->mem.release_all();
    if (b->h_scal) (void)hipHostFree(b->h_scal);
    if (b->h_j) (void)hipHostFree(b->h_j);
    if (b->h_int) (void)hipHostFree(b->h_int);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    for (hipEvent_t e : b->pev) (void)hipEventDestroy(e);
    for (hipStream_t q : b->ps) (void)hipStreamDestroy(q);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
}

}  // extern "C"
