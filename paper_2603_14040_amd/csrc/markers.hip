// Marker <-> grid transfers and RK4 marker advection (Sec. "Interpolation
// Between Markers and Grid", Sec. "Advection of Lagrangian Markers",
// eq. rk4_method), behind the tph_markers_* entry points of tephra.h.
//
// Marker -> grid without atomics: markers are binned by the node-grid cell
// that contains them (the cell whose four corners are the nodes they weight)
// with a stable least-significant-digit radix sort of (cell, marker) pairs
// written here (8-bit digits, one pass per digit; see k_digit_count); each
// cell then sums, in sorted order, the weighted values and weights its
// markers give to its four corners, and each node adds the partial sums of
// its (up to) four cells in a fixed order.  Every sum has one writer and a
// fixed order, so results are bitwise reproducible.  Grid -> marker and RK4
// are one thread per marker; all four RK4 stages run in registers, the
// velocity grids are read through the caches.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/tephra.h"
#include "devmem.h"
#include "solver_internal.h"

struct tph_markers {
    int nx = 0, ny = 0;
    double lx = 0, ly = 0, dx = 0, dy = 0;
    int capacity = 0;
    hipStream_t st = nullptr;
    uint32_t* keys[2] = {nullptr, nullptr};
    int32_t* vals[2] = {nullptr, nullptr};
    int32_t* hist = nullptr;       // radix sort: per-(digit, tile) counts, then their scan
    int32_t* chunk = nullptr;      // radix sort: scan of the per-chunk totals of hist
    int32_t* cstart = nullptr;     // per cell: first sorted position
    int32_t* cend = nullptr;       // one past the last
    double* partial = nullptr;     // per cell: 4 corners x (sum w phi, sum w)
    int sorted = 0;                // which key/value buffer holds the sorted pairs
    // the current binning
    int kind = -1;
    int n = 0;
    const double* xm = nullptr;
    const double* ym = nullptr;
    tph::DeviceArena mem;          // device workspace (through the allocator current at creation)
};

namespace {

void tph_internal_set_error_m(const std::string& m) { tph_internal_set_error(m); }

// node grid of a kind: node (i, j) at (x0 + j dx, y0 + i dy), i in [imin, imax], j in [jmin, jmax]
struct NodeGrid {
    double x0, y0, dx, dy;
    int imin, imax, jmin, jmax;
    int pitch;                     // nx + 2: the caller's dense array layout
    double idx, idy;               // 1 / dx, 1 / dy (interpolation multiplies instead of dividing)
};

NodeGrid node_grid(const tph_markers* h, int kind) {
    NodeGrid q{};
    q.dx = h->dx;
    q.dy = h->dy;
    q.pitch = h->nx + 2;
    switch (kind) {
        case TPH_NODES_BASIC: q = {0.0, 0.0, h->dx, h->dy, 0, h->ny, 0, h->nx, h->nx + 2}; break;
        case TPH_NODES_CELL: q = {-0.5 * h->dx, -0.5 * h->dy, h->dx, h->dy, 1, h->ny, 1, h->nx, h->nx + 2}; break;
        case TPH_NODES_VX: q = {0.0, -0.5 * h->dy, h->dx, h->dy, 0, h->ny + 1, 0, h->nx, h->nx + 2}; break;
        default: q = {-0.5 * h->dx, 0.0, h->dx, h->dy, 0, h->ny, 0, h->nx + 1, h->nx + 2}; break;
    }
    q.idx = 1.0 / h->dx;
    q.idy = 1.0 / h->dy;
    return q;
}

// cells of the binning: lower-left node index (i, j) in [0, ny] x [0, nx] for both scatter kinds
__device__ __forceinline__ uint32_t cell_key(const NodeGrid& q, int nx, int ny, double x, double y) {
    int j = (int)floor((x - q.x0) / q.dx);
    int i = (int)floor((y - q.y0) / q.dy);
    j = j < 0 ? 0 : (j > nx ? nx : j);
    i = i < 0 ? 0 : (i > ny ? ny : i);
    return (uint32_t)(i * (nx + 1) + j);
}

__global__ __launch_bounds__(256) void k_bin(NodeGrid q, int nx, int ny, int n, const double* __restrict__ xm,
                                             const double* __restrict__ ym, uint32_t* __restrict__ keys,
                                             int32_t* __restrict__ vals) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    keys[m] = cell_key(q, nx, ny, xm[m], ym[m]);
    vals[m] = m;
}

// ---------------------------------------------------------------------------
// Stable radix sort of (key, marker) pairs, 8-bit digits, least significant
// first.  A tile of kTile = 4096 pairs goes to one workgroup of 4 waves; wave
// w owns pairs [w * 1024, (w + 1) * 1024) of its tile and walks them in 16
// rounds of 64 consecutive pairs.  In a round, the lanes holding the same
// digit find each other with 8 ballots (one per digit bit); a lane's rank
// among them is the number of such lanes below it, added to the wave's
// running count of that digit (kept in LDS, bumped by the highest lane of
// each group).  Ranks therefore follow the pair order, which makes the sort
// stable, and no atomic operation is involved.
//   k_digit_count:  per tile, the count of each digit -> hist[d * ntiles + t]
//   k_scan_chunks / k_scan_top: exclusive scan of hist in that (digit-major)
//                   order, as per-chunk scans plus a scan of the chunk totals
//   k_digit_scatter: ranks again, then writes each pair to
//                   scan[d * ntiles + t] + (its rank in the tile)
// ---------------------------------------------------------------------------
constexpr int kWaves = 4;
constexpr int kRounds = 16;
constexpr int kTile = kWaves * kRounds * 64;     // 4096 pairs per workgroup
constexpr int kChunk = 4096;                     // scan chunk (entries)

// Counts of the 256 digits over this wave's 1024 pairs of tile t, and (when
// rank is non-null) each pair's rank among the wave's pairs of its digit.
__device__ __forceinline__ void wave_rank(const uint32_t* __restrict__ keys, int n, int t, int shift,
                                          int* __restrict__ wcnt, uint32_t* dig, int* rank) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = lane ? ((1ull << lane) - 1ull) : 0ull;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        const long long m = (long long)t * kTile + (long long)w * (kRounds * 64) + k * 64 + lane;
        const bool valid = m < n;
        const uint32_t d = valid ? (keys[m] >> shift) & 255u : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        // every lane of a group reads the count before its highest lane advances it: the read
        // precedes the write in program order, and a wave's LDS operations complete in order
        const int base = valid ? wcnt[d] : 0;
        if (dig) dig[k] = d;
        if (rank) rank[k] = base + __popcll(peers & below);
        if (valid && 63 - __clzll(peers) == lane) wcnt[d] = base + __popcll(peers);
    }
}

__global__ __launch_bounds__(256) void k_digit_count(const uint32_t* __restrict__ keys, int n, int ntiles, int shift,
                                                     int32_t* __restrict__ hist) {
    __shared__ int cnt[kWaves][256];
    const int w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * 256; d += blockDim.x) (&cnt[0][0])[d] = 0;
    __syncthreads();
    wave_rank(keys, n, blockIdx.x, shift, cnt[w], nullptr, nullptr);
    __syncthreads();
    const int d = threadIdx.x;                       // 256 threads: one digit each
    int tot = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) tot += cnt[q][d];
    hist[(size_t)d * ntiles + blockIdx.x] = tot;
}

// exclusive scan of each chunk of kChunk entries in place; chunk totals to sums
__global__ __launch_bounds__(256) void k_scan_chunks(int32_t* __restrict__ a, long long len,
                                                     int32_t* __restrict__ sums) {
    __shared__ int part[256];
    const long long base = (long long)blockIdx.x * kChunk + threadIdx.x * (kChunk / 256);
    int v[kChunk / 256];
    int s = 0;
#pragma unroll
    for (int q = 0; q < kChunk / 256; ++q) {
        v[q] = base + q < len ? a[base + q] : 0;
        s += v[q];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan of the 256 thread totals
    for (int off = 1; off < 256; off <<= 1) {
        const int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int run = part[threadIdx.x] - s;                 // exclusive prefix of this thread
#pragma unroll
    for (int q = 0; q < kChunk / 256; ++q) {
        if (base + q < len) a[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

// exclusive scan of the chunk totals (at most kChunk of them), one workgroup
__global__ __launch_bounds__(256) void k_scan_top(int32_t* __restrict__ sums, int nchunks) {
    __shared__ int part[256];
    const int per = kChunk / 256;
    int v[kChunk / 256];
    int s = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const int i = threadIdx.x * per + q;
        v[q] = i < nchunks ? sums[i] : 0;
        s += v[q];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int run = part[threadIdx.x] - s;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const int i = threadIdx.x * per + q;
        if (i < nchunks) sums[i] = run;
        run += v[q];
    }
}

__global__ __launch_bounds__(256) void k_digit_scatter(const uint32_t* __restrict__ kin,
                                                       const int32_t* __restrict__ vin, int n, int ntiles, int shift,
                                                       const int32_t* __restrict__ scan,
                                                       const int32_t* __restrict__ chunk,
                                                       uint32_t* __restrict__ kout, int32_t* __restrict__ vout) {
    __shared__ int cnt[kWaves][256];
    __shared__ int tile_base[kWaves][256];          // global start of each (wave, digit) run
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * 256; d += blockDim.x) (&cnt[0][0])[d] = 0;
    __syncthreads();
    uint32_t dig[kRounds];
    int rank[kRounds];
    wave_rank(kin, n, blockIdx.x, shift, cnt[w], dig, rank);
    __syncthreads();
    {
        const int d = threadIdx.x;
        const long long e = (long long)d * ntiles + blockIdx.x;
        int off = scan[e] + chunk[e / kChunk];
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            tile_base[q][d] = off;
            off += cnt[q][d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        const long long m = (long long)blockIdx.x * kTile + (long long)w * (kRounds * 64) + k * 64 + lane;
        if (m < n) {
            const int pos = tile_base[w][dig[k]] + rank[k];
            kout[pos] = kin[m];
            vout[pos] = vin[m];
        }
    }
}

__global__ __launch_bounds__(256) void k_ranges(int n, const uint32_t* __restrict__ keys, int32_t* __restrict__ cstart,
                                                int32_t* __restrict__ cend) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) cstart[k] = p;
    if (p == n - 1 || keys[p + 1] != k) cend[k] = p + 1;
}

// Per cell, in sorted (stable: marker index) order: sums of w phi and w for
// its four corners.  A workgroup owns 256 consecutive cells, whose markers
// occupy one contiguous run of the sorted order.  The run goes through LDS
// in chunks of kStage markers: the workgroup reads the sorted marker indices
// and gathers x, y and phi with neighbouring lanes on neighbouring entries;
// then every thread walks its own cell's part of the chunk from LDS.  The
// products and sums per cell are those of a direct loop over the cell's
// markers, in the same order.  Slots are padded by one per 16 entries: the
// cells of neighbouring lanes start about 16 markers apart, which would
// otherwise put their reads on the same LDS banks.
constexpr int kStage = 1024;
constexpr int kStageSlots = kStage + kStage / 16;
__device__ __forceinline__ int stage_slot(int t) { return t + (t >> 4); }

__global__ __launch_bounds__(256) void k_cell_partials(NodeGrid q, int nx, int ny, const int32_t* __restrict__ cstart,
                                                       const int32_t* __restrict__ cend,
                                                       const int32_t* __restrict__ order,
                                                       const double* __restrict__ xm, const double* __restrict__ ym,
                                                       const double* __restrict__ phi, double* __restrict__ partial) {
    __shared__ double sx[kStageSlots], sy[kStageSlots], sf[kStageSlots];
    __shared__ int run_lo[4], run_hi[4];
    const int ncell = (nx + 1) * (ny + 1);
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < ncell;
    const int b = live ? cstart[c] : 0, e = live ? cend[c] : 0;     // empty cells: b == e
    // run of the workgroup: first start and last end over its non-empty cells
    int lo = b < e ? b : INT_MAX, hi = b < e ? e : 0;
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    if ((threadIdx.x & 63) == 0) {
        run_lo[threadIdx.x >> 6] = lo;
        run_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    const int P0 = min(min(run_lo[0], run_lo[1]), min(run_lo[2], run_lo[3]));
    const int P1 = max(max(run_hi[0], run_hi[1]), max(run_hi[2], run_hi[3]));
    const int i = live ? c / (nx + 1) : 0, j = c - i * (nx + 1);
    const double xj = q.x0 + j * q.dx, yi = q.y0 + i * q.dy;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    constexpr int KS = kStage / 256;
    for (int base = P0; base < P1; base += kStage) {
        const int cnt = min(kStage, P1 - base);
        int m[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int t = threadIdx.x + k * 256;
            m[k] = t < cnt ? order[base + t] : -1;
        }
        double vx[KS], vy[KS], vf[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            vx[k] = m[k] >= 0 ? xm[m[k]] : 0.0;
            vy[k] = m[k] >= 0 ? ym[m[k]] : 0.0;
            vf[k] = m[k] >= 0 ? phi[m[k]] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int t = stage_slot(threadIdx.x + k * 256);
            sx[t] = vx[k];
            sy[t] = vy[k];
            sf[t] = vf[k];
        }
        __syncthreads();
        const int pe = min(e, base + cnt);
        for (int p = max(b, base); p < pe; ++p) {
            const int t = stage_slot(p - base);
            const double rx = (sx[t] - xj) / q.dx, ry = (sy[t] - yi) / q.dy;
            const double f = sf[t];
            const double w00 = (1.0 - rx) * (1.0 - ry), w01 = rx * (1.0 - ry), w10 = (1.0 - rx) * ry, w11 = rx * ry;
            s[0] += w00 * f;
            s[1] += w00;
            s[2] += w01 * f;
            s[3] += w01;
            s[4] += w10 * f;
            s[5] += w10;
            s[6] += w11 * f;
            s[7] += w11;
        }
        __syncthreads();
    }
    if (!live) return;
    double* out = partial + (size_t)c * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = s[k];
}

// node (i, j) = corner (1,1) of cell (i-1, j-1), (1,0) of (i-1, j), (0,1) of (i, j-1), (0,0) of (i, j)
__global__ __launch_bounds__(256) void k_nodes(NodeGrid q, int nx, int ny, const double* __restrict__ partial,
                                               double fill, double* __restrict__ grid) {
    const int j = q.jmin + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int i = q.imin + (int)blockIdx.y;
    if (j > q.jmax || i > q.imax) return;
    double num = 0.0, den = 0.0;
    const int ci[4] = {i - 1, i - 1, i, i};
    const int cj[4] = {j - 1, j, j - 1, j};
    const int corner[4] = {3, 2, 1, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (ci[k] < 0 || ci[k] > ny || cj[k] < 0 || cj[k] > nx) continue;
        const double* pp = partial + ((size_t)ci[k] * (nx + 1) + cj[k]) * 8 + 2 * corner[k];
        num += pp[0];
        den += pp[1];
    }
    grid[(size_t)i * q.pitch + j] = den > 0.0 ? num / den : fill;
}

// (the cell found by a multiplication may differ from the divided one for a
// marker on a cell edge; both cells give the same value there)
__device__ __forceinline__ double interp(const NodeGrid& q, const double* __restrict__ grid, double x, double y) {
    const double tx = (x - q.x0) * q.idx, ty = (y - q.y0) * q.idy;
    int j = (int)floor(tx);
    int i = (int)floor(ty);
    j = j < q.jmin ? q.jmin : (j > q.jmax - 1 ? q.jmax - 1 : j);
    i = i < q.imin ? q.imin : (i > q.imax - 1 ? q.imax - 1 : i);
    double rx = tx - j, ry = ty - i;
    rx = rx < 0.0 ? 0.0 : (rx > 1.0 ? 1.0 : rx);
    ry = ry < 0.0 ? 0.0 : (ry > 1.0 ? 1.0 : ry);
    const double* g0 = grid + (size_t)i * q.pitch + j;
    const double* g1 = g0 + q.pitch;
    return (1.0 - rx) * (1.0 - ry) * g0[0] + rx * (1.0 - ry) * g0[1] + (1.0 - rx) * ry * g1[0] + rx * ry * g1[1];
}

__global__ __launch_bounds__(256) void k_from_grid(NodeGrid q, int n, const double* __restrict__ xm,
                                                   const double* __restrict__ ym, const double* __restrict__ grid,
                                                   double* __restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    out[m] = interp(q, grid, xm[m], ym[m]);
}

__global__ __launch_bounds__(256) void k_rk4(NodeGrid qx, NodeGrid qy, double lx, double ly, int n,
                                             double* __restrict__ xm, double* __restrict__ ym,
                                             const double* __restrict__ vx, const double* __restrict__ vy, double dt) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    auto clampx = [&](double v) { return v < 0.0 ? 0.0 : (v > lx ? lx : v); };
    auto clampy = [&](double v) { return v < 0.0 ? 0.0 : (v > ly ? ly : v); };
    const double x = xm[m], y = ym[m];
    const double k1x = interp(qx, vx, x, y), k1y = interp(qy, vy, x, y);
    double sx = clampx(x + 0.5 * dt * k1x), sy = clampy(y + 0.5 * dt * k1y);
    const double k2x = interp(qx, vx, sx, sy), k2y = interp(qy, vy, sx, sy);
    sx = clampx(x + 0.5 * dt * k2x);
    sy = clampy(y + 0.5 * dt * k2y);
    const double k3x = interp(qx, vx, sx, sy), k3y = interp(qy, vy, sx, sy);
    sx = clampx(x + dt * k3x);
    sy = clampy(y + dt * k3y);
    const double k4x = interp(qx, vx, sx, sy), k4y = interp(qy, vy, sx, sy);
    xm[m] = clampx(x + dt / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x));
    ym[m] = clampy(y + dt / 6.0 * (k1y + 2.0 * k2y + 2.0 * k3y + k4y));
}

inline unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

#define M_HIP(call)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            tph_internal_set_error_m(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
            return TPH_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)

constexpr int kMaxMarkers = 1 << 28;   // keeps the scan of the digit counts within one top-level workgroup

int key_bits(const tph_markers* h) {
    const uint64_t ncell = (uint64_t)(h->nx + 1) * (uint64_t)(h->ny + 1);
    int b = 1;
    while (b < 32 && (1ull << b) < ncell) ++b;
    return b;
}

}  // namespace

extern "C" {

tph_status tph_markers_create(int32_t nx, int32_t ny, double lx, double ly, int32_t capacity, void* hip_stream,
                              tph_markers** out) {
    tph_internal_set_error_m("");
    if (!out) {
        tph_internal_set_error_m("out is NULL");
        return TPH_ERR_INVALID;
    }
    *out = nullptr;
    if (nx < 1 || ny < 1 || (int64_t)(nx + 2) * (ny + 2) > (int64_t)1 << 30 || !(lx > 0) || !(ly > 0) ||
        !std::isfinite(lx) || !std::isfinite(ly) || capacity < 1 || capacity > kMaxMarkers) {
        tph_internal_set_error_m("need nx, ny >= 1 (grid at most 2^30 entries), positive finite lx, ly and capacity "
                                 "in [1, 2^28]");
        return TPH_ERR_INVALID;
    }
    tph_markers* h = new tph_markers();
    h->nx = nx;
    h->ny = ny;
    h->lx = lx;
    h->ly = ly;
    h->dx = lx / nx;
    h->dy = ly / ny;
    h->capacity = capacity;
    h->st = (hipStream_t)hip_stream;
    h->mem.a = tph::default_allocator();
    const size_t ncell = (size_t)(nx + 1) * (ny + 1);
    std::string what;
    hipError_t e = hipSuccess;
    auto get = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = h->mem.alloc(p, bytes, &what);
    };
    for (int k = 0; k < 2; ++k) {
        get((void**)&h->keys[k], (size_t)capacity * sizeof(uint32_t));
        get((void**)&h->vals[k], (size_t)capacity * sizeof(int32_t));
    }
    get((void**)&h->cstart, ncell * sizeof(int32_t));
    get((void**)&h->cend, ncell * sizeof(int32_t));
    get((void**)&h->partial, ncell * 8 * sizeof(double));
    const long long ntiles = (capacity + kTile - 1) / kTile;
    get((void**)&h->hist, (size_t)ntiles * 256 * sizeof(int32_t));
    get((void**)&h->chunk, (size_t)((ntiles * 256 + kChunk - 1) / kChunk) * sizeof(int32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        tph_markers_destroy(h);
        tph_internal_set_error_m("marker workspace: " + what);
        return e == hipErrorOutOfMemory ? TPH_ERR_OOM : TPH_ERR_HIP;
    }
    *out = h;
    return TPH_OK;
}

void tph_markers_destroy(tph_markers* h) {
    if (!h) return;
    if (h->st) (void)hipStreamSynchronize(h->st);
    h->mem.release_all();
    delete h;
}

tph_status tph_markers_bin(tph_markers* h, int32_t kind, int32_t n, const double* xm, const double* ym) {
    tph_internal_set_error_m("");
    if (!h || (n > 0 && (!xm || !ym))) {
        tph_internal_set_error_m("handle, xm and ym are required");
        return TPH_ERR_INVALID;
    }
    if (kind != TPH_NODES_BASIC && kind != TPH_NODES_CELL) {
        tph_internal_set_error_m("marker -> grid transfers go to TPH_NODES_BASIC or TPH_NODES_CELL");
        return TPH_ERR_INVALID;
    }
    if (n < 0 || n > h->capacity) {
        tph_internal_set_error_m("n must be in [0, capacity]");
        return TPH_ERR_INVALID;
    }
    const NodeGrid q = node_grid(h, kind);
    const size_t ncell = (size_t)(h->nx + 1) * (h->ny + 1);
    M_HIP(hipMemsetAsync(h->cstart, 0, ncell * sizeof(int32_t), h->st));
    M_HIP(hipMemsetAsync(h->cend, 0, ncell * sizeof(int32_t), h->st));
    h->kind = kind;
    h->n = n;
    h->xm = xm;
    h->ym = ym;
    h->sorted = 0;
    if (n == 0) return TPH_OK;
    hipLaunchKernelGGL(k_bin, dim3(blocks(n)), dim3(256), 0, h->st, q, h->nx, h->ny, n, xm, ym, h->keys[0],
                       h->vals[0]);
    M_HIP(hipGetLastError());
    const int ntiles = (n + kTile - 1) / kTile;
    const long long len = (long long)ntiles * 256;
    const int nchunks = (int)((len + kChunk - 1) / kChunk);
    int cur = 0;
    for (int shift = 0; shift < key_bits(h); shift += 8) {
        hipLaunchKernelGGL(k_digit_count, dim3(ntiles), dim3(256), 0, h->st, h->keys[cur], n, ntiles, shift, h->hist);
        hipLaunchKernelGGL(k_scan_chunks, dim3(nchunks), dim3(256), 0, h->st, h->hist, len, h->chunk);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, h->st, h->chunk, nchunks);
        hipLaunchKernelGGL(k_digit_scatter, dim3(ntiles), dim3(256), 0, h->st, h->keys[cur], h->vals[cur], n, ntiles,
                           shift, h->hist, h->chunk, h->keys[1 - cur], h->vals[1 - cur]);
        M_HIP(hipGetLastError());
        cur = 1 - cur;
    }
    h->sorted = cur;
    hipLaunchKernelGGL(k_ranges, dim3(blocks(n)), dim3(256), 0, h->st, n, h->keys[h->sorted], h->cstart, h->cend);
    M_HIP(hipGetLastError());
    return TPH_OK;
}

tph_status tph_markers_to_grid(tph_markers* h, const double* phi_m, double fill, double* grid) {
    tph_internal_set_error_m("");
    if (!h || !grid || (h->n > 0 && !phi_m)) {
        tph_internal_set_error_m("handle, phi_m and grid are required");
        return TPH_ERR_INVALID;
    }
    if (h->kind < 0) {
        tph_internal_set_error_m("no binning: call tph_markers_bin first");
        return TPH_ERR_INVALID;
    }
    const NodeGrid q = node_grid(h, h->kind);
    const int ncell = (h->nx + 1) * (h->ny + 1);
    hipLaunchKernelGGL(k_cell_partials, dim3(blocks(ncell)), dim3(256), 0, h->st, q, h->nx, h->ny, h->cstart, h->cend,
                       h->vals[h->sorted], h->xm, h->ym, phi_m, h->partial);
    M_HIP(hipGetLastError());
    const dim3 grid_((unsigned)((q.jmax - q.jmin + 1 + 255) / 256), (unsigned)(q.imax - q.imin + 1));
    hipLaunchKernelGGL(k_nodes, grid_, dim3(256), 0, h->st, q, h->nx, h->ny, h->partial, fill, grid);
    M_HIP(hipGetLastError());
    return TPH_OK;
}

tph_status tph_markers_from_grid(tph_markers* h, int32_t kind, int32_t n, const double* xm, const double* ym,
                                 const double* grid, double* phi_m) {
    tph_internal_set_error_m("");
    if (!h || (n > 0 && (!xm || !ym || !grid || !phi_m))) {
        tph_internal_set_error_m("handle, xm, ym, grid and phi_m are required");
        return TPH_ERR_INVALID;
    }
    if (kind < TPH_NODES_BASIC || kind > TPH_NODES_VY || n < 0) {
        tph_internal_set_error_m("bad node kind or marker count");
        return TPH_ERR_INVALID;
    }
    if (n == 0) return TPH_OK;
    hipLaunchKernelGGL(k_from_grid, dim3(blocks(n)), dim3(256), 0, h->st, node_grid(h, kind), n, xm, ym, grid, phi_m);
    M_HIP(hipGetLastError());
    return TPH_OK;
}

tph_status tph_markers_advect_rk4(tph_markers* h, int32_t n, double* xm, double* ym, const double* vx,
                                  const double* vy, double dt) {
    tph_internal_set_error_m("");
    if (!h || (n > 0 && (!xm || !ym || !vx || !vy))) {
        tph_internal_set_error_m("handle, xm, ym, vx and vy are required");
        return TPH_ERR_INVALID;
    }
    if (n < 0 || !std::isfinite(dt)) {
        tph_internal_set_error_m("n must be >= 0 and dt finite");
        return TPH_ERR_INVALID;
    }
    if (n == 0) return TPH_OK;
    hipLaunchKernelGGL(k_rk4, dim3(blocks(n)), dim3(256), 0, h->st, node_grid(h, TPH_NODES_VX),
                       node_grid(h, TPH_NODES_VY), h->lx, h->ly, n, xm, ym, vx, vy, dt);
    M_HIP(hipGetLastError());
    return TPH_OK;
}

tph_status tph_markers_sync(tph_markers* h) {
    tph_internal_set_error_m("");
    if (!h) {
        tph_internal_set_error_m("handle is NULL");
        return TPH_ERR_INVALID;
    }
    M_HIP(hipStreamSynchronize(h->st));
    return TPH_OK;
}

}  // extern "C"
