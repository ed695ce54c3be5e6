// Handle-free residual norms that allocate nothing: tph_energy_residual_noalloc.
//
// The same quantities as tph_energy_residual (relative energy residual, Sec.
// "Residual Norms") and tph_info.res_l2 (plain relative l2 residual), for a
// state (vx, vy, p) of the problem given directly by its grid, viscosities,
// density and gravity, with no solver workspace.  The only device memory
// beyond the caller's inputs and outputs is a file-scope array of reduction
// partials, `scratch`, whose device address is looked up once per device.
//
// Kernel 1 (k_res_tiles): a fixed grid of at most kMaxBlocks workgroups walks
// the 64 x 4-cell tiles of the grid; each tile and its one-node frame is
// staged in LDS from the caller's dense (ny + 2) x (nx + 2) arrays, with the
// velocity walls set to zero and the ghosts mirrored per boundary condition
// while staging (the caller's ghost and wall entries are never read), so
// the stencils of stencil.h run on LDS.  Every workgroup writes its four
// partial sums (energy-weighted |b - A x|^2 and |b|^2, plain |b - A x|^2 and
// |b|^2).  Kernel 2 (k_res_finish, one workgroup) sums the partials in a
// fixed order and writes the two ratios.  Both are deterministic.
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/tephra.h"
#include "common.h"
#include "reduce.h"
#include "solver_internal.h"
#include "stencil.h"

namespace tph {
namespace {
constexpr int kMaxBlocks = 2048;             // workgroups of kernel 1
constexpr int kParts = 4;                    // partial sums per workgroup
}  // namespace
}  // namespace tph

// Reduction partials of every call on this device (kMaxBlocks * kParts
// doubles = 64 KiB), held by each device until the process ends.  In host
// code this name is not a device address: the host passes the per-device
// address from hipGetSymbolAddress (scratch_for) to the kernels.
static __device__ __align__(256) double scratch[tph::kMaxBlocks * tph::kParts];

namespace tph {
namespace {

constexpr int TX = 64;                       // tile columns (one wavefront per row)
constexpr int TY = 4;                        // tile rows
constexpr int LP = TX + 2;                   // LDS row pitch: tile + one node each side
constexpr int LR = TY + 2;                   // LDS rows
constexpr int kMaxSide = 32768;              // largest nx, ny accepted
constexpr int kMaxDevices = 64;

struct Prob {
    int nx, ny, pitch;                        // pitch = nx + 2 (the caller's dense rows)
    double idx, idy, gx, gy;
    LevelC<double> k;
};

// velocity and pressure entries as the solver sees them: walls zero,
// ghosts mirrored from the interior, nothing read outside the equation rows
__device__ __forceinline__ double vx_at(const Prob& q, const double* __restrict__ vx, int i, int j) {
    if (i < 0 || i > q.ny + 1 || j <= 0 || j >= q.nx) return 0.0;
    if (i == 0) return q.k.mirS * vx[(size_t)q.pitch + j];
    if (i == q.ny + 1) return q.k.mirN * vx[(size_t)q.ny * q.pitch + j];
    return vx[(size_t)i * q.pitch + j];
}

__device__ __forceinline__ double vy_at(const Prob& q, const double* __restrict__ vy, int i, int j) {
    if (i <= 0 || i >= q.ny || j < 0 || j > q.nx + 1) return 0.0;
    if (j == 0) return q.k.mirW * vy[(size_t)i * q.pitch + 1];
    if (j == q.nx + 1) return q.k.mirE * vy[(size_t)i * q.pitch + q.nx];
    return vy[(size_t)i * q.pitch + j];
}

__device__ __forceinline__ double at(const double* __restrict__ a, const Prob& q, int i, int j, int lo, int hi_i,
                                     int hi_j) {
    if (i < lo || j < lo || i > hi_i || j > hi_j) return 0.0;
    return a[(size_t)i * q.pitch + j];
}

__global__ __launch_bounds__(256) void k_res_tiles(Prob q, const double* __restrict__ eb,
                                                  const double* __restrict__ ep, const double* __restrict__ rho,
                                                  const double* __restrict__ vx, const double* __restrict__ vy,
                                                  const double* __restrict__ p, double* __restrict__ part) {
    __shared__ double s_vx[LR * LP], s_vy[LR * LP], s_p[LR * LP], s_eb[LR * LP], s_ep[LR * LP], s_rho[LR * LP];
    const int tid = threadIdx.y * TX + threadIdx.x;
    const int tiles_x = (q.nx + TX - 1) / TX;
    const int ntiles = tiles_x * ((q.ny + TY - 1) / TY);
    double ne = 0.0, de = 0.0, n2 = 0.0, d2 = 0.0;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int i0 = (t / tiles_x) * TY + 1;      // first owned row / column
        const int j0 = (t % tiles_x) * TX + 1;
        __syncthreads();                            // the previous tile's readers are done
        for (int e = tid; e < LR * LP; e += TX * TY) {
            const int i = i0 - 1 + e / LP;
            const int j = j0 - 1 + e % LP;
            s_vx[e] = vx_at(q, vx, i, j);
            s_vy[e] = vy_at(q, vy, i, j);
            s_p[e] = at(p, q, i, j, 1, q.ny, q.nx);
            s_eb[e] = at(eb, q, i, j, 0, q.ny, q.nx);
            s_ep[e] = at(ep, q, i, j, 1, q.ny, q.nx);
            s_rho[e] = at(rho, q, i, j, 0, q.ny, q.nx);
        }
        __syncthreads();
        const int i = i0 + threadIdx.y;
        const int j = j0 + threadIdx.x;
        if (i <= q.ny && j <= q.nx) {
            const int c = (threadIdx.y + 1) * LP + threadIdx.x + 1;
            if (j < q.nx) {
                const double a = lx_row(s_vx, s_vy, s_eb, s_ep, c, LP, q.idx, q.idy) - (s_p[c + 1] - s_p[c]) * q.idx;
                const double w = 1.0 / sqrt(-lx_diag(s_eb, s_ep, c, LP, i, q.ny, q.k));
                const double b = -q.gx * 0.5 * (s_rho[c - LP] + s_rho[c]);
                const double r = b - a;
                ne += (r * w) * (r * w);
                de += (b * w) * (b * w);
                n2 += r * r;
                d2 += b * b;
            }
            if (i < q.ny) {
                const double a = ly_row(s_vx, s_vy, s_eb, s_ep, c, LP, q.idx, q.idy) - (s_p[c + LP] - s_p[c]) * q.idy;
                const double w = 1.0 / sqrt(-ly_diag(s_eb, s_ep, c, LP, j, q.nx, q.k));
                const double b = -q.gy * 0.5 * (s_rho[c - 1] + s_rho[c]);
                const double r = b - a;
                ne += (r * w) * (r * w);
                de += (b * w) * (b * w);
                n2 += r * r;
                d2 += b * b;
            }
            {
                const double r = -((s_vx[c] - s_vx[c - 1]) * q.idx + (s_vy[c] - s_vy[c - LP]) * q.idy);
                const double sw = sqrt(wp_weight(s_ep[c], q.k));
                ne += (r * sw) * (r * sw);
                n2 += r * r;
            }
        }
    }
    const double sums[kParts] = {ne, de, n2, d2};
#pragma unroll
    for (int m = 0; m < kParts; ++m) {
        const double s = block_sum(sums[m]);
        if (tid == 0) part[blockIdx.x * kParts + m] = s;
    }
}

__global__ __launch_bounds__(256) void k_res_finish(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ out) {
    double v[kParts] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
        for (int m = 0; m < kParts; ++m) v[m] += part[b * kParts + m];
    double s[kParts];
#pragma unroll
    for (int m = 0; m < kParts; ++m) s[m] = block_sum(v[m]);
    if (threadIdx.x == 0) {
        out[0] = s[1] > 0.0 ? sqrt(s[0] / s[1]) : sqrt(s[0]);
        out[1] = s[3] > 0.0 ? sqrt(s[2] / s[3]) : sqrt(s[2]);
    }
}

// device address of `scratch`, looked up once per device with that device current
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_for(int dev, double** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace tph

using namespace tph;

extern "C" tph_status tph_energy_residual_noalloc(const tph_desc* desc, const double* eta_b, const double* eta_p,
                                                   const double* rho_b, double gx, double gy, const double* vx,
                                                   const double* vy, const double* p, double* out,
                                                   void* hip_stream) {
    tph_internal_set_error("");
    if (!desc) { tph_internal_set_error("desc is NULL"); return TPH_ERR_INVALID; }
    if (!eta_b || !eta_p || !rho_b || !vx || !vy || !p || !out) {
        tph_internal_set_error("eta_b, eta_p, rho_b, vx, vy, p and out are required");
        return TPH_ERR_INVALID;
    }
    if (desc->nx < 2 || desc->ny < 2 || desc->nx > kMaxSide || desc->ny > kMaxSide) {
        tph_internal_set_error("tph_energy_residual_noalloc: nx and ny must lie in [2, 32768]");
        return TPH_ERR_INVALID;
    }
    if (!(desc->lx > 0.0) || !(desc->ly > 0.0) || !std::isfinite(desc->lx) || !std::isfinite(desc->ly)) {
        tph_internal_set_error("lx and ly must be positive and finite");
        return TPH_ERR_INVALID;
    }
    for (int w = 0; w < 4; ++w)
        if (desc->bc[w] != TPH_FREE_SLIP && desc->bc[w] != TPH_NO_SLIP) {
            tph_internal_set_error("bc must be TPH_FREE_SLIP or TPH_NO_SLIP on every wall");
            return TPH_ERR_INVALID;
        }
    if (!std::isfinite(gx) || !std::isfinite(gy)) { tph_internal_set_error("gravity must be finite"); return TPH_ERR_INVALID; }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) {
        tph_internal_set_error("device ordinal out of range");
        return TPH_ERR_INVALID;
    }
    double* part = nullptr;
    if (e == hipSuccess) e = scratch_for(dev, &part);
    if (e != hipSuccess) {
        tph_internal_set_error(std::string("HIP error in tph_energy_residual_noalloc: ") + hipGetErrorString(e));
        return TPH_ERR_HIP;
    }
    Prob q;
    q.nx = desc->nx;
    q.ny = desc->ny;
    q.pitch = desc->nx + 2;
    Geom g{};
    g.nx = desc->nx;
    g.ny = desc->ny;
    g.pitch = q.pitch;
    g.dx = desc->lx / desc->nx;
    g.dy = desc->ly / desc->ny;
    for (int w = 0; w < 4; ++w) g.mir[w] = desc->bc[w] == TPH_NO_SLIP ? -1.0f : 1.0f;
    q.k = level_consts<double>(g);
    q.idx = q.k.idx;
    q.idy = q.k.idy;
    q.gx = gx;
    q.gy = gy;
    const int ntiles = ((q.nx + TX - 1) / TX) * ((q.ny + TY - 1) / TY);
    const int nblk = ntiles < kMaxBlocks ? ntiles : kMaxBlocks;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_res_tiles, dim3(nblk), dim3(TX, TY), 0, st, q, eta_b, eta_p, rho_b, vx, vy, p, part);
    hipLaunchKernelGGL(k_res_finish, dim3(1), dim3(256), 0, st, part, nblk, out);
    e = hipGetLastError();
    if (e != hipSuccess) {
        tph_internal_set_error(std::string("HIP error in tph_energy_residual_noalloc: ") + hipGetErrorString(e));
        return TPH_ERR_HIP;
    }
    return TPH_OK;
}
