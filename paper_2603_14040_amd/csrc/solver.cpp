// Host side of the solver: level hierarchy, V-cycle driver, flexible GMRES
// and the C ABI declared in include/tephra.h.
//
// Method (Ch. 4): FGMRES(m) in FP64 on A x = b (Sec. "Comparison with
// FGMRES") with the Uzawa step as variable right preconditioner (Sec. "Uzawa
// Iteration as a Fixed Point Method"), one geometric-multigrid V-cycle on L
// inside it (Sec. "Multigrid Cycles").  The Krylov inner product is the
// energy inner product of Sec. "Residual Norms": the basis is stored scaled
// by W^(1/2), W = diag(-L)^(-1) (+) eta_p / (2/dx^2 + 2/dy^2), so plain
// Euclidean dot products give energy norms and the least-squares residual
// estimate is the relative energy residual itself.  Each restart recomputes
// the true FP64 residual, which is the iterative-refinement step of the
// mixed-precision mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tephra.h"
#include "common.h"
#include "devmem.h"
#include "kernels.h"
#include "solver_internal.h"
#include "stencil_dev.h"

using namespace tph;

namespace {

thread_local std::string g_last_error;

void set_error(const std::string& m) { g_last_error = m; }

#define TPH_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
            return TPH_ERR_HIP;                                                             \
        }                                                                                   \
    } while (0)

#define TPH_TRY(expr)                          \
    do {                                       \
        tph_status s_ = (expr);                \
        if (s_ != TPH_OK) return s_;           \
    } while (0)

// slots of the device scalar buffer
constexpr int kSlotH1 = 0;                        // kMaxRestart + 1 entries
constexpr int kSlotH2 = kSlotH1 + kMaxRestart + 1;
constexpr int kSlotNrm = kSlotH2 + kMaxRestart + 1;
constexpr int kSlotY = kSlotNrm + 1;              // kMaxRestart entries
constexpr int kSlotMisc = kSlotY + kMaxRestart;   // 8 entries
constexpr int kScalars = kSlotMisc + 8;

struct LevelBuf {
    Geom g;
    double* eb64 = nullptr;
    double* ep64 = nullptr;
    void* eb = nullptr;          // viscosities in the V-cycle type
    void* ep = nullptr;
    void* ex[2] = {nullptr, nullptr};
    void* ey[2] = {nullptr, nullptr};
    void* rx = nullptr;
    void* ry = nullptr;
    void* tx = nullptr;
    void* ty = nullptr;
    int nu_pre = 0, nu_post = 0;
};

}  // namespace

struct tph_solver {
    tph_desc d{};
    hipStream_t st = nullptr;
    int nlev = 0;
    LevelBuf lev[kMaxLevels];
    double* Minv = nullptr;
    double** gj_table = nullptr; // device {Minv, ncoarse} for the LDS Gauss-Jordan (null: ncoarse too large)
    double* gj_work = nullptr;   // pivot row and column of the device-wide Gauss-Jordan (larger ncoarse)
    double* cont_eb = nullptr;   // continuation: blended viscosities in the caller's dense layout (lazy)
    double* cont_ep = nullptr;
    int ncoarse = 0;
    int lc = -1;                 // first level handled by the single-workgroup coarse kernel (-1: none)
    unsigned msw_mask = 0;       // levels smoothed in multi-sweep passes (resolved desc.msweep)
    unsigned shape_mask = 0;     // levels using the small tile shape (resolved desc.tile_shape)
    size_t lc_lds = 0;           // its LDS bytes
    int max_lds = 65536;         // device limit of LDS per workgroup
    size_t F = 0;                // elements of one field allocation
    size_t n3 = 0;               // elements of a three-field vector
    double* x = nullptr;         // solution vector
    double* b = nullptr;         // right-hand side of set_coefficients
    double* b2 = nullptr;        // right-hand side of a solve_rhs / adjoint call
    double* t1 = nullptr;        // scratch vectors
    double* t2 = nullptr;
    double* t3 = nullptr;        // inner residual of the multi-step preconditioner
    double* V = nullptr;         // (m + 1) basis vectors
    double* Z = nullptr;         // m preconditioned vectors
    double* rho = nullptr;       // staged fields (FP64)
    double* fxe = nullptr;
    double* fye = nullptr;
    double* gtmp[3] = {nullptr, nullptr, nullptr};
    double* partial = nullptr;   // reduction partials
    size_t partial_len = 0;
    double* dscal = nullptr;     // device scalars
    double* hscal = nullptr;     // pinned host mirror (mapped, coherent)
    double* hscal_dev = nullptr; // its device address: reductions write results there directly
    unsigned* hseq = nullptr;    // mapped host word: sequence number written by the last reduction
    unsigned* hseq_dev = nullptr;
    unsigned seq = 0;
    double gx = 0, gy = 0;
    bool has_fx = false, has_fy = false;
    bool ready = false;
    double bnorm = 0;
    double t_setup_ms = 0;
    long long reorth_count = 0;  // second Gram-Schmidt passes taken (diagnostic)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // optional event timing of one kernel class inside solves (the finest-level
    // smoother or the Uzawa link, tph_kernel_timing_target)
    bool ktime = false;
    int ktarget = TPH_KERNEL_SMOOTH;
    int kstride = 1;              // time every kstride-th launch
    long long kcount = 0;
    std::vector<hipEvent_t> kev;  // 2 per recorded launch
    int kev_used = 0;
    int kdropped = 0;
    double kbytes = 0.0;
    DeviceArena mem;              // device workspace (through the allocator current at creation)
    int vc_cycle = 0;             // V-cycle index inside the current preconditioner application (RAS shifts)
    long long vcycles = 0;        // V-cycles run since the current solve started
    // captured preconditioner applications, one per (v, z, w, energy, link) set
    struct PGraph {
        const double* v;
        const double* z;
        const double* w;
        bool energy, link;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<PGraph> pgraphs;
    bool graph_broken = false;    // capture failed once: launch eagerly from then on
    // graphs are captured on and launched into a stream of the library's own
    // (the caller's stream may be the legacy default stream, which cannot be
    // captured), joined to the caller's stream by events before and after
    hipStream_t gst = nullptr;
    hipEvent_t gev0 = nullptr, gev1 = nullptr;
    bool mixed() const { return d.precision == TPH_MIXED; }
    bool ras() const { return d.smoother == TPH_SMOOTH_RAS || d.smoother == TPH_SMOOTH_RAS_MIXED; }
};

namespace {

Vec3 vec3(const tph_solver* s, double* raw) { return Vec3{raw + (kAlign - 1), s->F}; }

constexpr int kMaxTimedLaunches = 8192;

// Timing of one finest-level smoothing launch (only while timing is on): the
// launch receives a pair of events that take the kernel's own start and end
// time stamps (hipExtLaunchKernel), so no marker packet sits between kernels.
struct KTime {
    hipEvent_t t0 = nullptr, t1 = nullptr;
};

KTime ktic(tph_solver* s, int l, int kind = TPH_KERNEL_SMOOTH) {
    KTime k;
    if (!s->ktime || l != 0 || kind != s->ktarget) return k;
    if (s->kcount++ % s->kstride != 0) return k;    // every kstride-th finest-level launch
    if (s->kev_used + 2 > (int)s->kev.size()) {
        ++s->kdropped;
        return k;
    }
    k.t0 = s->kev[s->kev_used];
    k.t1 = s->kev[s->kev_used + 1];
    return k;
}

void ktoc(tph_solver* s, const KTime& k, double words, size_t wbytes) {
    if (!k.t0) return;
    s->kev_used += 2;
    s->kbytes += words * (double)s->lev[0].g.nx * (double)s->lev[0].g.ny * (double)wbytes;
}

// Algorithmic bytes per cell of one Uzawa link pass (uzawa_link_cell): the
// correction e (2 words of the V-cycle type), the pressure source, eta_b and
// eta_p, z_old (3 FP64 words) after the first step; writes z (3 FP64); then
// kLinkNext reads r (3 FP64) and writes the next right-hand side (2 words of
// the V-cycle type) and its pressure part, kLinkApply writes w (3 FP64).
double link_bytes_per_cell(int mode, bool acc, size_t tbytes) {
    double b = 2.0 * tbytes + 8.0 * (1 + 2) + (acc ? 24.0 : 0.0) + 24.0;
    if (mode == kLinkNext) b += 24.0 + 2.0 * tbytes + 8.0;
    else if (mode == kLinkApply) b += 24.0;
    return b;
}

tph_status dev_alloc(tph_solver* s, void** p, size_t bytes) {
    std::string what;
    const hipError_t e = s->mem.alloc(p, bytes, &what);
    if (e != hipSuccess) {
        set_error(what);
        return e == hipErrorOutOfMemory ? TPH_ERR_OOM : TPH_ERR_HIP;
    }
    TPH_HIP(hipMemsetAsync(*p, 0, bytes, s->st));
    return TPH_OK;
}

// one field of level geometry g in element type of `bytes_per`; returns base (entry (0,0))
tph_status alloc_field(tph_solver* s, const Geom& g, size_t bytes_per, void** base) {
    void* raw = nullptr;
    TPH_TRY(dev_alloc(s, &raw, field_alloc(g) * bytes_per));
    *base = (char*)raw + (kAlign - 1) * bytes_per;
    return TPH_OK;
}

int level_sweeps(int nu, double growth, int l) {
    const double v = std::ceil(nu * std::pow(growth, l) - 1e-9);
    return (int)std::min(v, 256.0);
}

// cells of the next coarser level along one axis for coarsening factor f: n / f
// rounded to the nearest integer (halves up), at least 2
int coarse_cells(int n, double f) {
    const int c = (int)std::floor(n / f + 0.5);
    return c < 2 ? 2 : c;
}

tph_status validate_desc(const tph_desc* d, int* nlev_out) {
    if (!d) { set_error("desc is NULL"); return TPH_ERR_INVALID; }
    if (d->nx < 2 || d->ny < 2) { set_error("nx and ny must be >= 2"); return TPH_ERR_INVALID; }
    if ((int64_t)(d->nx + 2) * (d->ny + 2) > (int64_t)1 << 30) { set_error("grid too large"); return TPH_ERR_INVALID; }
    if (!(d->lx > 0) || !(d->ly > 0) || !std::isfinite(d->lx) || !std::isfinite(d->ly)) {
        set_error("lx and ly must be positive and finite");
        return TPH_ERR_INVALID;
    }
    for (int w = 0; w < 4; ++w)
        if (d->bc[w] != TPH_FREE_SLIP && d->bc[w] != TPH_NO_SLIP) { set_error("bad boundary condition"); return TPH_ERR_INVALID; }
    if (d->precision != TPH_FP64 && d->precision != TPH_MIXED) { set_error("bad precision"); return TPH_ERR_INVALID; }
    if (d->smoother != TPH_SMOOTH_JACOBI && d->smoother != TPH_SMOOTH_GS && d->smoother != TPH_SMOOTH_RAS &&
        d->smoother != TPH_SMOOTH_RAS_MIXED) {
        set_error("bad smoother");
        return TPH_ERR_INVALID;
    }
    if (d->smoother == TPH_SMOOTH_RAS || d->smoother == TPH_SMOOTH_RAS_MIXED) {
        if (d->ras_tile != 8 && d->ras_tile != 16 && d->ras_tile != 32) { set_error("ras_tile must be 8, 16 or 32"); return TPH_ERR_INVALID; }
        if (d->ras_inner < 1 || d->ras_inner > 16) { set_error("ras_inner must be in [1, 16]"); return TPH_ERR_INVALID; }
    }
    if (d->eta_mean != TPH_MEAN_ARITHMETIC && d->eta_mean != TPH_MEAN_GEOMETRIC) { set_error("bad eta_mean"); return TPH_ERR_INVALID; }
    if (d->nu_pre < 0 || d->nu_post < 0 || d->nu_pre > 256 || d->nu_post > 256) { set_error("bad sweep counts"); return TPH_ERR_INVALID; }
    if (!(d->nu_growth >= 1.0) || d->nu_growth > 4.0) { set_error("nu_growth must be in [1, 4]"); return TPH_ERR_INVALID; }
    if (!(d->omega > 0.0) || d->omega > 2.0) { set_error("omega must be in (0, 2]"); return TPH_ERR_INVALID; }
    if (!(d->alpha > 0.0) || !std::isfinite(d->alpha)) { set_error("alpha must be positive"); return TPH_ERR_INVALID; }
    if (!(d->rtol > 0.0) || !(d->rtol < 1.0)) { set_error("rtol must be in (0, 1)"); return TPH_ERR_INVALID; }
    if (d->accel != TPH_ACCEL_FGMRES && d->accel != TPH_ACCEL_GCR && d->accel != TPH_ACCEL_ANDERSON) {
        set_error("accel must be TPH_ACCEL_FGMRES, TPH_ACCEL_GCR or TPH_ACCEL_ANDERSON");
        return TPH_ERR_INVALID;
    }
    if (d->accel == TPH_ACCEL_ANDERSON) {
        if (d->restart < 0 || d->restart > kMaxRestart) { set_error("Anderson depth (restart) must be in [0, 64]"); return TPH_ERR_INVALID; }
        if (!(d->beta > 0.0) || d->beta > 1.0) { set_error("beta must be in (0, 1]"); return TPH_ERR_INVALID; }
    } else if (d->restart < 1 || d->restart > kMaxRestart) {
        set_error("restart must be in [1, 64]");
        return TPH_ERR_INVALID;
    }
    if (d->max_iters < 1) { set_error("max_iters must be >= 1"); return TPH_ERR_INVALID; }
    if (d->uzawa_steps < 1 || d->uzawa_steps > 16) { set_error("uzawa_steps must be in [1, 16]"); return TPH_ERR_INVALID; }
    if (d->fused != 0 && d->fused != 1) { set_error("fused must be 0 or 1"); return TPH_ERR_INVALID; }
    if (d->msweep < -1 || d->tile_shape < -1) { set_error("msweep and tile_shape must be -1 or a level mask"); return TPH_ERR_INVALID; }
    if (d->graph != 0 && d->graph != 1) { set_error("graph must be 0 or 1"); return TPH_ERR_INVALID; }
    if (d->coarse_level < -2) { set_error("coarse_level must be -2, -1 or a level index"); return TPH_ERR_INVALID; }
    if (!(d->coarsen == 2.0 || (d->coarsen >= 1.25 && d->coarsen <= 4.0))) {
        set_error("coarsen must be 2 or in [1.25, 4]");
        return TPH_ERR_INVALID;
    }
    const bool general = d->coarsen != 2.0;
    if (general && d->fused) {
        set_error("coarsening factors other than 2 run with fused = 0 (the LDS-tiled kernels assume halving)");
        return TPH_ERR_INVALID;
    }
    int nlev = d->levels;
    if (nlev == 0) {
        nlev = 1;
        int nx = d->nx, ny = d->ny;
        if (general) {
            while (coarse_cells(nx, d->coarsen) >= 8 && coarse_cells(ny, d->coarsen) >= 8 && nlev < kMaxLevels) {
                nx = coarse_cells(nx, d->coarsen);
                ny = coarse_cells(ny, d->coarsen);
                ++nlev;
            }
        } else {
            while (nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= 8 && ny / 2 >= 8 && nlev < kMaxLevels) {
                nx /= 2;
                ny /= 2;
                ++nlev;
            }
        }
    }
    if (nlev < 1 || nlev > kMaxLevels) { set_error("levels must be in [1, 16]"); return TPH_ERR_INVALID; }
    int cx = d->nx, cy = d->ny;
    if (general) {
        for (int l = 1; l < nlev; ++l) {
            cx = coarse_cells(cx, d->coarsen);
            cy = coarse_cells(cy, d->coarsen);
        }
    } else {
        const int f = 1 << (nlev - 1);
        if (d->nx % f || d->ny % f) { set_error("nx and ny must be divisible by 2^(levels-1)"); return TPH_ERR_INVALID; }
        cx = d->nx / f;
        cy = d->ny / f;
    }
    if (cx < 2 || cy < 2) { set_error("coarsest level must have at least 2 x 2 cells"); return TPH_ERR_INVALID; }
    const int nc = cy * (cx - 1) + (cy - 1) * cx;
    if (nc > 4096) { set_error("coarsest level too large for the dense FP64 solve (max 4096 unknowns)"); return TPH_ERR_INVALID; }
    if (d->coarse_level >= 0) {
        const int l = d->coarse_level;
        if (l >= nlev - 1 || (int64_t)(d->nx >> l) * (d->ny >> l) > 64 * 64) {
            set_error("coarse_level " + std::to_string(l) + " is not a level of at most 64 x 64 cells above the coarsest");
            return TPH_ERR_INVALID;
        }
    }
    *nlev_out = nlev;
    return TPH_OK;
}

template <typename T>
T* as(void* p) { return (T*)p; }

// ------------------------------------------------------- RAS smoothing
// Output k (0-based) of SplitMix64 started from `state` (Steele, Lea and
// Flood, 2014): the RAS tile shifts are draws of it.
uint64_t splitmix64(uint64_t state, uint64_t k) {
    uint64_t z = state + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint64_t kRasMaxOuter = 256;

bool ras_level(const tph_solver* s, int l) {
    return s->d.smoother == TPH_SMOOTH_RAS || (s->d.smoother == TPH_SMOOTH_RAS_MIXED && l > 0);
}

// nu sweeps of the RAS-type temporal-blocking smoother on level l:
// ceil(nu / ras_inner) outer iterations, one launch each, with shifts drawn
// for (V-cycle of this preconditioner application, level, leg, outer, axis);
// from_zero: the first launch starts from e = 0 and writes buffer 0.
template <typename T>
tph_status ras_smooth(tph_solver* s, int l, int nu, bool from_zero, int leg, int* cur) {
    LevelBuf& L = s->lev[l];
    const int TT = s->d.ras_tile, inner = s->d.ras_inner;
    const int nout = (nu + inner - 1) / inner;
    for (int t = 0; t < nout; ++t) {
        const uint64_t key = ((((uint64_t)s->vc_cycle * kMaxLevels + (uint64_t)l) * 2 + (uint64_t)leg) * kRasMaxOuter +
                              (uint64_t)t) * 2;
        const int si = (int)(splitmix64(s->d.seed, key) % (uint64_t)TT);
        const int sj = (int)(splitmix64(s->d.seed, key + 1) % (uint64_t)TT);
        const bool z = from_zero && t == 0;
        const int out = z ? 0 : 1 - *cur;
        const KTime tk = ktic(s, l);
        TPH_HIP(launch_ras_tile<T>(L.g, TT, si, sj, inner, z, z ? nullptr : as<T>(L.ex[*cur]),
                                   z ? nullptr : as<T>(L.ey[*cur]), as<T>(L.ex[out]), as<T>(L.ey[out]), as<T>(L.rx),
                                   as<T>(L.ry), as<T>(L.eb), as<T>(L.ep), (T)s->d.omega, s->st));
        ktoc(s, tk, z ? 6.0 : 8.0, sizeof(T));
        *cur = out;
    }
    return TPH_OK;
}

// ----------------------------------------------------------------- V-cycle
template <typename T>
tph_status vcycle(tph_solver* s, int l, int* cur_out) {
    LevelBuf& L = s->lev[l];
    const Geom& g = L.g;
    hipStream_t st = s->st;
    T* eb = as<T>(L.eb);
    T* ep = as<T>(L.ep);
    T* rx = as<T>(L.rx);
    T* ry = as<T>(L.ry);
    const T om = (T)s->d.omega;
    if (l == s->nlev - 1) {
        TPH_HIP(launch_coarse_solve<T>(g, s->Minv, rx, ry, as<T>(L.ex[0]), as<T>(L.ey[0]), st));
        *cur_out = 0;
        return TPH_OK;
    }
    int cur = 0;
    const bool jac = s->d.smoother != TPH_SMOOTH_GS;     // RAS_MIXED: Jacobi on the finest level
    const bool ras = ras_level(s, l);
    auto sweeps = [&](int nu, bool from_zero) -> tph_status {
        if (ras) return ras_smooth<T>(s, l, nu, from_zero, from_zero ? 0 : 1, &cur);
        for (int k = 0; k < nu; ++k) {
            const bool z = from_zero && k == 0;
            if (jac) {
                const int out = z ? 0 : 1 - cur;
                TPH_HIP(launch_jacobi<T>(g, z ? nullptr : as<T>(L.ex[cur]), z ? nullptr : as<T>(L.ey[cur]),
                                         as<T>(L.ex[out]), as<T>(L.ey[out]), rx, ry, eb, ep, om, st));
                cur = out;
            } else {
                T* ex = as<T>(L.ex[cur]);
                T* ey = as<T>(L.ey[cur]);
                TPH_HIP(launch_gs_half<T>(g, 0, 0, ex, ey, rx, ry, eb, ep, om, z, st));
                TPH_HIP(launch_gs_half<T>(g, 0, 1, ex, ey, rx, ry, eb, ep, om, false, st));
                TPH_HIP(launch_gs_half<T>(g, 1, 0, ex, ey, rx, ry, eb, ep, om, false, st));
                TPH_HIP(launch_gs_half<T>(g, 1, 1, ex, ey, rx, ry, eb, ep, om, false, st));
            }
        }
        return TPH_OK;
    };
    if (L.nu_pre == 0) {
        TPH_HIP(launch_zero_vel<T>(g, as<T>(L.ex[0]), as<T>(L.ey[0]), st));
        cur = 0;
    } else {
        TPH_TRY(sweeps(L.nu_pre, true));
    }
    TPH_HIP(launch_vel_residual<T>(g, as<T>(L.ex[cur]), as<T>(L.ey[cur]), rx, ry, eb, ep, as<T>(L.tx),
                                   as<T>(L.ty), st));
    LevelBuf& C = s->lev[l + 1];
    TPH_HIP(launch_restrict_res<T>(g, C.g, as<T>(L.tx), as<T>(L.ty), as<T>(C.rx), as<T>(C.ry), st));
    int ccur = 0;
    TPH_TRY(vcycle<T>(s, l + 1, &ccur));
    TPH_HIP(launch_prolong_add<T>(g, C.g, as<T>(C.ex[ccur]), as<T>(C.ey[ccur]), as<T>(L.ex[cur]), as<T>(L.ey[cur]),
                                  st));
    TPH_TRY(sweeps(L.nu_post, false));
    *cur_out = cur;
    return TPH_OK;
}

template <typename T>
tph_status vcycle_fused(tph_solver* s, int l, int* cur_out);

// One level of the fused V-cycle in multi-sweep passes: pre-smoothing from
// zero in passes of up to two Gauss-Seidel sweeps, the last one also forming
// the residual and restricting it to the next level; after the coarse
// correction, post-smoothing in passes of up to two sweeps, the first one
// applying the prolongation.  Same sweeps, same result as the one-sweep
// launches; fewer launches and one read of r and eta per pass.
template <typename T>
tph_status vcycle_msweep(tph_solver* s, int l, int* cur_out) {
    LevelBuf& L = s->lev[l];
    LevelBuf& C = s->lev[l + 1];
    const Geom& g = L.g;
    hipStream_t st = s->st;
    T* eb = as<T>(L.eb);
    T* ep = as<T>(L.ep);
    T* rx = as<T>(L.rx);
    T* ry = as<T>(L.ry);
    const T om = (T)s->d.omega;
    const int shape = (int)((s->shape_mask >> l) & 1u);
    int cur = 0;
    int mode = kTileZero;
    for (int left = L.nu_pre; left > 0;) {
        const int ns = left >= 2 ? 2 : 1;
        const int rr = left == ns ? 1 : 0;
        const bool zero = mode == kTileZero;
        const int dst = zero ? 0 : 1 - cur;
        const KTime tk = ktic(s, l);
        TPH_HIP(launch_gs_tile<T>(g, C.g, ns, mode, rr, shape, zero ? nullptr : as<T>(L.ex[cur]),
                                  zero ? nullptr : as<T>(L.ey[cur]), as<T>(L.ex[dst]), as<T>(L.ey[dst]), rx, ry, eb, ep,
                                  nullptr, nullptr, rr ? as<T>(C.rx) : nullptr, rr ? as<T>(C.ry) : nullptr, om, st,
                                  tk.t0, tk.t1));
        ktoc(s, tk, (zero ? 6.0 : 8.0) + (rr ? 0.5 : 0.0), sizeof(T));
        cur = dst;
        mode = kTilePlain;
        left -= ns;
    }
    int ccur = 0;
    TPH_TRY(vcycle_fused<T>(s, l + 1, &ccur));
    mode = kTileProlong;
    for (int left = L.nu_post; left > 0;) {
        const int ns = left >= 2 ? 2 : 1;
        const bool pro = mode == kTileProlong;
        const KTime tk = ktic(s, l);
        TPH_HIP(launch_gs_tile<T>(g, C.g, ns, mode, 0, shape, as<T>(L.ex[cur]), as<T>(L.ey[cur]), as<T>(L.ex[1 - cur]),
                                  as<T>(L.ey[1 - cur]), rx, ry, eb, ep, pro ? as<T>(C.ex[ccur]) : nullptr,
                                  pro ? as<T>(C.ey[ccur]) : nullptr, nullptr, nullptr, om, st, tk.t0, tk.t1));
        ktoc(s, tk, pro ? 8.5 : 8.0, sizeof(T));
        cur = 1 - cur;
        mode = kTilePlain;
        left -= ns;
    }
    *cur_out = cur;
    return TPH_OK;
}


// V-cycle with the fused kernels: LDS-tiled smoothing sweeps (first one
// from zero, first post-sweep with the prolongation fused in), fused
// residual + restriction, and the coarse tail in one workgroup.
template <typename T>
tph_status vcycle_fused(tph_solver* s, int l, int* cur_out) {
    LevelBuf& L = s->lev[l];
    const Geom& g = L.g;
    hipStream_t st = s->st;
    T* eb = as<T>(L.eb);
    T* ep = as<T>(L.ep);
    T* rx = as<T>(L.rx);
    T* ry = as<T>(L.ry);
    const T om = (T)s->d.omega;
    const int sm = s->d.smoother;
    if (l == s->lc) {
        CoarseArgs<T> a{};
        a.nl = s->nlev - l;
        a.nc = s->ncoarse;
        a.smoother = sm;
        a.omega = om;
        for (int q = 0; q < a.nl; ++q) {
            const LevelBuf& Q = s->lev[l + q];
            a.g[q] = Q.g;
            a.eb[q] = as<T>(Q.eb);
            a.ep[q] = as<T>(Q.ep);
            a.nu_pre[q] = Q.nu_pre;
            a.nu_post[q] = Q.nu_post;
        }
        a.rx = rx;
        a.ry = ry;
        a.ex = as<T>(L.ex[0]);
        a.ey = as<T>(L.ey[0]);
        a.Minv = s->Minv;
        TPH_HIP(launch_coarse_cycle<T>(a, s->lc_lds, s->max_lds, st));
        *cur_out = 0;
        return TPH_OK;
    }
    if (l == s->nlev - 1) {
        TPH_HIP(launch_coarse_solve<T>(g, s->Minv, rx, ry, as<T>(L.ex[0]), as<T>(L.ey[0]), st));
        *cur_out = 0;
        return TPH_OK;
    }
    int cur = 0;
    if (((s->msw_mask >> l) & 1u) && L.nu_pre > 0 && L.nu_post > 0) return vcycle_msweep<T>(s, l, cur_out);
    if (ras_level(s, l)) {
        // RAS launches, fused residual + restriction, separate prolongation
        LevelBuf& C = s->lev[l + 1];
        if (L.nu_pre == 0) TPH_HIP(launch_zero_vel<T>(g, as<T>(L.ex[0]), as<T>(L.ey[0]), st));
        else TPH_TRY(ras_smooth<T>(s, l, L.nu_pre, true, 0, &cur));
        TPH_HIP(launch_res_restrict<T>(g, C.g, as<T>(L.ex[cur]), as<T>(L.ey[cur]), rx, ry, eb, ep, as<T>(C.rx),
                                       as<T>(C.ry), st));
        int ccur = 0;
        TPH_TRY(vcycle_fused<T>(s, l + 1, &ccur));
        TPH_HIP(launch_prolong_add<T>(g, C.g, as<T>(C.ex[ccur]), as<T>(C.ey[ccur]), as<T>(L.ex[cur]),
                                      as<T>(L.ey[cur]), st));
        TPH_TRY(ras_smooth<T>(s, l, L.nu_post, false, 1, &cur));
        *cur_out = cur;
        return TPH_OK;
    }
    if (L.nu_pre == 0) {
        TPH_HIP(launch_zero_vel<T>(g, as<T>(L.ex[0]), as<T>(L.ey[0]), st));
    } else {
        KTime tk = ktic(s, l);
        TPH_HIP(launch_smooth_tile<T>(g, nullptr, sm, 1, nullptr, nullptr, as<T>(L.ex[0]), as<T>(L.ey[0]), rx, ry, eb,
                                      ep, nullptr, nullptr, om, st, tk.t0, tk.t1));
        ktoc(s, tk, 6.0, sizeof(T));
        for (int k = 1; k < L.nu_pre; ++k) {
            tk = ktic(s, l);
            TPH_HIP(launch_smooth_tile<T>(g, nullptr, sm, 0, as<T>(L.ex[cur]), as<T>(L.ey[cur]), as<T>(L.ex[1 - cur]),
                                          as<T>(L.ey[1 - cur]), rx, ry, eb, ep, nullptr, nullptr, om, st,
                                          tk.t0, tk.t1));
            ktoc(s, tk, 8.0, sizeof(T));
            cur = 1 - cur;
        }
    }
    LevelBuf& C = s->lev[l + 1];
    TPH_HIP(launch_res_restrict<T>(g, C.g, as<T>(L.ex[cur]), as<T>(L.ey[cur]), rx, ry, eb, ep, as<T>(C.rx),
                                   as<T>(C.ry), st));
    int ccur = 0;
    TPH_TRY(vcycle_fused<T>(s, l + 1, &ccur));
    if (L.nu_post == 0) {
        TPH_HIP(launch_prolong_add<T>(g, C.g, as<T>(C.ex[ccur]), as<T>(C.ey[ccur]), as<T>(L.ex[cur]),
                                      as<T>(L.ey[cur]), st));
    } else {
        KTime tk = ktic(s, l);
        TPH_HIP(launch_smooth_tile<T>(g, &C.g, sm, 2, as<T>(L.ex[cur]), as<T>(L.ey[cur]), as<T>(L.ex[1 - cur]),
                                      as<T>(L.ey[1 - cur]), rx, ry, eb, ep, as<T>(C.ex[ccur]), as<T>(C.ey[ccur]), om,
                                      st, tk.t0, tk.t1));
        ktoc(s, tk, 8.5, sizeof(T));
        cur = 1 - cur;
        for (int k = 1; k < L.nu_post; ++k) {
            tk = ktic(s, l);
            TPH_HIP(launch_smooth_tile<T>(g, nullptr, sm, 0, as<T>(L.ex[cur]), as<T>(L.ey[cur]), as<T>(L.ex[1 - cur]),
                                          as<T>(L.ey[1 - cur]), rx, ry, eb, ep, nullptr, nullptr, om, st,
                                          tk.t0, tk.t1));
            ktoc(s, tk, 8.0, sizeof(T));
            cur = 1 - cur;
        }
    }
    *cur_out = cur;
    return TPH_OK;
}

// z = M^{-1} v applied uzawa_steps times as a stationary iteration from z = 0:
// step 1: z = M^{-1} r; step k: z += M^{-1} (r - A z).  `energy`: v holds
// W^(1/2) r (a Krylov basis vector).  With wraw (the Krylov apply inside
// FGMRES and GCR) or `link`, each step's exit is one link pass: the last one
// ends the step and, with wraw, also forms w = W^(1/2) A z there; the others
// form the next step's right-hand side.  z alternates between zraw and t1
// (the last step writes zraw), the pressure residual between t3 and t2.
// Without either, each step runs as separate residual / entry / V-cycle /
// exit kernels.
template <typename T>
tph_status precondition_t(tph_solver* s, double* vraw, double* zraw, bool energy, double* wraw, bool link) {
    LevelBuf& L = s->lev[0];
    const Vec3 v = vec3(s, vraw), z = vec3(s, zraw);
    const bool fused = s->d.fused == 1;
    const int S = s->d.uzawa_steps;
    if (wraw || link) {
        const Vec3 zb[2] = {z, vec3(s, s->t1)};
        double* tpb[2] = {vec3(s, s->t3).p(), vec3(s, s->t2).p()};
        TPH_HIP(launch_precond_in<T>(L.g, v, L.eb64, L.ep64, energy, as<T>(L.rx), as<T>(L.ry), s->st));
        for (int q = 0; q < S; ++q) {
            s->vc_cycle = q;
            int cur = 0;
            if (fused) TPH_TRY(vcycle_fused<T>(s, 0, &cur));
            else TPH_TRY(vcycle<T>(s, 0, &cur));
            LinkArgs<T> a{};
            a.ex = as<T>(L.ex[cur]);
            a.ey = as<T>(L.ey[cur]);
            a.zold = zb[(S - q) & 1];
            a.acc = q > 0 ? 1 : 0;
            a.srcp = q == 0 ? v.p() : tpb[(q - 1) & 1];
            a.src_scaled = (q == 0 && energy) ? 1 : 0;
            a.alpha = s->d.alpha;
            a.zout = zb[(S - 1 - q) & 1];
            a.r = v;
            a.r_scaled = energy ? 1 : 0;
            a.rx = as<T>(L.rx);
            a.ry = as<T>(L.ry);
            a.tp = tpb[q & 1];
            a.wout = wraw ? vec3(s, wraw) : Vec3{nullptr, 0};
            a.w_scaled = energy ? 1 : 0;
            const int mode = q < S - 1 ? kLinkNext : (wraw ? kLinkApply : kLinkStore);
            const KTime tk = ktic(s, 0, TPH_KERNEL_LINK);
            TPH_HIP(launch_uzawa_link<T>(L.g, a, mode, L.eb64, L.ep64, s->st, tk.t0, tk.t1));
            ktoc(s, tk, link_bytes_per_cell(mode, a.acc != 0, sizeof(T)), 1);
        }
        return TPH_OK;
    }
    for (int step = 0; step < S; ++step) {
        s->vc_cycle = step;
        Vec3 src = v;
        bool src_scaled = energy;
        if (step > 0) {
            // t = r - A z (FP64), with r unscaled on the fly from v
            const Vec3 t = vec3(s, s->t3);
            TPH_HIP(launch_outer_residual(L.g, z, &v, L.eb64, L.ep64, t, ResMode::kResidual, false, nullptr, nullptr,
                                          s->st, energy));
            src = t;
            src_scaled = false;
        }
        TPH_HIP(launch_precond_in<T>(L.g, src, L.eb64, L.ep64, src_scaled, as<T>(L.rx), as<T>(L.ry), s->st));
        int cur = 0;
        if (fused) TPH_TRY(vcycle_fused<T>(s, 0, &cur));
        else TPH_TRY(vcycle<T>(s, 0, &cur));
        TPH_HIP(launch_precond_out<T>(L.g, as<T>(L.ex[cur]), as<T>(L.ey[cur]), src, L.ep64, src_scaled, s->d.alpha, z,
                                      s->st, step > 0));
    }
    return TPH_OK;
}

tph_status precondition_eager(tph_solver* s, double* vraw, double* zraw, bool energy, double* wraw, bool link) {
    return s->mixed() ? precondition_t<float>(s, vraw, zraw, energy, wraw, link)
                      : precondition_t<double>(s, vraw, zraw, energy, wraw, link);
}

// One preconditioner application.  On the linked path (inside the
// accelerators) with desc.graph set, the ~10 launches per Uzawa step are
// captured on first use for each distinct (v, z, w) and replayed as one
// graph launch afterwards: every kernel argument is fixed per solver (the
// level buffers, the RAS shifts of step q, the coefficients live in device
// memory), so a replay launches exactly the kernels of the eager path.
// Kernel time stamps need per-launch events, so timed solves run eagerly.
tph_status precondition(tph_solver* s, double* vraw, double* zraw, bool energy, double* wraw = nullptr,
                        bool link = false) {
    s->vcycles += s->d.uzawa_steps;
    if (!s->d.graph || s->graph_broken || s->ktime || !(wraw || link))
        return precondition_eager(s, vraw, zraw, energy, wraw, link);
    const tph_solver::PGraph* hit = nullptr;
    for (const auto& pg : s->pgraphs)
        if (pg.v == vraw && pg.z == zraw && pg.w == wraw && pg.energy == energy && pg.link == link) hit = &pg;
    if (!hit) {
        if (!s->gst) {
            if (hipStreamCreateWithFlags(&s->gst, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->gev0, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s->gev1, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                s->graph_broken = true;
                return precondition_eager(s, vraw, zraw, energy, wraw, link);
            }
        }
        tph_solver::PGraph pg{vraw, zraw, wraw, energy, link, nullptr, nullptr};
        if (hipStreamBeginCapture(s->gst, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            s->graph_broken = true;
            return precondition_eager(s, vraw, zraw, energy, wraw, link);
        }
        hipStream_t user = s->st;
        s->st = s->gst;                          // every launcher enqueues on s->st
        const tph_status st = precondition_eager(s, vraw, zraw, energy, wraw, link);
        s->st = user;
        const hipError_t e = hipStreamEndCapture(s->gst, &pg.graph);
        if (st != TPH_OK || e != hipSuccess || !pg.graph ||
            hipGraphInstantiate(&pg.exec, pg.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (pg.graph) (void)hipGraphDestroy(pg.graph);
            s->graph_broken = true;
            if (st != TPH_OK) return st;
            return precondition_eager(s, vraw, zraw, energy, wraw, link);
        }
        s->pgraphs.push_back(pg);
        hit = &s->pgraphs.back();
    }
    TPH_HIP(hipEventRecord(s->gev0, s->st));
    TPH_HIP(hipStreamWaitEvent(s->gst, s->gev0, 0));
    TPH_HIP(hipGraphLaunch(hit->exec, s->gst));
    TPH_HIP(hipEventRecord(s->gev1, s->gst));
    TPH_HIP(hipStreamWaitEvent(s->st, s->gev1, 0));
    return TPH_OK;
}

// reduce partial rows into `k` device scalars at slot; with to_host the same
// kernel also writes them into the mapped host mirror (no copy launch).  A
// reduction with `signal` (k == 1) ends the values the host is about to read:
// it also posts the next sequence number, which wait_signal() polls.
tph_status reduce_to(tph_solver* s, int nblk, int k, int slot, bool to_host = false, bool signal = false) {
    TPH_HIP(launch_reduce_rows(s->partial, nblk, k, s->dscal + slot, s->st, to_host ? s->hscal_dev + slot : nullptr,
                               signal ? s->hseq_dev : nullptr, signal ? ++s->seq : 0u));
    return TPH_OK;
}

// Wait until the last signalling reduction has posted its sequence number.
// Polling the mapped word avoids the wake-up latency of a stream
// synchronisation; past ~2 s of polling (a stalled device) it falls back to
// hipStreamSynchronize, which also reports any device error.
tph_status wait_signal(tph_solver* s) {
    const volatile unsigned* flag = s->hseq;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0; *flag != s->seq; ++spin) {
        if ((spin & 1023u) == 1023u &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2000)) {
            TPH_HIP(hipStreamSynchronize(s->st));
            if (*flag != s->seq) {
                set_error("reduction signal not observed after the stream completed");
                return TPH_ERR_HIP;
            }
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return TPH_OK;
}

tph_status fetch(tph_solver* s, int slot, int k) {
    TPH_HIP(hipMemcpyAsync(s->hscal + slot, s->dscal + slot, k * sizeof(double), hipMemcpyDeviceToHost, s->st));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

// ||W^(1/2) (b - A x)||^2 into dscal[slot]; out receives the scaled residual
tph_status energy_residual_vec(tph_solver* s, double* xraw, double* braw, double* outraw, int slot,
                               bool to_host = false) {
    const LevelBuf& L = s->lev[0];
    int nblk = 0;
    Vec3 b = vec3(s, braw);
    TPH_HIP(launch_outer_residual(L.g, vec3(s, xraw), &b, L.eb64, L.ep64, vec3(s, outraw), ResMode::kResidual, true,
                                  s->partial, &nblk, s->st));
    return reduce_to(s, nblk, 1, slot, to_host, to_host);
}

// GCR's residual recurrence |r_new|^2 = |r|^2 - alpha^2 is replaced by the
// norm of the updated residual once it falls below this fraction of the
// |r|^2 it started from, the cycle's or that of the last such replacement
// (it holds about 1e4 times its rounding error there).
constexpr double kPythFloor = 1e-10;

// Rounding floor of the relative energy residual at iterate x: eps times the
// energy norm of the row magnitudes |b| + |A| |x|, over the energy norm of b.
// The FP64 residual b - A x cannot be resolved below roughly this value.
tph_status rounding_floor(tph_solver* s, double* xraw, double* braw, double bnorm, double* out) {
    const LevelBuf& L = s->lev[0];
    int nblk = 0;
    TPH_HIP(launch_residual_magnitude(L.g, vec3(s, xraw), vec3(s, braw), L.eb64, L.ep64, s->partial, &nblk, s->st));
    TPH_TRY(reduce_to(s, nblk, 1, kSlotMisc + 4, true, true));
    TPH_TRY(wait_signal(s));
    *out = 2.220446049250313e-16 * std::sqrt(s->hscal[kSlotMisc + 4]) / (bnorm > 0.0 ? bnorm : 1.0);
    return TPH_OK;
}

// A residual that has not fallen by 10% over three restarts is taken as
// stagnation only within this factor of the rounding floor; above it the
// solve keeps going (slow convergence is not a floor).
constexpr double kFloorMargin = 100.0;

tph_status copy_in(tph_solver* s, const Geom& g, double* base, const double* user) {
    const size_t w = (size_t)(g.nx + 2) * sizeof(double);
    TPH_HIP(hipMemcpy2DAsync(base, (size_t)g.pitch * sizeof(double), user, w, w, g.ny + 2, hipMemcpyDeviceToDevice,
                             s->st));
    return TPH_OK;
}

tph_status copy_out(tph_solver* s, const Geom& g, double* user, const double* base) {
    const size_t w = (size_t)(g.nx + 2) * sizeof(double);
    TPH_HIP(hipMemcpy2DAsync(user, w, base, (size_t)g.pitch * sizeof(double), w, g.ny + 2, hipMemcpyDeviceToDevice,
                             s->st));
    return TPH_OK;
}

tph_status load_solution(tph_solver* s, double* raw, const double* vx, const double* vy, const double* p) {
    const Geom& g = s->lev[0].g;
    Vec3 x = vec3(s, raw);
    if (vx) TPH_TRY(copy_in(s, g, x.vx(), vx)); else TPH_HIP(hipMemsetAsync(raw, 0, s->F * sizeof(double), s->st));
    if (vy) TPH_TRY(copy_in(s, g, x.vy(), vy)); else TPH_HIP(hipMemsetAsync(raw + s->F, 0, s->F * sizeof(double), s->st));
    if (p) TPH_TRY(copy_in(s, g, x.p(), p)); else TPH_HIP(hipMemsetAsync(raw + 2 * s->F, 0, s->F * sizeof(double), s->st));
    TPH_HIP(launch_fill_bc<double>(g, x.vx(), x.vy(), s->st));
    return TPH_OK;
}

tph_status store_solution(tph_solver* s, const double* raw, double* vx, double* vy, double* p) {
    const Geom& g = s->lev[0].g;
    Vec3 x = vec3(s, (double*)raw);
    if (vx) TPH_TRY(copy_out(s, g, vx, x.vx()));
    if (vy) TPH_TRY(copy_out(s, g, vy, x.vy()));
    if (p) TPH_TRY(copy_out(s, g, p, x.p()));
    return TPH_OK;
}

// p -= mean(p) over the cells
tph_status remove_pressure_mean(tph_solver* s, double* raw) {
    const Geom& g = s->lev[0].g;
    Vec3 x = vec3(s, raw);
    int nblk = 0;
    TPH_HIP(launch_p_sum(g, x.p(), s->partial, &nblk, s->st));
    TPH_TRY(reduce_to(s, nblk, 1, kSlotMisc + 1));
    TPH_HIP(launch_p_shift(g, x.p(), s->dscal + kSlotMisc + 1, s->st));
    return TPH_OK;
}

// --------------------------------------------------------------- FGMRES
tph_status fgmres(tph_solver* s, double* braw, tph_info* info) {
    const int m = s->d.restart;
    const size_t n3 = s->n3;
    const int nblk_flat = flat_blocks(n3);
    auto Vk = [&](int k) { return s->V + (size_t)k * n3; };
    auto Zk = [&](int k) { return s->Z + (size_t)k * n3; };
    const auto t0 = std::chrono::steady_clock::now();

    // ||W^(1/2) b||: residual of x = 0
    {
        TPH_HIP(hipMemsetAsync(s->t2, 0, n3 * sizeof(double), s->st));
        TPH_TRY(energy_residual_vec(s, s->t2, braw, s->t1, kSlotMisc, true));
        TPH_TRY(wait_signal(s));
    }
    const double bnorm = std::sqrt(s->hscal[kSlotMisc]);
    if (!std::isfinite(bnorm)) { set_error("right-hand side is not finite"); return TPH_ERR_NONFINITE; }

    int its = 0, restarts = 0;
    double est = 0.0, true_res = 0.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
    tph_status result = TPH_NOT_CONVERGED;
    // stagnation guard: below the FP64 rounding floor of b - A x the true
    // residual stops decreasing; give up after three restarts without a 10% gain
    double best_true = HUGE_VAL;
    int stalled = 0;
    bool stagnated = false;
    while (true) {
        // true residual r = W^(1/2) (b - A x) into V_0
        TPH_TRY(energy_residual_vec(s, s->x, braw, Vk(0), kSlotMisc, true));
        TPH_TRY(wait_signal(s));
        const double beta = std::sqrt(s->hscal[kSlotMisc]);
        if (!std::isfinite(beta)) { set_error("non-finite residual during the solve"); return TPH_ERR_NONFINITE; }
        true_res = bnorm > 0 ? beta / bnorm : beta;
        if (bnorm == 0.0 || true_res <= s->d.rtol) { result = TPH_OK; break; }
        if (its >= s->d.max_iters) break;
        if (true_res > 0.9 * best_true) {
            if (++stalled >= 3) {
                double floor_ = 0.0;
                TPH_TRY(rounding_floor(s, s->x, braw, bnorm, &floor_));
                if (true_res <= kFloorMargin * floor_) { stagnated = true; break; }
                stalled = 0;
            }
        } else {
            stalled = 0;
        }
        best_true = std::min(best_true, true_res);
        ++restarts;
        TPH_HIP(launch_scale_by_rnorm(Vk(0), Vk(0), n3, s->dscal + kSlotMisc, s->st));
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            // z_j = M^{-1} v_j and w = W^(1/2) A z_j (the apply fused into the last Uzawa step's exit)
            TPH_TRY(precondition(s, Vk(j), Zk(j), true, Vk(j + 1)));
            double* w = Vk(j + 1);
            // classical Gram-Schmidt with selective re-orthogonalisation: one
            // projection pass, and a second only when the norm drops below
            // 1/sqrt(2) of its value before the projection (cancellation)
            TPH_HIP(launch_multidot(Vk(0), n3, j + 1, w, n3, s->partial, nblk_flat, s->st, j + 1));
            TPH_TRY(reduce_to(s, nblk_flat, j + 2, kSlotH1, true));  // h (j+1) and |w|^2 at kSlotH1 + j + 1
            TPH_HIP(launch_axpy_dot(w, Vk(0), n3, j + 1, s->dscal + kSlotH1, n3, false, 0, s->partial, nblk_flat,
                                    s->st));
            TPH_TRY(reduce_to(s, nblk_flat, 1, kSlotNrm, true, true));
            TPH_TRY(wait_signal(s));
            double* col = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = s->hscal[kSlotH1 + i];
            const double w2_before = s->hscal[kSlotH1 + j + 1];
            if (s->hscal[kSlotNrm] < 0.5 * w2_before) {
                TPH_HIP(launch_multidot(Vk(0), n3, j + 1, w, n3, s->partial, nblk_flat, s->st));
                TPH_TRY(reduce_to(s, nblk_flat, j + 1, kSlotH2, true));
                TPH_HIP(launch_axpy_dot(w, Vk(0), n3, j + 1, s->dscal + kSlotH2, n3, false, 0, s->partial, nblk_flat,
                                        s->st));
                TPH_TRY(reduce_to(s, nblk_flat, 1, kSlotNrm, true, true));
                TPH_TRY(wait_signal(s));
                for (int i = 0; i <= j; ++i) col[i] += s->hscal[kSlotH2 + i];
                ++s->reorth_count;
            }
            TPH_HIP(launch_scale_by_rnorm(w, w, n3, s->dscal + kSlotNrm, s->st));
            const double hn = std::sqrt(s->hscal[kSlotNrm]);
            col[j + 1] = hn;
            if (!std::isfinite(hn)) { set_error("non-finite value in the Krylov basis"); return TPH_ERR_NONFINITE; }
            for (int i = 0; i < j; ++i) {
                const double a = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = a;
            }
            const double rr = std::hypot(col[j], col[j + 1]);
            cs[j] = rr > 0 ? col[j] / rr : 1.0;
            sn[j] = rr > 0 ? col[j + 1] / rr : 0.0;
            col[j] = rr;
            col[j + 1] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            est = std::fabs(gv[j + 1]) / bnorm;
            if (info && info->history && its < info->history_len) info->history[its] = est;
            ++its;
            jdone = j + 1;
            if (est <= s->d.rtol || its >= s->d.max_iters || hn == 0.0) break;
        }
        // y = R^{-1} g, x += Z y
        for (int i = jdone - 1; i >= 0; --i) {
            double t = gv[i];
            for (int k = i + 1; k < jdone; ++k) t -= H[(size_t)k * (m + 1) + i] * y[k];
            y[i] = t / H[(size_t)i * (m + 1) + i];
        }
        TPH_HIP(hipMemcpyAsync(s->dscal + kSlotY, y.data(), jdone * sizeof(double), hipMemcpyHostToDevice, s->st));
        TPH_HIP(launch_update_x(s->x, s->Z, n3, jdone, s->dscal + kSlotY, n3, s->st));
    }
    TPH_TRY(remove_pressure_mean(s, s->x));
    TPH_HIP(hipStreamSynchronize(s->st));
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iters = its;
        info->restarts = restarts;
        info->res_energy = true_res;
        info->res_estimate = its ? est : true_res;
        info->t_setup_ms = s->t_setup_ms;
        info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (result == TPH_NOT_CONVERGED)
        set_error(std::string(stagnated ? "FGMRES stagnated at the rounding floor of the residual" : "FGMRES reached max_iters") +
                  " with relative energy residual " + std::to_string(true_res));
    return result;
}

// ------------------------------------------------------------------ GCR
// Restarted flexible GCR(m) (Alg. "Flexible GCR(m)") in the energy inner
// product: r and the directions w = A z are stored scaled by W^(1/2), as the
// FGMRES basis.  V_0 holds r, V_{i+1} the normalised w_i, Z_i the raw
// preconditioned z_i.  The projected, normalised z'_i of the algorithm are
// the combinations z' = Z C with C upper triangular (C e_i = (e_i - sum_j
// h_j C e_j) / nu_i), so x += sum_i alpha_i z'_i is applied once per cycle as
// x += Z (C alpha): the same iterate, without rewriting z and x every step.  The Gram-Schmidt projection against the earlier w's is one classical
// pass whose coefficients come from one multi-dot, with the norm of the
// projected vector from Pythagoras.  Pythagoras' |w_perp|^2 = |w|^2 - |h|^2
// is off by about eps |w|^2, and one classical pass leaves w_perp out of
// orthogonality by about eps |w| / |w_perp|: both stay near 1e-13 relative
// while |w_perp|^2 >= kCgsTrust |w|^2, ample for an FP64 solve to 1e-8.
// Below that the projection is carried out explicitly and repeated once if
// it still cancels (|w_perp|^2 < |w|^2 / 2 after it), as for the FGMRES
// basis.  Normalising the pair, x += alpha z and r -= alpha w are one
// kernel.  alpha = <r, w_i> is taken from the same multi-dot, before the
// projection: r is orthogonal to the earlier w's, so both agree up to
// rounding.  |r|^2 then drops by alpha^2, which gives the convergence
// estimate without another reduction; each restart recomputes the true
// residual.
constexpr double kCgsTrust = 1e-6;

tph_status gcr(tph_solver* s, double* braw, tph_info* info) {
    const int m = s->d.restart;
    const size_t n3 = s->n3;
    const int nblk = flat_blocks(n3);
    auto Vk = [&](int k) { return s->V + (size_t)k * n3; };
    auto Zk = [&](int k) { return s->Z + (size_t)k * n3; };
    const auto t0 = std::chrono::steady_clock::now();
    {
        TPH_HIP(hipMemsetAsync(s->t2, 0, n3 * sizeof(double), s->st));
        TPH_TRY(energy_residual_vec(s, s->t2, braw, s->t1, kSlotMisc, true));
        TPH_TRY(wait_signal(s));
    }
    const double bnorm = std::sqrt(s->hscal[kSlotMisc]);
    if (!std::isfinite(bnorm)) { set_error("right-hand side is not finite"); return TPH_ERR_NONFINITE; }

    int its = 0, restarts = 0;
    double est = 0.0, true_res = 0.0;
    tph_status result = TPH_NOT_CONVERGED;
    double best_true = HUGE_VAL;
    int stalled = 0;
    bool stagnated = false;
    GcrStepArgs a{};
    std::vector<double> C((size_t)m * m), alph(m), ycoef(m);
    while (true) {
        TPH_TRY(energy_residual_vec(s, s->x, braw, Vk(0), kSlotMisc, true));
        TPH_TRY(wait_signal(s));
        const double beta = std::sqrt(s->hscal[kSlotMisc]);
        if (!std::isfinite(beta)) { set_error("non-finite residual during the solve"); return TPH_ERR_NONFINITE; }
        true_res = bnorm > 0 ? beta / bnorm : beta;
        if (bnorm == 0.0 || true_res <= s->d.rtol) { result = TPH_OK; break; }
        if (its >= s->d.max_iters) break;
        if (true_res > 0.9 * best_true) {
            if (++stalled >= 3) {
                double floor_ = 0.0;
                TPH_TRY(rounding_floor(s, s->x, braw, bnorm, &floor_));
                if (true_res <= kFloorMargin * floor_) { stagnated = true; break; }
                stalled = 0;
            }
        } else {
            stalled = 0;
        }
        best_true = std::min(best_true, true_res);
        ++restarts;
        double rho2 = beta * beta;
        double ref2 = rho2;            // |r|^2 of the last exact evaluation
        int done = 0;
        for (int i = 0; i < m; ++i) {
            double* w = Vk(i + 1);
            double* z = Zk(i);
            // z = M^{-1} r and w = W^(1/2) A z (the apply fused into the last Uzawa step's exit)
            TPH_TRY(precondition(s, Vk(0), z, true, w));
            // <r, w>, <w_j, w> (j < i) and |w|^2 in one pass
            TPH_HIP(launch_multidot(Vk(0), n3, i + 1, w, n3, s->partial, nblk, s->st, i + 1));
            TPH_TRY(reduce_to(s, nblk, i + 2, kSlotH1, true));
            TPH_HIP(launch_post_seq(s->hseq_dev, ++s->seq, s->st));
            TPH_TRY(wait_signal(s));
            const double c = s->hscal[kSlotH1];
            const double w2 = s->hscal[kSlotH1 + i + 1];
            double h2 = 0.0;
            for (int j = 0; j < i; ++j) {
                a.hw[j] = a.hz[j] = s->hscal[kSlotH1 + 1 + j];
                h2 += a.hz[j] * a.hz[j];
            }
            double nu2 = w2 - h2;
            a.orth_w = 1;
            if (i > 0 && !(nu2 >= kCgsTrust * w2)) {
                TPH_HIP(launch_axpy_dot(w, Vk(1), n3, i, s->dscal + kSlotH1 + 1, n3, false, 0, s->partial, nblk,
                                        s->st));
                TPH_TRY(reduce_to(s, nblk, 1, kSlotNrm, true, true));
                TPH_TRY(wait_signal(s));
                nu2 = s->hscal[kSlotNrm];
                if (nu2 < 0.5 * w2) {
                    TPH_HIP(launch_multidot(Vk(1), n3, i, w, n3, s->partial, nblk, s->st));
                    TPH_TRY(reduce_to(s, nblk, i, kSlotH2, true));
                    TPH_HIP(launch_axpy_dot(w, Vk(1), n3, i, s->dscal + kSlotH2, n3, false, 0, s->partial, nblk,
                                            s->st));
                    TPH_TRY(reduce_to(s, nblk, 1, kSlotNrm, true, true));
                    TPH_TRY(wait_signal(s));
                    for (int j = 0; j < i; ++j) a.hz[j] += s->hscal[kSlotH2 + j];
                    nu2 = s->hscal[kSlotNrm];
                    ++s->reorth_count;
                }
                a.orth_w = 0;   // w already projected; z takes the accumulated coefficients
            }
            if (!std::isfinite(nu2) || !std::isfinite(c)) {
                set_error("non-finite value in the GCR directions");
                return TPH_ERR_NONFINITE;
            }
            if (!(nu2 > 0.0)) break;   // the new direction adds nothing: restart
            const double nu = std::sqrt(nu2);
            // column i of C: (e_i - sum_j hz_j C e_j) / nu
            for (int k = 0; k <= i; ++k) {
                double t = k == i ? 1.0 : 0.0;
                for (int j = k; j < i; ++j) t -= a.hz[j] * C[(size_t)j * m + k];
                C[(size_t)i * m + k] = t / nu;
            }
            a.w = w;
            a.W0 = Vk(1);
            a.z = nullptr;             // z and x: once per cycle below
            a.Z0 = nullptr;
            a.x = nullptr;
            a.r = Vk(0);
            a.stride = n3;
            a.n = n3;
            a.i = i;
            a.inv_nu = 1.0 / nu;
            a.alpha = c / nu;
            TPH_HIP(launch_gcr_step(a, s->st));
            alph[i] = a.alpha;
            done = i + 1;
            rho2 = std::max(rho2 - a.alpha * a.alpha, 0.0);
            // rho2 carries a rounding error of a few eps times the |r|^2 it
            // started from (each step subtracts a term of nearly its own
            // size), so it cannot resolve |r| below about sqrt(eps) of that
            // start; once it falls to kPythFloor times it, the norm of the
            // updated residual r itself replaces it and becomes the new start
            // (the later steps subtract terms of the new, smaller size)
            if (rho2 <= kPythFloor * ref2) {
                TPH_HIP(launch_multidot(Vk(0), n3, 1, Vk(0), n3, s->partial, nblk, s->st));
                TPH_TRY(reduce_to(s, nblk, 1, kSlotMisc + 5, true, true));
                TPH_TRY(wait_signal(s));
                rho2 = s->hscal[kSlotMisc + 5];
                ref2 = rho2;
            }
            est = std::sqrt(rho2) / bnorm;
            if (info && info->history && its < info->history_len) info->history[its] = est;
            ++its;
            if (est <= s->d.rtol || its >= s->d.max_iters) break;
        }
        // x += Z (C alpha) over the directions of this cycle
        if (done > 0) {
            for (int k = 0; k < done; ++k) {
                double t = 0.0;
                for (int i = k; i < done; ++i) t += C[(size_t)i * m + k] * alph[i];
                ycoef[k] = t;
            }
            TPH_HIP(hipMemcpyAsync(s->dscal + kSlotY, ycoef.data(), done * sizeof(double), hipMemcpyHostToDevice,
                                   s->st));
            TPH_HIP(launch_update_x(s->x, s->Z, n3, done, s->dscal + kSlotY, n3, s->st));
        }
    }
    TPH_TRY(remove_pressure_mean(s, s->x));
    TPH_HIP(hipStreamSynchronize(s->st));
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iters = its;
        info->restarts = restarts;
        info->res_energy = true_res;
        info->res_estimate = its ? est : true_res;
        info->t_setup_ms = s->t_setup_ms;
        info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (result == TPH_NOT_CONVERGED)
        set_error(std::string(stagnated ? "GCR stagnated at the rounding floor of the residual" : "GCR reached max_iters") +
                  " with relative energy residual " + std::to_string(true_res));
    return result;
}

// ------------------------------------------------------------- Anderson
// alpha minimising |sum_i alpha_i f_i|_2 subject to sum_i alpha_i = 1, from
// the Gram matrix G (n x n, row-major) of the window f_0 .. f_{n-1}.
// Eliminating the constraint (alpha_{n-1} = 1 - sum of the others) leaves the
// normal equations N g = -q, N_ij = (f_i - f_l).(f_j - f_l),
// q_i = (f_i - f_l).f_l (l = n - 1), which are solved by Cholesky with
// diagonal pivoting; directions whose pivot falls below 1e-13 of the largest
// diagonal entry are dropped (a rank-deficient window), their coefficients
// left at zero.
void aa_coefficients(const std::vector<double>& G, int n, std::vector<double>& alpha) {
    alpha.assign(n, 0.0);
    alpha[n - 1] = 1.0;
    const int k = n - 1;
    if (k == 0) return;
    const int l = n - 1;
    std::vector<double> N((size_t)k * k), rhs(k);
    std::vector<int> perm(k);
    double dmax = 0.0;
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j < k; ++j)
            N[(size_t)i * k + j] = G[(size_t)i * n + j] - G[(size_t)i * n + l] - G[(size_t)l * n + j] + G[(size_t)l * n + l];
        rhs[i] = -(G[(size_t)i * n + l] - G[(size_t)l * n + l]);
        perm[i] = i;
        dmax = std::max(dmax, N[(size_t)i * k + i]);
    }
    if (!(dmax > 0.0)) return;
    int r = 0;
    for (; r < k; ++r) {
        int p = r;
        for (int t = r + 1; t < k; ++t)
            if (N[(size_t)t * k + t] > N[(size_t)p * k + p]) p = t;
        if (!(N[(size_t)p * k + p] > 1e-13 * dmax)) break;
        if (p != r) {
            for (int t = 0; t < k; ++t) std::swap(N[(size_t)r * k + t], N[(size_t)p * k + t]);
            for (int t = 0; t < k; ++t) std::swap(N[(size_t)t * k + r], N[(size_t)t * k + p]);
            std::swap(rhs[r], rhs[p]);
            std::swap(perm[r], perm[p]);
        }
        const double d = std::sqrt(N[(size_t)r * k + r]);
        N[(size_t)r * k + r] = d;
        for (int t = r + 1; t < k; ++t) N[(size_t)t * k + r] /= d;
        for (int t = r + 1; t < k; ++t)
            for (int u = r + 1; u <= t; ++u) {
                N[(size_t)t * k + u] -= N[(size_t)t * k + r] * N[(size_t)u * k + r];
                N[(size_t)u * k + t] = N[(size_t)t * k + u];
            }
    }
    // L y = rhs, L^T g = y on the leading r x r block
    std::vector<double> y(r);
    for (int i = 0; i < r; ++i) {
        double t = rhs[i];
        for (int j = 0; j < i; ++j) t -= N[(size_t)i * k + j] * y[j];
        y[i] = t / N[(size_t)i * k + i];
    }
    double sum = 0.0;
    for (int i = r - 1; i >= 0; --i) {
        double t = y[i];
        for (int j = i + 1; j < r; ++j) t -= N[(size_t)j * k + i] * y[j];
        y[i] = t / N[(size_t)i * k + i];
    }
    for (int i = 0; i < r; ++i) {
        alpha[perm[i]] = y[i];
        sum += y[i];
    }
    alpha[l] = 1.0 - sum;
}

// AA(m) with mixing beta (Alg. "Anderson Acceleration(m) with Mixing") on the
// Uzawa fixed-point map G(x) = x + M^{-1}(b - A x).  A ring of m + 1 slots
// holds the iterates x_i (V_0 .. V_m) and their corrections f_i = G(x_i) - x_i
// (Z_0 .. Z_m); iterate k lives in slot k mod (m + 1) and V_{m+1} takes the
// residual.  Per iteration, behind one host wait: the energy residual of x_k
// and its norm, f_k = M^{-1}(b - A x_k) through the link path, and the new
// row of the Gram matrix of the window (dot products over the unknowns).  The
// host then solves the constrained least-squares problem and one kernel
// forms x_{k+1} = sum_i alpha_i (x_i + beta f_i), which is the paper's
// (1 - beta) sum alpha_i x_i + beta sum alpha_i G(x_i).  The first step is
// x_1 = G(x_0).  When x_k has converged, the f_k computed alongside its
// residual is not used.
tph_status anderson(tph_solver* s, double* braw, tph_info* info) {
    const int m = s->d.restart;
    const int ns = m + 1;
    const double beta_mix = s->d.beta;
    const size_t n3 = s->n3;
    const Geom& g0 = s->lev[0].g;
    const int nblk_u = unknown_dot_blocks(g0);
    auto Xk = [&](long long k) { return s->V + (size_t)(k % ns) * n3; };
    auto Fk = [&](long long k) { return s->Z + (size_t)(k % ns) * n3; };
    double* R = s->V + (size_t)ns * n3;
    const auto t0 = std::chrono::steady_clock::now();
    {
        TPH_HIP(hipMemsetAsync(s->t2, 0, n3 * sizeof(double), s->st));
        TPH_TRY(energy_residual_vec(s, s->t2, braw, s->t1, kSlotMisc, true));
        TPH_TRY(wait_signal(s));
    }
    const double bnorm = std::sqrt(s->hscal[kSlotMisc]);
    if (!std::isfinite(bnorm)) { set_error("right-hand side is not finite"); return TPH_ERR_NONFINITE; }
    TPH_HIP(hipMemcpyAsync(Xk(0), s->x, n3 * sizeof(double), hipMemcpyDeviceToDevice, s->st));

    std::vector<double> gram((size_t)ns * ns, 0.0), Gw, alpha, cx, cf;
    std::vector<const double*> xs, fs;
    long long k = 0;
    double true_res = 0.0, best = HUGE_VAL;
    int stalled = 0;
    const int stall_limit = std::max(30, 3 * ns);
    bool stagnated = false;
    tph_status result = TPH_NOT_CONVERGED;
    while (true) {
        const int mk = (int)std::min<long long>(m, k);
        // residual of x_k and its norm
        {
            const LevelBuf& L = s->lev[0];
            int nblk = 0;
            Vec3 b = vec3(s, braw);
            TPH_HIP(launch_outer_residual(L.g, vec3(s, Xk(k)), &b, L.eb64, L.ep64, vec3(s, R), ResMode::kResidual,
                                          true, s->partial, &nblk, s->st));
            TPH_TRY(reduce_to(s, nblk, 1, kSlotMisc, true));
        }
        const bool more = k < s->d.max_iters;
        if (more) {
            TPH_TRY(precondition(s, R, Fk(k), true, nullptr, true));
            // f_k . f_i over the window (oldest first) and |f_k|^2
            fs.clear();
            for (long long i = k - mk; i < k; ++i) fs.push_back(Fk(i));
            TPH_HIP(launch_multidot_unknowns(g0, s->F, fs.data(), mk, Fk(k), s->partial, nblk_u, s->st, mk));
            TPH_TRY(reduce_to(s, nblk_u, mk + 1, kSlotH1, true));
        }
        TPH_HIP(launch_post_seq(s->hseq_dev, ++s->seq, s->st));
        TPH_TRY(wait_signal(s));
        const double rn = std::sqrt(s->hscal[kSlotMisc]);
        if (!std::isfinite(rn)) { set_error("non-finite residual during the solve"); return TPH_ERR_NONFINITE; }
        true_res = bnorm > 0 ? rn / bnorm : rn;
        if (k > 0 && info && info->history && k - 1 < info->history_len) info->history[k - 1] = true_res;
        if (bnorm == 0.0 || true_res <= s->d.rtol) { result = TPH_OK; break; }
        if (!more) break;
        if (true_res <= 0.9 * best) {
            best = true_res;
            stalled = 0;
        } else if (++stalled >= stall_limit) {
            double floor_ = 0.0;
            TPH_TRY(rounding_floor(s, Xk(k), braw, bnorm, &floor_));
            if (true_res <= kFloorMargin * floor_) {
                stagnated = true;
                break;
            }
            stalled = 0;
        }
        // Gram row of f_k, then the window's Gram matrix (oldest first)
        const int sk = (int)(k % ns);
        for (int c = 0; c < mk; ++c) {
            const int sc = (int)((k - mk + c) % ns);
            const double v = s->hscal[kSlotH1 + c];
            gram[(size_t)sk * ns + sc] = v;
            gram[(size_t)sc * ns + sk] = v;
        }
        gram[(size_t)sk * ns + sk] = s->hscal[kSlotH1 + mk];
        if (!std::isfinite(gram[(size_t)sk * ns + sk])) {
            set_error("non-finite value in the Anderson corrections");
            return TPH_ERR_NONFINITE;
        }
        const int n = mk + 1;
        if (k == 0) {
            alpha.assign(1, 1.0);
        } else {
            Gw.assign((size_t)n * n, 0.0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    Gw[(size_t)i * n + j] = gram[(size_t)((k - mk + i) % ns) * ns + (size_t)((k - mk + j) % ns)];
            aa_coefficients(Gw, n, alpha);
        }
        xs.clear();
        fs.clear();
        cx.assign(n, 0.0);
        cf.assign(n, 0.0);
        const double bm = k == 0 ? 1.0 : beta_mix;   // x_1 = G(x_0)
        for (int i = 0; i < n; ++i) {
            xs.push_back(Xk(k - mk + i));
            fs.push_back(Fk(k - mk + i));
            cx[i] = alpha[i];
            cf[i] = bm * alpha[i];
            if (!std::isfinite(alpha[i])) {
                set_error("non-finite Anderson coefficients");
                return TPH_ERR_NONFINITE;
            }
        }
        // the output slot is the oldest iterate's when the window is full: it comes first
        TPH_HIP(launch_mix(Xk(k + 1), xs.data(), cx.data(), fs.data(), cf.data(), n, n3, s->st));
        ++k;
    }
    TPH_HIP(hipMemcpyAsync(s->x, Xk(k), n3 * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    TPH_TRY(remove_pressure_mean(s, s->x));
    TPH_HIP(hipStreamSynchronize(s->st));
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iters = (int32_t)k;
        info->restarts = 0;
        info->res_energy = true_res;
        info->res_estimate = true_res;
        info->t_setup_ms = s->t_setup_ms;
        info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (result == TPH_NOT_CONVERGED)
        set_error(std::string(stagnated ? "Anderson acceleration stagnated at the rounding floor of the residual" : "Anderson acceleration reached max_iters") +
                  " with relative energy residual " + std::to_string(true_res));
    return result;
}

// plain relative l2 residual ||b - A x||_2 / ||b||_2 over every equation row
// (no energy weights; Sec. "Residual Norms" reports both): the two squared
// norms are reduced into the mapped host scalars, read after the stream has
// drained (plain_residual_read)
tph_status plain_residual_enqueue(tph_solver* s, double* xraw, double* braw) {
    const LevelBuf& L = s->lev[0];
    int nblk = 0;
    Vec3 b = vec3(s, braw);
    TPH_HIP(launch_outer_residual(L.g, vec3(s, xraw), &b, L.eb64, L.ep64, vec3(s, s->t1), ResMode::kResidual, false,
                                  s->partial, &nblk, s->st));
    TPH_TRY(reduce_to(s, nblk, 1, kSlotMisc + 2, true));
    TPH_HIP(hipMemsetAsync(s->t2, 0, s->n3 * sizeof(double), s->st));
    TPH_HIP(launch_outer_residual(L.g, vec3(s, s->t2), &b, L.eb64, L.ep64, vec3(s, s->t1), ResMode::kResidual, false,
                                  s->partial, &nblk, s->st));
    return reduce_to(s, nblk, 1, kSlotMisc + 3, true);
}

double plain_residual_read(const tph_solver* s) {
    const double rr = std::sqrt(s->hscal[kSlotMisc + 2]), bb = std::sqrt(s->hscal[kSlotMisc + 3]);
    return bb > 0.0 ? rr / bb : rr;
}

tph_status accelerate(tph_solver* s, double* braw, tph_info* info) {
    s->vcycles = 0;
    tph_status r;
    switch (s->d.accel) {
        case TPH_ACCEL_GCR: r = gcr(s, braw, info); break;
        case TPH_ACCEL_ANDERSON: r = anderson(s, braw, info); break;
        default: r = fgmres(s, braw, info); break;
    }
    if (r >= 0 && info) {
        info->vcycles = (int32_t)std::min<long long>(s->vcycles, INT32_MAX);
        const std::string msg = g_last_error;          // keep a not-converged message
        TPH_TRY(plain_residual_enqueue(s, s->x, braw));
        TPH_HIP(hipStreamSynchronize(s->st));
        info->res_l2 = plain_residual_read(s);
        g_last_error = msg;
    }
    return r;
}

tph_status require_ready(tph_solver* s) {
    if (!s) { set_error("solver is NULL"); return TPH_ERR_INVALID; }
    if (!s->ready) { set_error("tph_set_coefficients has not succeeded on this solver"); return TPH_ERR_INVALID; }
    return TPH_OK;
}

template <typename T>
tph_status alloc_level_t(tph_solver* s, LevelBuf& L, bool share64) {
    if (share64) {
        L.eb = L.eb64;
        L.ep = L.ep64;
    } else {
        TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.eb));
        TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.ep));
    }
    for (int k = 0; k < 2; ++k) {
        TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.ex[k]));
        TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.ey[k]));
    }
    TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.rx));
    TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.ry));
    TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.tx));
    TPH_TRY(alloc_field(s, L.g, sizeof(T), &L.ty));
    return TPH_OK;
}

tph_status create_impl(const tph_desc* desc, void* stream, tph_solver* s) {
    int nlev = 0;
    TPH_TRY(validate_desc(desc, &nlev));
    s->d = *desc;
    s->st = (hipStream_t)stream;
    s->nlev = nlev;
    for (int l = 0; l < nlev; ++l) {
        Geom& g = s->lev[l].g;
        if (desc->coarsen != 2.0) {
            g.nx = l == 0 ? desc->nx : coarse_cells(s->lev[l - 1].g.nx, desc->coarsen);
            g.ny = l == 0 ? desc->ny : coarse_cells(s->lev[l - 1].g.ny, desc->coarsen);
        } else {
            g.nx = desc->nx >> l;
            g.ny = desc->ny >> l;
        }
        g.pitch = pitch_for(g.nx);
        g.dx = desc->lx / g.nx;
        g.dy = desc->ly / g.ny;
        for (int w = 0; w < 4; ++w) g.mir[w] = desc->bc[w] == TPH_FREE_SLIP ? 1.0f : -1.0f;
        s->lev[l].nu_pre = level_sweeps(desc->nu_pre, desc->nu_growth, l);
        s->lev[l].nu_post = level_sweeps(desc->nu_post, desc->nu_growth, l);
        TPH_TRY(alloc_field(s, g, sizeof(double), (void**)&s->lev[l].eb64));
        TPH_TRY(alloc_field(s, g, sizeof(double), (void**)&s->lev[l].ep64));
        if (s->mixed()) TPH_TRY(alloc_level_t<float>(s, s->lev[l], false));
        else TPH_TRY(alloc_level_t<double>(s, s->lev[l], true));
    }
    const Geom& g0 = s->lev[0].g;
    s->F = field_alloc(g0);
    s->n3 = 3 * s->F;
    const size_t vb = s->n3 * sizeof(double);
    TPH_TRY(dev_alloc(s, (void**)&s->x, vb));
    TPH_TRY(dev_alloc(s, (void**)&s->b, vb));
    TPH_TRY(dev_alloc(s, (void**)&s->b2, vb));
    TPH_TRY(dev_alloc(s, (void**)&s->t1, vb));
    TPH_TRY(dev_alloc(s, (void**)&s->t2, vb));
    TPH_TRY(dev_alloc(s, (void**)&s->t3, vb));
    // FGMRES: m + 1 basis vectors, m preconditioned ones; GCR: r and m
    // directions w, m directions z; Anderson: m + 1 iterates and the residual,
    // m + 1 corrections
    TPH_TRY(dev_alloc(s, (void**)&s->V, vb * (desc->restart + 2)));
    TPH_TRY(dev_alloc(s, (void**)&s->Z, vb * (desc->restart + 1)));
    void* p = nullptr;
    TPH_TRY(alloc_field(s, g0, sizeof(double), &p)); s->rho = (double*)p;
    TPH_TRY(alloc_field(s, g0, sizeof(double), &p)); s->fxe = (double*)p;
    TPH_TRY(alloc_field(s, g0, sizeof(double), &p)); s->fye = (double*)p;
    for (int k = 0; k < 3; ++k) { TPH_TRY(alloc_field(s, g0, sizeof(double), &p)); s->gtmp[k] = (double*)p; }
    const int nb_cells = (int)(((g0.nx + 2 + kCellBX - 1) / kCellBX) * ((g0.ny + 2 + kCellBY - 1) / kCellBY));
    s->partial_len = (size_t)std::max(nb_cells * 2, (kMaxRestart + 2) * 2048);
    TPH_TRY(dev_alloc(s, (void**)&s->partial, s->partial_len * sizeof(double)));
    TPH_TRY(dev_alloc(s, (void**)&s->dscal, kScalars * sizeof(double)));
    s->ncoarse = coarse_unknowns(s->lev[nlev - 1].g);
    {
        int dev = 0, lim = 0;
        TPH_HIP(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lim > 0)
            s->max_lds = lim;
    }
    s->lc = -1;
    // the coarse tail smooths with Jacobi or Gauss-Seidel only: the RAS smoothers run level by level
    if (desc->fused && nlev >= 2 && s->ncoarse <= 2048 && desc->coarse_level != -2 && !s->ras()) {
        // a level qualifies when its tail fits in one workgroup's LDS (leaving
        // room for the kernel's static tables) and its per-sweep work suits one
        // workgroup (<= 64 x 64 cells); default: the finest such level
        const size_t budget = (size_t)std::min(s->max_lds, 160 * 1024) - 8 * 1024;
        auto fits = [&](int l, size_t* need_out) {
            Geom gs[kMaxLevels];
            for (int q = l; q < nlev; ++q) gs[q - l] = s->lev[q].g;
            const size_t need = s->mixed() ? coarse_cycle_lds_bytes<float>(gs, nlev - l, s->ncoarse)
                                           : coarse_cycle_lds_bytes<double>(gs, nlev - l, s->ncoarse);
            *need_out = need;
            return s->lev[l].g.nx * s->lev[l].g.ny <= 64 * 64 && need <= budget;
        };
        size_t need = 0;
        if (desc->coarse_level >= 0) {
            const int l = desc->coarse_level;
            if (l >= nlev - 1 || !fits(l, &need)) {
                set_error("coarse_level " + std::to_string(l) + " does not fit the single-workgroup coarse tail");
                return TPH_ERR_INVALID;
            }
            s->lc = l;
            s->lc_lds = need;
        } else {
            for (int l = 0; l < nlev - 1; ++l) {
                if (fits(l, &need)) {
                    s->lc = l;
                    s->lc_lds = need;
                    break;
                }
            }
        }
    }
    s->msw_mask = 0;
    s->shape_mask = 0;
    if (desc->fused && desc->smoother == TPH_SMOOTH_GS) {
        const unsigned all = nlev >= 32 ? ~0u : ((1u << nlev) - 1u);
        s->msw_mask = desc->msweep < 0 ? (all & ~1u) : ((unsigned)desc->msweep & all);
        if (desc->tile_shape >= 0) {
            s->shape_mask = (unsigned)desc->tile_shape & all;
        } else {
            for (int l = 0; l < nlev; ++l) {
                const Geom& g = s->lev[l].g;
                const int tw = 64, th = s->mixed() ? 16 : 8;
                const long tiles = (long)((g.nx + tw - 1) / tw) * ((g.ny + th - 1) / th);
                if (tiles < 512) s->shape_mask |= 1u << l;
            }
        }
    }
    TPH_TRY(dev_alloc(s, (void**)&s->Minv, (size_t)s->ncoarse * s->ncoarse * sizeof(double)));
    if (s->ncoarse <= kGJLds) {
        struct { double* m; int n; int pad; } tab{s->Minv, s->ncoarse, 0};
        TPH_TRY(dev_alloc(s, (void**)&s->gj_table, sizeof(tab)));
        TPH_HIP(hipMemcpyAsync(s->gj_table, &tab, sizeof(tab), hipMemcpyHostToDevice, s->st));
        TPH_HIP(hipStreamSynchronize(s->st));
    } else {
        TPH_TRY(dev_alloc(s, (void**)&s->gj_work, 2 * (size_t)s->ncoarse * sizeof(double)));
    }
    TPH_HIP(hipHostMalloc((void**)&s->hscal, kScalars * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    TPH_HIP(hipHostGetDevicePointer((void**)&s->hscal_dev, s->hscal, 0));
    TPH_HIP(hipHostMalloc((void**)&s->hseq, 64, hipHostMallocMapped | hipHostMallocCoherent));
    TPH_HIP(hipHostGetDevicePointer((void**)&s->hseq_dev, s->hseq, 0));
    *s->hseq = 0;
    s->seq = 0;
    TPH_HIP(hipEventCreate(&s->ev0));
    TPH_HIP(hipEventCreate(&s->ev1));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

// Back-to-back launches of one kernel between two events on the solver's stream.
template <typename T>
tph_status time_kernel_t(tph_solver* s, int kind, int reps, double* ms, double* bytes) {
    LevelBuf& L = s->lev[0];
    const Geom& g = L.g;
    hipStream_t st = s->st;
    const double cells = (double)g.nx * g.ny;
    const double W = sizeof(T);
    T* eb = as<T>(L.eb);
    T* ep = as<T>(L.ep);
    const T om = (T)s->d.omega;
    double words = 0.0;
    // Krylov / Anderson vector kernels: i = restart / 2 earlier GCR pairs; restart + 1 Anderson slots
    // (zero coefficients: the launches stream the same bytes whatever the values)
    const int gcr_i = std::min(s->d.restart / 2, s->d.restart - 1 < 0 ? 0 : s->d.restart - 1);
    const int mix_n = s->d.restart + 1;
    std::vector<const double*> mix_x(mix_n), mix_f(mix_n);
    std::vector<double> mix_c(mix_n, 0.0);
    for (int v = 0; v < mix_n; ++v) {
        mix_x[v] = s->V + (size_t)v * s->n3;
        mix_f[v] = s->Z + (size_t)v * s->n3;
    }
    auto one = [&](int r) -> tph_status {
        switch (kind) {
            case TPH_KERNEL_SMOOTH:
                if (ras_level(s, 0)) {
                    const int a = r & 1;
                    TPH_HIP(launch_ras_tile<T>(g, s->d.ras_tile, 0, 0, s->d.ras_inner, false, as<T>(L.ex[a]),
                                               as<T>(L.ey[a]), as<T>(L.ex[1 - a]), as<T>(L.ey[1 - a]), as<T>(L.rx),
                                               as<T>(L.ry), eb, ep, om, st));
                } else if (s->d.fused) {
                    const int a = r & 1;
                    TPH_HIP(launch_smooth_tile<T>(g, nullptr, s->d.smoother, 0, as<T>(L.ex[a]), as<T>(L.ey[a]),
                                                  as<T>(L.ex[1 - a]), as<T>(L.ey[1 - a]), as<T>(L.rx), as<T>(L.ry), eb,
                                                  ep, nullptr, nullptr, om, st));
                } else if (s->d.smoother == TPH_SMOOTH_JACOBI) {
                    const int a = r & 1;
                    TPH_HIP(launch_jacobi<T>(g, as<T>(L.ex[a]), as<T>(L.ey[a]), as<T>(L.ex[1 - a]), as<T>(L.ey[1 - a]),
                                             as<T>(L.rx), as<T>(L.ry), eb, ep, om, st));
                } else {
                    TPH_HIP(launch_gs_half<T>(g, (r >> 1) & 1, r & 1, as<T>(L.ex[0]), as<T>(L.ey[0]), as<T>(L.rx),
                                              as<T>(L.ry), eb, ep, om, false, st));
                }
                break;
            case TPH_KERNEL_APPLY:
                TPH_HIP(launch_outer_residual(g, vec3(s, s->Z), nullptr, L.eb64, L.ep64, vec3(s, s->t1),
                                              ResMode::kApply, true, nullptr, nullptr, st));
                break;
            case TPH_KERNEL_RESIDUAL:
                TPH_HIP(launch_vel_residual<T>(g, as<T>(L.ex[0]), as<T>(L.ey[0]), as<T>(L.rx), as<T>(L.ry), eb, ep,
                                               as<T>(L.tx), as<T>(L.ty), st));
                break;
            case TPH_KERNEL_GCR_STEP: {
                GcrStepArgs a{};
                const int i = gcr_i;
                a.w = s->V + (size_t)(i + 1) * s->n3;
                a.W0 = s->V + s->n3;
                a.z = nullptr;             // the step as the solve runs it: w and r
                a.Z0 = nullptr;
                a.x = nullptr;
                a.r = s->V;
                a.stride = s->n3;
                a.n = s->n3;
                a.i = i;
                a.orth_w = 1;
                a.inv_nu = 1.0;
                a.alpha = 0.0;
                TPH_HIP(launch_gcr_step(a, st));
                break;
            }
            case TPH_KERNEL_AA_MIX: {
                TPH_HIP(launch_mix(s->V + (size_t)(mix_n) * s->n3, mix_x.data(), mix_c.data(), mix_f.data(),
                                   mix_c.data(), mix_n, s->n3, st));
                break;
            }
            case TPH_KERNEL_RESTRICT:
                if (s->d.fused)
                    TPH_HIP(launch_res_restrict<T>(g, s->lev[1].g, as<T>(L.ex[0]), as<T>(L.ey[0]), as<T>(L.rx),
                                                   as<T>(L.ry), eb, ep, as<T>(s->lev[1].rx), as<T>(s->lev[1].ry), st));
                else
                    TPH_HIP(launch_restrict_res<T>(g, s->lev[1].g, as<T>(L.tx), as<T>(L.ty), as<T>(s->lev[1].rx),
                                                   as<T>(s->lev[1].ry), st));
                break;
            default:
                TPH_HIP(launch_prolong_add<T>(g, s->lev[1].g, as<T>(s->lev[1].ex[0]), as<T>(s->lev[1].ey[0]),
                                              as<T>(L.ex[0]), as<T>(L.ey[0]), st));
                break;
        }
        return TPH_OK;
    };
    switch (kind) {
        case TPH_KERNEL_SMOOTH:
            // Jacobi: read e (2), r (2), eta_b, eta_p; write e (2).  GS colour
            // half-sweep: read both velocities, eta_b, eta_p and half of one r;
            // write half of one component.
            // a fused sweep (either smoother) reads e, r, eta_b, eta_p and writes e
            // a RAS launch: read e, r, eta_b, eta_p once for ras_inner sweeps, write e
            words = (s->d.fused || s->d.smoother != TPH_SMOOTH_GS) ? 8.0 : 5.0;
            break;
        case TPH_KERNEL_APPLY: words = 8.0; break;          // read vx, vy, p, eta_b, eta_p; write 3
        case TPH_KERNEL_RESIDUAL: words = 8.0; break;       // read e (2), r (2), eta_b, eta_p; write t (2)
        case TPH_KERNEL_RESTRICT:                           // fused: read e, r, eta_b, eta_p, write 2 coarse (1/4)
            words = s->d.fused ? 6.5 : 2.5;                 // separate: read t (2), write 2 coarse
            break;
        case TPH_KERNEL_GCR_STEP:                           // read i earlier vectors; w, r read + written
            words = (gcr_i + 4.0) * (double)s->n3 / cells;
            break;
        case TPH_KERNEL_AA_MIX:                             // read 2n vectors, write 1 (+ re-read/write per chunk)
            words = (2.0 * mix_n + 1.0 + 2.0 * ((mix_n + kVecSetMax - 1) / kVecSetMax - 1)) * (double)s->n3 / cells;
            break;
        default: words = 5.0; break;                        // read 2 coarse (1/4), e (2); write e (2)
    }
    const bool fp64_kernel = kind == TPH_KERNEL_APPLY || kind == TPH_KERNEL_GCR_STEP || kind == TPH_KERNEL_AA_MIX;
    const double wbytes = fp64_kernel ? 8.0 : W;
    TPH_TRY(one(0));                                     // warm
    TPH_HIP(hipEventRecord(s->ev0, st));
    for (int r = 0; r < reps; ++r) TPH_TRY(one(r));
    TPH_HIP(hipEventRecord(s->ev1, st));
    TPH_HIP(hipEventSynchronize(s->ev1));
    float el = 0.f;
    TPH_HIP(hipEventElapsedTime(&el, s->ev0, s->ev1));
    if (ms) *ms = (double)el / reps;
    if (bytes) *bytes = words * wbytes * cells;
    return TPH_OK;
}

// Coefficient setup in two halves: enqueue every step on the solver's stream
// (the coarsest factorisation only with `factor`; a batch factors all its
// problems in one launch), then wait and check.  The validity counts are
// written by the reduction straight into the mapped host block.
tph_status setup_enqueue(tph_solver* s, const double* eta_b, const double* eta_p, const double* rho_b, double gx,
                         double gy, const double* fx_extra, const double* fy_extra, bool factor) {
    if (!s) { set_error("solver is NULL"); return TPH_ERR_INVALID; }
    if (!eta_b || !eta_p || !rho_b) { set_error("eta_b, eta_p and rho_b are required"); return TPH_ERR_INVALID; }
    if (!std::isfinite(gx) || !std::isfinite(gy)) { set_error("gravity must be finite"); return TPH_ERR_INVALID; }
    s->ready = false;
    const Geom& g0 = s->lev[0].g;
    TPH_HIP(hipEventRecord(s->ev0, s->st));
    TPH_TRY(copy_in(s, g0, s->lev[0].eb64, eta_b));
    TPH_TRY(copy_in(s, g0, s->lev[0].ep64, eta_p));
    TPH_TRY(copy_in(s, g0, s->rho, rho_b));
    s->has_fx = fx_extra != nullptr;
    s->has_fy = fy_extra != nullptr;
    if (fx_extra) TPH_TRY(copy_in(s, g0, s->fxe, fx_extra));
    if (fy_extra) TPH_TRY(copy_in(s, g0, s->fye, fy_extra));
    int nblk = 0;
    TPH_HIP(launch_check_coeffs(g0, s->lev[0].eb64, s->lev[0].ep64, s->rho, s->has_fx ? s->fxe : nullptr,
                                s->has_fy ? s->fye : nullptr, s->partial, &nblk, s->st));
    TPH_HIP(launch_reduce_rows(s->partial, nblk, 2, s->dscal + kSlotMisc + 2, s->st, s->hscal_dev + kSlotMisc + 2));
    s->gx = gx;
    s->gy = gy;
    TPH_HIP(launch_rhs(g0, s->rho, gx, gy, s->has_fx ? s->fxe : nullptr, s->has_fy ? s->fye : nullptr,
                       vec3(s, s->b), s->st));
    for (int l = 1; l < s->nlev; ++l)
        TPH_HIP(launch_restrict_eta(s->lev[l - 1].g, s->lev[l].g, s->lev[l - 1].eb64, s->lev[l - 1].ep64,
                                    s->lev[l].eb64, s->lev[l].ep64, s->d.eta_mean == TPH_MEAN_GEOMETRIC, s->st));
    if (s->mixed()) {
        CastList cl{};
        for (int l = 0; l < s->nlev; ++l) {
            const size_t n = field_alloc(s->lev[l].g);
            cl.src[cl.count] = s->lev[l].eb64 - (kAlign - 1);
            cl.dst[cl.count] = (float*)s->lev[l].eb - (kAlign - 1);
            cl.n[cl.count++] = n;
            cl.src[cl.count] = s->lev[l].ep64 - (kAlign - 1);
            cl.dst[cl.count] = (float*)s->lev[l].ep - (kAlign - 1);
            cl.n[cl.count++] = n;
        }
        TPH_HIP(launch_cast_list(cl, s->st));
    }
    const LevelBuf& C = s->lev[s->nlev - 1];
    TPH_HIP(launch_coarse_assemble(C.g, C.eb64, C.ep64, s->Minv, s->st));
    if (factor) TPH_HIP(launch_gauss_jordan(s->Minv, s->ncoarse, s->st, s->gj_table, s->gj_work));
    TPH_HIP(hipEventRecord(s->ev1, s->st));
    return TPH_OK;
}

tph_status setup_finish(tph_solver* s) {
    TPH_HIP(hipStreamSynchronize(s->st));
    float ms = 0.f;
    TPH_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->t_setup_ms = ms;
    if (s->hscal[kSlotMisc + 2] != 0.0) {
        set_error("viscosity must be finite and positive (" + std::to_string((long long)s->hscal[kSlotMisc + 2]) +
                  " bad entries)");
        return TPH_ERR_INVALID;
    }
    if (s->hscal[kSlotMisc + 3] != 0.0) { set_error("density or extra force is not finite"); return TPH_ERR_NONFINITE; }
    s->ready = true;
    return TPH_OK;
}

// Viscosity minimum of the caller's dense (ny+2) x (nx+2) fields (basic
// nodes and cells), returned on the host.
tph_status eta_min_dense(tph_solver* s, const double* eta_b, const double* eta_p, double* m) {
    Geom gd = s->lev[0].g;
    gd.pitch = gd.nx + 2;
    TPH_HIP(launch_eta_min(gd, eta_b, eta_p, s->partial, s->dscal + kSlotMisc + 4, s->st));
    TPH_TRY(fetch(s, kSlotMisc + 4, 1));
    *m = s->hscal[kSlotMisc + 4];
    return TPH_OK;
}

}  // namespace

// ============================================================ internal view
tph_status tph_internal_setup_enqueue(tph_solver* s, const double* eta_b, const double* eta_p, const double* rho_b,
                                      double gx, double gy) {
    return setup_enqueue(s, eta_b, eta_p, rho_b, gx, gy, nullptr, nullptr, false);
}

tph_status tph_internal_setup_finish(tph_solver* s) { return setup_finish(s); }

TphSolverView tph_internal_view(const tph_solver* s) {
    TphSolverView v{};
    v.nlev = s->nlev;
    v.lc = s->lc;
    v.lc_lds = s->lc_lds;
    v.ncoarse = s->ncoarse;
    for (int l = 0; l < s->nlev; ++l) {
        const LevelBuf& L = s->lev[l];
        v.g[l] = L.g;
        v.eb[l] = L.eb;
        v.ep[l] = L.ep;
        for (int k = 0; k < 2; ++k) {
            v.ex[l][k] = L.ex[k];
            v.ey[l][k] = L.ey[k];
        }
        v.rx[l] = L.rx;
        v.ry[l] = L.ry;
        v.nu_pre[l] = L.nu_pre;
        v.nu_post[l] = L.nu_post;
    }
    v.Minv = s->Minv;
    v.eb64 = s->lev[0].eb64;
    v.ep64 = s->lev[0].ep64;
    v.x = s->x;
    v.b = s->b;
    v.V = s->V;
    v.Z = s->Z;
    v.t1 = s->t1;
    v.t2 = s->t2;
    v.t3 = s->t3;
    v.F = s->F;
    v.n3 = s->n3;
    return v;
}

void tph_internal_set_error(const std::string& msg) { g_last_error = msg; }

tph_status tph_internal_load_solution(tph_solver* s, const double* vx, const double* vy, const double* p) {
    return load_solution(s, s->x, vx, vy, p);
}

tph_status tph_internal_rounding_floor(tph_solver* s, double bnorm, double* out) {
    return rounding_floor(s, s->x, s->b, bnorm, out);
}

tph_status tph_internal_plain_residual_enqueue(tph_solver* s) { return plain_residual_enqueue(s, s->x, s->b); }
double tph_internal_plain_residual_read(const tph_solver* s) { return plain_residual_read(s); }

tph_status tph_internal_finish_solution(tph_solver* s, double* vx, double* vy, double* p) {
    TPH_TRY(remove_pressure_mean(s, s->x));
    return store_solution(s, s->x, vx, vy, p);
}

// ====================================================================== C ABI
extern "C" {

void tph_desc_default(tph_desc* d, int32_t nx, int32_t ny) {
    if (!d) return;
    std::memset(d, 0, sizeof(*d));
    d->nx = nx;
    d->ny = ny;
    d->lx = 1.0;
    d->ly = 1.0;
    for (int w = 0; w < 4; ++w) d->bc[w] = TPH_FREE_SLIP;
    d->precision = TPH_MIXED;
    d->levels = 0;
    d->smoother = TPH_SMOOTH_GS;
    d->nu_pre = 2;
    d->nu_post = 2;
    d->nu_growth = 1.0;
    d->omega = 1.0;
    d->alpha = 1.0;
    d->eta_mean = TPH_MEAN_ARITHMETIC;
    d->rtol = 1e-8;
    d->restart = 20;
    d->accel = TPH_ACCEL_FGMRES;
    d->beta = 1.0;
    d->ras_tile = 32;
    d->ras_inner = 4;
    d->seed = 0;
    d->graph = 0;
    d->pad_ = 0;
    d->coarsen = 2.0;
    d->max_iters = 500;
    d->uzawa_steps = 2;
    d->fused = 1;
    d->msweep = -1;
    d->tile_shape = -1;
    d->coarse_level = -1;
}

tph_status tph_create(const tph_desc* desc, void* hip_stream, tph_solver** out) {
    g_last_error.clear();
    if (!out) { set_error("out is NULL"); return TPH_ERR_INVALID; }
    *out = nullptr;
    int nlev = 0;
    TPH_TRY(validate_desc(desc, &nlev));       // host-only checks before any HIP call
    tph_solver* s = new tph_solver();
    s->mem.a = default_allocator();
    const tph_status st = create_impl(desc, hip_stream, s);
    if (st != TPH_OK) {
        const std::string msg = g_last_error;
        tph_destroy(s);
        g_last_error = msg;
        return st;
    }
    *out = s;
    return TPH_OK;
}

tph_status tph_set_coefficients(tph_solver* s, const double* eta_b, const double* eta_p, const double* rho_b,
                                double gx, double gy, const double* fx_extra, const double* fy_extra) {
    g_last_error.clear();
    TPH_TRY(setup_enqueue(s, eta_b, eta_p, rho_b, gx, gy, fx_extra, fy_extra, true));
    return setup_finish(s);
}

tph_status tph_solve(tph_solver* s, double* vx, double* vy, double* p, tph_info* info) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!vx || !vy || !p) { set_error("vx, vy and p are required"); return TPH_ERR_INVALID; }
    TPH_TRY(load_solution(s, s->x, vx, vy, p));
    const tph_status r = accelerate(s, s->b, info);
    if (r < 0) return r;
    TPH_TRY(store_solution(s, s->x, vx, vy, p));
    TPH_HIP(hipStreamSynchronize(s->st));
    return r;
}

tph_status tph_lithostatic_pressure(tph_solver* s, const double* rho_b, double gy, double* p) {
    g_last_error.clear();
    if (!s) { set_error("solver is NULL"); return TPH_ERR_INVALID; }
    if (!rho_b || !p) { set_error("rho_b and p are required"); return TPH_ERR_INVALID; }
    if (!std::isfinite(gy)) { set_error("gravity must be finite"); return TPH_ERR_INVALID; }
    const Geom& g = s->lev[0].g;
    TPH_TRY(copy_in(s, g, s->gtmp[2], rho_b));
    const Vec3 t = vec3(s, s->t3);
    TPH_HIP(hipMemsetAsync(s->t3, 0, s->n3 * sizeof(double), s->st));
    TPH_HIP(launch_lithostatic(g, s->gtmp[2], gy, t.p(), s->st));
    TPH_TRY(remove_pressure_mean(s, s->t3));
    TPH_TRY(copy_out(s, g, p, t.p()));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

tph_status tph_solve_continuation(tph_solver* s, const double* eta_b, const double* eta_p, const double* rho_b,
                                  double gx, double gy, const double* thetas, int32_t nthetas, double stage_rtol,
                                  int32_t lithostatic, double* vx, double* vy, double* p, tph_info* info) {
    g_last_error.clear();
    if (!s) { set_error("solver is NULL"); return TPH_ERR_INVALID; }
    if (!eta_b || !eta_p || !rho_b || !vx || !vy || !p) {
        set_error("eta_b, eta_p, rho_b, vx, vy and p are required");
        return TPH_ERR_INVALID;
    }
    if (!thetas || nthetas < 1 || nthetas > 64) { set_error("thetas must hold 1..64 values"); return TPH_ERR_INVALID; }
    for (int k = 0; k < nthetas; ++k) {
        if (!(thetas[k] >= 0.0 && thetas[k] <= 1.0) || (k > 0 && thetas[k] < thetas[k - 1])) {
            set_error("thetas must be non-decreasing values in [0, 1]");
            return TPH_ERR_INVALID;
        }
    }
    if (thetas[nthetas - 1] != 1.0) { set_error("the last theta must be 1 (the original viscosity)"); return TPH_ERR_INVALID; }
    if (!(stage_rtol > 0.0 && stage_rtol < 1.0)) { set_error("stage_rtol must be in (0, 1)"); return TPH_ERR_INVALID; }
    if (lithostatic != 0 && lithostatic != 1) { set_error("lithostatic must be 0 or 1"); return TPH_ERR_INVALID; }
    const Geom& g = s->lev[0].g;
    const size_t nd = (size_t)(g.ny + 2) * (g.nx + 2);
    if (!s->cont_eb) {
        TPH_TRY(dev_alloc(s, (void**)&s->cont_eb, nd * sizeof(double)));
        TPH_TRY(dev_alloc(s, (void**)&s->cont_ep, nd * sizeof(double)));
    }
    double m = 0.0;
    TPH_TRY(eta_min_dense(s, eta_b, eta_p, &m));
    if (!(m > 0.0) || !std::isfinite(m)) { set_error("viscosity must be finite and positive"); return TPH_ERR_INVALID; }
    // initial guess: the lithostatic pressure with zero velocity, or the caller's fields
    if (lithostatic) {
        TPH_HIP(hipMemsetAsync(s->x, 0, s->n3 * sizeof(double), s->st));
        TPH_TRY(copy_in(s, g, s->gtmp[2], rho_b));
        TPH_HIP(launch_lithostatic(g, s->gtmp[2], gy, vec3(s, s->x).p(), s->st));
    } else {
        TPH_TRY(load_solution(s, s->x, vx, vy, p));
    }
    const double rtol = s->d.rtol;
    tph_info tot{};
    tph_status r = TPH_OK;
    for (int k = 0; k < nthetas && r >= 0; ++k) {
        TPH_HIP(launch_blend(eta_b, s->cont_eb, nd, thetas[k], m, s->st));
        TPH_HIP(launch_blend(eta_p, s->cont_ep, nd, thetas[k], m, s->st));
        TPH_TRY(setup_enqueue(s, s->cont_eb, s->cont_ep, rho_b, gx, gy, nullptr, nullptr, true));
        TPH_TRY(setup_finish(s));
        tph_info st{};
        if (info && info->history && tot.iters < info->history_len) {
            st.history = info->history + tot.iters;
            st.history_len = info->history_len - tot.iters;
        }
        s->d.rtol = k == nthetas - 1 ? rtol : std::max(stage_rtol, rtol);
        r = accelerate(s, s->b, &st);
        s->d.rtol = rtol;
        tot.iters += st.iters;
        tot.restarts += st.restarts;
        tot.vcycles += st.vcycles;
        tot.res_l2 = st.res_l2;
        tot.res_energy = st.res_energy;
        tot.res_estimate = st.res_estimate;
        tot.t_setup_ms += s->t_setup_ms;
        tot.t_solve_ms += st.t_solve_ms;
        // an intermediate stage that stops short of stage_rtol still gives the next one its start
        if (r == TPH_NOT_CONVERGED && k < nthetas - 1) r = TPH_OK;
    }
    if (r < 0) return r;
    TPH_TRY(store_solution(s, s->x, vx, vy, p));
    TPH_HIP(hipStreamSynchronize(s->st));
    if (info) {
        double* h = info->history;
        const int32_t hl = info->history_len;
        *info = tot;
        info->history = h;
        info->history_len = hl;
    }
    return r;
}

tph_status tph_solve_rhs(tph_solver* s, const double* fx, const double* fy, const double* fp, double* vx, double* vy,
                         double* p, tph_info* info) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!vx || !vy || !p) { set_error("vx, vy and p are required"); return TPH_ERR_INVALID; }
    TPH_TRY(load_solution(s, s->b2, fx, fy, fp));
    TPH_TRY(load_solution(s, s->x, vx, vy, p));
    const tph_status r = accelerate(s, s->b2, info);
    if (r < 0) return r;
    TPH_TRY(store_solution(s, s->x, vx, vy, p));
    TPH_HIP(hipStreamSynchronize(s->st));
    return r;
}

tph_status tph_apply(tph_solver* s, const double* vx, const double* vy, const double* p, double* ax, double* ay,
                     double* ap) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!vx || !vy || !p || !ax || !ay || !ap) { set_error("all six arrays are required"); return TPH_ERR_INVALID; }
    TPH_TRY(load_solution(s, s->t2, vx, vy, p));
    const LevelBuf& L = s->lev[0];
    TPH_HIP(launch_outer_residual(L.g, vec3(s, s->t2), nullptr, L.eb64, L.ep64, vec3(s, s->t1), ResMode::kApply,
                                  false, nullptr, nullptr, s->st));
    TPH_TRY(store_solution(s, s->t1, ax, ay, ap));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

tph_status tph_precondition_apply(tph_solver* s, const double* rx, const double* ry, const double* rp, double* zx,
                                  double* zy, double* zp, double* wx, double* wy, double* wp) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!rx || !ry || !rp || !zx || !zy || !zp || !wx || !wy || !wp) {
        set_error("all nine arrays are required");
        return TPH_ERR_INVALID;
    }
    const Geom& g = s->lev[0].g;
    Vec3 r = vec3(s, s->b2);
    TPH_TRY(copy_in(s, g, r.vx(), rx));
    TPH_TRY(copy_in(s, g, r.vy(), ry));
    TPH_TRY(copy_in(s, g, r.p(), rp));
    // z and w in the accelerator workspace, free outside a solve: z (a
    // solution-type vector, mirrored ghosts) in the first preconditioned
    // slot, w (residual-type) in the second basis slot.  Basis vectors must
    // stay zero outside the equation rows (the Krylov kernels stream every
    // entry), so z must not go there.
    double* zb = s->Z;
    double* wb = s->V + s->n3;
    TPH_HIP(hipMemsetAsync(zb, 0, s->n3 * sizeof(double), s->st));
    TPH_HIP(hipMemsetAsync(wb, 0, s->n3 * sizeof(double), s->st));
    TPH_TRY(precondition(s, s->b2, zb, false, wb));
    TPH_TRY(store_solution(s, zb, zx, zy, zp));
    TPH_TRY(store_solution(s, wb, wx, wy, wp));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

tph_status tph_precondition(tph_solver* s, const double* rx, const double* ry, const double* rp, double* zx,
                            double* zy, double* zp) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!rx || !ry || !rp || !zx || !zy || !zp) { set_error("all six arrays are required"); return TPH_ERR_INVALID; }
    const Geom& g = s->lev[0].g;
    Vec3 r = vec3(s, s->t2);
    TPH_TRY(copy_in(s, g, r.vx(), rx));
    TPH_TRY(copy_in(s, g, r.vy(), ry));
    TPH_TRY(copy_in(s, g, r.p(), rp));
    TPH_HIP(hipMemsetAsync(s->t1, 0, s->n3 * sizeof(double), s->st));
    TPH_TRY(precondition(s, s->t2, s->t1, false));
    TPH_TRY(store_solution(s, s->t1, zx, zy, zp));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

tph_status tph_energy_residual(tph_solver* s, const double* vx, const double* vy, const double* p, double* out) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!vx || !vy || !p || !out) { set_error("vx, vy, p and out are required"); return TPH_ERR_INVALID; }
    TPH_TRY(load_solution(s, s->t2, vx, vy, p));
    TPH_TRY(energy_residual_vec(s, s->t2, s->b, s->t1, kSlotMisc));
    TPH_HIP(hipMemsetAsync(s->t2, 0, s->n3 * sizeof(double), s->st));
    TPH_TRY(energy_residual_vec(s, s->t2, s->b, s->t1, kSlotMisc + 1));
    TPH_TRY(fetch(s, kSlotMisc, 2));
    const double num = s->hscal[kSlotMisc], den = s->hscal[kSlotMisc + 1];
    *out = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
    return TPH_OK;
}

tph_status tph_level_shape(tph_solver* s, int32_t level, int32_t* nx, int32_t* ny) {
    g_last_error.clear();
    if (!s) { set_error("solver is NULL"); return TPH_ERR_INVALID; }
    if (level < 0 || level >= s->nlev) { set_error("level out of range"); return TPH_ERR_INVALID; }
    if (nx) *nx = s->lev[level].g.nx;
    if (ny) *ny = s->lev[level].g.ny;
    return TPH_OK;
}

tph_status tph_level_plan(tph_solver* s, int32_t level, int32_t* kind, int32_t* shape) {
    g_last_error.clear();
    if (!s) { set_error("solver is NULL"); return TPH_ERR_INVALID; }
    if (level < 0 || level >= s->nlev) { set_error("level out of range"); return TPH_ERR_INVALID; }
    int k = 0;
    if (s->d.fused) {
        const LevelBuf& L = s->lev[level];
        if (s->lc >= 0 && level >= s->lc) k = 2;
        else if (level == s->nlev - 1) k = 3;
        else if (ras_level(s, level)) k = 4;
        else if (((s->msw_mask >> level) & 1u) && L.nu_pre > 0 && L.nu_post > 0) k = 1;
    }
    if (kind) *kind = k;
    if (shape) *shape = (int32_t)((s->shape_mask >> level) & 1u);
    return TPH_OK;
}

tph_status tph_level_viscosity(tph_solver* s, int32_t level, double* eta_b, double* eta_p) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (level < 0 || level >= s->nlev) { set_error("level out of range"); return TPH_ERR_INVALID; }
    const LevelBuf& L = s->lev[level];
    if (eta_b) TPH_TRY(copy_out(s, L.g, eta_b, L.eb64));
    if (eta_p) TPH_TRY(copy_out(s, L.g, eta_p, L.ep64));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

tph_status tph_solve_adjoint(tph_solver* s, const double* gvx, const double* gvy, const double* gp, double* lvx,
                             double* lvy, double* lp, tph_info* info) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!lvx || !lvy || !lp) { set_error("lvx, lvy and lp are required"); return TPH_ERR_INVALID; }
    // A is symmetric: the adjoint solve is the forward solve with right-hand side g
    TPH_HIP(hipMemsetAsync(s->b2, 0, s->n3 * sizeof(double), s->st));
    const Geom& g = s->lev[0].g;
    Vec3 r = vec3(s, s->b2);
    if (gvx) TPH_TRY(copy_in(s, g, r.vx(), gvx));
    if (gvy) TPH_TRY(copy_in(s, g, r.vy(), gvy));
    if (gp) TPH_TRY(copy_in(s, g, r.p(), gp));
    // the output pressure of a solve is mean-free and ghosts mirror their owners:
    // project the incoming gradient accordingly (this also makes the system consistent)
    TPH_HIP(launch_fold_ghost_grad(g, r, s->st));
    TPH_TRY(remove_pressure_mean(s, s->b2));
    TPH_HIP(hipMemsetAsync(s->x, 0, s->n3 * sizeof(double), s->st));
    const tph_status st = accelerate(s, s->b2, info);
    if (st < 0) return st;
    TPH_TRY(store_solution(s, s->x, lvx, lvy, lp));
    TPH_HIP(hipStreamSynchronize(s->st));
    return st;
}

tph_status tph_coeff_gradient(tph_solver* s, const double* vx, const double* vy, const double* p, const double* lvx,
                              const double* lvy, const double* lp, double* g_eta_b, double* g_eta_p, double* g_rho_b) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (!vx || !vy || !lvx || !lvy) { set_error("forward and adjoint velocities are required"); return TPH_ERR_INVALID; }
    const Geom& g = s->lev[0].g;
    TPH_TRY(load_solution(s, s->t1, vx, vy, p));
    TPH_TRY(load_solution(s, s->t2, lvx, lvy, lp));
    for (int k = 0; k < 3; ++k)
        TPH_HIP(hipMemsetAsync(s->gtmp[k] - (kAlign - 1), 0, field_alloc(g) * sizeof(double), s->st));
    TPH_HIP(launch_coeff_gradient(g, vec3(s, s->t1), vec3(s, s->t2), s->gx, s->gy, g_eta_b ? s->gtmp[0] : nullptr,
                                  g_eta_p ? s->gtmp[1] : nullptr, g_rho_b ? s->gtmp[2] : nullptr, s->st));
    if (g_eta_b) TPH_TRY(copy_out(s, g, g_eta_b, s->gtmp[0]));
    if (g_eta_p) TPH_TRY(copy_out(s, g, g_eta_p, s->gtmp[1]));
    if (g_rho_b) TPH_TRY(copy_out(s, g, g_rho_b, s->gtmp[2]));
    TPH_HIP(hipStreamSynchronize(s->st));
    return TPH_OK;
}

tph_status tph_time_kernel(tph_solver* s, int32_t kind, int32_t reps, double* ms_per_launch,
                           double* bytes_per_launch) {
    g_last_error.clear();
    TPH_TRY(require_ready(s));
    if (reps < 1 || kind < TPH_KERNEL_SMOOTH || kind > TPH_KERNEL_AA_MIX) {
        set_error("bad kernel kind or repetition count");
        return TPH_ERR_INVALID;
    }
    if ((kind == TPH_KERNEL_RESTRICT || kind == TPH_KERNEL_PROLONG) && s->nlev < 2) {
        set_error("transfer kernels need at least two levels");
        return TPH_ERR_INVALID;
    }
    const tph_status st = s->mixed() ? time_kernel_t<float>(s, kind, reps, ms_per_launch, bytes_per_launch)
                                     : time_kernel_t<double>(s, kind, reps, ms_per_launch, bytes_per_launch);
    return st;
}

tph_status tph_kernel_timing(tph_solver* s, int32_t enable) {
    g_last_error.clear();
    if (!s) { set_error("null handle"); return TPH_ERR_INVALID; }
    if (enable < 0 || enable > 1024) { set_error("enable must be 0 (off) or a sampling stride in [1, 1024]"); return TPH_ERR_INVALID; }
    if (enable && s->kev.empty()) {
        s->kev.assign(2 * kMaxTimedLaunches, nullptr);
        for (auto& e : s->kev) {
            const hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) {
                for (auto& q : s->kev)
                    if (q) (void)hipEventDestroy(q);
                s->kev.clear();
                set_error(std::string("hipEventCreate: ") + hipGetErrorString(err));
                return TPH_ERR_HIP;
            }
        }
    }
    s->ktime = enable > 0;
    s->kstride = enable > 0 ? enable : 1;
    s->kcount = 0;
    return TPH_OK;
}

tph_status tph_kernel_timing_target(tph_solver* s, int32_t kind) {
    g_last_error.clear();
    if (!s) { set_error("null handle"); return TPH_ERR_INVALID; }
    if (kind != TPH_KERNEL_SMOOTH && kind != TPH_KERNEL_LINK) {
        set_error("the timing target must be TPH_KERNEL_SMOOTH or TPH_KERNEL_LINK");
        return TPH_ERR_INVALID;
    }
    s->ktarget = kind;
    s->kcount = 0;
    return TPH_OK;
}

tph_status tph_kernel_timing_read(tph_solver* s, int32_t* launches, double* total_ms, double* total_bytes,
                                  int32_t* dropped) {
    g_last_error.clear();
    if (!s) { set_error("null handle"); return TPH_ERR_INVALID; }
    double ms = 0.0;
    if (s->kev_used > 0) {
        TPH_HIP(hipEventSynchronize(s->kev[s->kev_used - 1]));
        for (int q = 0; q < s->kev_used; q += 2) {
            float t = 0.0f;
            TPH_HIP(hipEventElapsedTime(&t, s->kev[q], s->kev[q + 1]));
            ms += t;
        }
    }
    if (launches) *launches = s->kev_used / 2;
    if (total_ms) *total_ms = ms;
    if (total_bytes) *total_bytes = s->kbytes;
    if (dropped) *dropped = s->kdropped;
    s->kev_used = 0;
    s->kdropped = 0;
    s->kbytes = 0.0;
    return TPH_OK;
}

void tph_destroy(tph_solver* s) {
    if (!s) return;
    if (s->st || !s->mem.empty()) (void)hipStreamSynchronize(s->st);
    if (s->gst) (void)hipStreamSynchronize(s->gst);
    s->mem.release_all();
    if (s->hscal) (void)hipHostFree(s->hscal);
    if (s->hseq) (void)hipHostFree(s->hseq);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    for (auto& e : s->kev)
        if (e) (void)hipEventDestroy(e);
    for (auto& pg : s->pgraphs) {
        if (pg.exec) (void)hipGraphExecDestroy(pg.exec);
        if (pg.graph) (void)hipGraphDestroy(pg.graph);
    }
    if (s->gst) {
        (void)hipStreamSynchronize(s->gst);
        (void)hipStreamDestroy(s->gst);
    }
    if (s->gev0) (void)hipEventDestroy(s->gev0);
    if (s->gev1) (void)hipEventDestroy(s->gev1);
    delete s;
}

tph_status tph_set_allocator(tph_solver* s, void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
    g_last_error.clear();
    if ((alloc == nullptr) != (free_fn == nullptr)) {
        set_error("alloc and free must both be given or both be NULL");
        return TPH_ERR_INVALID;
    }
    Allocator a;
    a.alloc = alloc;
    a.free = free_fn;
    a.ctx = alloc ? ctx : nullptr;
    if (s) s->mem.a = a;
    else set_default_allocator(a);
    return TPH_OK;
}

const char* tph_last_error(void) { return g_last_error.c_str(); }

const char* tph_version(void) { return "tephra 0.1.0 (gfx950)"; }

}  // extern "C"
