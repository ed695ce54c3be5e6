// Host-side launchers of the HIP kernels (one translation unit per family).
// Every launcher enqueues on `st` and returns the launch status.
#pragma once
#include "common.h"

namespace tph {

// ---------------------------------------------------------------- stencil.hip
// out = scale * (b - A x)  (b may be null: out = scale * (-A x) if negate, else scale * A x)
// scale = sqrt(energy weight) when `energy` is set, else 1.  Writes equation
// rows only.  partial (nullable): per-block sums of out^2, nblk entries.
enum class ResMode { kResidual = 0, kApply = 1 };
// b_scaled: b holds W^(1/2) b (an energy-scaled Krylov vector) and is unscaled on the fly
hipError_t launch_outer_residual(const Geom& g, Vec3 x, const Vec3* b, const double* eb, const double* ep,
                                 Vec3 out, ResMode mode, bool energy, double* partial, int* nblk_out,
                                 hipStream_t st, bool b_scaled = false);
// per-block sums of the squared energy-weighted row magnitudes |b| + |A| |x|
hipError_t launch_residual_magnitude(const Geom& g, Vec3 x, Vec3 b, const double* eb, const double* ep,
                                    double* partial, int* nblk_out, hipStream_t st);
// walls to zero, ghosts mirrored, for a solution-type vx / vy pair
template <typename T>
hipError_t launch_fill_bc(const Geom& g, T* vx, T* vy, hipStream_t st);
// every entry of a velocity correction pair to zero
template <typename T>
hipError_t launch_zero_vel(const Geom& g, T* ex, T* ey, hipStream_t st);
// damped Jacobi sweep: e_out = e_in + omega (r - L e_in) / diag (e_in == null: zero guess)
template <typename T>
hipError_t launch_jacobi(const Geom& g, const T* ex_in, const T* ey_in, T* ex_out, T* ey_out,
                         const T* rx, const T* ry, const T* eb, const T* ep, T omega, hipStream_t st);
// one colour half-sweep of damped Gauss-Seidel on component comp (0 vx, 1 vy), colour col
template <typename T>
hipError_t launch_gs_half(const Geom& g, int comp, int col, T* ex, T* ey, const T* rx, const T* ry,
                          const T* eb, const T* ep, T omega, bool zero_guess, hipStream_t st);
// t = r - L e (velocity rows)
template <typename T>
hipError_t launch_vel_residual(const Geom& g, const T* ex, const T* ey, const T* rx, const T* ry,
                               const T* eb, const T* ep, T* tx, T* ty, hipStream_t st);
// preconditioner entry: level-0 right-hand side r = v / sqrt(w_v) (energy) or v
template <typename T>
hipError_t launch_precond_in(const Geom& g, Vec3 v, const double* eb, const double* ep, bool energy,
                             T* rx, T* ry, hipStream_t st);
// preconditioner exit: z_v = (double) e; z_p = alpha eta_p (r_p - D z_v)
// (accumulate: z_v += e, z_p += alpha eta_p (r_p - D e))
template <typename T>
struct LinkArgs;
// one pass linking two Uzawa steps (mode kLinkNext), the last step and the
// Krylov apply (kLinkApply) or ending the last step (kLinkStore); see
// uzawa_link_cell
template <typename T>
hipError_t launch_uzawa_link(const Geom& g, const LinkArgs<T>& a, int mode, const double* eb, const double* ep,
                             hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
template <typename T>
hipError_t launch_precond_out(const Geom& g, const T* ex, const T* ey, Vec3 v, const double* ep,
                              bool energy, double alpha, Vec3 z, hipStream_t st, bool accumulate = false);
// right-hand side f = -rho g (+ extra) at velocity rows, 0 at continuity rows
// lithostatic pressure at the cells (ghosts untouched), viscosity minimum
// (partial: one slot per 64 x 4 block of the basic grid; out: 1 value), and
// the continuation blend out = (1 - theta) m + theta in over n entries
hipError_t launch_lithostatic(const Geom& g, const double* rho, double gy, double* p, hipStream_t st);
hipError_t launch_eta_min(const Geom& g, const double* eb, const double* ep, double* partial, double* out,
                          hipStream_t st);
hipError_t launch_blend(const double* in, double* out, size_t n, double theta, double m, hipStream_t st);
hipError_t launch_rhs(const Geom& g, const double* rho, double gx, double gy, const double* fxe,
                      const double* fye, Vec3 b, hipStream_t st);
// per-block counts of invalid coefficients: [bad eta, nonfinite rho/force]
hipError_t launch_check_coeffs(const Geom& g, const double* eb, const double* ep, const double* rho,
                               const double* fxe, const double* fye, double* partial, int* nblk_out,
                               hipStream_t st);
// coefficient gradient (adjoint): outputs nullable
hipError_t launch_coeff_gradient(const Geom& g, Vec3 x, Vec3 lam, double gx, double gy,
                                 double* g_eb, double* g_ep, double* g_rho, hipStream_t st);
// adjoint right-hand side: fold gradients of ghost entries onto their interior owners
hipError_t launch_fold_ghost_grad(const Geom& g, Vec3 v, hipStream_t st);
// Cell block of the one-thread-per-cell kernels (operator apply, residuals,
// Uzawa entry, exit and link passes, coefficient checks, and the batch's cell
// work items): kCellBX x kCellBY cells, one thread each.  The per-block
// reduction partials are sized from it.
constexpr int kCellBX = 64;
constexpr int kCellBY = 4;

// FP64 -> FP32 casts of whole arrays in one launch (the viscosities of every level)
struct CastList {
    const double* src[2 * kMaxLevels];
    float* dst[2 * kMaxLevels];
    size_t n[2 * kMaxLevels];
    int count;
};
hipError_t launch_cast_list(const CastList& c, hipStream_t st);

// --------------------------------------------------------------- transfer.hip
// coarse viscosities from fine ones (normalised bilinear gather; geometric = log-mean)
hipError_t launch_restrict_eta(const Geom& gf, const Geom& gc, const double* ebf, const double* epf,
                               double* ebc, double* epc, bool geometric, hipStream_t st);
template <typename T>
hipError_t launch_restrict_res(const Geom& gf, const Geom& gc, const T* tx, const T* ty, T* rx, T* ry,
                               hipStream_t st);
template <typename T>
hipError_t launch_prolong_add(const Geom& gf, const Geom& gc, const T* ecx, const T* ecy, T* ex, T* ey,
                              hipStream_t st);

// ----------------------------------------------------------------- coarse.hip
int coarse_unknowns(const Geom& g);
// dense M = -L (n x n row-major, FP64) of the level, then in-place inverse
hipError_t launch_coarse_assemble(const Geom& g, const double* eb, const double* ep, double* M,
                                  hipStream_t st);
// In-place inverse of the n x n SPD matrix M (row-major) by Gauss-Jordan
// elimination.  n <= kGJLds: one workgroup in LDS, which needs `table`:
// device memory holding {M, (int)n} as written by the caller (a pointer
// followed by an int).  Larger n: 2 n launches over the device with `work`
// = 2 n doubles of device scratch.
constexpr int kGJLds = 136;    // largest n inverted by one workgroup (registers, 2 n doubles of LDS)
hipError_t launch_gauss_jordan(double* M, int n, hipStream_t st, double** table, double* work);
// one workgroup per matrix: mats[i] (device array of device pointers), sizes
// ns[i] <= kGJLds, nmax = max ns[i]
hipError_t launch_gauss_jordan_batched(double* const* mats, const int* ns, int count, int nmax, hipStream_t st);
size_t gauss_jordan_lds_bytes(int n);
// e = L^{-1} r = -M^{-1} r with M^{-1} stored; r, e level fields (ghosts of e
// written); one wave per row, 4 rows per workgroup
template <typename T>
hipError_t launch_coarse_solve(const Geom& g, const double* Minv, const T* rx, const T* ry, T* ex, T* ey,
                               hipStream_t st);

// -------------------------------------------------------------------- ras.hip
// one outer iteration of the RAS-type temporal-blocking Jacobi smoother:
// tile x tile tiles (8, 16 or 32) with boundaries at rows 1 + si + k tile and
// columns 1 + sj + k tile, `inner` damped Jacobi sweeps per tile with the
// outside held at the input state; zero: the input is zero (exi, eyi unused).
// The output buffers must differ from the inputs.
template <typename T>
hipError_t launch_ras_tile(const Geom& g, int tile, int si, int sj, int inner, bool zero, const T* exi, const T* eyi,
                           T* exo, T* eyo, const T* rx, const T* ry, const T* eb, const T* ep, T omega,
                           hipStream_t st);

// ----------------------------------------------------------------- krylov.hip
int flat_blocks(size_t n);
// partial[i * nblk + b] = sum over block b of V_i . w (any nv, in chunks of 8); when
// norm_slot >= 0 also partial[norm_slot * nblk + b] = block sums of w . w
hipError_t launch_multidot(const double* V0, size_t vstride, int nv, const double* w, size_t n,
                           double* partial, int nblk, hipStream_t st, int norm_slot = -1);
// w -= sum_i h[i] V_i, then partial[i * nblk + b] = block sums of V_i . w (nv entries)
// and, when norm_slot >= 0, partial[norm_slot * nblk + b] = block sums of w . w
hipError_t launch_axpy_dot(double* w, const double* V0, size_t vstride, int nv, const double* h,
                           size_t n, bool want_dots, int norm_slot, double* partial, int nblk,
                           hipStream_t st);
// out[i] = sum_b partial[i * nblk + b], i < k  (fixed order: deterministic)
// row sums of partial (k rows of nblk) into out; also into host_out (a device
// pointer to mapped coherent host memory) when it is not null.  With k == 1
// and host_seq not null, the kernel then writes seq to *host_seq (mapped host
// memory) after a system-scope fence, so a host that sees seq there also sees
// every value written to host memory by this and earlier kernels.
hipError_t launch_reduce_rows(const double* partial, int nblk, int k, double* out, hipStream_t st,
                              double* host_out = nullptr, unsigned* host_seq = nullptr, unsigned seq = 0);
// dst = src / sqrt(*nrm2)
hipError_t launch_scale_by_rnorm(double* dst, const double* src, size_t n, const double* nrm2,
                                 hipStream_t st);
// dst = src * (1 / *beta)
hipError_t launch_scale_by_rbeta(double* dst, const double* src, size_t n, const double* beta,
                                 hipStream_t st);
// x += sum_j y[j] Z_j  (k <= 8 per launch)
hipError_t launch_update_x(double* x, const double* Z0, size_t zstride, int k, const double* y,
                           size_t n, hipStream_t st);
// flexible GCR step (see k_gcr_step): coefficients by value, i <= kMaxRestart
struct GcrStepArgs {
    double* w;               // in: new direction A z (energy-scaled); out: w^ (normalised)
    const double* W0;        // earlier w^_0 .. w^_{i-1}, stride apart
    double* z;               // in: preconditioned z; out: z' (same combination as w); null: skip z, x
    const double* Z0;        // earlier z'_0 .. z'_{i-1}
    double* x;
    double* r;               // energy-scaled residual
    size_t stride, n;
    int i, orth_w;
    double inv_nu, alpha;
    double hw[kMaxRestart];
    double hz[kMaxRestart];
};
hipError_t launch_gcr_step(const GcrStepArgs& a, hipStream_t st);
// Anderson: dot products over the unknowns of three-field solution vectors
// (vecs[i] and f are raw vector pointers, fields fstride apart), in chunks of
// 8; partial rows as launch_multidot.  nblk = unknown_dot_blocks(g).
constexpr int kVecSetMax = 8;
struct VecSet { const double* v[kVecSetMax]; };
int unknown_dot_blocks(const Geom& g);
hipError_t launch_multidot_unknowns(const Geom& g, size_t fstride, const double* const* vecs, int nv,
                                    const double* f, double* partial, int nblk, hipStream_t st, int norm_slot);
// out = sum_v cx[v] X[v] + cf[v] F[v] over n entries; out may alias X[0] (and
// no other input)
struct MixArgs {
    double* out;
    size_t n;
    int nv, acc;
    const double* X[kVecSetMax];
    const double* F[kVecSetMax];
    double cx[kVecSetMax];
    double cf[kVecSetMax];
};
hipError_t launch_mix(double* out, const double* const* X, const double* cx, const double* const* F,
                      const double* cf, int nv, size_t n, hipStream_t st);
// writes seq to mapped host memory after every earlier kernel of the stream
hipError_t launch_post_seq(unsigned* host_seq, unsigned seq, hipStream_t st);
// sum of p over cells -> partial; then p -= mean
hipError_t launch_p_sum(const Geom& g, const double* p, double* partial, int* nblk_out, hipStream_t st);
hipError_t launch_p_shift(const Geom& g, double* p, const double* sum, hipStream_t st);

// ------------------------------------------------------------------ fused.hip
template <typename T>
struct CoarseArgs {
    int nl;                          // levels handled: 0 = top (read rx, ry; write ex, ey), nl-1 = coarsest
    int nc;                          // unknowns of the coarsest level (dense FP64 solve)
    int smoother;                    // TPH_SMOOTH_*
    T omega;
    Geom g[kMaxLevels];
    const T* eb[kMaxLevels];
    const T* ep[kMaxLevels];
    int nu_pre[kMaxLevels];
    int nu_post[kMaxLevels];
    const T* rx;
    const T* ry;
    T* ex;
    T* ey;
    const double* Minv;
};
template <typename T>
size_t coarse_cycle_lds_bytes(const Geom* g, int nl, int nc);
// mode: 0 plain sweep, 1 from a zero initial guess, 2 prolongation + correction then sweep
enum TileMode { kTilePlain = 0, kTileZero = 1, kTileProlong = 2 };
template <typename T>
hipError_t launch_smooth_tile(const Geom& g, const Geom* gc, int smoother, int mode, const T* exi, const T* eyi,
                              T* exo, T* eyo, const T* rx, const T* ry, const T* eb, const T* ep, const T* ecx,
                              const T* ecy, T omega, hipStream_t st, hipEvent_t t0 = nullptr,
                              hipEvent_t t1 = nullptr);
template <typename T>
hipError_t launch_res_restrict(const Geom& gf, const Geom& gc, const T* ex, const T* ey, const T* rx, const T* ry,
                               const T* eb, const T* ep, T* rcx, T* rcy, hipStream_t st);
template <typename T>
hipError_t launch_coarse_cycle(const CoarseArgs<T>& a, size_t lds_bytes, int max_lds, hipStream_t st);
// Gauss-Seidel on LDS tiles, ns (1 or 2) full sweeps per pass; mode as
// above; rr = 1 adds the residual and its restriction to the coarse level gc
// (rcx, rcy); shape 0 / 1 selects the large / small tile.  The tile
// launchers take optional events (t0, t1) that receive the start and end
// time stamps of the kernel itself.
template <typename T>
hipError_t launch_gs_tile(const Geom& g, const Geom& gc, int ns, int mode, int rr, int shape, const T* exi,
                          const T* eyi, T* exo, T* eyo, const T* rx, const T* ry, const T* eb, const T* ep,
                          const T* ecx, const T* ecy, T* rcx, T* rcy, T omega, hipStream_t st,
                          hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

}  // namespace tph
