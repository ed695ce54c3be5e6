/*
 * tephra: matrix-free geometric-multigrid solver of the 2D incompressible
 * variable-viscosity Stokes equations on the stress-conservative staggered
 * grid, for AMD Instinct MI355X (gfx950).
 *
 * The problem (Ch. 3 "Conservation of Mass and Momentum", Ch. 4
 * "Stress-Conservative Finite Differences", eq. stokes_saddle):
 *
 *     [ L  G ] [v]   [f]      L v = div_h(eta (grad_h v + grad_h v^T))
 *     [ D  0 ] [p] = [0],     G p = -grad_h p,  D v = div_h v,
 *
 * with f = -rho g (gravity moved to the right-hand side) plus an optional
 * extra body force.  The solver is an FP64 accelerator (Ch. 4
 * "Accelerators": flexible GMRES(m), flexible GCR(m) or Anderson
 * acceleration AA(m, beta)) around the Uzawa step (Sec. "Uzawa Iteration as
 * a Fixed Point Method"): a geometric multigrid V-cycle on L (Sec.
 * "Multigrid Cycles") followed by the viscosity-scaled pressure update.  The
 * stopping test is the relative energy residual of Sec. "Residual Norms".
 *
 * ARRAY CONVENTION (all field arguments).  A problem of nx x ny cells uses
 * dense row-major FP64 arrays of (ny + 2) x (nx + 2) entries, row index i
 * along y, column index j along x (Ch. 4 "Staggered Grid Layout"):
 *   basic node (i, j) at (j dx, i dy), i in [0, ny], j in [0, nx]: eta_b, rho_b
 *   cell centre (i, j) at ((j - 1/2) dx, (i - 1/2) dy), i, j in [1, n]: eta_p, p
 *   vx (i, j) at (j dx, (i - 1/2) dy): unknowns i in [1, ny], j in [1, nx - 1]
 *   vy (i, j) at ((j - 1/2) dx, i dy): unknowns i in [1, ny - 1], j in [1, nx]
 * Entries outside those ranges are ignored on input.  Velocity outputs hold
 * zero on the walls and mirrored ghosts (+1 free slip, -1 no slip) outside
 * them; pressure outputs have zero mean over the nx*ny cells; residual-type
 * outputs (tph_apply) are zero outside the equation rows.
 *
 * POINTERS AND OWNERSHIP.  Every field pointer is a DEVICE pointer on the
 * device current when the solver was created (for example a torch tensor's
 * data_ptr()).  The caller owns it; the library never keeps it after the call
 * returns.  tph_set_coefficients copies what it needs into library-owned
 * device workspace.
 *
 * STREAMS.  All work is enqueued on the hipStream_t given to tph_create.
 * Entry points that report scalars (solve, energy residual) synchronise that
 * stream before returning.
 *
 * ERRORS.  Every entry point returns a tph_status; nothing is thrown across
 * the ABI.  A human-readable message for the calling thread's last failure
 * is available from tph_last_error().  Descriptor and size checks run on the
 * host before any device work.  Viscosity that is not finite and positive,
 * or a non-finite density / force, is detected by a device check inside
 * tph_set_coefficients (TPH_ERR_INVALID / TPH_ERR_NONFINITE).  A solve that
 * exhausts max_iters returns TPH_NOT_CONVERGED (a warning: the best iterate
 * is written and the info block filled).
 *
 * THREADING.  A handle must not be used from two threads at once.
 */
#ifndef TEPHRA_H
#define TEPHRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TPH_OK = 0,
    TPH_NOT_CONVERGED = 1,
    TPH_ERR_INVALID = -1,
    TPH_ERR_OOM = -2,
    TPH_ERR_HIP = -3,
    TPH_ERR_NONFINITE = -4,
    TPH_ERR_UNSUPPORTED = -5
} tph_status;

/* Per-wall velocity condition (Ch. 3 "Boundary Conditions"). */
enum { TPH_FREE_SLIP = 0, TPH_NO_SLIP = 1 };
/* Wall order in tph_desc.bc: west (x = 0), east (x = lx), south (row 0), north (row ny). */
enum { TPH_WEST = 0, TPH_EAST = 1, TPH_SOUTH = 2, TPH_NORTH = 3 };
/* TPH_FP64: V-cycle in FP64.  TPH_MIXED: V-cycle smoothing and transfers in
 * FP32; outer residual, Krylov orthogonalisation, coarsest solve and the
 * pressure step stay FP64. */
enum { TPH_FP64 = 0, TPH_MIXED = 1 };
/* Smoother on L (Sec. "Smoothers"): damped Jacobi (eq. damped_jacobi),
 * damped Gauss-Seidel (eq. sor_update) in four colour half-sweeps
 * (vx red, vx black, vy red, vy black; red = (i + j) even), or the RAS-type
 * temporal-blocking Jacobi of Alg. "RAS-Type Temporal Blocking" on every
 * level (TPH_SMOOTH_RAS) or below the finest level, which takes damped
 * Jacobi (TPH_SMOOTH_RAS_MIXED, the paper's "Mixed" configuration).  RAS:
 * each outer iteration (one launch) splits the velocity unknowns into
 * ras_tile x ras_tile tiles with boundaries at rows 1 + s_i + k ras_tile and
 * columns 1 + s_j + k ras_tile, and every tile runs ras_inner damped Jacobi
 * sweeps on its unknowns with the values outside it held at the state the
 * outer iteration started from; ceil(nu / ras_inner) outer iterations make
 * up a smoothing call of nu sweeps.  The shifts are SplitMix64 draws from
 * desc.seed at the counter ((((cycle * 16 + level) * 2 + leg) * 256 + outer)
 * * 2 + axis) modulo ras_tile, where cycle numbers the V-cycles of one
 * preconditioner application (0 .. uzawa_steps - 1) and leg is 0 (pre) or
 * 1 (post).  The RAS smoothers run without the single-workgroup coarse tail
 * and are not available to the batched solver. */
enum { TPH_SMOOTH_JACOBI = 0, TPH_SMOOTH_GS = 1, TPH_SMOOTH_RAS = 2, TPH_SMOOTH_RAS_MIXED = 3 };
/* Coarse-level viscosity: normalised bilinear restriction of eta
 * (arithmetic) or of log(eta) (geometric). */
enum { TPH_MEAN_ARITHMETIC = 0, TPH_MEAN_GEOMETRIC = 1 };
/* Accelerator around the Uzawa fixed-point map (Ch. 4 "Accelerators"):
 *   TPH_ACCEL_FGMRES    flexible GMRES(m) in the energy inner product, the
 *                       Uzawa step as right preconditioner (Sec. "Comparison
 *                       with FGMRES");
 *   TPH_ACCEL_GCR       restarted flexible GCR(m) (Alg. "Flexible GCR(m)")
 *                       in the same inner product: residual-minimising over
 *                       the preconditioned directions of a cycle;
 *   TPH_ACCEL_ANDERSON  Anderson acceleration with depth m and mixing beta
 *                       (Alg. "Anderson Acceleration(m) with Mixing") on
 *                       G(x) = x + M^{-1}(b - A x); its least-squares norm is
 *                       the Euclidean norm over the unknowns (vx, vy, p). */
enum { TPH_ACCEL_FGMRES = 0, TPH_ACCEL_GCR = 1, TPH_ACCEL_ANDERSON = 2 };

typedef struct tph_desc {
    int32_t nx, ny;        /* cells; each must be divisible by 2^(levels-1)
                              when coarsen = 2                                 */
    double lx, ly;         /* domain size, dx = lx / nx, dy = ly / ny        */
    int32_t bc[4];         /* TPH_FREE_SLIP / TPH_NO_SLIP per wall           */
    int32_t precision;     /* TPH_FP64 or TPH_MIXED                          */
    int32_t levels;        /* multigrid levels; 0 = automatic (coarsest side in [8, 16)
                              for coarsen = 2) */
    int32_t smoother;      /* TPH_SMOOTH_*                                    */
    int32_t nu_pre;        /* pre-smoothing sweeps on the finest level       */
    int32_t nu_post;       /* post-smoothing sweeps on the finest level      */
    double nu_growth;      /* sweeps on level l = ceil(nu * nu_growth^l)     */
    double omega;          /* smoother damping                                */
    double alpha;          /* Uzawa pressure relaxation                       */
    int32_t eta_mean;      /* TPH_MEAN_*                                      */
    double rtol;           /* relative energy residual target                 */
    int32_t restart;       /* m of the accelerator: FGMRES / GCR restart length
                              (1..64), Anderson depth (0..64)                 */
    int32_t max_iters;     /* total iterations (applications of the Uzawa
                              preconditioner)                                 */
    int32_t uzawa_steps;   /* Uzawa sweeps per preconditioner application (1..16):
                              z <- z + M^{-1}(r - A z), the fixed-point map of the
                              splitting A = M - N applied this many times         */
    int32_t fused;         /* 1: LDS-tiled fused smoother / residual-restriction
                              kernels and the single-workgroup coarse tail;
                              0: one kernel per colour half-sweep (reference)    */
    int32_t msweep;        /* levels whose smoothing runs in multi-sweep LDS passes
                              (bit l = level l): up to two Gauss-Seidel sweeps per
                              launch, the last pre-smoothing pass also forming the
                              residual and restricting it, the first post-smoothing
                              pass applying the prolongation; -1 = every level but
                              the finest.  Used with fused = 1 and the Gauss-Seidel
                              smoother, ignored otherwise                         */
    int32_t tile_shape;    /* levels whose LDS tiles use the small shape (bit l);
                              -1 = levels where the large shape gives fewer than
                              512 tiles                                           */
    int32_t coarse_level;  /* first level of the single-workgroup coarse tail
                              (fused = 1): -1 = the finest level of at most
                              64 x 64 cells whose tail fits in LDS; -2 = none (one
                              launch per level down to the coarsest); l >= 0 =
                              level l (rejected when it does not fit)          */
    int32_t accel;         /* TPH_ACCEL_*                                     */
    double beta;           /* Anderson mixing in (0, 1]; ignored otherwise    */
    int32_t ras_tile;      /* RAS tile side: 8, 16 or 32                      */
    int32_t ras_inner;     /* RAS local sweeps per outer iteration (1..16)    */
    uint64_t seed;         /* seed of the RAS tile shifts                     */
    int32_t graph;         /* 1: each preconditioner application inside a solve
                              (the Uzawa steps with their V-cycles and linked
                              exits) is captured once per distinct set of
                              vectors as a HIP graph and replayed; 0: every
                              kernel is launched on its own.  Same kernels and
                              results either way; while kernel timing is on
                              (tph_kernel_timing) applications run uncaptured.
                              Off by default: on MI355X the replays (launched
                              into a library stream joined by events) ran the
                              benchmark solve no faster than direct launches */
    int32_t pad_;          /* must be zero                                    */
    double coarsen;        /* coarsening factor between levels: 2 (exact halving;
                              sides divisible by 2^(levels-1)), or any value in
                              [1.25, 4] with fused = 0: level l+1 has
                              round(n_l / coarsen) cells per side (halves up, at
                              least 2), its nodes fall between fine nodes, and the
                              transfers use the normalised bilinear weights of
                              node coordinates with the fine index bounds of
                              Alg. "Bisect Bound" (the paper's sinker test
                              coarsens by 2.5); levels = 0 then coarsens while
                              both sides stay >= 8                             */
} tph_desc;

typedef struct tph_info {
    int32_t iters;         /* iterations (= preconditioner applications whose
                              result entered the returned iterate)           */
    int32_t restarts;      /* FGMRES / GCR restart cycles started (Anderson: 0) */
    double res_energy;     /* true relative energy residual of the result     */
    double res_estimate;   /* FGMRES / GCR recurrence estimate at exit
                              (Anderson: the true residual)                   */
    double t_setup_ms;     /* last tph_set_coefficients, device time          */
    double t_solve_ms;     /* this solve, host wall time                      */
    double* history;       /* optional caller-owned HOST buffer: estimate per iteration */
    int32_t history_len;   /* its capacity (entries)                          */
    int32_t vcycles;       /* V-cycles run by this solve: uzawa_steps per
                              preconditioner application, counting every
                              application (also one whose result the accelerator
                              did not keep)                                   */
    double res_l2;         /* plain relative residual ||b - A x||_2 / ||b||_2
                              over every equation row, no energy weights
                              (Sec. "Residual Norms" reports it beside the
                              energy residual)                                */
} tph_info;

typedef struct tph_solver tph_solver;

/* Fill *d with the defaults for an nx x ny unit-square free-slip problem:
 * mixed precision, automatic levels, coloured Gauss-Seidel (omega 1) with 2
 * pre- and 2 post-sweeps on every level, alpha 1, arithmetic coarse
 * viscosity, two Uzawa sweeps per preconditioner application, fused
 * kernels with the default multi-sweep levels and tile shapes (-1), rtol
 * 1e-8, FGMRES with restart 20, max_iters 500, beta 1, RAS tiles 32 x 32
 * with 4 inner sweeps and seed 0, no graph capture. */
void tph_desc_default(tph_desc* d, int32_t nx, int32_t ny);

/* Create a solver for the grid in *desc; hip_stream is a hipStream_t (NULL:
 * the null stream).  Allocates all device workspace (levels, Krylov basis)
 * through the process-wide allocator (tph_set_allocator).  Errors:
 * TPH_ERR_INVALID (sizes, levels, parameters), TPH_ERR_OOM (an allocation
 * failed; everything allocated before it has been freed again), TPH_ERR_HIP.
 * *out is NULL on failure. */
tph_status tph_create(const tph_desc* desc, void* hip_stream, tph_solver** out);

/* Device memory of the library's workspace (the shared simulation state of
 * Ch. 5 "Simulation State": the caller's memory manager, e.g. a framework's
 * caching allocator, can own it).  alloc(bytes, ctx) returns `bytes` of
 * device memory on the device current at the call, 256-byte aligned, or NULL
 * when it cannot (the library then returns TPH_ERR_OOM after freeing what it
 * had obtained); free(ptr, ctx) releases a block alloc returned.  Both NULL:
 * hipMalloc / hipFree (the initial state).  Exactly one NULL: TPH_ERR_INVALID.
 *   s == NULL: the process-wide default, read by every later tph_create,
 *              tph_batch_create and tph_markers_create (thread-safe).
 *   s != NULL: that solver's allocator for blocks it allocates from now on
 *              (workspace made on demand, e.g. by tph_solve_continuation);
 *              blocks it already holds stay where they are.
 * Every block is freed with the free function of the allocator that made it,
 * after the handle's stream has drained (tph_destroy and the other destroy
 * calls).  Pinned host memory (for scalars the host reads) is not device
 * workspace and is always taken from hipHostMalloc.  Returns TPH_OK. */
tph_status tph_set_allocator(tph_solver* s, void* (*alloc)(size_t bytes, void* ctx),
                             void (*free)(void* ptr, void* ctx), void* ctx);

/* Coefficient setup (hot-path step "coefficient setup"): copies eta_b,
 * eta_p (basic nodes, cell centres) and builds f = -rho_b g averaged to the
 * velocity nodes (x: mean of the basic nodes below/above; y: left/right) plus
 * fx_extra / fy_extra sampled at vx / vy nodes (both nullable); restricts the
 * viscosities down every level (normalised bilinear weights, Alg. "4-Color
 * Parallel Restriction" in gather form) and factors the coarsest operator in
 * FP64.  All arrays are device (ny+2) x (nx+2) FP64.  Must precede any solve
 * or apply. */
tph_status tph_set_coefficients(tph_solver* s, const double* eta_b, const double* eta_p,
                                const double* rho_b, double gx, double gy,
                                const double* fx_extra, const double* fy_extra);

/* Solve A [v; p] = [f; 0] to desc.rtol in the relative energy residual.
 * vx, vy, p: in = initial guess (unknown entries), out = solution.
 * info may be NULL.  Returns TPH_OK or TPH_NOT_CONVERGED (or an error). */
tph_status tph_solve(tph_solver* s, double* vx, double* vy, double* p, tph_info* info);

/* Lithostatic pressure (Sec. "Viscosity Rescaling and Initial Guess"): the
 * integral of rho g_y along y, discretely the hydrostatic balance of every
 * y-momentum row for zero velocity, p(i+1, j) - p(i, j) = gy dy (rho_b(i, j-1)
 * + rho_b(i, j)) / 2, with zero mean over the cells.  rho_b and p are device
 * (ny+2) x (nx+2) FP64 arrays; p's ghost and wall entries are written 0.
 * Needs only tph_create. */
tph_status tph_lithostatic_pressure(tph_solver* s, const double* rho_b, double gy, double* p);

/* Continuation solve (Sec. "Viscosity Rescaling and Initial Guess"): for
 * theta in thetas[0..nthetas-1] (non-decreasing in [0, 1], the last equal to
 * 1) the system with the computational viscosity (1 - theta) eta_min + theta
 * eta (eta_min: the smallest of eta_b over the basic nodes and eta_p over the
 * cells, both fields blended) is set up and solved from the previous stage's
 * solution, to max(stage_rtol, desc.rtol) for the intermediate stages (a
 * stage that stops short still hands its iterate on) and to desc.rtol for
 * the last.  lithostatic = 1 starts from zero velocity and the lithostatic
 * pressure (as tph_lithostatic_pressure), 0 from (vx, vy, p) as given.
 * Afterwards the solver holds the original coefficients, as after
 * tph_set_coefficients(eta_b, eta_p, rho_b, gx, gy).  info sums iterations,
 * restarts and times over the stages; res_energy is the last stage's; the
 * history (if given) is the concatenation of the stages'. */
tph_status tph_solve_continuation(tph_solver* s, const double* eta_b, const double* eta_p, const double* rho_b,
                                  double gx, double gy, const double* thetas, int32_t nthetas, double stage_rtol,
                                  int32_t lithostatic, double* vx, double* vy, double* p, tph_info* info);

/* Same with an explicit right-hand side (fx at vx rows, fy at vy rows, fp at
 * continuity rows), replacing the one from tph_set_coefficients for this call
 * only.  Used for the adjoint solve (A is symmetric, A = A^T). */
tph_status tph_solve_rhs(tph_solver* s, const double* fx, const double* fy, const double* fp,
                         double* vx, double* vy, double* p, tph_info* info);

/* (ax, ay, ap) = A (vx, vy, p) in FP64, matrix-free (Ch. 6 point-wise
 * operator and its mirror).  Outputs are zero outside the equation rows. */
tph_status tph_apply(tph_solver* s, const double* vx, const double* vy, const double* p,
                     double* ax, double* ay, double* ap);

/* One application of the Uzawa preconditioner (Sec. "Uzawa Iteration as a
 * Fixed Point Method", M = [[L, 0], [D, (alpha eta_p)^{-1}]]): starting from
 * z = 0, desc.uzawa_steps times z <- z + M^{-1}(r - A z), where one M^{-1}
 * application is z_v = one V-cycle on L z_v = r_v from zero (in the solver's
 * precision) and z_p = alpha eta_p (r_p - D z_v).  With levels = 1 and one
 * step this is the exact block-triangular solve.  Inputs are residual-type
 * arrays, outputs solution-type arrays. */
tph_status tph_precondition(tph_solver* s, const double* rx, const double* ry, const double* rp,
                            double* zx, double* zy, double* zp);

/* z = M^{-1} r exactly as tph_precondition, and w = A z, in one sequence:
 * the exit of every Uzawa step is a single pass over the grid that also
 * forms the next step's right-hand side, and the last one forms w, the
 * product an outer Krylov method needs next (Sec. "Uzawa Iteration as a
 * Fixed Point Method", Sec. "Comparison with FGMRES").  Arrays as in
 * tph_precondition (inputs) and tph_apply (w: zero outside the equation
 * rows). */
tph_status tph_precondition_apply(tph_solver* s, const double* rx, const double* ry, const double* rp,
                                  double* zx, double* zy, double* zp, double* wx, double* wy, double* wp);

/* Relative energy residual of (vx, vy, p) for the right-hand side of
 * tph_set_coefficients (Sec. "Global Relative Energy Residual"). */
tph_status tph_energy_residual(tph_solver* s, const double* vx, const double* vy,
                               const double* p, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual norms of (vx, vy, p) with no solver handle, no allocation, no
 * memset and no host synchronisation.
 *   out[0] = relative energy residual, as tph_energy_residual for a solver
 *            holding (eta_b, eta_p, rho_b, gx, gy) and no extra force;
 *   out[1] = plain relative l2 residual ||b - A x||_2 / ||b||_2, as
 *            tph_info.res_l2.
 * desc: only nx, ny (each in [2, 32768]; larger grids are rejected with
 * TPH_ERR_INVALID), lx, ly and bc are read.  All arrays are DEVICE arrays of
 * the current device in the dense (ny + 2) x (nx + 2) layout of the array
 * convention above (ghost and wall entries of vx, vy are ignored; viscosity
 * must be positive and finite, which is not checked here: a bad entry makes
 * the result NaN).  out: a DEVICE array of 2 doubles, written by a kernel on
 * hip_stream (a hipStream_t; NULL: the null stream); the call returns once
 * the two kernels are enqueued.  Reduction partials live in a 64 KiB
 * library-static device array that each device holds until the process
 * ends; every call on a device shares it, so calls that overlap on one
 * device (two streams, two threads) race and must be serialised by the
 * caller.  Errors: TPH_ERR_INVALID (arguments), TPH_ERR_HIP (launch). */
tph_status tph_energy_residual_noalloc(const tph_desc* desc, const double* eta_b, const double* eta_p,
                                       const double* rho_b, double gx, double gy, const double* vx,
                                       const double* vy, const double* p, double* out, void* hip_stream);

/* Copy the viscosities of multigrid level l (0 = finest) into device arrays
 * of that level's shape ((ny_l + 2) x (nx_l + 2), FP64). */
tph_status tph_level_viscosity(tph_solver* s, int32_t level, double* eta_b, double* eta_p);

/* Number of levels actually used, and level l's cell counts. */
tph_status tph_level_shape(tph_solver* s, int32_t level, int32_t* nx, int32_t* ny);

/* How level l is processed by the fused V-cycle (desc.fused = 1):
 * *kind = 0: one-sweep LDS tile launches (plus the fused residual-restriction),
 *         1: multi-sweep LDS passes, 2: inside the single-workgroup coarse
 *         tail, 3: coarsest level without the coarse tail (dense solve),
 *         4: RAS tile launches;
 * *shape = 1 if its tiles use the small shape.  With desc.fused = 0 every
 * level reports kind 0.  Either output may be NULL. */
tph_status tph_level_plan(tph_solver* s, int32_t level, int32_t* kind, int32_t* shape);

/* Adjoint solve A^T lam = g (A is symmetric, so this is the forward solver
 * with right-hand side g = (gvx, gvy, gp)); lam is written zero-mean in
 * pressure.  Any of gvx, gvy, gp may be NULL (zero). */
tph_status tph_solve_adjoint(tph_solver* s, const double* gvx, const double* gvy, const double* gp,
                             double* lvx, double* lvy, double* lp, tph_info* info);

/* Gradient of a functional J(v, p) with respect to the coefficients, given
 * the forward solution x = (vx, vy, p) and the adjoint lam = (lvx, lvy, lp):
 * dJ/d eta_p(c) = 2 (exx(lam) exx(x) + eyy(lam) eyy(x)) at cell centres,
 * dJ/d eta_b(b) = w_b gamma(lam) gamma(x) at basic nodes (gamma =
 * d vx/dy + d vy/dx with mirrored ghosts; w_b = 1 inside, 1/2 on a no-slip
 * wall), dJ/d rho_b = lam^T df/d rho_b.  Any output may be NULL. */
tph_status tph_coeff_gradient(tph_solver* s, const double* vx, const double* vy, const double* p,
                              const double* lvx, const double* lvy, const double* lp,
                              double* g_eta_b, double* g_eta_p, double* g_rho_b);

/* Kernels that tph_time_kernel can time. */
enum {
    TPH_KERNEL_SMOOTH = 0,   /* one finest-level smoother launch (fused: one full sweep on LDS tiles;
                                otherwise a Jacobi sweep or one GS colour half-sweep; RAS: one
                                outer iteration of ras_inner sweeps) */
    TPH_KERNEL_APPLY = 1,    /* FP64 matrix-free operator apply with energy scaling (Krylov step) */
    TPH_KERNEL_RESIDUAL = 2, /* finest-level velocity residual r - L e in the V-cycle type */
    TPH_KERNEL_RESTRICT = 3, /* finest -> second level residual restriction */
    TPH_KERNEL_PROLONG = 4,  /* second -> finest level prolongation and correction */
    TPH_KERNEL_GCR_STEP = 5, /* flexible GCR step update (Alg. "Flexible GCR(m)"): project and
                                normalise the new direction w against i = restart / 2 earlier
                                ones and update r (FP64, every entry of the vectors; x is
                                updated once per cycle) */
    TPH_KERNEL_AA_MIX = 6,   /* Anderson mixing x = sum_i alpha_i (x_i + beta f_i) over
                                restart + 1 stored pairs (FP64, every entry of the vectors) */
    TPH_KERNEL_LINK = 7      /* one Uzawa link pass (Sec. "Uzawa Iteration as a Fixed Point
                                Method"): z += e with the pressure update, then the next step's
                                FP64 residual or the Krylov apply; live timing only
                                (tph_kernel_timing_target), not tph_time_kernel */
};

/* Measurement hook: run `reps` back-to-back launches of one hot-path kernel
 * on the solver's stream between two HIP events and return the mean
 * duration per launch (*ms_per_launch) and the algorithmic bytes one launch
 * must move (*bytes_per_launch: each field word the operation reads or
 * writes, counted once).  Requires tph_set_coefficients; the kernels operate
 * on the solver's own workspace (the correction arrays, Krylov vectors and
 * the solution held between solves are modified; caller arrays are not). */
tph_status tph_time_kernel(tph_solver* s, int32_t kind, int32_t reps, double* ms_per_launch,
                           double* bytes_per_launch);

/* Measurement hook for the smoother inside real solves.  With enable = k
 * >= 1, every k-th finest-level smoothing launch of the fused V-cycle
 * (desc.fused = 1) made by later solves on this handle is launched with a
 * pair of HIP events that take the kernel's own start and end time stamps
 * (hipExtLaunchKernel; a timed launch delays the stream by a few
 * microseconds, hence the sampling); enable = 0 turns timing off.  Up to
 * 8192 launches are recorded between two reads,
 * later ones are counted in *dropped.  The events are created on the first
 * enable and live as long as the handle.  tph_kernel_timing_read waits for
 * the stream, returns the number of timed launches, their summed duration in
 * ms and their summed algorithmic bytes (per cell: zero-guess sweep 6 words
 * = read r (2), eta_b, eta_p, write e (2); sweep from an iterate 8 words;
 * sweep with fused prolongation 8.5 words, the coarse correction being a
 * quarter of two fields; plus 0.5 when the pass also restricts its residual),
 * then resets the counters. */
tph_status tph_kernel_timing(tph_solver* s, int32_t enable);
/* Kernel class that tph_kernel_timing times: TPH_KERNEL_SMOOTH (default; the
 * finest-level smoothing launches, bytes as above) or TPH_KERNEL_LINK (every
 * Uzawa link pass on the finest level; bytes per cell: e 2 words of the
 * V-cycle type, eta_b, eta_p and the pressure source 3 FP64 words, z_old 3
 * FP64 words after the first step, z written 3 FP64 words, plus r read 3
 * FP64 words and the next right-hand side written 2 V-cycle words + 1 FP64
 * word for a link into the next step, or w written 3 FP64 words for the
 * link into the Krylov apply).  Resets the sampling counter. */
tph_status tph_kernel_timing_target(tph_solver* s, int32_t kind);
tph_status tph_kernel_timing_read(tph_solver* s, int32_t* launches, double* total_ms, double* total_bytes,
                                  int32_t* dropped);

/* Release everything the solver owns.  NULL is allowed. */
void tph_destroy(tph_solver* s);

/* ---------------------------------------------------------------- batches
 * Many independent problems of uneven grid sizes solved together: every
 * V-cycle phase is one launch for the whole batch (work lists of (problem,
 * tile) items), the coarse tails run one workgroup per problem, and the
 * device work of one FGMRES iteration is captured once as a hipGraph and
 * replayed while every problem iterates; once some have converged, the
 * iteration is launched directly over work lists holding only the items of
 * the problems still iterating (converged problems are also masked on the
 * device).  All problems must
 * share precision, smoother, sweep counts (>= 1, nu_growth 1), omega, alpha,
 * eta_mean, restart, max_iters, uzawa_steps, rtol and msweep, use fused
 * kernels, and be large enough to have a coarse tail of at least one level
 * (any grid whose automatic hierarchy has >= 2 levels).  With Gauss-Seidel,
 * msweep selects the depths (bit d = level d of every problem; -1 = none,
 * unlike a single solve) smoothed in multi-sweep passes (FP32: up to two
 * sweeps per pass; FP64: one), the last pre-smoothing pass restricting the
 * residual and the first post-smoothing pass applying the prolongation;
 * tile_shape is not used.  Pointer-array arguments are HOST arrays of `count` DEVICE pointers
 * with the single-problem conventions. */
typedef struct tph_batch tph_batch;

tph_status tph_batch_create(int32_t count, const tph_desc* descs, void* hip_stream, tph_batch** out);
/* gxy: host array of 2 * count doubles (gx, gy per problem). */
tph_status tph_batch_set_coefficients(tph_batch* b, const double* const* eta_b, const double* const* eta_p,
                                      const double* const* rho_b, const double* gxy);
/* vx, vy, p: in = initial guesses, out = solutions; infos: host array of
 * `count` (nullable).  Returns TPH_NOT_CONVERGED if any problem did not. */
tph_status tph_batch_solve(tph_batch* b, double* const* vx, double* const* vy, double* const* p, tph_info* infos);
void tph_batch_destroy(tph_batch* b);

/* Message of the calling thread's last error ("" if none). */
const char* tph_last_error(void);

/* Library version string. */
const char* tph_version(void);

/* ------------------------------------------------------------------------
 * Markers (Ch. 4, Sec. "The Marker-in-Cell Method", Sec. "Interpolation
 * Between Markers and Grid", Sec. "Advection of Lagrangian Markers").
 *
 * Marker positions and values are DEVICE arrays of n FP64 entries (caller
 * owned); positions lie in [0, lx] x [0, ly].  Grid arrays use the dense
 * (ny + 2) x (nx + 2) convention of this header.  Node grids:
 *   TPH_NODES_BASIC (j dx, i dy),                i in [0, ny],     j in [0, nx]
 *   TPH_NODES_CELL  ((j - 1/2) dx, (i - 1/2) dy), i in [1, ny],     j in [1, nx]
 *   TPH_NODES_VX    (j dx, (i - 1/2) dy),         i in [0, ny + 1], j in [0, nx]
 *   TPH_NODES_VY    ((j - 1/2) dx, i dy),         i in [0, ny],     j in [0, nx + 1]
 * (vx and vy include the walls and the mirrored ghosts of a solver output).
 * Bilinear weights of a marker at (x, y) in the cell whose lower-left node
 * is (i, j): (1 - rx)(1 - ry), rx (1 - ry), (1 - rx) ry, rx ry on (i, j),
 * (i, j+1), (i+1, j), (i+1, j+1), with rx = (x - x_j) / dx, ry = (y - y_i) / dy.
 * All work is enqueued on the stream given at creation; tph_markers_sync
 * waits for it.
 * ------------------------------------------------------------------------ */
enum { TPH_NODES_BASIC = 0, TPH_NODES_CELL = 1, TPH_NODES_VX = 2, TPH_NODES_VY = 3 };

typedef struct tph_markers tph_markers;

/* Workspace for an nx x ny grid of size lx x ly and up to `capacity`
 * markers (sort buffers, per-cell ranges and partial sums).  Errors:
 * TPH_ERR_INVALID for bad sizes, TPH_ERR_OOM. */
tph_status tph_markers_create(int32_t nx, int32_t ny, double lx, double ly, int32_t capacity, void* hip_stream,
                              tph_markers** out);
void tph_markers_destroy(tph_markers* h);

/* Marker -> grid, step 1: bin the n markers by the cell of the `kind` node
 * grid (TPH_NODES_BASIC or TPH_NODES_CELL) that contains them, with a stable
 * sort of (cell, marker index).  xm and ym must stay valid and unchanged
 * until the last tph_markers_to_grid of this binning. */
tph_status tph_markers_bin(tph_markers* h, int32_t kind, int32_t n, const double* xm, const double* ym);

/* Marker -> grid, step 2 (any number of fields per binning): grid(i, j) =
 * sum_m w_m(i, j) phi_m / sum_m w_m(i, j) over the binned markers that reach
 * node (i, j) of the binned kind (normalised bilinear average), `fill` where
 * none does; entries outside the kind's node range are not written.
 * Weights that fall on nodes outside the range are dropped (the
 * normalisation absorbs them).  Without atomics: per-cell partial sums in
 * sorted order, then per-node sums of its four cells in a fixed order, so the
 * result is bitwise reproducible. */
tph_status tph_markers_to_grid(tph_markers* h, const double* phi_m, double fill, double* grid);

/* Grid -> marker: phi_m = the bilinear interpolation of the `kind` node
 * grid at each marker (the weights sum to one).  The cell is taken within
 * the kind's node range and rx, ry are clamped to [0, 1] (no
 * extrapolation). */
tph_status tph_markers_from_grid(tph_markers* h, int32_t kind, int32_t n, const double* xm, const double* ym,
                                 const double* grid, double* phi_m);

/* One classical RK4 step (eq. rk4_method) of dx/dt = v(x) for n markers, in
 * place, with v interpolated from the staggered velocity arrays vx, vy (a
 * solver output: walls and ghosts set) as in tph_markers_from_grid; every
 * stage position and the result are clamped to [0, lx] x [0, ly]. */
tph_status tph_markers_advect_rk4(tph_markers* h, int32_t n, double* xm, double* ym, const double* vx,
                                  const double* vy, double dt);

/* Wait for the marker stream (reports any device error). */
tph_status tph_markers_sync(tph_markers* h);

#ifdef __cplusplus
}
#endif
#endif /* TEPHRA_H */
