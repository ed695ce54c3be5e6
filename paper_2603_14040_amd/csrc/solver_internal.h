// Internal interface between the single-problem solver (solver.cpp) and the
// batched driver (batch.hip): a read-only view of one solver's workspace and
// the load / finish steps of a solve.  Not part of the public C ABI.
#pragma once
#include <string>

#include "../../include/tephra.h"
#include "common.h"

struct TphSolverView {
    int nlev;
    int lc;                       // level of the single-workgroup coarse tail (-1: none)
    size_t lc_lds;                // its LDS bytes
    int ncoarse;                  // unknowns of the coarsest level
    tph::Geom g[tph::kMaxLevels];
    void* eb[tph::kMaxLevels];    // viscosities in the V-cycle type
    void* ep[tph::kMaxLevels];
    void* ex[tph::kMaxLevels][2];
    void* ey[tph::kMaxLevels][2];
    void* rx[tph::kMaxLevels];
    void* ry[tph::kMaxLevels];
    int nu_pre[tph::kMaxLevels];
    int nu_post[tph::kMaxLevels];
    const double* Minv;
    const double* eb64;           // finest-level FP64 viscosities
    const double* ep64;
    double* x;                    // raw three-field vectors (allocation starts)
    double* b;
    double* V;                    // restart + 1 basis vectors, stride n3
    double* Z;
    double* t1;                   // scratch vectors (the Uzawa link's second z and pressure residual)
    double* t2;
    double* t3;
    size_t F, n3;
};

TphSolverView tph_internal_view(const tph_solver* s);
void tph_internal_set_error(const std::string& msg);
// copy an initial guess in (walls zeroed, ghosts mirrored)
tph_status tph_internal_load_solution(tph_solver* s, const double* vx, const double* vy, const double* p);
// coefficient setup of one problem, enqueued on its stream without the
// coarsest factorisation (the batch factors every problem in one launch),
// and its completion (waits for the stream, checks the coefficients)
tph_status tph_internal_setup_enqueue(tph_solver* s, const double* eta_b, const double* eta_p, const double* rho_b,
                                      double gx, double gy);
tph_status tph_internal_setup_finish(tph_solver* s);
// rounding floor of the relative energy residual of the solver's current
// iterate (waits for its stream)
tph_status tph_internal_rounding_floor(tph_solver* s, double bnorm, double* out);
// plain relative l2 residual of the solution held by the solver: enqueue the
// reductions on its stream, read the value after that stream has drained
tph_status tph_internal_plain_residual_enqueue(tph_solver* s);
double tph_internal_plain_residual_read(const tph_solver* s);
// remove the pressure mean of the solution and copy it out
tph_status tph_internal_finish_solution(tph_solver* s, double* vx, double* vy, double* p);
