"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (relative, as stated for this path): operator apply, energy
residual and coarse viscosities to rounding (<= 1e-13 / 1e-12); one FP64
preconditioner application to <= 1e-11, FP32 to <= 2e-5; solutions at a
1e-12 energy-residual target to <= 1e-7 (FP64) and <= 1e-6 (mixed) in the
relative L2 norm of velocity and of zero-mean pressure.
"""
import math

import numpy as np
import pytest
import torch

import paper_2603_14040_amd as tph
import workloads as wl
from oracle import adjoint as adj
from oracle import multigrid as mg
from oracle import stokes as st

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# One FP32 preconditioner application against the FP64 oracle: every output
# entry depends on a chain of at most S = steps * sum_l (nu_pre,l + nu_post,l
# + 2) FP32 stages (sweeps, transfers and casts), each adding a relative
# error of a few u = 2^-24 that the contractive cycle does not amplify.  The
# longest chain here is S = 68 (2 Uzawa steps, 3 levels, sweeps 2, 4, 8);
# with 4 u per stage, 68 * 4 * 6e-8 = 1.6e-5 < 2e-5.  The cases measure
# <= 4.6e-6.
FP32_PRECOND_TOL = 2e-5


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def solver_for(nx, ny, lx=1.0, ly=1.0, bc=(0, 0, 0, 0), **kw):
    print(f"[case] solver {nx}x{ny} lx={lx} ly={ly} bc={bc} {kw}", flush=True)
    return tph.Solver(nx, ny, lx, ly, bc=bc, device=DEV, **kw)


@pytest.mark.parametrize("shape,bc,ls", [((8, 8), (0, 0, 0, 0), (1.0, 1.0)),
                                         ((13, 7), (1, 1, 1, 1), (1.0, 1.3)),
                                         ((200, 96), (1, 0, 0, 1), (2.0, 1.0)),
                                         ((64, 64), (0, 1, 1, 0), (1.0, 1.0))])
def test_apply_matches_oracle_spmv(shape, bc, ls):
    nx, ny = shape
    eb, ep, rho = wl.random_fields(nx, ny, seed=nx + ny, eta_decades=3)
    vx, vy, p = wl.random_state(nx, ny, seed=3)
    g = st.Grid(nx, ny, ls[0], ls[1], bc)
    s = solver_for(nx, ny, ls[0], ls[1], bc, precision=tph.FP64)
    s.set_coefficients(T(eb), T(ep), T(rho), 0.3, -1.0)
    ax, ay, ap = s.apply(T(vx), T(vy), T(p))
    rx, ry, rp = st.apply(g, eb, ep, vx, vy, p)
    for got, ref in ((ax, rx), (ay, ry), (ap, rp)):
        assert relmax(N(got), ref) < 1e-13


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 0, 1, 0)])
def test_energy_residual_matches_oracle(bc):
    nx, ny = 48, 40
    eb, ep, rho = wl.random_fields(nx, ny, seed=5, eta_decades=2)
    vx, vy, p = wl.random_state(nx, ny, seed=8)
    g = st.Grid(nx, ny, 1.0, 1.0, bc)
    s = solver_for(nx, ny, bc=bc, precision=tph.FP64)
    s.set_coefficients(T(eb), T(ep), T(rho), 0.2, -1.0)
    got = s.energy_residual(T(vx), T(vy), T(p))
    A = st.assemble(g, eb, ep)
    b = st.rhs(g, rho, 0.2, -1.0)
    ref = st.energy_residual(g, A, st.to_vector(g, vx, vy, p), b, ep)
    assert got == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("mean", [tph.MEAN_ARITHMETIC, tph.MEAN_GEOMETRIC])
def test_level_viscosities_match_oracle(mean):
    nx, ny = 96, 64
    eb, ep, rho = wl.random_fields(nx, ny, seed=12, eta_decades=4)
    s = solver_for(nx, ny, precision=tph.MIXED, levels=4, eta_mean=mean)
    s.set_coefficients(T(eb), T(ep), T(rho))
    g = st.Grid(nx, ny)
    cb, cp = eb, ep
    for l in range(1, 4):
        cb, cp = mg.coarse_viscosity(g, cb, cp, "geometric" if mean == tph.MEAN_GEOMETRIC else "arithmetic")
        g = mg.coarsen(g)
        gb, gp = s.level_viscosity(l)
        gb, gp = N(gb), N(gp)
        assert relmax(gb[:g.ny + 1, :g.nx + 1], cb[:g.ny + 1, :g.nx + 1]) < 1e-13
        assert relmax(gp[1:g.ny + 1, 1:g.nx + 1], cp[1:g.ny + 1, 1:g.nx + 1]) < 1e-13


PRECOND_CASES = [
    # (nx, ny, bc, levels, smoother, nu, growth, omega, alpha, steps)
    (16, 16, (0, 0, 0, 0), 1, tph.SMOOTH_JACOBI, 1, 1.0, 0.6, 1.0, 1),
    (16, 16, (0, 0, 0, 0), 2, tph.SMOOTH_JACOBI, 1, 1.0, 0.6, 1.0, 1),
    (32, 24, (1, 1, 0, 0), 3, tph.SMOOTH_JACOBI, 2, 2.0, 0.6, 1.5, 1),
    (32, 32, (0, 0, 0, 0), 3, tph.SMOOTH_GS, 2, 2.0, 1.0, 1.0, 2),
    (80, 48, (0, 1, 1, 0), 4, tph.SMOOTH_GS, 1, 2.0, 0.9, 2.0, 1),
    (130, 34, (1, 0, 0, 1), 2, tph.SMOOTH_JACOBI, 0, 1.0, 0.6, 1.0, 1),
    # sizes that run the LDS-tiled fine-level kernels (ragged tiles), the
    # fused residual-restriction and the single-workgroup coarse tail
    (256, 192, (0, 0, 0, 0), 4, tph.SMOOTH_GS, 2, 1.0, 1.0, 1.0, 2),
    (200, 72, (1, 0, 1, 1), 3, tph.SMOOTH_GS, 1, 1.0, 0.9, 1.0, 1),
    (192, 128, (0, 1, 0, 1), 3, tph.SMOOTH_JACOBI, 2, 1.0, 0.7, 1.2, 3),
    (136, 136, (1, 1, 1, 1), 4, tph.SMOOTH_GS, 3, 1.0, 1.0, 1.0, 1),
]


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
@pytest.mark.parametrize("case", PRECOND_CASES)
def test_preconditioner_matches_oracle_vcycle(case, prec, fused):
    nx, ny, bc, levels, sm, nu, growth, omega, alpha, steps = case
    eb, ep, rho = wl.random_fields(nx, ny, seed=nx * 7 + ny, eta_decades=2)
    rx, ry, rp = wl.random_state(nx, ny, seed=nx + 1)
    s = solver_for(nx, ny, bc=bc, precision=prec, levels=levels, smoother=sm, nu_pre=nu, nu_post=nu,
                   nu_growth=growth, omega=omega, alpha=alpha, uzawa_steps=steps, fused=bool(fused))
    s.set_coefficients(T(eb), T(ep), T(rho))
    zx, zy, zp = s.precondition(T(rx), T(ry), T(rp))
    sched = [min(256, math.ceil(nu * growth ** l - 1e-9)) for l in range(levels)]
    prm = mg.MGParams(levels=levels, nu_pre=sched, nu_post=sched, omega=omega,
                      smoother="jacobi" if sm == tph.SMOOTH_JACOBI else "gs", alpha=alpha)
    g = st.Grid(nx, ny, 1.0, 1.0, bc)
    levs = mg.build_hierarchy(g, eb, ep, prm)
    if steps == 1:
        ox, oy, op = mg.precondition(levs, prm, rx, ry, rp)
    else:
        ox, oy, op = mg.uzawa_preconditioner(levs, prm, st.assemble(g, eb, ep), rx, ry, rp, steps)
    tol = 1e-11 if prec == tph.FP64 else FP32_PRECOND_TOL
    gx_, gy_, gp_ = N(zx), N(zy), N(zp)
    v_ref = np.concatenate([ox[1:ny + 1, 1:nx].ravel(), oy[1:ny, 1:nx + 1].ravel()])
    v_got = np.concatenate([gx_[1:ny + 1, 1:nx].ravel(), gy_[1:ny, 1:nx + 1].ravel()])
    ev = np.linalg.norm(v_got - v_ref) / np.linalg.norm(v_ref)
    epr = np.linalg.norm(gp_[1:ny + 1, 1:nx + 1] - op[1:ny + 1, 1:nx + 1]) / np.linalg.norm(op[1:ny + 1, 1:nx + 1])
    print(f"[precond] rel err v {ev:.2e} p {epr:.2e}", flush=True)
    assert ev < tol and epr < tol
    # output contract: walls zero, ghosts mirrored
    assert np.all(gx_[:, 0] == 0) and np.all(gx_[:, nx] == 0)
    assert np.array_equal(gx_[0, 1:nx], (1 if bc[2] == 0 else -1) * gx_[1, 1:nx])
    assert np.array_equal(gy_[1:ny, nx + 1], (1 if bc[1] == 0 else -1) * gy_[1:ny, nx])


@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
def test_large_coarsest_system_matches_oracle_vcycle(prec):
    """A hierarchy whose coarsest level (32 x 38 cells, 2362 unknowns) is too
    large for the one-workgroup inverse and for the coarse tail: the
    device-wide Gauss-Jordan and the row-parallel dense solve give the
    oracle's V-cycle (exact coarsest solve)."""
    nx, ny, levels = 512, 608, 5
    eb, ep, rho = wl.random_fields(nx, ny, seed=71, eta_decades=2)
    rx, ry, rp = wl.random_state(nx, ny, seed=72)
    s = solver_for(nx, ny, bc=(1, 0, 0, 1), precision=prec, levels=levels, nu_pre=1, nu_post=1, omega=1.0,
                   alpha=1.0, uzawa_steps=1)
    s.set_coefficients(T(eb), T(ep), T(rho))
    zx, zy, zp = (N(t) for t in s.precondition(T(rx), T(ry), T(rp)))
    prm = mg.MGParams(levels=levels, nu_pre=[1] * levels, nu_post=[1] * levels, omega=1.0, smoother="gs",
                      alpha=1.0)
    g = st.Grid(nx, ny, 1.0, 1.0, (1, 0, 0, 1))
    ox, oy, op = mg.precondition(mg.build_hierarchy(g, eb, ep, prm), prm, rx, ry, rp)
    v_ref = np.concatenate([ox[1:ny + 1, 1:nx].ravel(), oy[1:ny, 1:nx + 1].ravel()])
    v_got = np.concatenate([zx[1:ny + 1, 1:nx].ravel(), zy[1:ny, 1:nx + 1].ravel()])
    ev = np.linalg.norm(v_got - v_ref) / np.linalg.norm(v_ref)
    epr = np.linalg.norm(zp[1:ny + 1, 1:nx + 1] - op[1:ny + 1, 1:nx + 1]) / np.linalg.norm(op[1:ny + 1, 1:nx + 1])
    print(f"[large coarsest] prec={prec} rel err v {ev:.2e} p {epr:.2e}", flush=True)
    tol = 1e-11 if prec == tph.FP64 else FP32_PRECOND_TOL
    assert ev < tol and epr < tol


# level plans of the fused V-cycle: (msweep mask, tile_shape mask, coarse_level);
# -1 = library default, coarse_level -2 = no single-workgroup coarse tail
PLANS = [(0, 0, -1), (-1, -1, -1), (0xFFFF, 0, -2), (0xFFFF, 0xFFFF, -1), (0, 0xFFFF, -2)]


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
@pytest.mark.parametrize("case", [c for c in PRECOND_CASES if c[4] == tph.SMOOTH_GS])
def test_multisweep_plans_match_oracle_vcycle(case, prec, plan):
    """Multi-sweep passes (two Gauss-Seidel sweeps per launch, residual and
    restriction fused into the last pre-smoothing pass, prolongation into the
    first post-smoothing pass) on every level, on none, and with either tile
    shape: the same V-cycle as the oracle's."""
    nx, ny, bc, levels, sm, nu, growth, omega, alpha, steps = case
    eb, ep, rho = wl.random_fields(nx, ny, seed=nx * 5 + ny, eta_decades=2)
    rx, ry, rp = wl.random_state(nx, ny, seed=nx + 3)
    msw, shp, cl = plan
    s = solver_for(nx, ny, bc=bc, precision=prec, levels=levels, smoother=sm, nu_pre=nu, nu_post=nu,
                   nu_growth=growth, omega=omega, alpha=alpha, uzawa_steps=steps, fused=True, msweep=msw,
                   tile_shape=shp, coarse_level=cl)
    s.set_coefficients(T(eb), T(ep), T(rho))
    zx, zy, zp = s.precondition(T(rx), T(ry), T(rp))
    sched = [min(256, math.ceil(nu * growth ** l - 1e-9)) for l in range(levels)]
    prm = mg.MGParams(levels=levels, nu_pre=sched, nu_post=sched, omega=omega, smoother="gs", alpha=alpha)
    g = st.Grid(nx, ny, 1.0, 1.0, bc)
    levs = mg.build_hierarchy(g, eb, ep, prm)
    if steps == 1:
        ox, oy, op = mg.precondition(levs, prm, rx, ry, rp)
    else:
        ox, oy, op = mg.uzawa_preconditioner(levs, prm, st.assemble(g, eb, ep), rx, ry, rp, steps)
    tol = 1e-11 if prec == tph.FP64 else FP32_PRECOND_TOL
    gx_, gy_, gp_ = N(zx), N(zy), N(zp)
    v_ref = np.concatenate([ox[1:ny + 1, 1:nx].ravel(), oy[1:ny, 1:nx + 1].ravel()])
    v_got = np.concatenate([gx_[1:ny + 1, 1:nx].ravel(), gy_[1:ny, 1:nx + 1].ravel()])
    ev = np.linalg.norm(v_got - v_ref) / np.linalg.norm(v_ref)
    epr = np.linalg.norm(gp_[1:ny + 1, 1:nx + 1] - op[1:ny + 1, 1:nx + 1]) / np.linalg.norm(op[1:ny + 1, 1:nx + 1])
    print(f"[msweep {plan}] rel err v {ev:.2e} p {epr:.2e}", flush=True)
    assert ev < tol and epr < tol
    assert np.all(gx_[:, 0] == 0) and np.all(gx_[:, nx] == 0)
    assert np.array_equal(gx_[0, 1:nx], (1 if bc[2] == 0 else -1) * gx_[1, 1:nx])
    assert np.array_equal(gy_[1:ny, nx + 1], (1 if bc[1] == 0 else -1) * gy_[1:ny, nx])


@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
@pytest.mark.parametrize("steps", [1, 2, 3, 4])
def test_precondition_apply_matches_separate_kernels(prec, steps):
    """The linked Uzawa exits (one pass per step, the last also forming A z)
    give the preconditioner of the separate exit / residual / entry kernels,
    and w = A z."""
    nx, ny, bc = 200, 72, (1, 0, 1, 1)
    eb, ep, rho = wl.random_fields(nx, ny, seed=91 + steps, eta_decades=2)
    rx, ry, rp = wl.random_state(nx, ny, seed=17 + steps)
    s = solver_for(nx, ny, bc=bc, precision=prec, uzawa_steps=steps, alpha=1.5)
    s.set_coefficients(T(eb), T(ep), T(rho))
    z_ref = [N(t) for t in s.precondition(T(rx), T(ry), T(rp))]
    z, w = s.precondition_apply(T(rx), T(ry), T(rp))
    z = [N(t) for t in z]
    w = [N(t) for t in w]
    w_ref = [N(t) for t in s.apply(*[T(t) for t in z])]
    tol = 1e-12 if prec == tph.FP64 else 2e-5
    sl = [np.s_[1:ny + 1, 1:nx], np.s_[1:ny, 1:nx + 1], np.s_[1:ny + 1, 1:nx + 1]]
    for a, b_, q in zip(z, z_ref, sl):
        err = relmax(a[q], b_[q])
        print(f"[link] z rel max err {err:.2e}", flush=True)
        assert err < tol
    for a, b_, q in zip(w, w_ref, sl):
        assert relmax(a[q], b_[q]) < 1e-12
    # output contract of z: ghosts mirrored, walls zero
    assert np.all(z[0][:, 0] == 0) and np.all(z[0][:, nx] == 0)
    assert np.array_equal(z[0][0, 1:nx], (1 if bc[2] == 0 else -1) * z[0][1, 1:nx])


def _check_solution_contract(nx, ny, bc, vx, vy, p):
    assert np.all(vx[:, 0] == 0) and np.all(vx[:, nx] == 0)
    assert np.all(vy[0, :] == 0) and np.all(vy[ny, :] == 0)
    ms, mn = (1 if bc[2] == 0 else -1), (1 if bc[3] == 0 else -1)
    assert np.array_equal(vx[0, 1:nx], ms * vx[1, 1:nx])
    assert np.array_equal(vx[ny + 1, 1:nx], mn * vx[ny, 1:nx])
    mw, me = (1 if bc[0] == 0 else -1), (1 if bc[1] == 0 else -1)
    assert np.array_equal(vy[1:ny, 0], mw * vy[1:ny, 1])
    assert np.array_equal(vy[1:ny, nx + 1], me * vy[1:ny, nx])
    pc = p[1:ny + 1, 1:nx + 1]
    assert abs(pc.mean()) <= 1e-12 * max(np.abs(pc).max(), 1e-300)


SOLVE_CASES = [
    ("sinker64", lambda: wl.sinker(64)),
    ("grf128", lambda: wl.random_viscosity(128)),
    ("noslip_rect", lambda: wl.sinker(48, ny=32, lx=1.5, ly=1.0, bc=(1, 1, 0, 1), gx=0.3, gy=-1.0,
                                      center=(0.7, 0.4), radius=0.15, eta_in=50.0)),
]


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
@pytest.mark.parametrize("name,make", SOLVE_CASES)
def test_solve_matches_oracle(name, make, prec, fused):
    pr = make()
    g = st.Grid(pr.nx, pr.ny, pr.lx, pr.ly, pr.bc)
    ref = st.solve(g, pr.eta_b, pr.eta_p, pr.rho_b, pr.gx, pr.gy)
    s = solver_for(pr.nx, pr.ny, pr.lx, pr.ly, pr.bc, precision=prec, rtol=1e-12, max_iters=2000,
                   fused=bool(fused))
    s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b), pr.gx, pr.gy)
    vx, vy, p, info = s.solve()
    # 1e-12 can sit below the FP64 rounding floor of the residual: either it is
    # reached, or the solver stops on stagnation within a few restarts
    assert info.status == "TPH_OK" or (info.res_energy < 1e-10 and info.restarts < 40)
    print(f"[{name}] prec={prec} iters={info.iters} restarts={info.restarts} res={info.res_energy:.3e}", flush=True)
    vx, vy, p = N(vx), N(vy), N(p)
    ev, ep_ = st.parity_errors(g, ref, vx, vy, p)
    tol = 1e-7 if prec == tph.FP64 else 1e-6
    print(f"[{name}] rel L2 v={ev:.3e} p={ep_:.3e}", flush=True)
    assert ev < tol and ep_ < tol
    _check_solution_contract(pr.nx, pr.ny, pr.bc, vx, vy, p)
    # the GPU-reported energy residual agrees with the oracle's for the returned fields
    A = st.assemble(g, pr.eta_b, pr.eta_p)
    b = st.rhs(g, pr.rho_b, pr.gx, pr.gy)
    oracle_res = st.energy_residual(g, A, st.to_vector(g, vx, vy, p), b, pr.eta_p)
    assert oracle_res < 1e-10


@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
def test_sinker_config_converges_to_1e8(prec):
    pr = wl.sinker(64)
    s = solver_for(64, 64, precision=prec)        # defaults: 4 levels, rtol 1e-8
    assert s.levels == 4
    s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b), pr.gx, pr.gy)
    vx, vy, p, info = s.solve(history=500)
    assert info.status == "TPH_OK" and info.res_energy <= 1e-8
    assert all(b <= a * 1.000001 for a, b in zip(info.history, info.history[1:]))  # FGMRES is monotone
    g = st.Grid(64, 64)
    A = st.assemble(g, pr.eta_b, pr.eta_p)
    b = st.rhs(g, pr.rho_b, pr.gx, pr.gy)
    oracle_res = st.energy_residual(g, A, st.to_vector(g, N(vx), N(vy), N(p)), b, pr.eta_p)
    assert oracle_res <= 1.0001e-8
    # the library's own energy residual (device reductions) agrees with the oracle's
    assert info.res_energy == pytest.approx(oracle_res, rel=1e-4)
    assert s.energy_residual(vx, vy, p) == pytest.approx(oracle_res, rel=1e-6)


def test_full_size_random_viscosity_residual_property():
    """1024^2 random-viscosity problem in the benchmark configuration: the
    oracle's assembled operator confirms the relative energy residual of the
    mixed-precision result, and FP64 and mixed solutions agree."""
    pr = wl.random_viscosity(1024)
    g = st.Grid(1024, 1024)
    sols = {}
    for prec in (tph.MIXED, tph.FP64):
        s = solver_for(1024, 1024, precision=prec)
        s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b), pr.gx, pr.gy)
        vx, vy, p, info = s.solve()
        print(f"[grf1024] prec={prec} iters={info.iters} res={info.res_energy:.3e} t={info.t_solve_ms:.1f}ms",
              flush=True)
        assert info.status == "TPH_OK"
        sols[prec] = (N(vx), N(vy), N(p))
        s.close()
    A = st.assemble(g, pr.eta_b, pr.eta_p)
    b = st.rhs(g, pr.rho_b, pr.gx, pr.gy)
    for prec, (vx, vy, p) in sols.items():
        assert st.energy_residual(g, A, st.to_vector(g, vx, vy, p), b, pr.eta_p) <= 1.0001e-8
    (ax, ay, ap), (bx, by, bp) = sols[tph.MIXED], sols[tph.FP64]
    v1 = np.concatenate([ax.ravel(), ay.ravel()])
    v2 = np.concatenate([bx.ravel(), by.ravel()])
    # both satisfy the 1e-8 energy-residual target; their difference is bounded
    # by the conditioning, checked loosely here
    assert np.linalg.norm(v1 - v2) / np.linalg.norm(v2) < 1e-4


def test_solve_is_deterministic():
    pr = wl.random_viscosity(64)
    s = solver_for(64, 64, precision=tph.MIXED)
    s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b))
    a = [N(t).copy() for t in s.solve()[:3]]
    b = [N(t).copy() for t in s.solve()[:3]]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_not_converged_is_reported():
    pr = wl.sinker(64)
    s = solver_for(64, 64, precision=tph.FP64, max_iters=3)
    s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b))
    vx, vy, p, info = s.solve()
    assert info.status == "TPH_NOT_CONVERGED" and info.iters == 3 and info.res_energy > 1e-8
    with pytest.raises(tph.TephraError):
        s.solve(raise_on_fail=True)


def test_invalid_coefficients_rejected():
    pr = wl.sinker(32)
    s = solver_for(32, 32)
    bad = pr.eta_p.copy()
    bad[5, 7] = 0.0
    with pytest.raises(tph.TephraError, match="TPH_ERR_INVALID"):
        s.set_coefficients(T(pr.eta_b), T(bad), T(pr.rho_b))
    badr = pr.rho_b.copy()
    badr[3, 3] = np.nan
    with pytest.raises(tph.TephraError, match="TPH_ERR_NONFINITE"):
        s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(badr))
    with pytest.raises(tph.TephraError, match="TPH_ERR_INVALID"):
        s.solve()                 # no valid coefficients loaded
    s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b))
    assert s.solve()[3].status == "TPH_OK"


@pytest.mark.parametrize("n", [32, 64, 128])
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1)])
def test_adjoint_gradient_matches_oracle(bc, n):
    """Misfit gradient with respect to eta_b, eta_p and rho_b from the FP64
    forward + adjoint solves and the gradient kernel, against the oracle's
    adjoint (direct solves, term-by-term derivative of the assembled
    operator): <= 1e-7 relative L2 per field."""
    base = wl.random_viscosity(n, ell=0.15, contrast=100.0)
    base.bc = bc
    g = st.Grid(n, n, 1.0, 1.0, bc)
    rng = np.random.default_rng(9)
    target = 0.01 * rng.standard_normal(n - 1)
    ref = adj.gradient(g, base.eta_b, base.eta_p, base.rho_b, 0.2, -1.0, target)
    s = solver_for(n, n, bc=bc, precision=tph.FP64, rtol=1e-13, max_iters=4000)
    eb = T(base.eta_b).requires_grad_(True)
    ep = T(base.eta_p).requires_grad_(True)
    rho = T(base.rho_b).requires_grad_(True)
    vx, vy, p = tph.StokesFunction.apply(eb, ep, rho, s, 0.2, -1.0)
    tt = T(target)
    J = 0.5 * g.dx * torch.sum((vx[n, 1:n] - tt) ** 2)
    assert float(J) == pytest.approx(ref["J"], rel=1e-7)
    J.backward()
    for got, key, sl in ((eb.grad, "g_eta_b", (slice(0, n + 1), slice(0, n + 1))),
                         (ep.grad, "g_eta_p", (slice(1, n + 1), slice(1, n + 1))),
                         (rho.grad, "g_rho_b", (slice(0, n + 1), slice(0, n + 1)))):
        a, b = N(got)[sl], ref[key][sl]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"[adjoint] n={n} bc={bc} {key} rel err {err:.2e}", flush=True)
        assert err < 1e-7, key


def test_adjoint_uses_the_forward_operator():
    """Two forwards on one solver, then the backward of the first: the
    gradient is that of the first problem's operator (the saved forward
    coefficients are loaded again), equal to a fresh single forward/backward."""
    n = 32
    p1 = wl.random_viscosity(n, ell=0.15, contrast=100.0)
    p2 = wl.random_viscosity(n, ell=0.1, contrast=1000.0, seed_field=77)
    s = solver_for(n, n, precision=tph.FP64, rtol=1e-13, max_iters=4000)

    def grads(order):
        outs = {}
        for k in order:
            pr = (p1, p2)[k]
            eb = T(pr.eta_b).requires_grad_(True)
            vx, vy, p = tph.StokesFunction.apply(eb, T(pr.eta_p), T(pr.rho_b), s, 0.0, -1.0)
            outs[k] = (eb, torch.sum(vx[n, 1:n] ** 2))
        return outs

    fresh = grads([0])
    fresh[0][1].backward()
    ref = N(fresh[0][0].grad)
    both = grads([0, 1])
    both[0][1].backward()                   # first problem's graph, after the second forward
    got = N(both[0][0].grad)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10


def test_adjoint_raises_when_the_forward_solve_does_not_converge():
    n = 32
    pr = wl.random_viscosity(n, ell=0.15, contrast=100.0)
    s = solver_for(n, n, precision=tph.FP64, rtol=1e-12, max_iters=2)
    eb = T(pr.eta_b).requires_grad_(True)
    with pytest.raises(tph.TephraError, match="did not converge"):
        tph.StokesFunction.apply(eb, T(pr.eta_p), T(pr.rho_b), s, 0.0, -1.0)


@pytest.mark.parametrize("steps,nu,msweep", [(1, 2, -1), (2, 2, 0b10), (3, 2, -1), (2, 1, 0b10), (2, 3, 0b10),
                                             (2, 2, 0), (2, 3, 0b101), (3, 1, 0b111)])
@pytest.mark.parametrize("prec", [tph.FP64, tph.MIXED])
def test_batched_solve_matches_oracle(prec, steps, nu, msweep):
    """Uneven problems in one batch: each result matches its own oracle solve
    (1, 2 and 3 Uzawa steps: the link passes alternate z between two buffers,
    so odd and even step counts end differently; 1-3 sweeps with multi-sweep
    passes on no depth (the batch default), on every depth but the finest,
    on chosen depths and on every depth, which changes the buffers each depth
    ends in).  The problems need different iteration counts, so the later
    iterations run over work lists compacted to the problems still
    iterating, and the second solve starts again from the full lists."""
    probs = [wl.sinker(64, radius=0.12, eta_in=30.0),
             wl.sinker(32, radius=0.2, eta_in=10.0),
             wl.random_viscosity(64, ell=0.15, contrast=100.0),
             wl.sinker(128, radius=0.08, eta_in=1e3),
             wl.sinker(48, ny=32, lx=1.5, ly=1.0, center=(0.6, 0.5), eta_in=5.0),
             wl.sinker(64, radius=0.15, eta_in=200.0, bc=(1, 1, 0, 1))]
    shapes = [(p.nx, p.ny, p.lx, p.ly, p.bc) for p in probs]
    print(f"[batch] prec={prec} steps={steps} nu={nu} msweep={msweep} shapes={shapes}", flush=True)
    bat = tph.Batch(shapes, device=DEV, precision=prec, rtol=1e-11, max_iters=2000, restart=16, uzawa_steps=steps,
                    nu_pre=nu, nu_post=nu, msweep=msweep)
    bat.set_coefficients([T(p.eta_b) for p in probs], [T(p.eta_p) for p in probs],
                         [T(p.rho_b) for p in probs], [(p.gx, p.gy) for p in probs])
    vx, vy, pp, infos = bat.solve()
    for k, pr in enumerate(probs):
        g = st.Grid(pr.nx, pr.ny, pr.lx, pr.ly, pr.bc)
        ref = st.solve(g, pr.eta_b, pr.eta_p, pr.rho_b, pr.gx, pr.gy)
        ev, epr = st.parity_errors(g, ref, N(vx[k]), N(vy[k]), N(pp[k]))
        print(f"[batch] problem {k} {pr.nx}x{pr.ny}: iters {infos[k].iters} res {infos[k].res_energy:.2e} "
              f"err v {ev:.2e} p {epr:.2e}", flush=True)
        tol = 1e-7 if prec == tph.FP64 else 1e-6
        assert infos[k].res_energy < 1e-10
        assert ev < tol and epr < tol
        assert infos[k].vcycles == infos[k].iters * steps
        assert 0.0 <= infos[k].res_l2 < 1e-6
        _check_solution_contract(pr.nx, pr.ny, pr.bc, N(vx[k]), N(vy[k]), N(pp[k]))
    # the problems stop at different iterations: the compacted work lists were used
    assert len({i.iters for i in infos}) > 1
    # a second solve on the same batch (graph replay, masks and full lists reset) gives the same answer
    vx2, vy2, pp2, infos2 = bat.solve()
    for k in range(len(probs)):
        assert np.array_equal(N(vx[k]), N(vx2[k])) and np.array_equal(N(pp[k]), N(pp2[k]))
    bat.close()


def _eta_from_logvisc(m, n):
    """eta_p = 10**m at cell centres; eta_b = 10**(mean of m over the touching cells) (torch, differentiable)."""
    ep = torch.ones((n + 2, n + 2), dtype=torch.float64, device=m.device)
    ep = ep.index_put((torch.arange(1, n + 1, device=m.device)[:, None],
                       torch.arange(1, n + 1, device=m.device)[None, :]), 10.0 ** m)
    mp = torch.nn.functional.pad(m, (1, 1, 1, 1))
    one = torch.nn.functional.pad(torch.ones_like(m), (1, 1, 1, 1))
    s = mp[:-1, :-1] + mp[1:, :-1] + mp[:-1, 1:] + mp[1:, 1:]
    c = one[:-1, :-1] + one[1:, :-1] + one[:-1, 1:] + one[1:, 1:]
    eb = torch.nn.functional.pad(10.0 ** (s / c), (0, 1, 0, 1), value=1.0)
    return eb, ep


def test_adjoint_gradient_finite_differences_full_size():
    """Surface-velocity misfit on the 1024^2 random field: d J / d log10(eta)
    from the adjoint solve against central differences (h = 1e-3) on 64
    seeded cells, all solves mixed precision at a tight tolerance.

    A one-cell perturbation moves the surface velocity by a tiny fraction of
    its size, so two independent solves to a residual relative to ||b||
    would difference away most of their digits.  Each perturbed solution is
    therefore formed as v0 + d with A(m +- h) d = b - A(m +- h) v0 (v0: the
    solution at m): exactly the perturbed solution, with a solver error
    relative to the small correction instead of to v."""
    n = 1024
    base, m, m_true, cells = wl.adjoint_problem(n)
    s = solver_for(n, n, precision=tph.MIXED, rtol=1e-11, max_iters=3000)
    rho = T(base.rho_b)
    gx, gy = base.gx, base.gy
    eb_t, ep_t = wl.logvisc_to_eta(m_true, n, n)
    s.set_coefficients(T(eb_t), T(ep_t), rho, gx, gy)
    target = s.solve()[0][n, 1:n].clone()

    def J_of_v(vx):
        return 0.5 * (1.0 / n) * torch.sum((vx[n, 1:n] - target) ** 2)

    def J_of(mm):
        eb, ep = _eta_from_logvisc(mm, n)
        vx, vy, p = tph.StokesFunction.apply(eb, ep, rho, s, gx, gy)
        return J_of_v(vx)

    mt = T(m).requires_grad_(True)
    J = J_of(mt)
    J.backward()
    grad = N(mt.grad)
    gmax = np.abs(grad).max()
    # base solution and right-hand side b = (-g rho averaged to the velocity nodes, 0)
    with torch.no_grad():
        eb0, ep0 = _eta_from_logvisc(T(m), n)
        s.set_coefficients(eb0, ep0, rho, gx, gy)
        vx0, vy0, p0, _ = s.solve()
        bx, by = torch.zeros_like(rho), torch.zeros_like(rho)
        bx[1:n + 1, 1:n] = -gx * 0.5 * (rho[0:n, 1:n] + rho[1:n + 1, 1:n])
        by[1:n, 1:n + 1] = -gy * 0.5 * (rho[1:n, 0:n] + rho[1:n, 1:n + 1])
        ax, ay, ap = s.apply(vx0, vy0, p0)
        r0 = torch.cat([(bx - ax)[1:n + 1, 1:n].ravel(), (by - ay)[1:n, 1:n + 1].ravel()])
        bn = torch.cat([bx[1:n + 1, 1:n].ravel(), by[1:n, 1:n + 1].ravel()])
        assert float(torch.linalg.norm(r0) / torch.linalg.norm(bn)) < 1e-6   # b is the solver's own
        assert float(J_of_v(vx0)) == pytest.approx(float(J), rel=1e-9)

        def J_pert(mm):
            eb, ep = _eta_from_logvisc(mm, n)
            s.set_coefficients(eb, ep, rho, gx, gy)
            ax, ay, ap = s.apply(vx0, vy0, p0)
            dvx, dvy, dp, info = s.solve_rhs(bx - ax, by - ay, -ap)
            assert info.res_energy < 1e-9
            return float(J_of_v(vx0 + dvx))

        h = 1e-3
        errs = []
        for (ci, cj) in cells:
            i, j = int(ci) - 1, int(cj) - 1
            mp_, mm_ = T(m), T(m)
            mp_[i, j] += h
            mm_[i, j] -= h
            fd = (J_pert(mp_) - J_pert(mm_)) / (2 * h)
            errs.append(abs(grad[i, j] - fd) / max(abs(fd), 1e-3 * gmax))
    print(f"[adjoint-fd] J={float(J):.4e} max rel err {max(errs):.2e} median {np.median(errs):.2e}", flush=True)
    assert max(errs) < 1e-4
