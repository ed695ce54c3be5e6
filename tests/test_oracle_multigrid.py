"""Pins of the oracle's multigrid pieces.

* restriction: against a literal run of the paper's 4-colour scatter
  algorithm (bisection bounds, per-colour accumulation of w u and w,
  normalisation) in plain loops, with half-open cell footprints; constants
  are restricted to themselves.
* prolongation: reproduces bilinear fields exactly; in the interior it is 4x
  the transpose of the restriction.
* coloured Gauss-Seidel: no coupling inside a colour, so it equals a
  sequential point-by-point Gauss-Seidel over the same ordering.
* V-cycle: one level is the exact solve; as a stationary iteration the
  V-cycle converges at an h-independent rate.
* Uzawa preconditioner with exact velocity solve equals the block
  triangular solve with M; the pressure sign makes the stationary iteration
  contract (reading documented in the oracle).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import multigrid as mg
from oracle import stokes as st


def _bisect_bound(x, xt):
    lo, hi = 0, len(x) - 1
    while lo < hi:
        m = (lo + hi) // 2
        if x[m] < xt:
            lo = m + 1
        else:
            hi = m
    return lo


def _four_colour_restriction(xf, yf, uf, xc, yc):
    """Normalised bilinear scatter following Alg. "4-Color Parallel
    Restriction": bounds by bisection, four colour sweeps over coarse cells,
    each fine node visited by exactly one cell (half-open footprints; the
    last cell also takes its end line), normalisation at the end."""
    ny_c, nx_c = len(yc), len(xc)
    uc = np.zeros((ny_c, nx_c))
    wc = np.zeros((ny_c, nx_c))
    dX, dY = xc[1] - xc[0], yc[1] - yc[0]
    ib = [_bisect_bound(yf, yc[k]) if yf[-1] >= yc[k] else len(yf) for k in range(ny_c)]
    jb = [_bisect_bound(xf, xc[k]) if xf[-1] >= xc[k] else len(xf) for k in range(nx_c)]
    for cy in (0, 1):
        for cx in (0, 1):
            for I in range(cy, ny_c - 1, 2):
                for J in range(cx, nx_c - 1, 2):
                    i_end = ib[I + 1] + (1 if I + 1 == ny_c - 1 else 0)
                    j_end = jb[J + 1] + (1 if J + 1 == nx_c - 1 else 0)
                    for i in range(ib[I], min(i_end, len(yf))):
                        for j in range(jb[J], min(j_end, len(xf))):
                            for di, dj in ((0, 0), (1, 0), (0, 1), (1, 1)):
                                rx = abs(xf[j] - xc[J + dj]) / dX
                                ry = abs(yf[i] - yc[I + di]) / dY
                                w = (1 - rx) * (1 - ry)
                                uc[I + di, J + dj] += w * uf[i, j]
                                wc[I + di, J + dj] += w
    out = np.zeros_like(uc)
    ok = wc > 0
    out[ok] = uc[ok] / wc[ok]
    return out


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
@pytest.mark.parametrize("shape", [(4, 4), (8, 6), (6, 10)])
def test_restriction_matches_four_colour_algorithm(kind, shape):
    nx, ny = shape
    g = st.Grid(nx, ny, 1.0, 1.5)
    gc = mg.coarsen(g)
    rng = np.random.default_rng(nx * 31 + ny)
    u = rng.standard_normal((ny + 2, nx + 2))
    (xf, inx), (yf, iny) = mg.axis_coords(g, kind)
    (xc, _), (yc, _) = mg.axis_coords(gc, kind)
    ref = _four_colour_restriction(xf[inx], yf[iny], u[np.ix_(iny, inx)], xc, yc)
    got = mg.restrict(g, kind, u)
    # coarse nodes inside the coarse domain
    (_, cinx), (_, ciny) = mg.axis_coords(gc, kind)
    sel = np.ix_(ciny, cinx)
    assert np.allclose(got[sel], ref[sel], rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
def test_restriction_of_constant_is_constant(kind):
    g = st.Grid(8, 12)
    u = np.full((14, 10), 3.25)
    out = mg.restrict(g, kind, u)
    gc = mg.coarsen(g)
    (_, cinx), (_, ciny) = mg.axis_coords(gc, kind)
    assert np.allclose(out[np.ix_(ciny, cinx)], 3.25, rtol=1e-15)


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
def test_prolongation_exact_for_bilinear_fields(kind):
    gf = st.Grid(8, 6, 2.0, 1.0)
    gc = mg.coarsen(gf)
    (xc, _), (yc, _) = mg.axis_coords(gc, kind)
    (xf, inx), (yf, iny) = mg.axis_coords(gf, kind)
    f = lambda x, y: 1.5 - 0.7 * x + 2.0 * y + 0.3 * x * y
    uc = f(xc[None, :], yc[:, None])
    uf = mg.prolong(gc, kind, uc, gf)
    # fine nodes inside the span of the coarse lattice
    sx = (xf >= xc[0]) & (xf <= xc[-1]) & inx
    sy_ = (yf >= yc[0]) & (yf <= yc[-1]) & iny
    sel = np.ix_(sy_, sx)
    assert np.allclose(uf[sel], f(xf[None, :], yf[:, None])[sel], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
def test_prolongation_is_four_times_restriction_transpose_in_interior(kind):
    gf = st.Grid(16, 16)
    gc = mg.coarsen(gf)
    rng = np.random.default_rng(4)
    u = np.zeros((18, 18))
    c = np.zeros((10, 10))
    u[5:13, 5:13] = rng.standard_normal((8, 8))     # away from every boundary
    c[3:7, 3:7] = rng.standard_normal((4, 4))
    ru = mg.restrict(gf, kind, u)
    pc = mg.prolong(gc, kind, c, gf)
    assert 4.0 * np.sum(ru * c) == pytest.approx(np.sum(u * pc), rel=1e-13)


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (1, 0, 1, 0)])
def test_colored_gs_equals_sequential_gs(bc):
    g = st.Grid(5, 4, 1.0, 1.0, bc)
    eb, ep, _ = wl.random_fields(5, 4, seed=21)
    lev = mg.Level(g, eb, ep)
    Ld = lev.L.toarray()
    for c in lev.colors:        # no coupling between two nodes of one colour
        blk = Ld[np.ix_(c, c)]
        assert np.count_nonzero(blk - np.diag(np.diag(blk))) == 0
    rng = np.random.default_rng(2)
    r = rng.standard_normal(Ld.shape[0])
    e0 = rng.standard_normal(Ld.shape[0])
    omega = 0.8
    e = e0.copy()
    for _ in range(2):
        for c in lev.colors:
            for k in c:
                e[k] = e[k] + omega * (r[k] - Ld[k] @ e) / Ld[k, k]
    got = mg.colored_gs(lev, e0, r, omega, 2)
    assert np.allclose(got, e, rtol=1e-13, atol=1e-13)


def test_jacobi_definition_pointwise():
    g = st.Grid(4, 4)
    eb, ep, _ = wl.random_fields(4, 4, seed=8)
    lev = mg.Level(g, eb, ep)
    Ld = lev.L.toarray()
    rng = np.random.default_rng(1)
    r = rng.standard_normal(Ld.shape[0])
    e = rng.standard_normal(Ld.shape[0])
    omega = 0.6
    ref = np.array([(1 - omega) * e[k] + omega * (r[k] - sum(Ld[k, m] * e[m] for m in range(len(e)) if m != k)) / Ld[k, k]
                    for k in range(len(e))])
    assert np.allclose(mg.jacobi(lev, e, r, omega, 1), ref, rtol=1e-13, atol=1e-13)


def test_single_level_vcycle_is_exact_solve():
    g = st.Grid(8, 8)
    eb, ep, _ = wl.random_fields(8, 8, seed=3)
    prm = mg.MGParams(levels=1, nu_pre=[2], nu_post=[2])
    levs = mg.build_hierarchy(g, eb, ep, prm)
    r = np.random.default_rng(0).standard_normal(g.n_vx + g.n_vy)
    e = mg.vcycle(levs, prm, 0, r)
    assert np.allclose(levs[0].L @ e, r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("smoother", ["jacobi", "gs"])
def test_vcycle_convergence_is_h_independent(smoother):
    rates = []
    for n in (16, 32, 64):
        g = st.Grid(n, n)
        one = np.ones((n + 2, n + 2))
        levels = int(np.log2(n)) - 1          # coarsest 4 x 4 cells
        prm = mg.MGParams(levels=levels, nu_pre=[2] * levels, nu_post=[2] * levels,
                          omega=0.6 if smoother == "jacobi" else 1.0, smoother=smoother)
        levs = mg.build_hierarchy(g, one, one, prm)
        L = levs[0].L
        rng = np.random.default_rng(n)
        xs = rng.standard_normal(L.shape[0])
        b = L @ xs
        e = np.zeros_like(b)
        errs = []
        for _ in range(8):
            e = e + mg.vcycle(levs, prm, 0, b - L @ e)
            errs.append(np.linalg.norm(e - xs))
        rates.append((errs[-1] / errs[-4]) ** (1 / 3))
    # Jacobi (omega 0.6) and coloured GS (omega 1) contract by about 0.45 and
    # 0.14 per V(2,2) cycle on this operator; the rate must not grow with n
    assert max(rates) < (0.5 if smoother == "jacobi" else 0.2)
    assert max(rates) - min(rates) < 0.1


def _block_M(g, A, eta_p, alpha):
    nv = g.n_vx + g.n_vy
    L = A[:nv, :nv]
    D = A[nv:, :nv]
    d = 1.0 / (alpha * eta_p[1:g.ny + 1, 1:g.nx + 1].ravel())
    return sp.bmat([[L, None], [D, sp.diags(d)]], format="csc")


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 0, 1, 0)])
def test_uzawa_preconditioner_is_block_triangular_solve(bc):
    g = st.Grid(6, 8, 1.0, 1.0, bc)
    eb, ep, _ = wl.random_fields(6, 8, seed=17, eta_decades=3)
    alpha = 1.7
    prm = mg.MGParams(levels=1, nu_pre=[1], nu_post=[1], alpha=alpha)
    levs = mg.build_hierarchy(g, eb, ep, prm)
    rx, ry, rp = wl.random_state(6, 8, seed=5)
    zx, zy, zp = mg.precondition(levs, prm, rx, ry, rp)
    A = st.assemble(g, eb, ep)
    M = _block_M(g, A, ep, alpha)
    z = spla.spsolve(M, st.to_vector(g, rx, ry, rp))
    assert np.allclose(st.to_vector(g, zx, zy, zp), z, rtol=1e-11, atol=1e-11)
    # splitting: N = M - A has zero velocity columns, so (M - A) x does not see v
    N = (M - A.tocsc()).toarray()
    nv = g.n_vx + g.n_vy
    assert np.abs(N[:, :nv]).max() == 0.0


def test_uzawa_stationary_iteration_contracts_with_adopted_sign():
    """x <- x + M^{-1}(b - A x) with an exact velocity solve converges for the
    adopted pressure sign (spectral radius of I - M^{-1}A below one)."""
    n = 8
    g = st.Grid(n, n)
    one = np.ones((n + 2, n + 2))
    A = st.assemble(g, one, one).toarray()
    nv = g.n_vx + g.n_vy
    for alpha, bound in ((1.0, 0.75), (2.0, 0.6)):
        M = _block_M(g, sp.csr_matrix(A), one, alpha).toarray()
        T = np.eye(g.n) - np.linalg.solve(M, A)
        # restrict to zero-mean pressures (the null space is invariant)
        P = np.eye(g.n)
        P[nv:, nv:] -= 1.0 / g.n_p
        rho = np.max(np.abs(np.linalg.eigvals(P @ T @ P)))
        assert rho < bound
    # the printed sign (M with -(alpha eta)^{-1}) expands the pressure error
    Mneg = _block_M(g, sp.csr_matrix(A), one, -1.0).toarray()
    T = np.eye(g.n) - np.linalg.solve(Mneg, A)
    assert np.max(np.abs(np.linalg.eigvals(T))) > 1.2


def test_coarse_viscosity_means():
    g = st.Grid(8, 8)
    eb, ep, _ = wl.random_fields(8, 8, seed=6)
    cb, cp = mg.coarse_viscosity(g, eb, ep)
    # interior coarse basic node = 9-point full weighting of the fine nodes around it
    w = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    assert cb[2, 2] == pytest.approx(np.sum(w * eb[3:6, 3:6]), rel=1e-14)
    # interior coarse cell = 16-point (1,3,3,1)^2 / 64 weighting
    w4 = np.outer([1, 3, 3, 1], [1, 3, 3, 1]) / 64.0
    assert cp[2, 2] == pytest.approx(np.sum(w4 * ep[2:6, 2:6]), rel=1e-14)
    gb, gp = mg.coarse_viscosity(g, eb, ep, mean="geometric")
    assert gp[2, 2] == pytest.approx(np.exp(np.sum(w4 * np.log(ep[2:6, 2:6]))), rel=1e-13)
    assert np.all(cb[:5, :5] > 0) and np.all(cp[1:5, 1:5] > 0)


def test_uzawa_steps_converge_to_exact_solution():
    """Many sweeps of the stationary Uzawa iteration with an exact velocity
    solve converge to A^{-1} b (contraction shown above), and one sweep is the
    single preconditioner application."""
    n = 8
    g = st.Grid(n, n)
    eb, ep, _ = wl.random_fields(n, n, seed=4, eta_decades=1)
    prm = mg.MGParams(levels=1, nu_pre=[1], nu_post=[1], alpha=1.0)
    levs = mg.build_hierarchy(g, eb, ep, prm)
    A = st.assemble(g, eb, ep)
    rx, ry, rp = wl.random_state(n, n, seed=2)
    rp[1:n + 1, 1:n + 1] -= rp[1:n + 1, 1:n + 1].mean()        # consistent right-hand side
    one = mg.uzawa_preconditioner(levs, prm, A, rx, ry, rp, 1)
    ref1 = mg.precondition(levs, prm, rx, ry, rp)
    for a, b in zip(one, ref1):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13)
    zx, zy, zp = mg.uzawa_preconditioner(levs, prm, A, rx, ry, rp, 250)
    b = st.to_vector(g, rx, ry, rp)
    x, _ = st.solve_system(g, A, b)
    got = st.to_vector(g, zx, zy, zp)
    nv = g.n_vx + g.n_vy
    got[nv:] -= got[nv:].mean()
    assert np.allclose(got, x, rtol=1e-8, atol=1e-8 * np.abs(x).max())


# ---------------------------------------------------------------------------
# coarsening by factors other than 2 (the paper's sinker test coarsens by 2.5)
# ---------------------------------------------------------------------------
def test_bisect_bound_is_the_smallest_index_not_below_the_target():
    """Alg. "Bisect Bound" returns the smallest i with x[i] >= x_t; against a
    linear scan on random sorted arrays with repeats and exact hits."""
    rng = np.random.default_rng(17)
    for n in (1, 2, 3, 7, 64, 101):
        x = np.sort(rng.integers(0, 20, n).astype(np.float64))
        for xt in list(x) + list(rng.uniform(-1.0, 21.0, 10)):
            idx = [i for i in range(n) if x[i] >= xt]
            want = idx[0] if idx else n - 1
            assert mg.bisect_bound(x, xt) == want
    assert mg.bisect_bound(np.linspace(0, 1, 11), 0.35) == int(np.searchsorted(np.linspace(0, 1, 11), 0.35))


@pytest.mark.parametrize("n,f,want", [(500, 2.5, 200), (200, 2.5, 80), (96, 2.5, 38), (601, 2.5, 240),
                                      (64, 2.0, 32), (10, 3.0, 3), (3, 2.5, 2)])
def test_coarse_cell_counts(n, f, want):
    assert mg.coarse_cells(n, f) == want


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
@pytest.mark.parametrize("shape,f", [((10, 15), 2.5), ((12, 9), 3.0), ((9, 7), 1.5), ((25, 20), 2.5)])
def test_general_ratio_restriction_matches_four_colour_algorithm(kind, shape, f):
    """Normalised bilinear restriction onto a coarse grid whose nodes fall
    between fine nodes equals the literal scatter of Alg. "4-Color Parallel
    Restriction" with bisection bounds."""
    nx, ny = shape
    g = st.Grid(nx, ny, 1.0, 1.5)
    gc = mg.coarsen(g, f)
    rng = np.random.default_rng(nx * 7 + ny)
    u = rng.standard_normal((ny + 2, nx + 2))
    (xf, inx), (yf, iny) = mg.axis_coords(g, kind)
    (xc, _), (yc, _) = mg.axis_coords(gc, kind)
    ref = _four_colour_restriction(xf[inx], yf[iny], u[np.ix_(iny, inx)], xc, yc)
    got = mg.restrict(g, kind, u, gc)
    (_, cinx), (_, ciny) = mg.axis_coords(gc, kind)
    sel = np.ix_(ciny, cinx)
    assert np.allclose(got[sel], ref[sel], rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
def test_general_ratio_restriction_of_constant_is_constant(kind):
    g = st.Grid(25, 30, 1.0, 1.2)
    gc = mg.coarsen(g, 2.5)
    out = mg.restrict(g, kind, np.full((32, 27), -1.75), gc)
    (_, cinx), (_, ciny) = mg.axis_coords(gc, kind)
    assert np.allclose(out[np.ix_(ciny, cinx)], -1.75, rtol=1e-15)


@pytest.mark.parametrize("kind", ["vx", "vy", "p", "basic"])
@pytest.mark.parametrize("f", [2.5, 3.0, 1.5])
def test_general_ratio_prolongation_exact_for_bilinear_fields(kind, f):
    gf = st.Grid(15, 12, 2.0, 1.0)
    gc = mg.coarsen(gf, f)
    (xc, _), (yc, _) = mg.axis_coords(gc, kind)
    (xf, inx), (yf, iny) = mg.axis_coords(gf, kind)
    fn = lambda x, y: 0.5 + 1.3 * x - 0.4 * y + 0.9 * x * y
    uf = mg.prolong(gc, kind, fn(xc[None, :], yc[:, None]), gf)
    sx = (xf >= xc[0]) & (xf <= xc[-1]) & inx
    sy_ = (yf >= yc[0]) & (yf <= yc[-1]) & iny
    sel = np.ix_(sy_, sx)
    assert np.allclose(uf[sel], fn(xf[None, :], yf[:, None])[sel], rtol=1e-13, atol=1e-13)


def test_vcycle_with_factor_2_5_coarsening_contracts():
    """The sinker-test hierarchy shape: coarsening by 2.5 per level (50 x 60
    -> 20 x 24 -> 8 x 10); the V-cycle as a stationary iteration on L
    contracts, and does so at a rate close to the factor-2 hierarchy's."""
    nx, ny = 50, 60
    eb, ep, _ = wl.random_fields(nx, ny, seed=5, eta_decades=1.0)
    g = st.Grid(nx, ny, 1.0, 1.2)
    rates = {}
    for f, levels in ((2.5, 3), (2.0, 2)):
        prm = mg.MGParams(levels=levels, nu_pre=[2] * levels, nu_post=[2] * levels, omega=1.0, smoother="gs",
                          coarsen=f)
        levs = mg.build_hierarchy(g, eb, ep, prm)
        if f == 2.5:
            assert [(lv.g.nx, lv.g.ny) for lv in levs] == [(50, 60), (20, 24), (8, 10)]
        L = levs[0].L
        rng = np.random.default_rng(3)
        x_true = rng.standard_normal(L.shape[0])
        b = L @ x_true
        x = np.zeros_like(b)
        errs = []
        for _ in range(8):
            x = x + mg.vcycle(levs, prm, 0, b - L @ x)
            errs.append(np.linalg.norm(x - x_true))
        rates[f] = (errs[-1] / errs[2]) ** (1 / 5)
    assert rates[2.5] < 0.5
    assert rates[2.5] < 1.5 * rates[2.0] + 0.05
