"""Pins of the CPU oracle's operator, right-hand side and direct solve.

Each test checks the oracle against something other than itself: the
printed listing (golden fixture), the dissipation functional (a variational
characterisation), a manufactured closed-form solution (second-order
convergence), the hydrostatic closed form, symmetry / definiteness /
null-space statements of Ch. 4, and the mirror symmetry of the centred sinker.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import sympy as sy

import workloads as wl
from oracle import stokes as st

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BCS = [(0, 0, 0, 0), (1, 1, 1, 1), (1, 0, 0, 1), (0, 1, 1, 0)]


def test_listing_coefficients_golden():
    d = json.load(open(os.path.join(GOLD, "listing_vx_row.json")))
    pt = d["point"]
    g = st.Grid(pt["nx"], pt["ny"], pt["lx"], pt["ly"])
    assert g.dx == pt["dx"] and g.dy == pt["dy"]
    eb, ep, _ = wl.random_fields(g.nx, g.ny, seed=7)
    i, j = pt["i"], pt["j"]
    v = d["viscosity"]
    ep[i, j] = v["etaA = eta_p[i,j]"]
    ep[i, j + 1] = v["etaB = eta_p[i,j+1]"]
    eb[i - 1, j] = v["eta1 = eta_b[i-1,j]"]
    eb[i, j] = v["eta2 = eta_b[i,j]"]
    A = st.assemble(g, eb, ep).toarray()
    ivx, ivy, ip = st.index_maps(g)
    row = A[ivx[i, j]]
    maps = {"vx": ivx, "vy": ivy, "p": ip}
    seen = set()
    for c in d["coefficients"]:
        col = maps[c["field"]][i + c["di"], j + c["dj"]]
        assert col >= 0
        assert row[col] == pytest.approx(c["value"], rel=1e-14), c["name"]
        seen.add(col)
    # no other entries in that row
    others = [k for k in np.nonzero(row)[0] if k not in seen]
    assert others == []


def _energy(g, eb, ep, vx, vy):
    """Half the discrete dissipation: sum_c eta_p (exx^2 + eyy^2)
    + 1/2 sum_b w_b eta_b gamma_b^2, with midpoint weights at cell centres and
    trapezoid weights w_b (1 interior, 1/2 edge, 1/4 corner) at basic nodes.
    Velocity arrays carry mirrored ghosts and zero walls."""
    nx, ny, dx, dy = g.nx, g.ny, g.dx, g.dy
    exx = (vx[1:ny + 1, 1:nx + 1] - vx[1:ny + 1, 0:nx]) / dx
    eyy = (vy[1:ny + 1, 1:nx + 1] - vy[0:ny, 1:nx + 1]) / dy
    e1 = np.sum(ep[1:ny + 1, 1:nx + 1] * (exx ** 2 + eyy ** 2))
    gam = ((vx[1:ny + 2, 0:nx + 1] - vx[0:ny + 1, 0:nx + 1]) / dy
           + (vy[0:ny + 1, 1:nx + 2] - vy[0:ny + 1, 0:nx + 1]) / dx)
    wy = np.ones(ny + 1)
    wy[[0, -1]] = 0.5
    wx = np.ones(nx + 1)
    wx[[0, -1]] = 0.5
    e2 = 0.5 * np.sum(wy[:, None] * wx[None, :] * eb[:ny + 1, :nx + 1] * gam ** 2)
    return e1 + e2


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(3, 3), (4, 5), (7, 4)])
def test_velocity_block_is_minus_hessian_of_dissipation(bc, shape):
    nx, ny = shape
    g = st.Grid(nx, ny, 1.3, 0.7, bc)
    eb, ep, _ = wl.random_fields(nx, ny, seed=11 + nx * ny)
    A = st.assemble(g, eb, ep)
    nv = g.n_vx + g.n_vy
    L = A[:nv, :nv].toarray()
    rng = np.random.default_rng(3)
    for _ in range(4):
        a = rng.standard_normal(g.n)
        b = rng.standard_normal(g.n)
        a[nv:] = 0
        b[nv:] = 0
        ax, ay, _ = st.to_arrays(g, a)
        bx, by, _ = st.to_arrays(g, b)
        sx, sy_, _ = st.to_arrays(g, a + b)
        dx_, dy_, _ = st.to_arrays(g, a - b)
        # v^T L w = -(E(v+w) - E(v-w)) / 2 for the quadratic form E = 1/2 v^T H v
        lhs = a[:nv] @ L @ b[:nv]
        rhs = -(_energy(g, eb, ep, sx, sy_) - _energy(g, eb, ep, dx_, dy_)) / 2.0
        assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-11 * abs(lhs))


@pytest.mark.parametrize("bc", BCS)
def test_symmetric_negative_definite_nullspace(bc):
    g = st.Grid(6, 5, 1.0, 1.0, bc)
    eb, ep, _ = wl.random_fields(6, 5, seed=5, eta_decades=4)
    A = st.assemble(g, eb, ep)
    assert abs(A - A.T).max() == 0.0
    nv = g.n_vx + g.n_vy
    sla.cholesky(-A[:nv, :nv].toarray())       # -L SPD
    ones_p = np.zeros(g.n)
    ones_p[nv:] = 1.0
    assert np.abs(A @ ones_p).max() < 1e-12     # constant pressure in the null space
    # the null space is exactly one-dimensional: the bordered system is regular
    K = st.bordered(g, A).toarray()
    assert np.linalg.matrix_rank(K) == K.shape[0]


def test_gradient_is_minus_divergence_transpose():
    g = st.Grid(5, 4, 1.0, 2.0, (1, 0, 1, 0))
    eb, ep, _ = wl.random_fields(5, 4, seed=2)
    A = st.assemble(g, eb, ep).toarray()
    nv = g.n_vx + g.n_vy
    G = A[:nv, nv:]
    D = A[nv:, :nv]
    assert np.array_equal(G, D.T)
    # D is the discrete divergence: for a velocity sampled from a linear field
    # with zero wall normal components... use a divergence check on
    # v = (x (1 - x), 0) whose divergence is 1 - 2x at cell centres
    nx, ny = g.nx, g.ny
    vx = np.zeros((ny + 2, nx + 2))
    xj = np.arange(nx + 2) * g.dx
    vx[:, :] = (xj * (g.lx - xj))[None, :]
    vx[:, 0] = vx[:, nx] = 0
    vy = np.zeros_like(vx)
    x = st.to_vector(g, vx, vy, np.zeros_like(vx))
    div = (D @ x[:nv]).reshape(ny, nx)
    xc = (np.arange(1, nx + 1) - 0.5) * g.dx
    assert np.allclose(div, (g.lx - 2 * xc)[None, :], rtol=0, atol=1e-12)


def test_energy_weights_golden():
    d = json.load(open(os.path.join(GOLD, "energy_weights.json")))
    g = st.Grid(d["nx"], d["ny"], d["lx"], d["ly"])
    eb = np.full((g.ny + 2, g.nx + 2), d["eta"])
    ep = eb.copy()
    A = st.assemble(g, eb, ep)
    w = st.energy_weights(g, A, ep)
    ivx, ivy, ip = st.index_maps(g)
    assert w[ivx[2, 3]] == pytest.approx(d["interior_vx_weight"], rel=1e-14)
    assert w[ivy[2, 3]] == pytest.approx(d["interior_vy_weight"], rel=1e-14)
    assert w[ip[2, 3]] == pytest.approx(d["pressure_weight"], rel=1e-14)


@pytest.mark.parametrize("g_vec", [(0.0, -1.0), (0.7, -0.3), (-2.0, 0.0)])
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (1, 0, 0, 1)])
def test_hydrostatic_closed_form(g_vec, bc):
    """Uniform density: v = 0 and p = rho0 (g . x) + const exactly."""
    nx, ny = 9, 7
    g = st.Grid(nx, ny, 1.5, 1.0, bc)
    eb, ep, _ = wl.random_fields(nx, ny, seed=9, eta_decades=3)
    rho0 = 1.7
    rho = np.full((ny + 2, nx + 2), rho0)
    sol = st.solve(g, eb, ep, rho, g_vec[0], g_vec[1])
    xc = (np.arange(nx + 2) - 0.5) * g.dx
    yc = (np.arange(ny + 2) - 0.5) * g.dy
    pex = rho0 * (g_vec[0] * xc[None, :] + g_vec[1] * yc[:, None])
    pex = pex[1:ny + 1, 1:nx + 1]
    pex -= pex.mean()
    scale = max(np.abs(pex).max(), 1.0)
    assert np.abs(sol.vx).max() < 1e-12 * scale
    assert np.abs(sol.vy).max() < 1e-12 * scale
    assert np.abs(sol.p[1:ny + 1, 1:nx + 1] - pex).max() < 1e-12 * scale
    assert abs(sol.dropped_residual) < 1e-12 * scale


def _mms_fields():
    x, y = sy.symbols("x y")
    psi = sy.sin(sy.pi * x) * sy.sin(sy.pi * y)
    vx = sy.diff(psi, y)
    vy = -sy.diff(psi, x)
    p = sy.cos(sy.pi * x) * sy.cos(sy.pi * y)
    eta = sy.exp(x * y)
    sxx = 2 * eta * sy.diff(vx, x)
    syy = 2 * eta * sy.diff(vy, y)
    sxy = eta * (sy.diff(vx, y) + sy.diff(vy, x))
    fx = sy.diff(sxx, x) + sy.diff(sxy, y) - sy.diff(p, x)
    fy = sy.diff(sxy, x) + sy.diff(syy, y) - sy.diff(p, y)
    return [sy.lambdify((x, y), e, "numpy") for e in (vx, vy, p, eta, fx, fy)]


def test_manufactured_solution_second_order():
    """Free-slip manufactured solution with eta = exp(xy): O(h^2) in v and p."""
    F = _mms_fields()
    errs = []
    for n in (16, 32, 64):
        g = st.Grid(n, n)
        h = 1.0 / n
        i = np.arange(n + 2)[:, None] * 1.0
        j = np.arange(n + 2)[None, :] * 1.0
        full = np.ones((n + 2, n + 2))
        eb = F[3](j * h, i * h) * full
        ep = F[3]((j - 0.5) * h, (i - 0.5) * h) * full
        fx = F[4](j * h, (i - 0.5) * h) * full
        fy = F[5]((j - 0.5) * h, i * h) * full
        sol = st.solve(g, eb, ep, np.zeros_like(full), 0.0, 0.0, fx, fy)
        ex = F[0](j * h, (i - 0.5) * h) * full
        ey = F[1]((j - 0.5) * h, i * h) * full
        pe = (F[2]((j - 0.5) * h, (i - 0.5) * h) * full)[1:n + 1, 1:n + 1]
        pe = pe - pe.mean()
        ev = np.sqrt((np.sum((sol.vx - ex)[1:n + 1, 1:n] ** 2)
                      + np.sum((sol.vy - ey)[1:n, 1:n + 1] ** 2)) * h * h)
        ep_ = np.sqrt(np.sum((sol.p[1:n + 1, 1:n + 1] - pe) ** 2) * h * h)
        errs.append((ev, ep_))
    for (a, b), (c, d) in zip(errs[:-1], errs[1:]):
        assert np.log2(a / c) > 1.9
        assert np.log2(b / d) > 1.9


def test_constant_viscosity_reduces_to_mac_laplacian():
    """Constant eta and a discretely divergence-free v: L v = eta * 5-point
    Laplacian of each component at interior nodes (classical MAC scheme)."""
    n = 8
    g = st.Grid(n, n)
    eta = 2.5
    full = np.full((n + 2, n + 2), eta)
    A = st.assemble(g, full, full)
    nv = g.n_vx + g.n_vy
    # discretely divergence-free field from a stream function at basic nodes
    rng = np.random.default_rng(1)
    psi = np.zeros((n + 1, n + 1))
    psi[1:n, 1:n] = rng.standard_normal((n - 1, n - 1))
    vx = np.zeros((n + 2, n + 2))
    vy = np.zeros((n + 2, n + 2))
    vx[1:n + 1, 0:n + 1] = (psi[1:n + 1, :] - psi[0:n, :]) / g.dy
    vy[0:n + 1, 1:n + 1] = -(psi[:, 1:n + 1] - psi[:, 0:n]) / g.dx
    st.fill_ghosts(g, vx, vy)
    x = st.to_vector(g, vx, vy, np.zeros_like(vx))
    assert np.abs((A @ x)[nv:]).max() < 1e-10      # divergence free
    Lv = (A[:nv, :nv] @ x[:nv])
    ax, ay, _ = st.to_arrays(g, np.concatenate([Lv, np.zeros(g.n_p)]))
    # interior vx nodes away from every wall: i in [2, n-1], j in [2, n-2]
    I = slice(2, n)
    J = slice(2, n - 1)
    lap = eta * ((vx[2:n, 3:n] - 2 * vx[I, J] + vx[2:n, 1:n - 2]) / g.dx ** 2
                 + (vx[3:n + 1, J] - 2 * vx[I, J] + vx[1:n - 1, J]) / g.dy ** 2)
    assert np.allclose(ax[I, J], lap, rtol=1e-12, atol=1e-9)


def test_sinker_mirror_symmetry_and_divergence():
    p = wl.sinker(32, radius=0.1, eta_in=1e3)
    g = st.Grid(p.nx, p.ny, bc=p.bc)
    sol = st.solve(g, p.eta_b, p.eta_p, p.rho_b, p.gx, p.gy)
    n = p.nx
    vx = sol.vx[1:n + 1, 0:n + 1]
    vy = sol.vy[0:n + 1, 1:n + 1]
    pp = sol.p[1:n + 1, 1:n + 1]
    s = np.abs(vy).max()
    assert s > 0
    # vx odd, vy and p even under x -> 1 - x
    assert np.abs(vx + vx[:, ::-1]).max() < 1e-10 * s
    assert np.abs(vy - vy[:, ::-1]).max() < 1e-10 * s
    assert np.abs(pp - pp[:, ::-1]).max() < 1e-7 * np.abs(pp).max()
    # dense inclusion moves along g = (0, -1): vy < 0 at the centre
    assert sol.vy[n // 2, n // 2] < 0
    div = ((sol.vx[1:n + 1, 1:n + 1] - sol.vx[1:n + 1, 0:n]) / g.dx
           + (sol.vy[1:n + 1, 1:n + 1] - sol.vy[0:n, 1:n + 1]) / g.dy)
    assert np.abs(div).max() < 1e-8 * s / g.dx
    assert abs(pp.sum()) < 1e-10 * np.abs(pp).max() * pp.size
    assert sol.residual_energy < 1e-11
