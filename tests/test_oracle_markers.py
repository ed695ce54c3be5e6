"""Pins of the oracle's marker <-> grid interpolation and RK4 advection.

* marker -> grid: one marker on each node returns its own value (the weight
  on its node is 1, on every other node 0); constant fields are reproduced;
  a lattice symmetric about every interior node reproduces a linear field
  there (the weighted mean position is the node); nodes no marker reaches
  get the fill value;
* grid -> marker: bilinear fields are reproduced exactly, node values at
  node positions, and the four weights sum to one (constants);
* RK4: with an affine velocity field v = A x + b (represented exactly by
  bilinear interpolation) one step equals the closed form
  x + dt (I + dt A / 2 + (dt A)^2 / 6 + (dt A)^3 / 24)(A x + b), which a
  wrong stage weight or stage position breaks; a uniform field moves every
  marker by dt v.
"""
import numpy as np
import pytest

from oracle import markers as mk
from oracle import stokes as st


def _nodes(g, kind):
    x0, y0, jmin, jmax, imin, imax = mk.node_grid(g, kind)
    I, J = np.meshgrid(np.arange(imin, imax + 1), np.arange(jmin, jmax + 1), indexing="ij")
    return I.ravel(), J.ravel(), x0 + J.ravel() * g.dx, y0 + I.ravel() * g.dy


@pytest.mark.parametrize("kind", ["basic", "cell"])
def test_marker_on_each_node_returns_its_value(kind):
    g = st.Grid(9, 7, 1.3, 0.8)
    I, J, x, y = _nodes(g, kind)
    phi = np.random.default_rng(1).standard_normal(len(x))
    out = mk.markers_to_grid(g, kind, x, y, phi)
    assert np.allclose(out[I, J], phi, rtol=0, atol=1e-14)


def _lattice(g, per=2):
    # per x per markers per basic cell at the (k + 1/2) / per fractions
    f = (np.arange(per) + 0.5) / per
    xs = (np.arange(g.nx)[:, None] + f[None, :]).ravel() * g.dx
    ys = (np.arange(g.ny)[:, None] + f[None, :]).ravel() * g.dy
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return X.ravel(), Y.ravel()


@pytest.mark.parametrize("kind", ["basic", "cell"])
def test_constant_and_linear_fields(kind):
    g = st.Grid(12, 10, 1.0, 0.7)
    xm, ym = _lattice(g, 2)
    out = mk.markers_to_grid(g, kind, xm, ym, np.full(len(xm), 3.25))
    x0, y0, jmin, jmax, imin, imax = mk.node_grid(g, kind)
    assert np.allclose(out[imin:imax + 1, jmin:jmax + 1], 3.25, rtol=0, atol=1e-13)
    lin = 0.5 + 2.0 * xm - 1.5 * ym
    out = mk.markers_to_grid(g, kind, xm, ym, lin)
    I, J, x, y = _nodes(g, kind)
    interior = (x > g.dx * 0.9) & (x < g.lx - g.dx * 0.9) & (y > g.dy * 0.9) & (y < g.ly - g.dy * 0.9)
    assert np.allclose(out[I[interior], J[interior]], (0.5 + 2.0 * x - 1.5 * y)[interior], rtol=0, atol=1e-12)


def test_unreached_nodes_get_fill():
    g = st.Grid(8, 8)
    out = mk.markers_to_grid(g, "basic", np.array([0.01]), np.array([0.02]), np.array([5.0]), fill=-7.0)
    assert out[0, 0] == 5.0 and out[0, 1] == 5.0 and out[1, 1] == 5.0
    assert out[4, 4] == -7.0 and np.sum(out[:9, :9] == -7.0) == 81 - 4


@pytest.mark.parametrize("kind", mk.KINDS)
def test_grid_to_markers_bilinear_exact(kind):
    g = st.Grid(10, 6, 2.0, 1.0)
    x0, y0, jmin, jmax, imin, imax = mk.node_grid(g, kind)
    J, I = np.meshgrid(np.arange(g.nx + 2), np.arange(g.ny + 2))
    X, Y = x0 + J * g.dx, y0 + I * g.dy
    f = lambda x, y: 1.0 + 0.3 * x - 2.0 * y + 0.7 * x * y
    grid = f(X, Y)
    rng = np.random.default_rng(2)
    # positions inside the span of the grid's nodes
    xm = rng.uniform(max(0.0, x0 + jmin * g.dx), min(g.lx, x0 + jmax * g.dx), 500)
    ym = rng.uniform(max(0.0, y0 + imin * g.dy), min(g.ly, y0 + imax * g.dy), 500)
    assert np.allclose(mk.grid_to_markers(g, kind, grid, xm, ym), f(xm, ym), rtol=0, atol=1e-12)
    Is, Js, xn, yn = _nodes(g, kind)
    assert np.allclose(mk.grid_to_markers(g, kind, grid, xn, yn), grid[Is, Js], rtol=0, atol=1e-12)
    assert np.allclose(mk.grid_to_markers(g, kind, np.full_like(grid, 2.5), xm, ym), 2.5)


def _affine_velocity(g, A, b):
    J, I = np.meshgrid(np.arange(g.nx + 2), np.arange(g.ny + 2))
    out = []
    for comp, kind in ((0, "vx"), (1, "vy")):
        x0, y0 = mk.node_grid(g, kind)[:2]
        X, Y = x0 + J * g.dx, y0 + I * g.dy
        out.append(A[comp, 0] * X + A[comp, 1] * Y + b[comp])
    return out


def test_rk4_affine_field_closed_form():
    g = st.Grid(16, 16)
    A = np.array([[0.3, -1.1], [0.9, -0.2]])
    b = np.array([0.05, -0.02])
    vx, vy = _affine_velocity(g, A, b)
    rng = np.random.default_rng(5)
    xm, ym = rng.uniform(0.3, 0.7, 200), rng.uniform(0.3, 0.7, 200)
    dt = 0.07
    nx_, ny_ = mk.rk4_advect(g, vx, vy, xm, ym, dt)
    X = np.stack([xm, ym])
    hA = dt * A
    P = np.eye(2) + hA / 2 + hA @ hA / 6 + hA @ hA @ hA / 24
    ref = X + dt * P @ (A @ X + b[:, None])
    assert np.allclose(nx_, ref[0], rtol=0, atol=1e-13) and np.allclose(ny_, ref[1], rtol=0, atol=1e-13)


def test_rk4_uniform_field_translates():
    g = st.Grid(8, 12, 1.0, 1.5)
    vx, vy = _affine_velocity(g, np.zeros((2, 2)), np.array([0.4, -0.25]))
    xm, ym = np.array([0.2, 0.5, 0.8]), np.array([0.7, 1.0, 1.2])
    nx_, ny_ = mk.rk4_advect(g, vx, vy, xm, ym, 0.3)
    assert np.allclose(nx_, xm + 0.12) and np.allclose(ny_, ym - 0.075)


def test_node_positions_follow_the_staggered_layout():
    # written out from the array convention, not from node_grid
    g = st.Grid(6, 5, 1.2, 1.0)
    dx, dy = g.dx, g.dy
    pos = {"basic": lambda i, j: (j * dx, i * dy), "cell": lambda i, j: ((j - 0.5) * dx, (i - 0.5) * dy),
           "vx": lambda i, j: (j * dx, (i - 0.5) * dy), "vy": lambda i, j: ((j - 0.5) * dx, i * dy)}
    for kind, f in pos.items():
        x, y = f(3, 2)
        if kind in ("basic", "cell"):
            out = mk.markers_to_grid(g, kind, np.array([x]), np.array([y]), np.array([4.0]), fill=0.0)
            assert out[3, 2] == pytest.approx(4.0, abs=1e-14)
            far = np.ones_like(out, dtype=bool)
            far[2:5, 1:4] = False
            assert np.all((out[far] == 0.0) | np.isnan(out[far]))
        grid = np.zeros((g.ny + 2, g.nx + 2))
        grid[3, 2] = 1.0
        assert mk.grid_to_markers(g, kind, grid, np.array([x]), np.array([y]))[0] == pytest.approx(1.0, abs=1e-14)
