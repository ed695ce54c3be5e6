"""Pins of the viscosity-rescaling and lithostatic-pressure oracle."""
import numpy as np

import workloads as wl
from oracle import continuation as co
from oracle import stokes as st


def _rows(g):
    nvx = g.ny * (g.nx - 1)
    nvy = (g.ny - 1) * g.nx
    return slice(0, nvx), slice(nvx, nvx + nvy), slice(nvx + nvy, None)


def test_lithostatic_pressure_balances_every_y_momentum_row():
    # random density, gravity along y only: zero velocity with p_litho leaves no y-momentum residual
    g = st.Grid(24, 16, 1.3, 0.9)
    eb, ep, rho = wl.random_fields(24, 16, seed=5, eta_decades=3)
    p = co.lithostatic_pressure(g, rho, -1.7)
    A = st.assemble(g, eb, ep)
    b = st.rhs(g, rho, 0.0, -1.7)
    x = st.to_vector(g, np.zeros((18, 26)), np.zeros((18, 26)), p)
    r = A @ x - b
    sx, sy, sp = _rows(g)
    assert np.abs(r[sy]).max() <= 1e-12 * np.abs(b[sy]).max()
    assert np.abs(r[sp]).max() == 0.0                    # zero velocity is divergence free
    assert np.abs(r[sx]).max() > 1e-6                     # horizontal density gradients drive flow
    assert abs(p[1:17, 1:25].mean()) < 1e-14


def test_lithostatic_pressure_is_the_hydrostatic_solution_for_uniform_density():
    g = st.Grid(20, 12)
    eb, ep, _ = wl.random_fields(20, 12, seed=2, eta_decades=2)
    rho = np.full((14, 22), 2.5)
    sol = st.solve(g, eb, ep, rho, 0.0, -1.0)
    p = co.lithostatic_pressure(g, rho, -1.0)
    assert np.abs(p[1:13, 1:21] - sol.p[1:13, 1:21]).max() < 1e-9
    # closed form: p = rho g_y y_c minus its mean
    yc = (np.arange(1, 13) - 0.5) / 12
    pc = 2.5 * -1.0 * yc
    pc -= pc.mean()
    assert np.abs(p[1:13, 1:21] - pc[:, None]).max() < 1e-13


def test_rescaled_viscosity_blend():
    g = st.Grid(10, 8)
    eb, ep, _ = wl.random_fields(10, 8, seed=9, eta_decades=4)
    m = co.eta_min(g, eb, ep)
    assert m == min(eb[:9, :11].min(), ep[1:9, 1:11].min())
    b1, p1 = co.rescaled_viscosity(g, eb, ep, 1.0)
    assert np.array_equal(b1, eb) and np.array_equal(p1, ep)
    b0, p0 = co.rescaled_viscosity(g, eb, ep, 0.0)
    assert np.all(b0 == m) and np.all(p0 == m)
    bh, ph = co.rescaled_viscosity(g, eb, ep, 0.5)
    assert np.all(bh[:9, :11] >= m) and np.all(bh[:9, :11] <= eb[:9, :11] + 1e-15)
    assert np.allclose(ph, 0.5 * (m + ep))
