"""Pins of the oracle's misfit gradient: central finite differences of the
misfit computed with independent direct solves (the gradient is exact up to
the O(h^2) difference error, which is checked against a tight bound)."""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as adj
from oracle import stokes as st


def _J(g, eb, ep, rho, gvec, target):
    sol = st.solve(g, eb, ep, rho, gvec[0], gvec[1])
    return adj.misfit(g, sol.vx, target)


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
def test_eta_and_rho_gradients_match_finite_differences(bc):
    nx, ny = 6, 5
    g = st.Grid(nx, ny, 1.0, 1.0, bc)
    eb, ep, rho = wl.random_fields(nx, ny, seed=31, eta_decades=1.5)
    gvec = (0.3, -1.0)
    rng = np.random.default_rng(4)
    target = rng.standard_normal(nx - 1) * 0.01
    out = adj.gradient(g, eb, ep, rho, gvec[0], gvec[1], target)
    picks_b = [(0, 0), (0, 3), (2, 2), (ny, nx - 1), (3, nx), (ny, 2)]
    picks_p = [(1, 1), (2, 4), (ny, nx), (3, 3)]
    for (i, j) in picks_b:
        h = 1e-5 * eb[i, j]
        e1, e2 = eb.copy(), eb.copy()
        e1[i, j] += h
        e2[i, j] -= h
        fd = (_J(g, e1, ep, rho, gvec, target) - _J(g, e2, ep, rho, gvec, target)) / (2 * h)
        assert out["g_eta_b"][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(out["J"]) / eb[i, j] + 1e-14)
    for (i, j) in picks_p:
        h = 1e-5 * ep[i, j]
        e1, e2 = ep.copy(), ep.copy()
        e1[i, j] += h
        e2[i, j] -= h
        fd = (_J(g, eb, e1, rho, gvec, target) - _J(g, eb, e2, rho, gvec, target)) / (2 * h)
        assert out["g_eta_p"][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-14)
    for (i, j) in [(0, 1), (2, 2), (ny, nx), (1, 0)]:
        h = 1e-4
        r1, r2 = rho.copy(), rho.copy()
        r1[i, j] += h
        r2[i, j] -= h
        fd = (_J(g, eb, ep, r1, gvec, target) - _J(g, eb, ep, r2, gvec, target)) / (2 * h)
        assert out["g_rho_b"][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-14)


def test_free_slip_boundary_nodes_have_zero_eta_b_gradient():
    nx = ny = 6
    g = st.Grid(nx, ny)
    eb, ep, rho = wl.random_fields(nx, ny, seed=2)
    target = np.zeros(nx - 1)
    out = adj.gradient(g, eb, ep, rho, 0.0, -1.0, target, with_rho=False)
    gb = out["g_eta_b"]
    assert np.all(gb[0, :nx + 1] == 0) and np.all(gb[ny, :nx + 1] == 0)
    assert np.all(gb[:ny + 1, 0] == 0) and np.all(gb[:ny + 1, nx] == 0)


def test_logvisc_chain_matches_finite_differences():
    n = 8
    base = wl.random_viscosity(n, ell=0.2, contrast=100.0)
    m = base.meta["m"]
    g = st.Grid(n, n)
    target = np.linspace(-0.01, 0.01, n - 1)

    def J_of_m(mm):
        eb, ep = wl.logvisc_to_eta(mm, n, n)
        return _J(g, eb, ep, base.rho_b, (0.0, -1.0), target)

    eb, ep = wl.logvisc_to_eta(m, n, n)
    out = adj.gradient(g, eb, ep, base.rho_b, 0.0, -1.0, target, with_rho=False)
    gm = adj.chain_to_logvisc(g, out["g_eta_b"], out["g_eta_p"], eb, ep)
    for (i, j) in [(0, 0), (3, 4), (7, 7), (0, 5)]:
        h = 1e-5
        m1, m2 = m.copy(), m.copy()
        m1[i, j] += h
        m2[i, j] -= h
        fd = (J_of_m(m1) - J_of_m(m2)) / (2 * h)
        assert gm[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-13)
