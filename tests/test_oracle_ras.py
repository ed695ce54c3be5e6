"""Pins of the oracle's RAS-type temporal-blocking smoother.

* the shift generator: SplitMix64 outputs published with its reference
  implementation (tests/golden/splitmix64.txt);
* the tiling: a partition of the velocity unknowns whose tile boundaries sit
  at rows 1 + s_i + k T and columns 1 + s_j + k T;
* special cases that reduce to textbook damped Jacobi: one inner sweep per
  outer iteration (any tiling), and one tile covering the level;
* the fixed-boundary reading: with many inner sweeps each tile reaches the
  exact solve of its block with every outside value frozen (a direct sparse
  solve per tile), so a wrong halo (a tile reading its neighbours' new
  values, or tiles sharing unknowns) fails;
* inside the V-cycle it contracts as a stationary iteration.
"""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import multigrid as mg
from oracle import ras
from oracle import stokes as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_published_outputs():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for seed, k, out in rows:
        assert ras.splitmix64(int(seed), int(k)) == int(out)


def _level(nx, ny, bc=(0, 0, 0, 0), seed=3):
    eb, ep, _ = wl.random_fields(nx, ny, seed=seed, eta_decades=2)
    return mg.Level(st.Grid(nx, ny, 1.0, 1.0, bc), eb, ep)


@pytest.mark.parametrize("shift,T", [((0, 0), 4), ((3, 1), 4), ((5, 7), 8), ((0, 2), 3)])
def test_tiles_partition_unknowns(shift, T):
    g = st.Grid(13, 11)
    I, J = ras.node_indices(g)
    ts = ras.tiles(g, shift, (T, T))
    allidx = np.sort(np.concatenate(ts))
    assert np.array_equal(allidx, np.arange(len(I)))
    for S in ts:
        ri = (I[S] - 1 - shift[0]) // T
        rj = (J[S] - 1 - shift[1]) // T
        assert len(set(ri)) == 1 and len(set(rj)) == 1
        lo_i = 1 + shift[0] + ri[0] * T
        lo_j = 1 + shift[1] + rj[0] * T
        assert np.all((I[S] >= lo_i) & (I[S] < lo_i + T)) and np.all((J[S] >= lo_j) & (J[S] < lo_j + T))


def test_one_inner_sweep_is_jacobi():
    lev = _level(20, 14, bc=(1, 0, 0, 1))
    rng = np.random.default_rng(1)
    r = rng.standard_normal(lev.L.shape[0])
    e0 = rng.standard_normal(lev.L.shape[0])
    got = ras.ras_jacobi(lev, e0, r, 0.7, 3, (4, 4), 1, [(1, 2), (3, 0), (2, 3)])
    ref = mg.jacobi(lev, e0, r, 0.7, 3)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("sweeps,inner,total", [(8, 4, 8), (5, 2, 6), (3, 4, 4)])
def test_single_tile_is_jacobi(sweeps, inner, total):
    # ceil(N_max / T_inner) outer iterations of T_inner sweeps each
    lev = _level(16, 12)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(lev.L.shape[0])
    got = ras.ras_jacobi(lev, np.zeros_like(r), r, 0.6, sweeps, (32, 32), inner, [(0, 0)] * 3)
    ref = mg.jacobi(lev, np.zeros_like(r), r, 0.6, total)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 0, 1)])
def test_many_inner_sweeps_reach_frozen_block_solve(bc):
    lev = _level(12, 10, bc=bc, seed=5)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(lev.L.shape[0])
    e0 = rng.standard_normal(lev.L.shape[0])
    shift, T = (1, 2), (4, 4)
    # omega 0.3 (the paper's velocity relaxation for this smoother) keeps the local Jacobi convergent
    got = ras.ras_jacobi(lev, e0, r, 0.3, 4000, T, 4000, [shift])
    ref = ras.block_solve(lev, e0, r, shift, T)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)
    # a different tiling gives a different block solve (the tiles matter)
    other = ras.block_solve(lev, e0, r, (0, 0), T)
    assert np.linalg.norm(other - ref) > 1e-3 * np.linalg.norm(ref)


def test_shifts_follow_the_generator():
    sh = ras.ras_shifts(7, 1, 2, 1, 3, (32, 16))
    for t, (si, sj) in enumerate(sh):
        assert si == ras.splitmix64(7, ras.ras_key(1, 2, 1, t, 0)) % 32
        assert sj == ras.splitmix64(7, ras.ras_key(1, 2, 1, t, 1)) % 16
        assert 0 <= si < 32 and 0 <= sj < 16
    keys = {ras.ras_key(c, l, g, t, a) for c in range(2) for l in range(16) for g in range(2)
            for t in range(4) for a in range(2)}
    assert len(keys) == 2 * 16 * 2 * 4 * 2


@pytest.mark.parametrize("smoother", ["ras", "ras_mixed"])
def test_vcycle_with_ras_contracts(smoother):
    n = 32
    eb, ep, _ = wl.random_fields(n, n, seed=9, eta_decades=1)
    g = st.Grid(n, n)
    prm = mg.MGParams(levels=3, nu_pre=[4] * 3, nu_post=[4] * 3, omega=0.6, smoother=smoother, ras_tile=8,
                      ras_inner=2, seed=11)
    levs = mg.build_hierarchy(g, eb, ep, prm)
    rng = np.random.default_rng(4)
    x_true = rng.standard_normal(levs[0].L.shape[0])
    r = levs[0].L @ x_true
    x = np.zeros_like(r)
    errs = []
    for c in range(6):
        x = x + mg.vcycle(levs, prm, 0, r - levs[0].L @ x, c)
        errs.append(np.linalg.norm(x - x_true))
    rate = (errs[-1] / errs[1]) ** (1 / 4)
    assert rate < 0.5
