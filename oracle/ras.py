"""RAS-type temporal-blocking Jacobi smoother (oracle; test infrastructure).

Only tests/, the smoke check and the CPU baseline of bench.py use this module.

What it computes (Ch. 4, Sec. "The Multigrid Method", subsection "RAS-Type
Jacobi Smoother", Alg. "RAS-Type Temporal Blocking"): the velocity unknowns
of one level are split into tiles of T_I x T_J nodes; each outer iteration
draws a shift (s_i, s_j), places the tile boundaries at the rows
i = 1 + s_i + k T_I and the columns j = 1 + s_j + k T_J, and lets every tile
run T_inner damped Jacobi sweeps (eq. damped_jacobi) on its own unknowns
while every value outside the tile stays at the state the outer iteration
started from; the tiles' results together form the next state (one writer
per unknown).  The number of outer iterations is ceil(N_max / T_inner).

Readings (where the text leaves a choice):

* Both velocity components share one tiling of the (i, j) index space: a
  tile owns the vx and the vy unknowns whose indices fall inside it.  A
  ghost value outside a wall mirrors the adjacent unknown, so it moves with
  that unknown's tile (the assembled operator has the ghosts eliminated).
* "Treating its outer boundaries as fixed": the values a tile reads outside
  itself are those at the start of the outer iteration.  The printed
  algorithm lets tiles run at once on shared buffers and accepts whichever
  value a neighbour has written (benign races); the fixed reading is the
  deterministic member of that family.
* The periodic wrap-around of the shifted tiling joins the first and last
  partial tiles of a row or column into one tile; no stencil couples the
  two pieces (they sit at opposite walls), so they are treated as separate
  partial tiles.
* The printed algorithm rounds the number of outer iterations up to an even
  count so that its two swapped buffers end in place; the count here is
  ceil(N_max / T_inner) without that rounding (the HIP path tracks which
  buffer holds the result).
* The shifts are random numbers the method draws: draw k of a smoothing
  call is the k-th output of SplitMix64 (Steele, Lea and Flood, 2014; the
  64-bit generator with increment 0x9E3779B97F4A7C15 and the two
  xor-shift-multiply finalisation rounds) seeded with the solver seed, at
  the counter ras_key(cycle, level, leg, outer, axis), reduced modulo the
  tile side.  `cycle` counts the V-cycles of one preconditioner call
  (0 .. uzawa_steps - 1), leg is 0 for pre- and 1 for post-smoothing.

Pins (tests/test_oracle_ras.py): T_inner = 1 and a tile covering the level
are plain damped Jacobi; with many inner sweeps each tile reaches the exact
block solve with frozen neighbours (a direct sparse solve per tile);
ownership is a partition with boundaries at the stated rows and columns;
SplitMix64 against a published output value.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import scipy.sparse.linalg as spla

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MAX_LEVELS = 16
MAX_OUTER = 256


def splitmix64(state: int, k: int) -> int:
    """Output k (0-based) of SplitMix64 started from `state`."""
    z = (state + (k + 1) * GOLDEN_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def ras_key(cycle: int, level: int, leg: int, outer: int, axis: int) -> int:
    return (((cycle * MAX_LEVELS + level) * 2 + leg) * MAX_OUTER + outer) * 2 + axis


def ras_shifts(seed: int, cycle: int, level: int, leg: int, n_outer: int, tile: Tuple[int, int]):
    """(s_i, s_j) of each outer iteration of one smoothing call."""
    return [(splitmix64(seed, ras_key(cycle, level, leg, t, 0)) % tile[0],
             splitmix64(seed, ras_key(cycle, level, leg, t, 1)) % tile[1]) for t in range(n_outer)]


def node_indices(g):
    """(i, j) of every velocity unknown of a level, in vector order [vx; vy]."""
    I, J = np.meshgrid(np.arange(1, g.ny + 1), np.arange(1, g.nx), indexing="ij")
    I2, J2 = np.meshgrid(np.arange(1, g.ny), np.arange(1, g.nx + 1), indexing="ij")
    return np.concatenate([I.ravel(), I2.ravel()]), np.concatenate([J.ravel(), J2.ravel()])


def tiles(g, shift: Tuple[int, int], tile: Tuple[int, int]) -> List[np.ndarray]:
    """Index sets of the velocity unknowns owned by each tile of one outer iteration."""
    I, J = node_indices(g)
    ti = (I - 1 - shift[0]) // tile[0]
    tj = (J - 1 - shift[1]) // tile[1]
    key = ti * (g.nx + 2) + tj
    return [np.flatnonzero(key == k) for k in np.unique(key)]


def ras_jacobi(lev, e: np.ndarray, r: np.ndarray, omega: float, sweeps: int, tile: Tuple[int, int],
               inner: int, shifts: Sequence[Tuple[int, int]]) -> np.ndarray:
    """RAS-type temporal-blocking damped Jacobi on L e = r; one shift per outer iteration."""
    n_outer = -(-sweeps // inner) if sweeps > 0 else 0
    assert len(shifts) >= n_outer
    L, d = lev.L.tocsr(), lev.diag
    for t in range(n_outer):
        old = e
        new = e.copy()
        for S in tiles(lev.g, shifts[t], tile):
            LS = L[S]
            y = old.copy()
            for _ in range(inner):
                y[S] = y[S] + omega * (r[S] - LS @ y) / d[S]
            new[S] = y[S]
        e = new
    return e


def block_solve(lev, e: np.ndarray, r: np.ndarray, shift: Tuple[int, int], tile: Tuple[int, int]) -> np.ndarray:
    """Each tile solved exactly with every outside value frozen (the limit of many inner sweeps)."""
    L = lev.L.tocsr()
    new = e.copy()
    for S in tiles(lev.g, shift, tile):
        mask = np.ones(len(e), dtype=bool)
        mask[S] = False
        rhs = r[S] - L[S][:, mask] @ e[mask]
        new[S] = spla.spsolve(L[S][:, S].tocsc(), rhs)
    return new
