"""Marker <-> grid interpolation and RK4 marker advection (oracle; test infrastructure).

Only tests/, the smoke check and the CPU baseline of bench.py use this module.

What it computes (Ch. 4, Sec. "Interpolation Between Markers and Grid" and
Sec. "Advection of Lagrangian Markers"):

* Bilinear weights: a marker at (x, y) inside the cell of a node grid whose
  lower-left node is (i, j) at (x_j, y_i) has r_x = x - x_j, r_y = y - y_i
  and the four weights (1 - r_x/dx)(1 - r_y/dy), (r_x/dx)(1 - r_y/dy),
  (1 - r_x/dx)(r_y/dy), (r_x/dx)(r_y/dy) on (i, j), (i, j+1), (i+1, j),
  (i+1, j+1).
* Marker -> grid: phi(i, j) = sum_m w_m(i, j) phi_m / sum_m w_m(i, j) over
  the markers that reach node (i, j); a node no marker reaches gets `fill`.
* Grid -> marker: phi_m = sum over the four nodes of w phi(i, j).
* RK4 (eq. rk4_method): k1 = v(x), k2 = v(x + dt/2 k1), k3 = v(x + dt/2 k2),
  k4 = v(x + dt k3), x <- x + dt/6 (k1 + 2 k2 + 2 k3 + k4), v interpolated
  from the staggered vx and vy grids (grid -> marker).

Node grids (index convention of the (ny + 2) x (nx + 2) arrays):
  "basic": (j dx, i dy), i in [0, ny], j in [0, nx]   (eta_b, rho_b)
  "cell":  ((j - 1/2) dx, (i - 1/2) dy), i in [1, ny], j in [1, nx]   (eta_p, p)
  "vx":    (j dx, (i - 1/2) dy), i in [0, ny + 1], j in [0, nx]   (walls and ghost rows included)
  "vy":    ((j - 1/2) dx, i dy), i in [0, ny], j in [0, nx + 1]

Readings (where the text leaves a choice):

* Marker -> grid: a marker contributes only to the nodes of the grid's own
  range; near a wall some of its four weights fall on nodes outside that
  range (the cell grid's half-cell rim) and are dropped, which the
  normalisation absorbs.
* Grid -> marker: the cell containing the marker is taken within the
  grid's range (the reference index is clamped so that its four nodes
  exist) and r/d is clamped to [0, 1], so a marker in the cell grid's
  half-cell rim takes the value of the nearest row or column of centres
  (no extrapolation).  For vx and vy the ranges include the wall and ghost
  nodes, so no clamping happens inside the domain.
* Positions leave the box only by round-off or an intermediate RK stage
  near a wall (the normal velocity vanishes on the walls); every stage
  position and the result are clamped to [0, lx] x [0, ly].  The paper's
  listing wraps positions with a modulo because its example domain is
  periodic; this solver's box has walls.

Pins (tests/test_oracle_markers.py): one marker per node returns its value;
constants are reproduced; a symmetric lattice reproduces linear fields at
interior nodes; grid -> marker reproduces bilinear fields exactly and node
values at nodes; RK4 on a linear velocity field (exactly representable)
equals the closed-form amplification sum_k (dt A)^k / k! for k <= 4, and a
uniform field moves markers by dt v.
"""
from __future__ import annotations

import numpy as np

from .stokes import Grid

KINDS = ("basic", "cell", "vx", "vy")


def node_grid(g: Grid, kind: str):
    """(x0, y0, jmin, jmax, imin, imax): node (i, j) sits at (x0 + j dx, y0 + i dy)."""
    if kind == "basic":
        return 0.0, 0.0, 0, g.nx, 0, g.ny
    if kind == "cell":
        return -0.5 * g.dx, -0.5 * g.dy, 1, g.nx, 1, g.ny
    if kind == "vx":
        return 0.0, -0.5 * g.dy, 0, g.nx, 0, g.ny + 1
    if kind == "vy":
        return -0.5 * g.dx, 0.0, 0, g.nx + 1, 0, g.ny
    raise ValueError(kind)


def markers_to_grid(g: Grid, kind: str, xm: np.ndarray, ym: np.ndarray, phi: np.ndarray,
                    fill: float = 0.0) -> np.ndarray:
    """Normalised bilinear marker -> grid average on an (ny + 2) x (nx + 2) array."""
    x0, y0, jmin, jmax, imin, imax = node_grid(g, kind)
    num = np.zeros((g.ny + 2, g.nx + 2))
    den = np.zeros((g.ny + 2, g.nx + 2))
    j = np.floor((xm - x0) / g.dx).astype(np.int64)
    i = np.floor((ym - y0) / g.dy).astype(np.int64)
    rx = (xm - (x0 + j * g.dx)) / g.dx
    ry = (ym - (y0 + i * g.dy)) / g.dy
    for di, dj, w in ((0, 0, (1 - rx) * (1 - ry)), (0, 1, rx * (1 - ry)), (1, 0, (1 - rx) * ry), (1, 1, rx * ry)):
        ii, jj = i + di, j + dj
        ok = (ii >= imin) & (ii <= imax) & (jj >= jmin) & (jj <= jmax)
        np.add.at(num, (ii[ok], jj[ok]), w[ok] * phi[ok])
        np.add.at(den, (ii[ok], jj[ok]), w[ok])
    out = np.full((g.ny + 2, g.nx + 2), np.nan)
    sl = (slice(imin, imax + 1), slice(jmin, jmax + 1))
    has = den[sl] > 0
    out[sl] = np.where(has, num[sl] / np.where(has, den[sl], 1.0), fill)
    return out


def grid_to_markers(g: Grid, kind: str, grid: np.ndarray, xm: np.ndarray, ym: np.ndarray) -> np.ndarray:
    """Bilinear grid -> marker interpolation."""
    x0, y0, jmin, jmax, imin, imax = node_grid(g, kind)
    j = np.clip(np.floor((xm - x0) / g.dx).astype(np.int64), jmin, jmax - 1)
    i = np.clip(np.floor((ym - y0) / g.dy).astype(np.int64), imin, imax - 1)
    rx = np.clip((xm - (x0 + j * g.dx)) / g.dx, 0.0, 1.0)
    ry = np.clip((ym - (y0 + i * g.dy)) / g.dy, 0.0, 1.0)
    return ((1 - rx) * (1 - ry) * grid[i, j] + rx * (1 - ry) * grid[i, j + 1]
            + (1 - rx) * ry * grid[i + 1, j] + rx * ry * grid[i + 1, j + 1])


def _clamp(g: Grid, x, y):
    return np.clip(x, 0.0, g.lx), np.clip(y, 0.0, g.ly)


def rk4_advect(g: Grid, vx: np.ndarray, vy: np.ndarray, xm: np.ndarray, ym: np.ndarray, dt: float):
    """One classical RK4 step of dx/dt = v(x) with v interpolated from the staggered grids."""
    def v(x, y):
        return grid_to_markers(g, "vx", vx, x, y), grid_to_markers(g, "vy", vy, x, y)

    k1x, k1y = v(xm, ym)
    k2x, k2y = v(*_clamp(g, xm + 0.5 * dt * k1x, ym + 0.5 * dt * k1y))
    k3x, k3y = v(*_clamp(g, xm + 0.5 * dt * k2x, ym + 0.5 * dt * k2y))
    k4x, k4y = v(*_clamp(g, xm + dt * k3x, ym + dt * k3y))
    return _clamp(g, xm + dt / 6.0 * (k1x + 2 * k2x + 2 * k3x + k4x), ym + dt / 6.0 * (k1y + 2 * k2y + 2 * k3y + k4y))
