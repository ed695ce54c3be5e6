"""Viscosity rescaling and lithostatic initial pressure (oracle; test infrastructure).

Only tests/, the smoke check and the CPU baseline of bench.py use this module.

What it computes (Ch. 4, Sec. "Viscosity Rescaling and Initial Guess"):

* The computational viscosity of a continuation stage,
      eta_comp = (1 - theta) eta_min + theta eta,
  with eta_min the smallest viscosity of the domain (over the cell-centre
  field eta_p and the basic-node field eta_b), applied to both fields.
  theta = 1 gives eta back; theta = 0 a uniform field.
* The lithostatic pressure, the integral of rho g_y along y from the first
  cell row.  Reading on this grid: the discrete hydrostatic balance of the
  y-momentum rows for zero velocity, p(i+1, j) - p(i, j) = g_y dy rho_y(i, j)
  with rho_y(i, j) = (rho_b(i, j-1) + rho_b(i, j)) / 2 the density at the
  vy node between the two cells (the same average as the right-hand side),
  starting from p(1, j) = 0; the zero-mean constant is removed.  With this
  reading every y-momentum residual of (v = 0, p_litho) is exactly zero, and
  for uniform density it is the hydrostatic solution.

The continuation itself changes only the path to the solution: the final
stage solves the system with the original viscosity, so the oracle for a
continuation solve is `stokes.solve` with the original fields.

Pins (tests/test_oracle_continuation.py): zero y-momentum residual through
the assembled operator for random density; equality with the hydrostatic
closed form for uniform density; theta = 1 / theta = 0 / monotone blend.
"""
from __future__ import annotations

import numpy as np

from .stokes import Grid


def eta_min(g: Grid, eta_b: np.ndarray, eta_p: np.ndarray) -> float:
    """Smallest viscosity over the basic nodes (0..ny, 0..nx) and cells (1..ny, 1..nx)."""
    return float(min(eta_b[0:g.ny + 1, 0:g.nx + 1].min(), eta_p[1:g.ny + 1, 1:g.nx + 1].min()))


def rescaled_viscosity(g: Grid, eta_b: np.ndarray, eta_p: np.ndarray, theta: float, emin: float = None):
    """(eta_b_comp, eta_p_comp) of one continuation stage."""
    m = eta_min(g, eta_b, eta_p) if emin is None else emin
    return (1.0 - theta) * m + theta * eta_b, (1.0 - theta) * m + theta * eta_p


def lithostatic_pressure(g: Grid, rho_b: np.ndarray, gy: float) -> np.ndarray:
    """Zero-mean lithostatic pressure on the (ny+2) x (nx+2) cell array (ghosts 0)."""
    p = np.zeros((g.ny + 2, g.nx + 2))
    for j in range(1, g.nx + 1):
        acc = 0.0
        for i in range(1, g.ny + 1):
            p[i, j] = acc
            if i < g.ny:
                acc += gy * g.dy * 0.5 * (rho_b[i, j - 1] + rho_b[i, j])
    p[1:g.ny + 1, 1:g.nx + 1] -= p[1:g.ny + 1, 1:g.nx + 1].mean()
    return p
