"""Assembled FP64 Stokes operator and direct solve (oracle; test infrastructure).

What it computes
----------------
The discrete incompressible variable-viscosity Stokes system of Ch. 4,
"Stress-Conservative Finite Differences" and "Fast Solver for the Stokes
System" (eq. stokes_saddle):

    [ L  G ] [v]   [f]
    [ D  0 ] [p] = [0],     L v = div_h(eta (grad_h v + grad_h v^T)),
                            G p = -grad_h p,  D v = div_h v.

Each momentum row is written exactly as the stress-conservative stencil: the
x-momentum row at vx(i, j) combines sigma'_xx differences at the two
neighbouring cell centres (viscosity eta_p), sigma'_xy differences at the two
neighbouring basic nodes (viscosity eta_b) and the pressure difference, which
reproduces the nine velocity coefficients, four cross coefficients and two
pressure coefficients of the point-wise x-momentum operator of Ch. 6 ("Kernel
Implementation").  The y row is its mirror.

Boundary conditions (Ch. 3, "Boundary Conditions"; Ch. 4 "Staggered Grid
Layout"): normal velocities on the walls are zero; the tangential velocity in
the ghost row/column outside a wall equals +1 (free slip) or -1 (no slip)
times the adjacent interior value.  Ghost references are eliminated when the
matrix is assembled.

Readings adopted where the text is silent or inconsistent
---------------------------------------------------------
* The y-momentum right-hand side is f = -rho g (the body force rho g moved
  to the right of "L v + G p = f"), with density averaged from the two basic
  nodes adjacent to each velocity node.  The printed "= rho g_y" would make
  pressure decrease along gravity, which contradicts the lithostatic
  initial guess of Ch. 4 "Viscosity Rescaling and Initial Guess".
* Pressure is unique up to a constant (Ch. 4 "Pressure Nullspace
  Elimination"); the oracle fixes one cell's pressure, which that section
  states is equivalent to the zero-mean condition, then removes the mean.

Index convention: arrays are (ny+2) x (nx+2); vx unknowns i in [1, ny],
j in [1, nx-1]; vy unknowns i in [1, ny-1], j in [1, nx]; p unknowns
i in [1, ny], j in [1, nx].  The unknown vector is [vx; vy; p], each block
row-major.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FREE_SLIP = 0
NO_SLIP = 1


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    lx: float = 1.0
    ly: float = 1.0
    bc: Tuple[int, int, int, int] = (FREE_SLIP,) * 4   # west, east, south, north

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    def mirror(self, wall: int) -> float:
        """Ghost = mirror * interior for the tangential velocity at a wall."""
        return 1.0 if self.bc[wall] == FREE_SLIP else -1.0

    @property
    def n_vx(self) -> int:
        return self.ny * (self.nx - 1)

    @property
    def n_vy(self) -> int:
        return (self.ny - 1) * self.nx

    @property
    def n_p(self) -> int:
        return self.nx * self.ny

    @property
    def n(self) -> int:
        return self.n_vx + self.n_vy + self.n_p


W, E, S, N = 0, 1, 2, 3


def index_maps(g: Grid):
    """Arrays (ny+2, nx+2) giving the unknown number of each entry or -1."""
    shp = (g.ny + 2, g.nx + 2)
    ivx = -np.ones(shp, dtype=np.int64)
    ivy = -np.ones(shp, dtype=np.int64)
    ip = -np.ones(shp, dtype=np.int64)
    ivx[1:g.ny + 1, 1:g.nx] = np.arange(g.n_vx).reshape(g.ny, g.nx - 1)
    ivy[1:g.ny, 1:g.nx + 1] = g.n_vx + np.arange(g.n_vy).reshape(g.ny - 1, g.nx)
    ip[1:g.ny + 1, 1:g.nx + 1] = g.n_vx + g.n_vy + np.arange(g.n_p).reshape(g.ny, g.nx)
    return ivx, ivy, ip


def _resolve(g: Grid, maps, field: str, I: np.ndarray, J: np.ndarray):
    """Map references field[I, J] to (unknown column, factor).

    Wall entries resolve to factor 0; ghost entries resolve to the mirrored
    interior unknown with factor +1 / -1 according to the wall's condition.
    """
    ivx, ivy, ip = maps
    I = I.copy()
    J = J.copy()
    fac = np.ones(I.shape)
    if field == "vx":
        lo = I == 0
        hi = I == g.ny + 1
        fac[lo] *= g.mirror(S)
        fac[hi] *= g.mirror(N)
        I[lo] = 1
        I[hi] = g.ny
        col = ivx[I, J]
    elif field == "vy":
        lo = J == 0
        hi = J == g.nx + 1
        fac[lo] *= g.mirror(W)
        fac[hi] *= g.mirror(E)
        J[lo] = 1
        J[hi] = g.nx
        col = ivy[I, J]
    else:
        col = ip[I, J]
    fac[col < 0] = 0.0          # walls: prescribed zero normal velocity
    col = np.where(col < 0, 0, col)
    return col, fac


def stencil_terms(g: Grid):
    """Yield the stencil terms of every equation row.

    Each term is (row, field, I, J, scale, eta_kind, eI, eJ): the row gets
    ``scale * eta_kind[eI, eJ] * field[I, J]`` (``eta_kind`` None: no
    viscosity factor).  A is linear in the viscosities, so this list also
    gives dA/d(eta) term by term.
    """
    dx, dy = g.dx, g.dy
    ivx, ivy, ip = index_maps(g)
    one = None

    # ---- x-momentum at vx(i, j):  d(sxx)/dx + d(sxy)/dy - dp/dx ----------
    I, J = np.meshgrid(np.arange(1, g.ny + 1), np.arange(1, g.nx), indexing="ij")
    I, J = I.ravel(), J.ravel()
    r = ivx[I, J]
    c = np.ones(I.shape)
    # sxx(i,j+1) - sxx(i,j), sxx(cell) = 2 eta_p(cell) (vx right face - vx left face) / dx
    yield r, "vx", I, J + 1, 2 * c / dx ** 2, "p", I, J + 1
    yield r, "vx", I, J, -2 * c / dx ** 2, "p", I, J + 1
    yield r, "vx", I, J, -2 * c / dx ** 2, "p", I, J
    yield r, "vx", I, J - 1, 2 * c / dx ** 2, "p", I, J
    # sxy(i,j) - sxy(i-1,j), sxy(b) = eta_b(b) ((vx above - vx below)/dy + (vy right - vy left)/dx)
    yield r, "vx", I + 1, J, c / dy ** 2, "b", I, J
    yield r, "vx", I, J, -c / dy ** 2, "b", I, J
    yield r, "vy", I, J + 1, c / (dx * dy), "b", I, J
    yield r, "vy", I, J, -c / (dx * dy), "b", I, J
    yield r, "vx", I, J, -c / dy ** 2, "b", I - 1, J
    yield r, "vx", I - 1, J, c / dy ** 2, "b", I - 1, J
    yield r, "vy", I - 1, J + 1, -c / (dx * dy), "b", I - 1, J
    yield r, "vy", I - 1, J, c / (dx * dy), "b", I - 1, J
    # -(p(i,j+1) - p(i,j)) / dx
    yield r, "p", I, J + 1, -c / dx, one, None, None
    yield r, "p", I, J, c / dx, one, None, None

    # ---- y-momentum at vy(i, j):  d(syx)/dx + d(syy)/dy - dp/dy ----------
    I, J = np.meshgrid(np.arange(1, g.ny), np.arange(1, g.nx + 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    r = ivy[I, J]
    c = np.ones(I.shape)
    yield r, "vy", I + 1, J, 2 * c / dy ** 2, "p", I + 1, J
    yield r, "vy", I, J, -2 * c / dy ** 2, "p", I + 1, J
    yield r, "vy", I, J, -2 * c / dy ** 2, "p", I, J
    yield r, "vy", I - 1, J, 2 * c / dy ** 2, "p", I, J
    yield r, "vx", I + 1, J, c / (dx * dy), "b", I, J
    yield r, "vx", I, J, -c / (dx * dy), "b", I, J
    yield r, "vy", I, J + 1, c / dx ** 2, "b", I, J
    yield r, "vy", I, J, -c / dx ** 2, "b", I, J
    yield r, "vx", I + 1, J - 1, -c / (dx * dy), "b", I, J - 1
    yield r, "vx", I, J - 1, c / (dx * dy), "b", I, J - 1
    yield r, "vy", I, J, -c / dx ** 2, "b", I, J - 1
    yield r, "vy", I, J - 1, c / dx ** 2, "b", I, J - 1
    yield r, "p", I + 1, J, -c / dy, one, None, None
    yield r, "p", I, J, c / dy, one, None, None

    # ---- continuity at p(i, j):  dvx/dx + dvy/dy -----------------------
    I, J = np.meshgrid(np.arange(1, g.ny + 1), np.arange(1, g.nx + 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    r = ip[I, J]
    c = np.ones(I.shape)
    yield r, "vx", I, J, c / dx, one, None, None
    yield r, "vx", I, J - 1, -c / dx, one, None, None
    yield r, "vy", I, J, c / dy, one, None, None
    yield r, "vy", I - 1, J, -c / dy, one, None, None


def assemble(g: Grid, eta_b: np.ndarray, eta_p: np.ndarray) -> sp.csr_matrix:
    """Assemble A = [[L, G], [D, 0]] (no pressure constraint) as CSR."""
    maps = index_maps(g)
    rows, cols, vals = [], [], []
    for r, field, I, J, scale, ek, eI, eJ in stencil_terms(g):
        col, fac = _resolve(g, maps, field, I, J)
        coef = scale if ek is None else scale * (eta_b if ek == "b" else eta_p)[eI, eJ]
        v = coef * fac
        keep = v != 0.0
        rows.append(r[keep])
        cols.append(col[keep])
        vals.append(v[keep])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.n, g.n)).tocsr()
    A.sum_duplicates()
    return A


def rhs(g: Grid, rho_b: np.ndarray, gx: float, gy: float,
        fx_extra: Optional[np.ndarray] = None,
        fy_extra: Optional[np.ndarray] = None) -> np.ndarray:
    """b = [f_x; f_y; 0] with f = -rho g (density averaged to velocity nodes)."""
    fx = -gx * 0.5 * (rho_b[0:g.ny, 1:g.nx] + rho_b[1:g.ny + 1, 1:g.nx])
    fy = -gy * 0.5 * (rho_b[1:g.ny, 0:g.nx] + rho_b[1:g.ny, 1:g.nx + 1])
    if fx_extra is not None:
        fx = fx + fx_extra[1:g.ny + 1, 1:g.nx]
    if fy_extra is not None:
        fy = fy + fy_extra[1:g.ny, 1:g.nx + 1]
    return np.concatenate([fx.ravel(), fy.ravel(), np.zeros(g.n_p)])


def to_vector(g: Grid, vx, vy, p) -> np.ndarray:
    return np.concatenate([vx[1:g.ny + 1, 1:g.nx].ravel(),
                           vy[1:g.ny, 1:g.nx + 1].ravel(),
                           p[1:g.ny + 1, 1:g.nx + 1].ravel()])


def fill_ghosts(g: Grid, vx: np.ndarray, vy: np.ndarray) -> None:
    """Walls to zero, ghosts to mirror * interior (in place)."""
    vx[:, 0] = 0.0
    vx[:, g.nx] = 0.0
    vx[:, g.nx + 1] = 0.0
    vx[0, :] = g.mirror(S) * vx[1, :]
    vx[g.ny + 1, :] = g.mirror(N) * vx[g.ny, :]
    vy[0, :] = 0.0
    vy[g.ny, :] = 0.0
    vy[g.ny + 1, :] = 0.0
    vy[:, 0] = g.mirror(W) * vy[:, 1]
    vy[:, g.nx + 1] = g.mirror(E) * vy[:, g.nx]


def to_arrays(g: Grid, x: np.ndarray):
    shp = (g.ny + 2, g.nx + 2)
    vx, vy, p = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    vx[1:g.ny + 1, 1:g.nx] = x[:g.n_vx].reshape(g.ny, g.nx - 1)
    vy[1:g.ny, 1:g.nx + 1] = x[g.n_vx:g.n_vx + g.n_vy].reshape(g.ny - 1, g.nx)
    p[1:g.ny + 1, 1:g.nx + 1] = x[g.n_vx + g.n_vy:].reshape(g.ny, g.nx)
    fill_ghosts(g, vx, vy)
    return vx, vy, p


def bordered(g: Grid, A: sp.spmatrix) -> sp.csr_matrix:
    """[[A, c], [c^T, 0]] with c the indicator of the pressure block."""
    c = np.zeros(g.n)
    c[g.n_vx + g.n_vy:] = 1.0
    col = sp.csr_matrix(c[:, None])
    return sp.bmat([[A, col], [col.T, None]], format="csc")


def solve_system(g: Grid, A: sp.spmatrix, b: np.ndarray):
    """Direct solve (SuperLU, one refinement step) of A x = b, zero-mean p.

    The constant-pressure null space is removed by fixing the pressure of the
    last cell at zero (Ch. 4 "Pressure Nullspace Elimination": fixing one
    node is equivalent to the zero-mean condition), which drops that cell's
    continuity row and pressure column; the mean is subtracted afterwards.
    For a consistent right-hand side (pressure rows summing to zero, as for
    every body-force problem) the dropped row is implied by the others.
    Returns (x, residual of the dropped row).
    """
    nv = g.n_vx + g.n_vy
    keep = np.arange(g.n - 1)
    Ar = A[keep][:, keep].tocsc()
    lu = spla.splu(Ar)
    br = b[keep]
    xr = lu.solve(br)
    # one step of iterative refinement with the same factors: partial
    # pivoting on the indefinite saddle-point matrix leaves a residual well
    # above the rounding floor, one correction removes it
    xr = xr + lu.solve(br - Ar @ xr)
    x = np.concatenate([xr, [0.0]])
    dropped = float(b[-1] - A.getrow(g.n - 1).dot(x)[0])
    x[nv:] -= x[nv:].mean()
    return x, dropped


@dataclass
class Solution:
    vx: np.ndarray
    vy: np.ndarray
    p: np.ndarray
    x: np.ndarray
    dropped_residual: float
    residual_energy: float


def solve(g: Grid, eta_b, eta_p, rho_b, gx: float, gy: float,
          fx_extra=None, fy_extra=None) -> Solution:
    """Exact solution of the discrete system (SuperLU), zero-mean pressure."""
    A = assemble(g, eta_b, eta_p)
    b = rhs(g, rho_b, gx, gy, fx_extra, fy_extra)
    x, lam = solve_system(g, A, b)
    vx, vy, p = to_arrays(g, x)
    res = energy_residual(g, A, x, b, eta_p)
    return Solution(vx, vy, p, x, float(lam), res)


def energy_weights(g: Grid, A: sp.spmatrix, eta_p: np.ndarray) -> np.ndarray:
    """Diagonal energy weights (Ch. 4 "Residual Norms").

    Velocity rows: 1 / diag(-L).  Pressure rows: eta_p / (2/dx^2 + 2/dy^2).
    """
    d = -A.diagonal()[: g.n_vx + g.n_vy]
    wp = eta_p[1:g.ny + 1, 1:g.nx + 1].ravel() / (2.0 / g.dx ** 2 + 2.0 / g.dy ** 2)
    return np.concatenate([1.0 / d, wp])


def energy_residual(g: Grid, A, x, b, eta_p) -> float:
    """Relative energy residual sqrt((|r_v|^2_{L~^-1} + |r_p|^2_{S~^-1}) / |f|^2_{L~^-1})."""
    w = energy_weights(g, A, eta_p)
    r = b - A @ x
    num = float(np.sum(w * r * r))
    den = float(np.sum(w * b * b))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def apply(g: Grid, eta_b, eta_p, vx, vy, p):
    """A (vx, vy, p) as arrays (residual-space arrays, zero outside rows)."""
    A = assemble(g, eta_b, eta_p)
    y = A @ to_vector(g, vx, vy, p)
    shp = (g.ny + 2, g.nx + 2)
    ax, ay, ap = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    ax[1:g.ny + 1, 1:g.nx] = y[:g.n_vx].reshape(g.ny, g.nx - 1)
    ay[1:g.ny, 1:g.nx + 1] = y[g.n_vx:g.n_vx + g.n_vy].reshape(g.ny - 1, g.nx)
    ap[1:g.ny + 1, 1:g.nx + 1] = y[g.n_vx + g.n_vy:].reshape(g.ny, g.nx)
    return ax, ay, ap


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def parity_errors(g: Grid, ref: Solution, vx, vy, p):
    """Relative L2 errors of velocity (vx, vy together) and zero-mean pressure."""
    v_ref = np.concatenate([ref.vx[1:g.ny + 1, 1:g.nx].ravel(), ref.vy[1:g.ny, 1:g.nx + 1].ravel()])
    v = np.concatenate([vx[1:g.ny + 1, 1:g.nx].ravel(), vy[1:g.ny, 1:g.nx + 1].ravel()])
    pr = ref.p[1:g.ny + 1, 1:g.nx + 1].ravel()
    pp = p[1:g.ny + 1, 1:g.nx + 1].ravel()
    return rel_l2(v, v_ref), rel_l2(pp - pp.mean(), pr - pr.mean())
