"""Plain references of the multigrid preconditioner (oracle; test infrastructure).

Everything here follows Ch. 4 "The Multigrid Method" and "Accelerators":

* restriction: normalised bilinear weighting, sum_w w r / sum_w w over every
  fine node inside the physical domain (Sec. "Restriction and Prolongation
  Operators", Alg. "4-Color Parallel Restriction").  The weights are computed
  from node coordinates with the hat function (1 - |r_x|)(1 - |r_y|) of
  Sec. "Interpolation Between Markers and Grid"; no weight table is typed in,
  so any coarsening factor works (the paper coarsens by 2.5 in its sinker
  test; ``coarsen``, ``coarse_cells``); ``bisect_bound`` is the index search
  of Alg. "Bisect Bound".
  The four-colour ordering of the algorithm only serves race-freedom of a
  parallel scatter; the sums it forms are the ones computed here.
* prolongation: bilinear interpolation whose weights sum to one, from the
  coarse field with its boundary ghosts mirrored first.
* coarse levels: the same stencil rediscretised with restricted viscosities
  (geometric multigrid, Sec. "Geometric vs Algebraic Multigrid").
* damped Jacobi (eq. damped_jacobi), the RAS-type temporal-blocking Jacobi
  of Alg. "RAS-Type Temporal Blocking" (module ``ras``; on every level or,
  as the paper's "Mixed" configuration, below the finest) and damped
  Gauss-Seidel with a parallel colouring (eq. sor_update); the colouring is vx-red, vx-black, vy-red,
  vy-black with red = (i + j) even, since the vx/vy cross terms couple the
  two velocity components at nodes of either parity.
* V-cycle (eq. multigrid_levels), exact coarsest solve.
* Uzawa preconditioner M^{-1} of the splitting A = M - N (Sec. "Uzawa
  Iteration as a Fixed Point Method"): z_v = V(r_v) ~ L^{-1} r_v, then the
  viscosity-scaled pressure step z_p = alpha eta_p (r_p - D z_v).

Reading (documented): with the paper's operators G = -grad_h, D = div_h and
L negative definite, D L^{-1} G is approximately -1/(2 eta) and the printed
update p += alpha eta D v makes the stationary Uzawa iteration expand the
pressure error by 1 + alpha/2; the sign is taken so that it contracts
(factor 1 - alpha/2), i.e. M = [[L, 0], [D, +(alpha eta)^{-1}]].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .stokes import Grid, assemble, index_maps, fill_ghosts, S, N, W, E
from .stokes import to_vector as st_to_vector, to_arrays as st_to_arrays_sol


def st_to_arrays_res(g: Grid, x: np.ndarray):
    """Residual-type arrays (zero outside the equation rows) from a vector."""
    shp = (g.ny + 2, g.nx + 2)
    ax, ay, ap = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    ax[1:g.ny + 1, 1:g.nx] = x[:g.n_vx].reshape(g.ny, g.nx - 1)
    ay[1:g.ny, 1:g.nx + 1] = x[g.n_vx:g.n_vx + g.n_vy].reshape(g.ny - 1, g.nx)
    ap[1:g.ny + 1, 1:g.nx + 1] = x[g.n_vx + g.n_vy:].reshape(g.ny, g.nx)
    return ax, ay, ap

# ---------------------------------------------------------------------------
# node coordinates of the four staggered grids (1D, separable)
# ---------------------------------------------------------------------------


def axis_coords(g: Grid, kind: str):
    """(x[j], inside_x[j]), (y[i], inside_y[i]) for j in [0, nx+1], i in [0, ny+1]."""
    j = np.arange(g.nx + 2, dtype=np.float64)
    i = np.arange(g.ny + 2, dtype=np.float64)
    node_x = kind in ("vx", "basic")      # x on basic-node columns
    node_y = kind in ("vy", "basic")      # y on basic-node rows
    x = j * g.dx if node_x else (j - 0.5) * g.dx
    y = i * g.dy if node_y else (i - 0.5) * g.dy
    in_x = (j <= g.nx) if node_x else ((j >= 1) & (j <= g.nx))
    in_y = (i <= g.ny) if node_y else ((i >= 1) & (i <= g.ny))
    return (x, in_x), (y, in_y)


def hat(t: np.ndarray) -> np.ndarray:
    return np.maximum(0.0, 1.0 - np.abs(t))


def coarse_cells(n: int, factor: float) -> int:
    """Cells of the next coarser level along one axis: n / factor rounded to
    the nearest integer (halves up), at least 2.  The paper coarsens its
    501 x 601-node sinker grid by 2.5 per level (Ch. 4, robustness test);
    with a factor that does not divide the cell count the coarse nodes fall
    between fine nodes, which the coordinate-based transfers below handle."""
    return max(2, int(np.floor(n / factor + 0.5)))


def coarsen(g: Grid, factor: float = 2.0) -> Grid:
    """The next coarser uniform grid on the same domain (factor 2: exact halving)."""
    if factor == 2.0:
        assert g.nx % 2 == 0 and g.ny % 2 == 0
        return Grid(g.nx // 2, g.ny // 2, g.lx, g.ly, g.bc)
    return Grid(coarse_cells(g.nx, factor), coarse_cells(g.ny, factor), g.lx, g.ly, g.bc)


def bisect_bound(x: np.ndarray, xt: float) -> int:
    """Smallest index i with x[i] >= xt in a non-decreasing array x (the last
    index when none is), by halving [0, n - 1] (Alg. "Bisect Bound")."""
    lo, hi = 0, len(x) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if x[mid] < xt:
            lo = mid + 1
        else:
            hi = mid
    return lo


# ---------------------------------------------------------------------------
# restriction and prolongation
# ---------------------------------------------------------------------------


def restrict(gf: Grid, kind: str, u: np.ndarray, gc: Optional[Grid] = None) -> np.ndarray:
    """Normalised bilinear restriction of a fine array to the coarse grid
    ``gc`` (default: the factor-2 coarsening of ``gf``).

    Every coarse node of the grid ``kind`` (entries [0, N+1]) receives
    sum w u / sum w over fine nodes inside the domain; coarse nodes with no
    contributing fine node are 0.  Values at fine walls enter with their
    stored value (zero for residuals).
    """
    gc = coarsen(gf) if gc is None else gc
    (xf, inxf), (yf, inyf) = axis_coords(gf, kind)
    (xc, _), (yc, _) = axis_coords(gc, kind)
    wx = hat((xf[None, :] - xc[:, None]) / gc.dx) * inxf[None, :]
    wy = hat((yf[None, :] - yc[:, None]) / gc.dy) * inyf[None, :]
    num = wy @ u @ wx.T
    den = wy.sum(axis=1)[:, None] * wx.sum(axis=1)[None, :]
    out = np.zeros_like(num)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out


def prolong(gc: Grid, kind: str, uc: np.ndarray, gf: Grid) -> np.ndarray:
    """Bilinear interpolation of a coarse array (ghosts already mirrored)."""
    (xf, _), (yf, _) = axis_coords(gf, kind)
    (xc, _), (yc, _) = axis_coords(gc, kind)
    px = hat((xf[:, None] - xc[None, :]) / gc.dx)
    py = hat((yf[:, None] - yc[None, :]) / gc.dy)
    return py @ uc @ px.T


def coarse_viscosity(gf: Grid, eta_b: np.ndarray, eta_p: np.ndarray,
                     mean: str = "arithmetic", gc: Optional[Grid] = None):
    """Coarse-level viscosities by normalised bilinear restriction to ``gc``
    (default: the factor-2 coarsening of ``gf``).

    ``mean='geometric'`` restricts log(eta) instead.  Unused entries are 1.
    """
    gc = coarsen(gf) if gc is None else gc
    if mean == "geometric":
        cb = np.exp(restrict(gf, "basic", np.log(eta_b), gc))
        cp = np.exp(restrict(gf, "p", np.log(eta_p), gc))
    else:
        cb = restrict(gf, "basic", eta_b, gc)
        cp = restrict(gf, "p", eta_p, gc)
    ob = np.ones((gc.ny + 2, gc.nx + 2))
    op = np.ones((gc.ny + 2, gc.nx + 2))
    ob[: gc.ny + 1, : gc.nx + 1] = cb[: gc.ny + 1, : gc.nx + 1]
    op[1: gc.ny + 1, 1: gc.nx + 1] = cp[1: gc.ny + 1, 1: gc.nx + 1]
    # fine entries outside the domain are excluded, so restrict() must not
    # have read them; unused fine entries could hold anything
    return ob, op


# ---------------------------------------------------------------------------
# velocity block helpers
# ---------------------------------------------------------------------------


@dataclass
class Level:
    g: Grid
    eta_b: np.ndarray
    eta_p: np.ndarray
    L: sp.csr_matrix = None
    diag: np.ndarray = None
    colors: List[np.ndarray] = field(default_factory=list)

    def __post_init__(self):
        A = assemble(self.g, self.eta_b, self.eta_p)
        nv = self.g.n_vx + self.g.n_vy
        self.L = A[:nv, :nv].tocsr()
        self.diag = self.L.diagonal()
        g = self.g
        I, J = np.meshgrid(np.arange(1, g.ny + 1), np.arange(1, g.nx), indexing="ij")
        par_x = ((I + J) % 2).ravel()
        I, J = np.meshgrid(np.arange(1, g.ny), np.arange(1, g.nx + 1), indexing="ij")
        par_y = ((I + J) % 2).ravel()
        ix = np.arange(g.n_vx)
        iy = g.n_vx + np.arange(g.n_vy)
        self.colors = [ix[par_x == 0], ix[par_x == 1], iy[par_y == 0], iy[par_y == 1]]


def vel_to_vec(g: Grid, ex: np.ndarray, ey: np.ndarray) -> np.ndarray:
    return np.concatenate([ex[1:g.ny + 1, 1:g.nx].ravel(), ey[1:g.ny, 1:g.nx + 1].ravel()])


def vec_to_vel(g: Grid, v: np.ndarray):
    shp = (g.ny + 2, g.nx + 2)
    ex, ey = np.zeros(shp), np.zeros(shp)
    ex[1:g.ny + 1, 1:g.nx] = v[:g.n_vx].reshape(g.ny, g.nx - 1)
    ey[1:g.ny, 1:g.nx + 1] = v[g.n_vx:].reshape(g.ny - 1, g.nx)
    fill_ghosts(g, ex, ey)
    return ex, ey


def jacobi(lev: Level, e: np.ndarray, r: np.ndarray, omega: float, sweeps: int) -> np.ndarray:
    """Damped Jacobi on L e = r: e <- e + omega D^{-1} (r - L e)."""
    for _ in range(sweeps):
        e = e + omega * (r - lev.L @ e) / lev.diag
    return e


def colored_gs(lev: Level, e: np.ndarray, r: np.ndarray, omega: float, sweeps: int) -> np.ndarray:
    """Damped coloured Gauss-Seidel: four half-sweeps per sweep.

    Nodes of one colour are not coupled to each other, so updating them all
    at once from the current residual equals the sequential Gauss-Seidel
    update over that colour.
    """
    e = e.copy()
    for _ in range(sweeps):
        for c in lev.colors:
            res = r[c] - lev.L[c] @ e
            e[c] = e[c] + omega * res / lev.diag[c]
    return e


# ---------------------------------------------------------------------------
# V-cycle and Uzawa preconditioner
# ---------------------------------------------------------------------------


@dataclass
class MGParams:
    levels: int
    nu_pre: Sequence[int]
    nu_post: Sequence[int]
    omega: float = 0.6
    smoother: str = "jacobi"        # "gs", "ras" (every level) or "ras_mixed" (Jacobi on the finest)
    alpha: float = 2.0
    eta_mean: str = "arithmetic"
    ras_tile: int = 32              # RAS tile side (T_I = T_J)
    ras_inner: int = 4              # RAS local sweeps per outer iteration
    seed: int = 0                   # RAS shift generator seed
    coarsen: float = 2.0            # coarsening factor between levels (coarse_cells)


def build_hierarchy(g: Grid, eta_b, eta_p, prm: MGParams) -> List[Level]:
    levs = [Level(g, eta_b, eta_p)]
    for _ in range(1, prm.levels):
        gc = coarsen(levs[-1].g, prm.coarsen)
        cb, cp = coarse_viscosity(levs[-1].g, levs[-1].eta_b, levs[-1].eta_p, prm.eta_mean, gc)
        levs.append(Level(gc, cb, cp))
    return levs


def _smoother(prm: MGParams, l: int, cycle: int):
    """The smoothing routine of level l: fn(lev, e, r, omega, sweeps, leg)."""
    ras_here = prm.smoother == "ras" or (prm.smoother == "ras_mixed" and l > 0)
    if ras_here:
        from .ras import ras_jacobi, ras_shifts
        T = (prm.ras_tile, prm.ras_tile)

        def fn(lev, e, r, omega, sweeps, leg):
            n_outer = -(-sweeps // prm.ras_inner) if sweeps > 0 else 0
            sh = ras_shifts(prm.seed, cycle, l, leg, n_outer, T)
            return ras_jacobi(lev, e, r, omega, sweeps, T, prm.ras_inner, sh)
        return fn
    base = colored_gs if prm.smoother == "gs" else jacobi
    return lambda lev, e, r, omega, sweeps, leg: base(lev, e, r, omega, sweeps)


def vcycle(levs: List[Level], prm: MGParams, l: int, r: np.ndarray, cycle: int = 0) -> np.ndarray:
    """Approximate L_l^{-1} r by one V-cycle from zero initial guess (`cycle`
    numbers the V-cycles of one preconditioner call: the RAS shifts depend on it)."""
    lev = levs[l]
    if l == len(levs) - 1:
        return spla.spsolve(lev.L.tocsc(), r)
    smooth = _smoother(prm, l, cycle)
    e = np.zeros_like(r)
    e = smooth(lev, e, r, prm.omega, prm.nu_pre[l], 0)
    res = r - lev.L @ e
    g, gc = lev.g, levs[l + 1].g
    rx, ry = vec_to_vel(g, res)
    # residual arrays: only unknown entries are meaningful, ghosts excluded
    rx[0, :] = 0.0
    rx[g.ny + 1, :] = 0.0
    ry[:, 0] = 0.0
    ry[:, g.nx + 1] = 0.0
    rcx = restrict(g, "vx", rx, gc)
    rcy = restrict(g, "vy", ry, gc)
    ec = vcycle(levs, prm, l + 1, vel_to_vec(gc, rcx, rcy), cycle)
    ecx, ecy = vec_to_vel(gc, ec)
    fx = prolong(gc, "vx", ecx, g)
    fy = prolong(gc, "vy", ecy, g)
    e = e + vel_to_vec(g, fx, fy)
    e = smooth(lev, e, r, prm.omega, prm.nu_post[l], 1)
    return e


def divergence(g: Grid, vx: np.ndarray, vy: np.ndarray) -> np.ndarray:
    """D v at cell centres (array), walls taken as zero."""
    out = np.zeros((g.ny + 2, g.nx + 2))
    out[1:g.ny + 1, 1:g.nx + 1] = ((vx[1:g.ny + 1, 1:g.nx + 1] - vx[1:g.ny + 1, 0:g.nx]) / g.dx
                                   + (vy[1:g.ny + 1, 1:g.nx + 1] - vy[0:g.ny, 1:g.nx + 1]) / g.dy)
    return out


def precondition(levs: List[Level], prm: MGParams, rx, ry, rp, cycle: int = 0):
    """One application of the Uzawa preconditioner M^{-1} to (r_v, r_p)."""
    g = levs[0].g
    zv = vcycle(levs, prm, 0, vel_to_vec(g, rx, ry), cycle)
    zx, zy = vec_to_vel(g, zv)
    dz = divergence(g, zx, zy)
    zp = np.zeros_like(rp)
    sl = (slice(1, g.ny + 1), slice(1, g.nx + 1))
    zp[sl] = prm.alpha * levs[0].eta_p[sl] * (rp[sl] - dz[sl])
    return zx, zy, zp


def uzawa_preconditioner(levs: List[Level], prm: MGParams, A, rx, ry, rp, steps: int):
    """`steps` sweeps of the Uzawa fixed-point iteration x <- x + M^{-1}(b - A x)
    from x = 0 (Sec. "Uzawa Iteration as a Fixed Point Method", preconditioned
    Richardson form), with b = (r_v, r_p)."""
    g = levs[0].g
    r = st_to_vector(g, rx, ry, rp)
    z = np.zeros_like(r)
    for step in range(steps):
        tx, ty, tp = st_to_arrays_res(g, r - A @ z)
        dx_, dy_, dp_ = precondition(levs, prm, tx, ty, tp, step)
        z = z + st_to_vector(g, dx_, dy_, dp_)
    return st_to_arrays_sol(g, z)


def default_schedule(levels: int, nu: int = 2, growth: float = 1.0):
    return [int(np.ceil(nu * growth ** l)) for l in range(levels)]
