"""Seeded synthetic inputs for the 2D variable-viscosity Stokes problem.

This module only *draws* inputs: material fields (viscosity at basic nodes and
at cell centres, density at basic nodes), gravity and boundary conditions.  It
holds none of the solver's arithmetic; both the CPU oracle and the GPU path
consume exactly the arrays produced here, bit for bit.

Array convention (staggered grid, Ch. 4 "Staggered Grid Layout"): a problem of
``nx`` x ``ny`` cells uses arrays of shape ``(ny + 2, nx + 2)``, row-major,
row index ``i`` along y and column index ``j`` along x.

* basic node ``(i, j)`` sits at ``(j*dx, i*dy)`` for ``i in [0, ny]``,
  ``j in [0, nx]``; it carries ``eta_b`` and ``rho_b``;
* cell centre ``(i, j)`` sits at ``((j-1/2)*dx, (i-1/2)*dy)`` for
  ``i in [1, ny]``, ``j in [1, nx]``; it carries ``eta_p`` (and pressure).

Entries outside those ranges are unused and set to 1 (viscosity) or 0
(density) so that no NaN ever reaches a kernel.

Recipes (all FP64, ``numpy.random.default_rng`` / PCG64):

* ``sinker``: one centred disc; a node is inside iff its squared distance to
  the centre is <= r^2 (closed disc), viscosity and density point-sampled.
* ``random_viscosity``: log10(eta_p) is a periodic Gaussian random field on
  the cell-centre lattice (Gaussian spectral filter with covariance
  exp(-r^2 / (2 l^2))), min/max normalised so the total contrast is exactly
  ``contrast``; eta_b = 10 ** (mean of log10 eta_p over the 1-4 cells that
  touch the node); rho_b = 1 - 0.01 log10(eta_b) + 0.01 N(0, 1).
* ``multi_inclusion``: discs painted in draw order over a background
  (eta = 1, rho = 0); later discs overwrite earlier ones.
* ``batch_sinkers``: independent sinkers of uneven square sizes.
* ``markers``: ``per_cell`` markers in every cell of a problem's grid at
  uniform random positions inside the cell (one seed), each carrying the
  viscosity eta_p of its cell and the density rho_b of the basic node
  nearest to it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

FREE_SLIP = 0
NO_SLIP = 1

__all__ = [
    "FREE_SLIP", "NO_SLIP", "Problem", "sinker", "grf", "random_viscosity",
    "multi_inclusion", "batch_sinkers", "adjoint_problem", "random_fields",
    "random_state", "logvisc_to_eta",
]


@dataclass
class Problem:
    """One Stokes problem: grid, material fields, gravity, boundary conditions.

    ``bc`` is per wall in the order (west x=0, east x=lx, south row 0,
    north row ny); each entry is ``FREE_SLIP`` or ``NO_SLIP``.
    """
    nx: int
    ny: int
    eta_b: np.ndarray
    eta_p: np.ndarray
    rho_b: np.ndarray
    gx: float = 0.0
    gy: float = -1.0
    lx: float = 1.0
    ly: float = 1.0
    bc: Tuple[int, int, int, int] = (FREE_SLIP,) * 4
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def _coords(nx: int, ny: int, lx: float, ly: float):
    dx, dy = lx / nx, ly / ny
    i = np.arange(ny + 2, dtype=np.float64)[:, None]
    j = np.arange(nx + 2, dtype=np.float64)[None, :]
    xb, yb = j * dx, i * dy                      # basic nodes
    xp, yp = (j - 0.5) * dx, (i - 0.5) * dy      # cell centres
    return (xb, yb), (xp, yp)


def _masks(nx: int, ny: int):
    basic = np.zeros((ny + 2, nx + 2), dtype=bool)
    basic[: ny + 1, : nx + 1] = True
    cell = np.zeros((ny + 2, nx + 2), dtype=bool)
    cell[1: ny + 1, 1: nx + 1] = True
    return basic, cell


def _paint_disc(nx, ny, lx, ly, cx, cy, r):
    (xb, yb), (xp, yp) = _coords(nx, ny, lx, ly)
    inb = (xb - cx) ** 2 + (yb - cy) ** 2 <= r * r
    inp = (xp - cx) ** 2 + (yp - cy) ** 2 <= r * r
    basic, cell = _masks(nx, ny)
    return inb & basic, inp & cell


def sinker(n: int, radius: float = 0.1, eta_in: float = 1e3,
           rho_in: float = 1.0, eta_out: float = 1.0, rho_out: float = 0.0,
           ny: Optional[int] = None, center=(0.5, 0.5), gx=0.0, gy=-1.0,
           lx=1.0, ly=1.0, bc=(FREE_SLIP,) * 4) -> Problem:
    """Centred circular inclusion in a uniform background (unit square)."""
    nx = n
    ny = n if ny is None else ny
    inb, inp = _paint_disc(nx, ny, lx, ly, center[0], center[1], radius)
    eta_b = np.full((ny + 2, nx + 2), eta_out)
    eta_p = np.full((ny + 2, nx + 2), eta_out)
    rho_b = np.zeros((ny + 2, nx + 2))
    basic, _ = _masks(nx, ny)
    rho_b[basic] = rho_out
    eta_b[inb] = eta_in
    eta_p[inp] = eta_in
    rho_b[inb] = rho_in
    return Problem(nx, ny, eta_b, eta_p, rho_b, gx, gy, lx, ly, tuple(bc),
                   name=f"sinker{nx}x{ny}",
                   meta=dict(radius=radius, eta_in=eta_in, rho_in=rho_in))


def grf(n: int, ell: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field on an n x n cell-centre lattice.

    White noise is filtered by the spectral factor exp(-(2 pi k)^2 s^2 / 2)
    with s = ell / sqrt(2), which gives the covariance exp(-r^2 / (2 ell^2))
    on the unit torus.  Returns the raw (unnormalised) real field.
    """
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n, d=1.0 / n)
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    s = ell / np.sqrt(2.0)
    filt = np.exp(-0.5 * (2.0 * np.pi) ** 2 * k2 * s * s)
    return np.real(np.fft.ifft2(np.fft.fft2(xi) * filt))


def logvisc_to_eta(m: np.ndarray, nx: int, ny: int):
    """Viscosity fields from a cell-centred log10-viscosity ``m`` (ny x nx).

    eta_p = 10 ** m at cell centres; eta_b at a basic node is 10 ** (mean of
    m over the 1-4 cells sharing that node).
    """
    eta_p = np.ones((ny + 2, nx + 2))
    eta_p[1: ny + 1, 1: nx + 1] = 10.0 ** m
    acc = np.zeros((ny + 1, nx + 1))
    cnt = np.zeros((ny + 1, nx + 1))
    # basic node (i, j) touches cells (i, j), (i+1, j), (i, j+1), (i+1, j+1)
    # in cell-centre indexing; with m indexed from 0 that is m[i-1 .. i, j-1 .. j].
    for di in (0, 1):
        for dj in (0, 1):
            acc[di: di + ny, dj: dj + nx] += m
            cnt[di: di + ny, dj: dj + nx] += 1.0
    eta_b = np.ones((ny + 2, nx + 2))
    eta_b[: ny + 1, : nx + 1] = 10.0 ** (acc / cnt)
    return eta_b, eta_p


def random_viscosity(n: int = 1024, ell: float = 0.05, contrast: float = 1e4,
                     seed_field: int = 2, seed_noise: int = 22,
                     gx=0.0, gy=-1.0, bc=(FREE_SLIP,) * 4) -> Problem:
    """Gaussian-random log-viscosity with a fixed total contrast."""
    g = grf(n, ell, seed_field)
    g = (g - g.min()) / (g.max() - g.min())
    decades = np.log10(contrast)
    m = decades * g - decades / 2.0
    eta_b, eta_p = logvisc_to_eta(m, n, n)
    rng = np.random.default_rng(seed_noise)
    zeta = rng.standard_normal((n + 1, n + 1))
    rho_b = np.zeros((n + 2, n + 2))
    rho_b[: n + 1, : n + 1] = (1.0 - 0.01 * np.log10(eta_b[: n + 1, : n + 1])
                               + 0.01 * zeta)
    return Problem(n, n, eta_b, eta_p, rho_b, gx, gy, 1.0, 1.0, tuple(bc),
                   name=f"grf{n}", meta=dict(m=m, ell=ell, contrast=contrast))


def multi_inclusion(n: int = 4096, count: int = 200, seed: int = 3,
                    rmin=0.005, rmax=0.03, gx=0.0, gy=-1.0) -> Problem:
    """Many discs of random radius, viscosity and density, painted in order."""
    rng = np.random.default_rng(seed)
    eta_b = np.ones((n + 2, n + 2))
    eta_p = np.ones((n + 2, n + 2))
    rho_b = np.zeros((n + 2, n + 2))
    dx = 1.0 / n
    ib = np.arange(n + 1)
    for _ in range(count):
        cx, cy = rng.uniform(0.0, 1.0, 2)
        r = rng.uniform(rmin, rmax)
        le = rng.uniform(-3.0, 3.0)
        rho = rng.uniform(-1.0, 1.0)
        # paint only the bounding box of the disc (same result as a full scan)
        lo_j = max(int(np.floor((cx - r) / dx)) - 1, 0)
        hi_j = min(int(np.ceil((cx + r) / dx)) + 2, n + 1)
        lo_i = max(int(np.floor((cy - r) / dx)) - 1, 0)
        hi_i = min(int(np.ceil((cy + r) / dx)) + 2, n + 1)
        jj = ib[lo_j:hi_j][None, :].astype(np.float64)
        ii = ib[lo_i:hi_i][:, None].astype(np.float64)
        inb = (jj * dx - cx) ** 2 + (ii * dx - cy) ** 2 <= r * r
        blk_b = (slice(lo_i, hi_i), slice(lo_j, hi_j))
        eta_b[blk_b][inb] = 10.0 ** le
        rho_b[blk_b][inb] = rho
        pi = np.arange(max(lo_i, 1), min(hi_i + 1, n + 1))
        pj = np.arange(max(lo_j, 1), min(hi_j + 1, n + 1))
        inp = (((pj[None, :] - 0.5) * dx - cx) ** 2
               + ((pi[:, None] - 0.5) * dx - cy) ** 2 <= r * r)
        blk_p = (slice(pi[0], pi[-1] + 1), slice(pj[0], pj[-1] + 1))
        eta_p[blk_p][inp] = 10.0 ** le
    return Problem(n, n, eta_b, eta_p, rho_b, gx, gy, 1.0, 1.0,
                   (FREE_SLIP,) * 4, name=f"multi{n}")


def batch_sinkers(count: int = 256, seed: int = 4,
                  sizes: Sequence[int] = (64, 128, 256, 512)) -> List[Problem]:
    """Independent centred sinkers with uneven square grid sizes."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(sizes[rng.integers(0, len(sizes))])
        r = rng.uniform(0.05, 0.2)
        lc = rng.uniform(1.0, 4.0)
        p = sinker(n, radius=r, eta_in=10.0 ** lc, rho_in=1.0)
        p.name = f"batch{k}_{n}"
        p.meta.update(log_contrast=lc)
        out.append(p)
    return out


def adjoint_problem(n: int = 1024, seed_pert: int = 5, seed_cells: int = 55,
                    n_cells: int = 64, amp: float = 0.2, ell: float = 0.05):
    """Inputs of the surface-velocity misfit gradient workload.

    Returns (base problem, m, m_true, probe cells).  ``m`` is the cell-centred
    log10 viscosity of the random-viscosity problem; ``m_true`` adds an
    independent random field (zero mean, unit std) scaled by ``amp``.  The
    density stays that of the base problem.  Probe cells are (i, j) cell
    indices in [1, n] drawn without replacement.
    """
    base = random_viscosity(n)
    m = base.meta["m"]
    gp = grf(n, ell, seed_pert)
    gp = (gp - gp.mean()) / gp.std()
    m_true = m + amp * gp
    rng = np.random.default_rng(seed_cells)
    flat = rng.choice(n * n, size=n_cells, replace=False)
    cells = np.stack([flat // n + 1, flat % n + 1], axis=1)
    return base, m, m_true, cells


def random_fields(nx: int, ny: int, seed: int, eta_decades: float = 2.0):
    """Random positive viscosities and random density (for operator tests)."""
    rng = np.random.default_rng(seed)
    eta_b = 10.0 ** rng.uniform(-eta_decades / 2, eta_decades / 2, (ny + 2, nx + 2))
    eta_p = 10.0 ** rng.uniform(-eta_decades / 2, eta_decades / 2, (ny + 2, nx + 2))
    rho_b = rng.uniform(-1.0, 1.0, (ny + 2, nx + 2))
    return eta_b, eta_p, rho_b


def random_state(nx: int, ny: int, seed: int):
    """Random (vx, vy, p) arrays of shape (ny+2, nx+2); only unknown entries
    are meaningful to a consumer (walls and ghosts are filled by it)."""
    rng = np.random.default_rng(seed)
    vx = rng.standard_normal((ny + 2, nx + 2))
    vy = rng.standard_normal((ny + 2, nx + 2))
    p = rng.standard_normal((ny + 2, nx + 2))
    return vx, vy, p


def markers(pr: "Problem", per_cell: int = 16, seed: int = 7):
    """Marker positions (x, y) and properties (eta, rho) for a problem; see the module recipes."""
    rng = np.random.default_rng(seed)
    nx, ny = pr.nx, pr.ny
    dx, dy = pr.lx / nx, pr.ly / ny
    ci = np.repeat(np.arange(ny), nx * per_cell)
    cj = np.tile(np.repeat(np.arange(nx), per_cell), ny)
    x = (cj + rng.random(ci.size)) * dx
    y = (ci + rng.random(ci.size)) * dy
    eta = pr.eta_p[ci + 1, cj + 1]
    rho = pr.rho_b[np.clip(np.rint(y / dy).astype(np.int64), 0, ny), np.clip(np.rint(x / dx).astype(np.int64), 0, nx)]
    return x, y, eta.astype(np.float64), rho.astype(np.float64)
