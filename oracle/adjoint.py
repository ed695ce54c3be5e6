"""Surface-velocity misfit and its gradient (oracle; test infrastructure).

Misfit: J = 1/2 dx sum_{j=1}^{nx-1} (vx[ny, j] - t_j)^2, the horizontal
velocity of the top row of vx nodes (the row next to the wall opposite to a
gravity vector (0, -1)) against a target profile t.

Gradient by the adjoint method for A(eta) x = b(rho):
    A^T lam = dJ/dx,   dJ/d(eta) = -lam^T (dA/d(eta)) x,   dJ/d(rho) = lam^T db/d(rho).
A is linear in the viscosities, so dA/d(eta) is read term by term off the
stencil term list of ``stokes.stencil_terms``; b is linear in the density.
No strain-rate formula is used here.  A is symmetric, but the oracle solves
with the transpose anyway.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .stokes import (Grid, assemble, rhs, index_maps, stencil_terms, _resolve,
                     solve_system, to_arrays, to_vector)


def misfit(g: Grid, vx: np.ndarray, target: np.ndarray) -> float:
    d = vx[g.ny, 1:g.nx] - target
    return 0.5 * g.dx * float(np.sum(d * d))


def misfit_grad_vx(g: Grid, vx: np.ndarray, target: np.ndarray) -> np.ndarray:
    """dJ/d(vx) as an array of the vx shape (zero outside the top row)."""
    out = np.zeros((g.ny + 2, g.nx + 2))
    out[g.ny, 1:g.nx] = g.dx * (vx[g.ny, 1:g.nx] - target)
    return out


def adjoint_solve(g: Grid, A, gx_arr, gy_arr, gp_arr):
    """lam with A^T lam = [g_vx; g_vy; g_p] (zero-mean pressure part)."""
    rhs_vec = to_vector(g, gx_arr, gy_arr, gp_arr)
    lam, _ = solve_system(g, A.T.tocsr(), rhs_vec)
    return lam


def eta_gradient(g: Grid, x: np.ndarray, lam: np.ndarray):
    """(-lam^T dA/d eta_b x, -lam^T dA/d eta_p x) as (ny+2, nx+2) arrays."""
    maps = index_maps(g)
    gb = np.zeros((g.ny + 2, g.nx + 2))
    gp = np.zeros((g.ny + 2, g.nx + 2))
    for r, field, I, J, scale, ek, eI, eJ in stencil_terms(g):
        if ek is None:
            continue
        col, fac = _resolve(g, maps, field, I, J)
        contrib = -lam[r] * scale * fac * x[col]
        np.add.at(gb if ek == "b" else gp, (eI, eJ), contrib)
    return gb, gp


def rho_gradient(g: Grid, lam: np.ndarray, gx: float, gy: float) -> np.ndarray:
    """lam^T db/d(rho_b): b is linear in rho_b, so differentiate by unit pokes
    of a linear map (exact): db/d rho_b[k] = rhs(e_k) - rhs(0)."""
    out = np.zeros((g.ny + 2, g.nx + 2))
    base = rhs(g, np.zeros((g.ny + 2, g.nx + 2)), gx, gy)
    for i in range(g.ny + 1):
        for j in range(g.nx + 1):
            e = np.zeros((g.ny + 2, g.nx + 2))
            e[i, j] = 1.0
            out[i, j] = float(lam @ (rhs(g, e, gx, gy) - base))
    return out


def gradient(g: Grid, eta_b, eta_p, rho_b, gx, gy, target, with_rho=True):
    """Forward solve, misfit, adjoint solve and all three gradients."""
    A = assemble(g, eta_b, eta_p)
    b = rhs(g, rho_b, gx, gy)
    x, _ = solve_system(g, A, b)
    vx, vy, p = to_arrays(g, x)
    J = misfit(g, vx, target)
    zeros = np.zeros_like(vx)
    lam = adjoint_solve(g, A, misfit_grad_vx(g, vx, target), zeros, zeros)
    gb, gp = eta_gradient(g, x, lam)
    grho = rho_gradient(g, lam, gx, gy) if with_rho else None
    lx, ly, lp = to_arrays(g, lam)
    return dict(J=J, vx=vx, vy=vy, p=p, lam=(lx, ly, lp), g_eta_b=gb, g_eta_p=gp,
                g_rho_b=grho)


def chain_to_logvisc(g: Grid, g_eta_b, g_eta_p, eta_b, eta_p):
    """dJ/dm for eta_p = 10**m and eta_b = 10**(mean of m over touching cells)."""
    ln10 = np.log(10.0)
    ny, nx = g.ny, g.nx
    gm = ln10 * eta_p[1:ny + 1, 1:nx + 1] * g_eta_p[1:ny + 1, 1:nx + 1]
    cnt = np.zeros((ny + 1, nx + 1))
    for di in (0, 1):
        for dj in (0, 1):
            cnt[di:di + ny, dj:dj + nx] += 1.0
    wb = ln10 * eta_b[:ny + 1, :nx + 1] * g_eta_b[:ny + 1, :nx + 1] / cnt
    for di in (0, 1):
        for dj in (0, 1):
            gm += wb[di:di + ny, dj:dj + nx]
    return gm
