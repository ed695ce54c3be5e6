"""Flexible GCR(m) and Anderson acceleration AA(m, beta) (oracle; test infrastructure).

Only tests/, the smoke check and the CPU baseline of bench.py use this module.

What it computes (Ch. 4, Sec. "Accelerators"):

* The Uzawa iteration is the preconditioned Richardson iteration
  x <- x + M_k^{-1} (b - A x) of the splitting A = M - N (subsection "Uzawa
  Iteration as a Fixed Point Method"); M_k^{-1} is one application of the
  inexact Uzawa preconditioner (a multigrid velocity solve and the
  viscosity-scaled pressure correction), which may change between
  applications.  Both accelerators below take it as a black box.

* `gcr`: restarted flexible GCR(m), Alg. "Flexible GCR(m)".  Each inner step
  preconditions the current residual (z = M_k^{-1} r), applies the operator
  (w = A z), orthogonalises w against the earlier w's of the cycle by
  modified Gram-Schmidt while applying the same combination to z, normalises
  both by |w|, and updates x += alpha z, r -= alpha w with alpha = <r, w>.
  The residual is carried over a restart (the paper's recurrence); only the
  stored directions are dropped.

* `anderson`: AA(m) with mixing beta, Alg. "Anderson Acceleration(m) with
  Mixing".  x^1 = G(x^0); then for k = 1, 2, ...: m_k = min(m, k), the last
  m_k + 1 fixed-point residuals r^i = G(x^i) - x^i form R^k, alpha^k
  minimises |R^k alpha|_2 over the coefficient vectors that sum to one, and
  x^{k+1} = (1 - beta) sum_i alpha_i x^i + beta sum_i alpha_i G(x^i).

Readings (where the text leaves a choice):

* GCR's dot products and norms are taken in the energy inner product
  <u, v> = sum W u v, W the diagonal energy weights of Sec. "Residual
  Norms", the norm in which the solver measures convergence; with W = 1 this
  is the printed Euclidean form.  (A plain Euclidean residual would weight
  the momentum rows by h^-2 against the continuity rows.)
* The Anderson norm |R alpha|_2 is the Euclidean norm over the unknowns
  (vx, vy, p) as printed: its residuals are solution-space corrections,
  whose velocity and pressure parts carry no grid-size factor.
* "Until convergence": the relative energy residual of the current iterate
  at most rtol, tested before every application of M_k^{-1} (GCR: after
  every update, on the carried residual).  One iteration is one application
  of M_k^{-1}; max_iters bounds them.
* The constrained least-squares problem is solved by eliminating the
  constraint (alpha_last = 1 - sum of the others) and a minimum-norm
  least-squares solve of the remaining unknowns.

Pins (tests/test_oracle_accelerators.py): GCR equals the minimal-residual
iterate over the span of the preconditioned directions, computed by brute
force (fixed and changing preconditioners, weighted norm); GCR(1) is the
local minimal-residual step; an exact preconditioner converges in one step.
AA with beta = 1 and unbounded depth equals G applied to the GMRES iterate
on the fixed-point residual (the equivalence the paper states for the linear
case), built by brute force over the Krylov space; AA(0, beta) is the damped
Picard iteration in closed form; a fixed point is stationary; a nonlinear
contraction converges.
"""
from __future__ import annotations

from typing import Callable, List, Optional, Tuple

import numpy as np


def gcr(apply_A: Callable[[np.ndarray], np.ndarray], precond: Callable[[np.ndarray], np.ndarray],
        b: np.ndarray, x0: np.ndarray, m: int, weights: Optional[np.ndarray] = None, rtol: float = 1e-8,
        max_iters: int = 500) -> Tuple[np.ndarray, int, List[float]]:
    """Restarted flexible GCR(m).  Returns (x, iterations, relative residual after each iteration)."""
    W = np.ones_like(b) if weights is None else weights

    def dot(u, v):
        return float(np.sum(W * u * v))

    bnorm = np.sqrt(dot(b, b))
    x = x0.copy()
    r = b - apply_A(x)
    hist: List[float] = []

    def rel(rv):
        n = np.sqrt(dot(rv, rv))
        return n / bnorm if bnorm > 0 else n

    if bnorm == 0.0 or rel(r) <= rtol:
        return x, 0, hist
    its = 0
    while its < max_iters:
        ws: List[np.ndarray] = []
        zs: List[np.ndarray] = []
        for _ in range(m):
            z = precond(r)
            w = apply_A(z)
            for wj, zj in zip(ws, zs):                 # modified Gram-Schmidt
                gamma = dot(w, wj) / dot(wj, wj)
                w = w - gamma * wj
                z = z - gamma * zj
            nu = np.sqrt(dot(w, w))
            w = w / nu
            z = z / nu
            alpha = dot(r, w)
            x = x + alpha * z
            r = r - alpha * w
            ws.append(w)
            zs.append(z)
            its += 1
            hist.append(rel(r))
            if hist[-1] <= rtol or its >= max_iters:
                return x, its, hist
    return x, its, hist


def constrained_lsq(R: np.ndarray) -> np.ndarray:
    """alpha minimising |R alpha|_2 subject to sum(alpha) = 1 (columns of R are the residuals)."""
    n = R.shape[1]
    if n == 1:
        return np.ones(1)
    last = R[:, -1]
    D = R[:, :-1] - last[:, None]                       # alpha = e_last + sum_i gamma_i (e_i - e_last)
    gamma = np.linalg.lstsq(D, -last, rcond=None)[0]
    return np.concatenate([gamma, [1.0 - gamma.sum()]])


def anderson(G: Callable[[np.ndarray], np.ndarray], x0: np.ndarray, m: int, beta: float,
             converged: Callable[[np.ndarray], bool], max_iters: int = 500,
             alphas: Optional[list] = None) -> Tuple[np.ndarray, int]:
    """AA(m) with mixing beta on x = G(x).  Returns (x, number of G evaluations).

    `converged(x)` is tested on every iterate before G is applied to it; the
    coefficient vectors are appended to `alphas` when it is given.
    """
    if converged(x0) or max_iters < 1:
        return x0.copy(), 0
    xs = [x0.copy()]
    gs = [G(x0)]
    its = 1
    x = gs[0].copy()                                     # x^1 = G(x^0)
    k = 1
    while its < max_iters and not converged(x):
        gx = G(x)
        its += 1
        xs.append(x)
        gs.append(gx)
        mk = min(m, k)
        X = np.stack(xs[-(mk + 1):], axis=1)
        GX = np.stack(gs[-(mk + 1):], axis=1)
        a = constrained_lsq(GX - X)
        if alphas is not None:
            alphas.append(a)
        x = (1.0 - beta) * (X @ a) + beta * (GX @ a)
        k += 1
        if len(xs) > m + 1:                              # older pairs are never used again
            xs.pop(0)
            gs.pop(0)
    return x, its


def uzawa_system(g, eta_b: np.ndarray, eta_p: np.ndarray, prm, steps: int):
    """(A, M_k^{-1}, W) of one Stokes problem on vectors of unknowns [vx; vy; p]:
    the assembled operator, `steps` Uzawa sweeps of the multigrid
    preconditioner with parameters `prm` as a callable, and the energy weights."""
    from .multigrid import build_hierarchy, st_to_arrays_res, uzawa_preconditioner
    from .stokes import assemble, energy_weights, to_vector

    A = assemble(g, eta_b, eta_p)
    levs = build_hierarchy(g, eta_b, eta_p, prm)

    def precond(r: np.ndarray) -> np.ndarray:
        rx, ry, rp = st_to_arrays_res(g, r)
        zx, zy, zp = uzawa_preconditioner(levs, prm, A, rx, ry, rp, steps)
        return to_vector(g, zx, zy, zp)

    return A, precond, energy_weights(g, A, eta_p)
