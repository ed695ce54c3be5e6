"""Pins of the oracle's accelerators (flexible GCR(m), Anderson AA(m, beta)).

Each check compares against something other than the oracle's own steps:

* GCR: the minimal-residual iterate over x0 + span{z_0 .. z_{k-1}} of the
  preconditioned directions it drew (brute-force weighted least squares),
  for a fixed and for a changing preconditioner; GCR(1) against the local
  minimal-residual step in closed form; an exact preconditioner converges
  in one iteration.  A dropped Gram-Schmidt term, a wrong sign of alpha, a
  missing update of z or a wrong normalisation breaks the first one.
* Anderson: with beta = 1 and depth at least the iteration count, on an
  affine map G(x) = T x + c the iterates are G applied to the GMRES iterates
  that minimise |G(x) - x|_2 over the Krylov space of I - T (built by brute
  force) -- the GMRES equivalence of the linear case stated with the
  algorithm; AA(0, beta) is the damped Picard iteration, in closed form
  through matrix powers; a fixed point is stationary; coefficients sum to
  one; a nonlinear contraction converges.
* Both accelerate the oracle's Uzawa iteration on a small Stokes problem to
  the direct solution.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import accelerators as acc
from oracle import multigrid as mg
from oracle import stokes as st


def _rand_system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    A = shift * np.eye(n) + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    return A, b, rng


def _min_res_over(A, b, x0, Z, w):
    """argmin_{x in x0 + span(Z)} |b - A x|_W by weighted least squares."""
    s = np.sqrt(w)
    r0 = b - A @ x0
    y = np.linalg.lstsq(s[:, None] * (A @ Z), s * r0, rcond=None)[0]
    return x0 + Z @ y


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_gcr_is_minimal_residual_over_preconditioned_directions(k):
    n = 40
    A, b, rng = _rand_system(n, 11)
    Minv = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    w = rng.uniform(0.2, 3.0, n)
    zs = []

    def pre(r):
        z = Minv @ r
        zs.append(z)
        return z

    x0 = rng.standard_normal(n)
    x, its, hist = acc.gcr(lambda v: A @ v, pre, b, x0, m=10, weights=w, rtol=0.0, max_iters=k)
    assert its == k
    ref = _min_res_over(A, b, x0, np.stack(zs, axis=1), w)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    # the carried residual history is that of the true residual, non-increasing
    wn = lambda r: np.sqrt(np.sum(w * r * r))
    assert hist[-1] == pytest.approx(wn(b - A @ x) / wn(b), rel=1e-9)
    assert all(h1 <= h0 * (1 + 1e-12) for h0, h1 in zip(hist, hist[1:]))


def test_gcr_flexible_preconditioner():
    # a preconditioner that changes every application (alternating matrices)
    n = 30
    A, b, rng = _rand_system(n, 5)
    P = [np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n) for _ in range(2)]
    zs = []

    def pre(r):
        z = P[len(zs) % 2] @ r
        zs.append(z)
        return z

    x, its, _ = acc.gcr(lambda v: A @ v, pre, b, np.zeros(n), m=8, rtol=0.0, max_iters=6)
    ref = _min_res_over(A, b, np.zeros(n), np.stack(zs, axis=1), np.ones(n))
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_gcr_restart_one_is_local_minimal_residual_step():
    n = 25
    A, b, rng = _rand_system(n, 8)
    w = rng.uniform(0.5, 2.0, n)
    x_ref = np.zeros(n)
    for _ in range(5):
        r = b - A @ x_ref
        q = A @ r
        x_ref = x_ref + np.sum(w * r * q) / np.sum(w * q * q) * r
    x, its, _ = acc.gcr(lambda v: A @ v, lambda r: r, b, np.zeros(n), m=1, weights=w, rtol=0.0, max_iters=5)
    assert its == 5
    assert np.allclose(x, x_ref, rtol=1e-11, atol=1e-13)


def test_gcr_exact_preconditioner_converges_in_one_step():
    n = 20
    A, b, _ = _rand_system(n, 3)
    x, its, hist = acc.gcr(lambda v: A @ v, lambda r: np.linalg.solve(A, r), b, np.zeros(n), m=5, rtol=1e-12)
    assert its == 1 and hist[0] <= 1e-13
    assert np.allclose(A @ x, b, atol=1e-12)


def test_gcr_zero_rhs_returns_initial_guess():
    A, _, _ = _rand_system(10, 2)
    x, its, hist = acc.gcr(lambda v: A @ v, lambda r: r, np.zeros(10), np.zeros(10), m=3)
    assert its == 0 and not hist and not x.any()


def _affine(n, seed, rho=0.8):
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((n, n))
    T *= rho / max(abs(np.linalg.eigvals(T)))
    c = rng.standard_normal(n)
    return T, c, rng


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_anderson_full_depth_equals_gmres_then_G(k):
    n = 30
    T, c, rng = _affine(n, 21)
    G = lambda x: T @ x + c
    x0 = rng.standard_normal(n)
    # GMRES on (I - T) x = c from x0: minimise |G(x) - x|_2 over x0 + K_k(I - T, f0)
    B = np.eye(n) - T
    f0 = G(x0) - x0
    K = [f0]
    for _ in range(k - 1):
        K.append(B @ K[-1])
    K = np.stack(K, axis=1)
    y = np.linalg.lstsq(B @ K, f0, rcond=None)[0]
    x_gm = x0 + K @ y
    x_aa, its = acc.anderson(G, x0, m=50, beta=1.0, converged=lambda x: False, max_iters=k + 1)
    assert its == k + 1
    ref = G(x_gm)
    assert np.linalg.norm(x_aa - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("beta", [1.0, 0.6])
def test_anderson_depth_zero_is_damped_picard(beta):
    n = 20
    T, c, rng = _affine(n, 4, rho=0.7)
    x0 = rng.standard_normal(n)
    xs = np.linalg.solve(np.eye(n) - T, c)
    K = 6
    x, its = acc.anderson(lambda x: T @ x + c, x0, m=0, beta=beta, converged=lambda x: False, max_iters=K)
    # x^1 = G(x^0), then x^{k+1} - x* = (I - beta (I - T)) (x^k - x*)
    E = np.linalg.matrix_power(np.eye(n) - beta * (np.eye(n) - T), K - 1) @ T
    assert np.allclose(x - xs, E @ (x0 - xs), rtol=1e-10, atol=1e-12)


def test_anderson_coefficients_sum_to_one_and_fixed_point_is_stationary():
    n = 15
    T, c, rng = _affine(n, 9)
    G = lambda x: T @ x + c
    alphas = []
    acc.anderson(G, rng.standard_normal(n), m=3, beta=0.7, converged=lambda x: False, max_iters=8, alphas=alphas)
    assert len(alphas) == 7
    assert [len(a) for a in alphas] == [2, 3, 4, 4, 4, 4, 4]
    for a in alphas:
        assert abs(a.sum() - 1.0) <= 1e-12
    xs = np.linalg.solve(np.eye(n) - T, c)
    x, _ = acc.anderson(G, xs, m=3, beta=0.7, converged=lambda x: False, max_iters=6)
    assert np.allclose(x, xs, rtol=1e-12, atol=1e-12)


def test_anderson_nonlinear_contraction():
    # componentwise x = 0.5 cos(x) + c: a contraction with a unique fixed point
    c = np.linspace(-1.0, 1.0, 12)
    G = lambda x: 0.5 * np.cos(x) + c
    res = lambda x: np.linalg.norm(G(x) - x)
    x, its = acc.anderson(G, np.zeros(12), m=5, beta=1.0, converged=lambda x: res(x) <= 1e-13, max_iters=100)
    assert res(x) <= 1e-13
    xp, itp = acc.anderson(G, np.zeros(12), m=0, beta=1.0, converged=lambda x: res(x) <= 1e-13, max_iters=100)
    assert its < itp


def _small_stokes(n=16, steps=2):
    g = st.Grid(n, n)
    prob = wl.random_viscosity(n, ell=0.15, contrast=1e3)
    levels = 3
    sched = [2] * levels
    prm = mg.MGParams(levels=levels, nu_pre=sched, nu_post=sched, omega=1.0, smoother="gs", alpha=1.5)
    A, pre, W = acc.uzawa_system(g, prob.eta_b, prob.eta_p, prm, steps)
    b = st.rhs(g, prob.rho_b, prob.gx, prob.gy)
    ref = st.solve(g, prob.eta_b, prob.eta_p, prob.rho_b, prob.gx, prob.gy)
    return g, A, pre, W, b, ref


def _errors(g, ref, x):
    vx, vy, p = st.to_arrays(g, x)
    return st.parity_errors(g, ref, vx, vy, p)


def test_gcr_accelerates_uzawa_to_direct_solution():
    g, A, pre, W, b, ref = _small_stokes()
    x, its, hist = acc.gcr(lambda v: A @ v, pre, b, np.zeros_like(b), m=10, weights=W, rtol=1e-12, max_iters=200)
    assert hist[-1] <= 1e-12 and its < 80
    ev, ep = _errors(g, ref, x)
    assert ev < 1e-8 and ep < 1e-8


def test_anderson_accelerates_uzawa_to_direct_solution():
    g, A, pre, W, b, ref = _small_stokes()
    G = lambda x: x + pre(b - A @ x)
    bn = np.sqrt(np.sum(W * b * b))
    conv = lambda x: np.sqrt(np.sum(W * (b - A @ x) ** 2)) <= 1e-12 * bn
    x, its = acc.anderson(G, np.zeros_like(b), m=8, beta=0.8, converged=conv, max_iters=300)
    assert conv(x) and its < 150
    ev, ep = _errors(g, ref, x)
    assert ev < 1e-8 and ep < 1e-8
    # and it beats the plain Uzawa iteration it accelerates
    xp, itp = acc.anderson(G, np.zeros_like(b), m=0, beta=1.0, converged=conv, max_iters=its)
    assert not conv(xp)
