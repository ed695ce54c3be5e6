"""Seeded input generators: determinism, shapes and the stated recipes."""
import numpy as np

import workloads as wl


def test_sinker_point_sampling_and_shapes():
    p = wl.sinker(64)
    assert p.eta_b.shape == (66, 66) and p.rho_b.shape == (66, 66)
    # basic node (32, 32) is the centre; (32, 32 + 6) is 6/64 = 0.094 < 0.1 away
    assert p.eta_b[32, 32] == 1e3 and p.eta_b[32, 38] == 1e3 and p.eta_b[32, 39] == 1.0
    assert p.rho_b[32, 32] == 1.0 and p.rho_b[0, 0] == 0.0
    # cell (33, 33) centre (0.5078, 0.5078) inside
    assert p.eta_p[33, 33] == 1e3 and p.eta_p[1, 1] == 1.0


def test_random_viscosity_contrast_and_determinism():
    a = wl.random_viscosity(64)
    b = wl.random_viscosity(64)
    assert np.array_equal(a.eta_b, b.eta_b) and np.array_equal(a.rho_b, b.rho_b)
    ep = a.eta_p[1:65, 1:65]
    assert np.isclose(ep.max() / ep.min(), 1e4, rtol=1e-12)
    # eta_b at an interior node is 10**(mean of the four touching cells' log10)
    m = a.meta["m"]
    assert np.isclose(np.log10(a.eta_b[5, 7]), m[4:6, 6:8].mean(), rtol=1e-13)
    # corner node touches one cell
    assert np.isclose(np.log10(a.eta_b[0, 0]), m[0, 0], rtol=1e-13)
    assert np.all(np.isfinite(a.rho_b))


def test_multi_inclusion_matches_full_scan():
    p = wl.multi_inclusion(128, count=20, seed=3)
    rng = np.random.default_rng(3)
    eb = np.ones((130, 130))
    ep = np.ones((130, 130))
    h = 1.0 / 128
    i = np.arange(130)[:, None]
    j = np.arange(130)[None, :]
    for _ in range(20):
        cx, cy = rng.uniform(0, 1, 2)
        r = rng.uniform(0.005, 0.03)
        le = rng.uniform(-3, 3)
        rng.uniform(-1, 1)
        inb = ((j * h - cx) ** 2 + (i * h - cy) ** 2 <= r * r) & (i <= 128) & (j <= 128)
        inp = (((j - .5) * h - cx) ** 2 + ((i - .5) * h - cy) ** 2 <= r * r) & (i >= 1) & (i <= 128) & (j >= 1) & (j <= 128)
        eb[inb] = 10 ** le
        ep[inp] = 10 ** le
    assert np.array_equal(eb, p.eta_b)
    assert np.array_equal(ep, p.eta_p)


def test_batch_sizes():
    ps = wl.batch_sinkers(16, seed=4)
    assert len(ps) == 16
    assert all(p.nx in (64, 128, 256, 512) and p.nx == p.ny for p in ps)
    assert all(10 <= p.meta["eta_in"] <= 1e4 for p in ps)
