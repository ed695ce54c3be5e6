"""The C ABI library loads and exports every function of include/tephra.h;
descriptor validation happens on the host before any HIP call (no GPU needed)."""
import ctypes
import os

import pytest

from paper_2603_14040_amd import _lib


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtephra.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_exports_every_declared_function(lib):
    names = _lib.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_struct_layout_matches_header(lib):
    # tph_desc: offsets follow the C layout (doubles 8-aligned)
    assert _lib.Desc.lx.offset == 8 and _lib.Desc.bc.offset == 24
    assert _lib.Desc.nu_growth.offset == 64 and _lib.Desc.rtol.offset == 96
    d = _lib.Desc()
    lib.tph_desc_default(ctypes.byref(d), 64, 32)
    assert (d.nx, d.ny, d.lx, d.precision, d.restart) == (64, 32, 1.0, _lib.MIXED, 20)
    assert d.rtol == 1e-8 and d.nu_growth == 1.0 and d.uzawa_steps == 2 and d.fused == 1
    assert d.msweep == -1 and d.tile_shape == -1 and d.coarse_level == -1
    assert d.accel == _lib.ACCEL_FGMRES and d.beta == 1.0
    assert _lib.Desc.accel.offset == 132 and _lib.Desc.beta.offset == 136
    assert _lib.Desc.ras_tile.offset == 144 and _lib.Desc.ras_inner.offset == 148 and _lib.Desc.seed.offset == 152
    assert (d.ras_tile, d.ras_inner, d.seed) == (32, 4, 0)
    assert _lib.Desc.graph.offset == 160 and d.graph == 0
    assert _lib.Desc.coarsen.offset == 168 and ctypes.sizeof(_lib.Desc) == 176 and d.coarsen == 2.0


def _create(lib, **kw):
    d = _lib.Desc()
    lib.tph_desc_default(ctypes.byref(d), kw.pop("nx", 64), kw.pop("ny", 64))
    for k, v in kw.items():
        setattr(d, k, v)
    h = ctypes.c_void_p()
    st = lib.tph_create(ctypes.byref(d), None, ctypes.byref(h))
    return st, h, lib.tph_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(nx=1), "nx and ny"),
    (dict(precision=7), "precision"),
    (dict(levels=6, nx=48, ny=48), "divisible"),
    (dict(levels=1, nx=128, ny=128), "coarsest level too large"),
    (dict(coarsen=2.5), "fused = 0"),
    (dict(coarsen=1.1, fused=0), "coarsen"),
    (dict(coarsen=5.0, fused=0), "coarsen"),
    (dict(restart=0), "restart"),
    (dict(restart=65), "restart"),
    (dict(omega=0.0), "omega"),
    (dict(rtol=0.0), "rtol"),
    (dict(nu_growth=0.5), "nu_growth"),
    (dict(lx=-1.0), "lx and ly"),
    (dict(uzawa_steps=0), "uzawa_steps"),
    (dict(fused=3), "fused"),
    (dict(msweep=-2), "msweep"),
    (dict(tile_shape=-5), "tile_shape"),
    (dict(coarse_level=-3), "coarse_level"),
    (dict(coarse_level=0, nx=256, ny=256), "coarse_level"),
    (dict(accel=3), "accel"),
    (dict(accel=1, restart=0), "restart"),
    (dict(accel=2, restart=-1), "Anderson depth"),
    (dict(accel=2, restart=65), "Anderson depth"),
    (dict(accel=2, beta=0.0), "beta"),
    (dict(accel=2, beta=1.5), "beta"),
    (dict(smoother=4), "smoother"),
    (dict(graph=2), "graph"),
    (dict(smoother=2, ras_tile=12), "ras_tile"),
    (dict(smoother=3, ras_inner=0), "ras_inner"),
    (dict(smoother=2, ras_inner=17), "ras_inner"),
])
def test_invalid_descriptor_rejected_on_host(lib, kw, needle):
    st, h, msg = _create(lib, **kw)
    assert st == -1 and not h.value
    assert needle in msg


def test_null_arguments_rejected(lib):
    assert lib.tph_create(None, None, None) == -1
    assert lib.tph_set_coefficients(None, None, None, None, 0.0, -1.0, None, None) == -1
    assert "NULL" in lib.tph_last_error().decode()
    assert lib.tph_solve(None, None, None, None, None) == -1
    lib.tph_destroy(None)
    assert lib.tph_version().decode().startswith("tephra")


def test_noalloc_residual_validates_on_the_host(lib):
    """tph_energy_residual_noalloc rejects bad arguments before any HIP call
    (pointers below are never dereferenced)."""
    fake = ctypes.c_void_p(256)
    d = _lib.Desc()
    lib.tph_desc_default(ctypes.byref(d), 8, 8)
    args = [fake, fake, fake, 0.0, -1.0, fake, fake, fake, fake, None]
    assert lib.tph_energy_residual_noalloc(None, *args) == -1
    for nx, ny in ((40000, 8), (8, 32769), (1, 8), (8, 0)):
        d.nx, d.ny = nx, ny
        assert lib.tph_energy_residual_noalloc(ctypes.byref(d), *args) == -1
        assert "[2, 32768]" in lib.tph_last_error().decode()
    d.nx, d.ny = 8, 8
    d.bc[1] = 5
    assert lib.tph_energy_residual_noalloc(ctypes.byref(d), *args) == -1
    assert "bc" in lib.tph_last_error().decode()
    d.bc[1] = 0
    d.lx = -1.0
    assert lib.tph_energy_residual_noalloc(ctypes.byref(d), *args) == -1
    d.lx = 1.0
    bad = list(args)
    bad[6] = None                       # vy
    assert lib.tph_energy_residual_noalloc(ctypes.byref(d), *bad) == -1
    assert "required" in lib.tph_last_error().decode()
