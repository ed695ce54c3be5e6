"""tph_energy_residual_noalloc (the entry point that allocates nothing)
against tph_energy_residual and tph_info.res_l2, through the C ABI.

* Two calls in a row on one device, the second on a smaller grid: each
  agrees with the solver-based entry point on the same state.
* States with garbage in the ghost and wall entries: both entry points
  ignore them, so the results agree.
* Captured in a HIP graph and replayed three times with eager changes of
  the state between replays: every replay equals an eager call.
* Oversized grids are rejected before any device work.

Tolerances: both sides form every residual entry with the same stencil
formulas in FP64 and differ only in the order of the sums (relative
differences ~1e-15 per sum); where the residual is small against the
right-hand side (an approximately solved state), the entries themselves
carry cancellation error ~eps |b| / |r|, so the comparison there is 1e-9.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2603_14040_amd as tph
from paper_2603_14040_amd import _lib
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _noalloc(lib, nx, ny, bc, eb, ep, rho, gx, gy, vx, vy, p, out, stream):
    d = tph._desc(lib, nx, ny, bc=bc)
    return lib.tph_energy_residual_noalloc(
        ctypes.byref(d), ctypes.c_void_p(eb.data_ptr()), ctypes.c_void_p(ep.data_ptr()),
        ctypes.c_void_p(rho.data_ptr()), gx, gy, ctypes.c_void_p(vx.data_ptr()), ctypes.c_void_p(vy.data_ptr()),
        ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))


def _case(nx, ny, bc, seed):
    eb, ep, rho = (_to(a) for a in wl.random_fields(nx, ny, seed, eta_decades=3.0))
    gx, gy = 0.3, -1.0
    return eb, ep, rho, gx, gy


@pytest.mark.parametrize("sizes", [((96, 80), (48, 40)), ((112, 88), (40, 24))])
def test_noalloc_matches_solver_entry_points_twice(sizes):
    lib = _lib.load()
    stream = torch.cuda.current_stream(DEV)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    bcs = [(tph.FREE_SLIP, tph.NO_SLIP, tph.FREE_SLIP, tph.NO_SLIP), (tph.NO_SLIP,) * 4]
    for k, ((nx, ny), bc) in enumerate(zip(sizes, bcs)):
        eb, ep, rho, gx, gy = _case(nx, ny, bc, 100 + k)
        with tph.Solver(nx, ny, bc=bc, precision=tph.FP64, rtol=1e-5, max_iters=200, device=DEV) as s:
            s.set_coefficients(eb, ep, rho, gx, gy)
            vx, vy, p, info = s.solve()
            # an approximately solved state: residual ~1e-5 of b
            assert _noalloc(lib, nx, ny, bc, eb, ep, rho, gx, gy, vx, vy, p, out, stream) == 0, \
                lib.tph_last_error()
            torch.cuda.synchronize()
            e_ref = s.energy_residual(vx, vy, p)
            got = out.cpu().numpy()
            assert got[0] == pytest.approx(e_ref, rel=1e-9)
            assert got[1] == pytest.approx(info.res_l2, rel=1e-9)
            assert got[0] == pytest.approx(info.res_energy, rel=1e-9)
            # a random state with garbage walls and ghosts: residual ~ b, no cancellation
            rs = [_to(a) for a in wl.random_state(nx, ny, 200 + k)]
            assert _noalloc(lib, nx, ny, bc, eb, ep, rho, gx, gy, *rs, out, stream) == 0
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert got[0] == pytest.approx(s.energy_residual(*rs), rel=1e-12)
            assert np.isfinite(got[1]) and got[1] > 0


def test_noalloc_replays_in_a_graph():
    lib = _lib.load()
    nx, ny = 72, 56
    bc = (tph.FREE_SLIP,) * 4
    eb, ep, rho, gx, gy = _case(nx, ny, bc, 7)
    vx, vy, p = (_to(a) for a in wl.random_state(nx, ny, 8))
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    eager = torch.zeros(2, dtype=torch.float64, device=DEV)
    side = torch.cuda.Stream(DEV)
    # first call outside the capture (looks up the scratch address)
    assert _noalloc(lib, nx, ny, bc, eb, ep, rho, gx, gy, vx, vy, p, out, torch.cuda.current_stream(DEV)) == 0
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side.wait_stream(torch.cuda.current_stream(DEV))
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            assert _noalloc(lib, nx, ny, bc, eb, ep, rho, gx, gy, vx, vy, p, out, side) == 0
    torch.cuda.synchronize()
    for r in range(3):
        vx.mul_(1.0 + 0.25 * r)             # eager change of the state between replays
        p.add_(0.5)
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert _noalloc(lib, nx, ny, bc, eb, ep, rho, gx, gy, vx, vy, p, eager,
                        torch.cuda.current_stream(DEV)) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, eager), (r, out, eager)


def test_noalloc_rejects_oversized_grids():
    lib = _lib.load()
    t = torch.zeros((4, 4), dtype=torch.float64, device=DEV)
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    for nx, ny in ((40000, 8), (8, 32769), (1, 8)):
        d = tph._desc(lib, 8, 8)
        d.nx, d.ny = nx, ny
        ptr = ctypes.c_void_p(t.data_ptr())
        st = lib.tph_energy_residual_noalloc(ctypes.byref(d), ptr, ptr, ptr, 0.0, -1.0, ptr, ptr, ptr,
                                             ctypes.c_void_p(out.data_ptr()), None)
        assert st == -1                     # TPH_ERR_INVALID
        assert "32768" in lib.tph_last_error().decode()
