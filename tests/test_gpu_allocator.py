"""The caller's device allocator (tph_set_allocator) through the C ABI.

* A counting allocator whose k-th allocation fails: tph_create,
  tph_batch_create and tph_markers_create return TPH_ERR_OOM for every k up
  to the number of blocks a successful create takes, and every block that
  was handed out has been freed when the call returns (allocations and
  frees balance); destroying a successful handle frees every block.
* A solver whose workspace comes from a counting allocator solves exactly as
  one on hipMalloc (bitwise equal results).
* The binding's default, torch's caching allocator: a solver's workspace
  shows up in torch.cuda.memory_allocated and is returned on close.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2603_14040_amd as tph
from paper_2603_14040_amd import _lib
import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


class Counting:
    """ctypes allocator callbacks over torch's caching allocator; fails the
    `fail_at`-th allocation (1-based, 0 = never)."""

    def __init__(self, fail_at=0):
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        self.frees = 0
        self.alloc_cb = _lib.ALLOC_FN(self._alloc)
        self.free_cb = _lib.FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        self.calls += 1
        if self.fail_at and self.calls == self.fail_at:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), device=0)
        self.live[p] = nbytes
        return p

    def _free(self, ptr, ctx):
        self.frees += 1
        assert ptr in self.live, "free of a block the allocator did not hand out"
        del self.live[ptr]
        torch.cuda.caching_allocator_delete(ptr)


def _use(c):
    lib = _lib.load()
    if c is None:
        tph.set_allocator("hip")
    else:
        assert lib.tph_set_allocator(None, c.alloc_cb, c.free_cb, None) == 0


@pytest.fixture(autouse=True)
def _restore_default_allocator():
    yield
    tph.set_allocator("torch")


def _desc(n, **kw):
    return tph._desc(_lib.load(), n, n, **kw)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _blocks_of(create):
    """Blocks a successful create takes (then destroyed): the count to sweep."""
    c = Counting()
    _use(c)
    h, st = create()
    assert st == 0, _lib.load().tph_last_error()
    n = c.calls
    assert n > 0 and len(c.live) == n
    return n, h, c


def _sweep(create, destroy, what):
    n, h, c = _blocks_of(create)
    destroy(h)
    assert not c.live and c.frees == n, f"{what}: destroy left {len(c.live)} blocks"
    print(f"[alloc] {what}: {n} blocks", flush=True)
    for k in range(1, n + 1):
        c = Counting(fail_at=k)
        _use(c)
        h, st = create()
        assert st == -2, f"{what}: failing allocation {k} of {n} gave status {st}"   # TPH_ERR_OOM
        assert not h.value
        assert "allocator returned NULL" in _lib.load().tph_last_error().decode()
        assert not c.live, f"{what}: {len(c.live)} blocks leaked when allocation {k} failed"
        assert c.frees == k - 1


def test_solver_create_reports_oom_and_frees_everything():
    lib = _lib.load()
    d = _desc(64, precision=tph.MIXED, restart=8)

    def create():
        h = ctypes.c_void_p()
        st = lib.tph_create(ctypes.byref(d), _stream(), ctypes.byref(h))
        return h, st

    _sweep(create, lib.tph_destroy, "tph_create 64^2 mixed")


def test_batch_create_reports_oom_and_frees_everything():
    lib = _lib.load()
    descs = (_lib.Desc * 3)()
    for k, n in enumerate((32, 64, 48)):
        descs[k] = _desc(n, precision=tph.MIXED, restart=8)

    def create():
        h = ctypes.c_void_p()
        st = lib.tph_batch_create(3, descs, _stream(), ctypes.byref(h))
        return h, st

    _sweep(create, lib.tph_batch_destroy, "tph_batch_create 3 problems")


def test_markers_create_reports_oom_and_frees_everything():
    lib = _lib.load()

    def create():
        h = ctypes.c_void_p()
        st = lib.tph_markers_create(32, 32, 1.0, 1.0, 4096, _stream(), ctypes.byref(h))
        return h, st

    _sweep(create, lib.tph_markers_destroy, "tph_markers_create")


def test_solver_on_a_caller_allocator_solves_as_on_hipmalloc():
    pr = wl.sinker(64)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    outs = []
    for c in (None, Counting()):
        _use(c)
        with tph.Solver(64, 64, precision=tph.MIXED, rtol=1e-10, device=DEV) as s:
            s.set_coefficients(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b), pr.gx, pr.gy)
            vx, vy, p, info = s.solve()
            torch.cuda.synchronize()
            outs.append((vx.cpu().numpy(), vy.cpu().numpy(), p.cpu().numpy(), info))
        if c is not None:
            assert c.calls > 0 and not c.live
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(a, b)
    assert outs[0][3].iters == outs[1][3].iters


def test_continuation_workspace_follows_the_solver_allocator():
    """tph_set_allocator on a live solver: blocks made on demand later (the
    continuation's blended viscosities) come from the new allocator."""
    lib = _lib.load()
    pr = wl.sinker(32, eta_in=1e3)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    _use(None)
    s = tph.Solver(32, 32, precision=tph.FP64, device=DEV)
    c = Counting()
    assert lib.tph_set_allocator(s._h, c.alloc_cb, c.free_cb, None) == 0
    s.solve_continuation(T(pr.eta_b), T(pr.eta_p), T(pr.rho_b), pr.gx, pr.gy)
    assert c.calls == 2 and len(c.live) == 2
    s.close()
    assert not c.live and c.frees == 2


def test_set_allocator_rejects_half_a_pair():
    lib = _lib.load()
    c = Counting()
    assert lib.tph_set_allocator(None, c.alloc_cb, _lib.FREE_FN(), None) == -1
    assert lib.tph_set_allocator(None, _lib.ALLOC_FN(), c.free_cb, None) == -1


def test_default_binding_allocator_is_torch_caching_allocator():
    tph.set_allocator("torch")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(DEV)
    s = tph.Solver(256, 256, precision=tph.MIXED, restart=8, device=DEV)
    during = torch.cuda.memory_allocated(DEV)
    s.close()
    after = torch.cuda.memory_allocated(DEV)
    # at least the 3-field FP64 vectors of the Krylov basis (10 x 3 x 258^2 x 8 B)
    assert during - before > 10 * 3 * 258 * 258 * 8
    assert after == before
