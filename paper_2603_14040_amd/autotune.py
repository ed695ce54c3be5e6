"""Autotuner of the solver's kernel plan and sweep schedule.

The converged answer of a solve does not depend on any parameter tuned
here: the V-cycle/Uzawa step is only the preconditioner of the accelerator
(flexible GMRES, GCR or Anderson), which converges to the same discrete
solution (the paper's Sec. "Accelerators" and its multigrid sections).  The
parameters trade work per iteration against the number of iterations and
map the work onto the chip differently, so the fastest choice depends on
the grid, the viscosity structure and the device.  The tuner measures
whole solves of the caller's own problem and keeps the fastest.

Knobs (all of them descriptor fields of tph_create):
  * per LDS-tiled level: one-sweep tile launches or multi-sweep passes
    (``msweep`` bit), large or small tile shape (``tile_shape`` bit);
  * the first level of the single-workgroup coarse tail (``coarse_level``);
  * pre- and post-smoothing sweeps and their growth per level (the paper's
    level-dependent schedule, nu_l = ceil(nu * growth^l));
  * Uzawa sweeps per preconditioner application (``uzawa_steps``, 1..16) and the
    Uzawa pressure relaxation ``alpha``; the smoother damping ``omega``;
  * the Krylov accelerator (flexible GMRES or GCR) and its restart length;
    for Anderson acceleration (tuned from an explicit knob list) the depth
    (``restart``) and the mixing ``beta``; for the RAS smoothers (also from
    an explicit list) the tile side and the inner sweeps.
Parameter sets that resolve to the same kernel plan on every level are
measured once.

Search: coordinate descent from the library defaults; each knob in turn
takes every candidate value with the others fixed, and a candidate is
adopted when it is faster by more than ``rel_gain``; passes repeat until
one changes nothing (at most ``rounds``).  A candidate is timed as the
median of ``reps`` solves from a zero initial guess to the target
residual, after one untimed solve; one that does not converge is
discarded.  Results go to a JSON database keyed by grid, precision,
device and library version.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import tempfile
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

Params = Dict[str, object]


# ---------------------------------------------------------------------------
# search (pure host logic)
# ---------------------------------------------------------------------------
@dataclass
class Knob:
    name: str
    candidates: Sequence[object]


@dataclass
class SearchResult:
    params: Params
    cost: float
    trials: List[Tuple[Params, float]] = field(default_factory=list)


def coordinate_search(measure: Callable[[Params], float], knobs: Sequence[Knob], start: Params,
                      rounds: int = 2, rel_gain: float = 0.02) -> SearchResult:
    """Coordinate descent over ``knobs`` from ``start``.

    ``measure`` returns the cost of a full parameter set (math.inf when the
    configuration is unusable).  Every distinct parameter set is measured
    at most once.
    """
    cache: Dict[str, float] = {}
    trials: List[Tuple[Params, float]] = []

    def cost(p: Params) -> float:
        key = json.dumps(p, sort_keys=True)
        if key not in cache:
            c = float(measure(dict(p)))
            cache[key] = c
            trials.append((dict(p), c))
        return cache[key]

    best = dict(start)
    best_cost = cost(best)
    for _ in range(max(1, rounds)):
        changed = False
        for kn in knobs:
            for v in kn.candidates:
                if best.get(kn.name) == v:
                    continue
                cand = dict(best)
                cand[kn.name] = v
                c = cost(cand)
                if c < best_cost * (1.0 - rel_gain):
                    best, best_cost, changed = cand, c, True
        if not changed:
            break
    return SearchResult(best, best_cost, trials)


# ---------------------------------------------------------------------------
# database
# ---------------------------------------------------------------------------
def default_db_path() -> str:
    return os.environ.get("TEPHRA_TUNING_DB", os.path.join(os.path.expanduser("~"), ".cache", "tephra_tuning.json"))


class TuningDB:
    """JSON file of tuned parameter sets (written atomically)."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or default_db_path()
        self.entries: Dict[str, dict] = {}
        if os.path.exists(self.path):
            with open(self.path) as fh:
                data = json.load(fh)
            if not isinstance(data, dict):
                raise ValueError(f"{self.path}: not a tuning database")
            self.entries = data

    @staticmethod
    def key(nx: int, ny: int, precision: int, device: str, version: str, tag: str = "") -> str:
        return f"{nx}x{ny}|prec{precision}|{device}|{version}" + (f"|{tag}" if tag else "")

    def get(self, key: str) -> Optional[dict]:
        return self.entries.get(key)

    def put(self, key: str, entry: dict) -> None:
        self.entries[key] = entry
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning", suffix=".json")
        with os.fdopen(fd, "w") as fh:
            json.dump(self.entries, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


# ---------------------------------------------------------------------------
# parameter sets <-> solver descriptor
# ---------------------------------------------------------------------------
def plan_to_masks(plan: Sequence[Tuple[int, int]], levels: Sequence[int]) -> Tuple[int, int]:
    """Per-tile-level (multisweep, small shape) choices -> (msweep, tile_shape) masks."""
    msw = shp = 0
    for (m, s), l in zip(plan, levels):
        msw |= (1 << l) if m else 0
        shp |= (1 << l) if s else 0
    return msw, shp


def solver_kwargs(p: Params, tile_levels: Sequence[int]) -> dict:
    """Solver keyword arguments of a parameter set (a joint ``krylov`` =
    (accelerator, restart) entry overrides ``accel`` and ``restart``)."""
    plan = [tuple(p[f"L{l}"]) for l in tile_levels]
    msw, shp = plan_to_masks(plan, tile_levels)
    accel, restart = (p["krylov"] if "krylov" in p else (p.get("accel", "fgmres"), p["restart"]))
    return dict(nu_pre=int(p["nu_pre"]), nu_post=int(p["nu_post"]), nu_growth=float(p.get("nu_growth", 1.0)),
                uzawa_steps=int(p["uzawa_steps"]), restart=int(restart), msweep=msw, tile_shape=shp,
                coarse_level=int(p.get("coarse_level", -1)), omega=float(p.get("omega", 1.0)),
                alpha=float(p.get("alpha", 1.0)), accel=str(accel),
                beta=float(p.get("beta", 1.0)), smoother=int(p.get("smoother", 1)),
                ras_tile=int(p.get("ras_tile", 32)), ras_inner=int(p.get("ras_inner", 4)))


# A second starting point of the search besides the library defaults: a
# short-restart GCR around a deeper Uzawa preconditioner with one sweep per
# leg.  Coordinate descent moves one knob at a time, and from the defaults
# (FGMRES(20), two Uzawa steps) it can settle where a better restart /
# accelerator / Uzawa-depth combination needs several knobs to move at once.
ALT_START: Params = {"krylov": ("gcr", 8), "uzawa_steps": 4, "alpha": 1.5, "nu_pre": 1, "nu_post": 1}


def knobs_for(tile_levels: Sequence[int], coarse_levels: Sequence[int] = (), nus=(1, 2, 3),
              growths=(1.0, 1.5, 2.0), uzawa=(1, 2, 3, 4, 6, 8, 12, 16), restarts=(5, 8, 10, 15, 20, 30, 50, 64),
              alphas=(1.0, 1.5, 1.75, 2.0, 3.0), omegas=(0.8, 1.0, 1.2),
              accels=("fgmres", "gcr")) -> List[Knob]:
    """Schedule knobs first (they move the iteration count), then the kernel plan.

    The Krylov accelerator (flexible GMRES or GCR, both residual-minimising
    over the preconditioned directions) is a knob beside its restart length."""
    ks = [Knob("alpha", list(alphas)), Knob("uzawa_steps", list(uzawa)), Knob("nu_pre", list(nus)),
          Knob("nu_post", list(nus)), Knob("omega", list(omegas)), Knob("nu_growth", list(growths)),
          Knob("krylov", [(a, r) for a in accels for r in restarts])]
    if coarse_levels:
        ks.append(Knob("coarse_level", [-1] + list(coarse_levels)))
    ks += [Knob(f"L{l}", [(0, 0), (0, 1), (1, 0), (1, 1)]) for l in tile_levels]
    return ks


# ---------------------------------------------------------------------------
# tuning a problem on the GPU
# ---------------------------------------------------------------------------
def schedule_knobs() -> List[Knob]:
    """Knobs that carry over between grid sizes of one recipe (no per-level plan)."""
    return [Knob("krylov", [(a, r) for a in ("fgmres", "gcr") for r in (8, 16, 30, 40, 48, 64)]),
            Knob("alpha", [1.0, 1.5, 1.75, 2.0, 3.0]),
            Knob("uzawa_steps", [1, 2, 3, 4, 6, 8, 12, 16]), Knob("nu_pre", [1, 2, 3]), Knob("nu_post", [1, 2, 3]),
            Knob("omega", [0.8, 1.0, 1.2])]


def tune(eta_b, eta_p, rho_b, gx: float = 0.0, gy: float = -1.0, *, precision: Optional[int] = None,
         lx: float = 1.0, ly: float = 1.0, bc=(0, 0, 0, 0), rtol: float = 1e-8, reps: int = 3, rounds: int = 2,
         rel_gain: float = 0.02, db: Optional[TuningDB] = None, tag: str = "", device=None,
         knobs: Optional[Sequence[Knob]] = None, log: Optional[Callable[[str], None]] = None,
         max_iters: int = 2000, start: Optional[dict] = None, starts: Optional[Sequence[dict]] = None,
         also: Optional[Sequence[tuple]] = None) -> dict:
    """Tune the solve of one problem (device FP64 arrays of shape (ny+2, nx+2)).

    Returns the database entry: ``params`` (Solver keyword arguments),
    ``ms`` (median solve time), ``iters``, ``trials`` and ``seconds``
    spent.  With ``db`` the entry is stored under the problem's key.
    ``start`` overrides entries of the starting point (schedule keys of
    ``solver_kwargs``, ``accel``, ``restart``, ``beta``, ``krylov``);
    ``starts`` lists further overrides, each the start of another descent
    (measured candidates are shared), and the fastest result wins.
    ``also`` lists further problems on the same grid, as (eta_b, eta_p,
    rho_b, gx, gy): a candidate's cost is then the mean of its median solve
    times over all the problems, so that a schedule is not picked for the
    iteration count of one instance (``ms`` and ``iters`` stay those of the
    first problem).
    """
    import torch
    from . import MIXED, Solver, _lib

    precision = MIXED if precision is None else precision
    ny, nx = eta_b.shape[0] - 2, eta_b.shape[1] - 2
    device = eta_b.device if device is None else device
    t_start = time.perf_counter()

    base = Solver(nx, ny, lx, ly, bc=bc, precision=precision, rtol=rtol, device=device)
    nlev = base.levels
    plan0 = [base.level_plan(l) for l in range(nlev)]
    lc0 = next((l for l, (k, _) in enumerate(plan0) if k == "coarse_tail"), nlev - 1)
    # levels that run tile kernels with the default coarse tail or one or two levels lower
    tile_levels = [l for l in range(min(lc0 + 2, nlev - 1))]
    coarse_levels = [l for l in (lc0 + 1, lc0 + 2) if l < nlev - 1 and lc0 < nlev - 1]
    d = base.desc
    init: Params = {"nu_pre": int(d.nu_pre), "nu_post": int(d.nu_post), "nu_growth": float(d.nu_growth),
                    "uzawa_steps": int(d.uzawa_steps), "restart": int(d.restart), "coarse_level": -1,
                    "omega": float(d.omega), "alpha": float(d.alpha), "accel": "fgmres", "beta": 1.0,
                    "smoother": int(d.smoother), "ras_tile": int(d.ras_tile), "ras_inner": int(d.ras_inner)}
    for l in tile_levels:
        k, s = plan0[l]
        init[f"L{l}"] = (1 if k == "multisweep" else 0, int(s))
    init["krylov"] = (init["accel"], init["restart"])
    for key, v in (start or {}).items():
        if key in init and not key.startswith("L"):
            init[key] = v
    if start and ("accel" in start or "restart" in start) and "krylov" not in start:
        init["krylov"] = (start.get("accel", init["krylov"][0]), start.get("restart", init["krylov"][1]))
    if start and ("msweep" in start or "tile_shape" in start):
        # a per-level plan given as descriptor masks (-1: that level's default)
        for l in tile_levels:
            m0, s0 = init[f"L{l}"]
            msw, shp = int(start.get("msweep", -1)), int(start.get("tile_shape", -1))
            init[f"L{l}"] = ((msw >> l) & 1 if msw >= 0 else m0, (shp >> l) & 1 if shp >= 0 else s0)
    base.close()
    del base

    iters: Dict[str, int] = {}       # effective plan -> iterations (first problem)
    seen: Dict[str, float] = {}       # effective plan -> cost
    first_ms: Dict[str, float] = {}   # effective plan -> median solve time of the first problem
    eff_of: Dict[str, str] = {}       # parameter set -> effective plan

    def measure(p: Params) -> float:
        kw = solver_kwargs(p, tile_levels)
        try:
            s = Solver(nx, ny, lx, ly, bc=bc, precision=precision, rtol=rtol, device=device, max_iters=max_iters,
                       **kw)
        except _lib.TephraError:
            return math.inf            # e.g. a coarse tail that does not fit
        try:
            # the plan the solver actually runs: sets that differ only in ignored bits are one candidate
            eff = json.dumps([kw["accel"], kw["beta"], kw["smoother"], kw["ras_tile"], kw["ras_inner"],
                              kw["nu_pre"], kw["nu_post"], kw["nu_growth"],
                              kw["uzawa_steps"], kw["restart"],
                              kw["omega"], kw["alpha"], [s.level_plan(l) for l in range(s.levels)]])
            eff_of[json.dumps(p, sort_keys=True)] = eff
            if eff in seen:
                return seen[eff]
            vx, vy, pp = s.zeros(), s.zeros(), s.zeros()
            costs, first_iters = [], None
            for prob in [(eta_b, eta_p, rho_b, gx, gy)] + list(also or ()):
                s.set_coefficients(*prob)
                ts = []
                for r in range(reps + 1):
                    vx.zero_(); vy.zero_(); pp.zero_()
                    torch.cuda.synchronize(device)
                    t0 = time.perf_counter()
                    info = s.solve(vx, vy, pp)[3]
                    torch.cuda.synchronize(device)
                    if info.status != "TPH_OK":
                        seen[eff] = math.inf
                        return math.inf
                    if r > 0:
                        ts.append(time.perf_counter() - t0)
                costs.append(statistics.median(ts) * 1e3)
                first_iters = info.iters if first_iters is None else first_iters
            c = statistics.mean(costs)
            seen[eff] = c
            first_ms[eff] = costs[0]
            iters[eff] = first_iters
            if log:
                log(f"[tune] {p} -> {c:.2f} ms, {first_iters} iterations")
            return c
        finally:
            s.close()

    ks = knobs if knobs is not None else knobs_for(tile_levels, coarse_levels)
    if not any(k.name == "krylov" for k in ks):
        init.pop("krylov", None)          # separate accel / restart knobs (or neither) drive those two
    res = coordinate_search(measure, ks, init, rounds=rounds, rel_gain=rel_gain)
    for extra in starts or ():
        p0 = dict(init)
        for key, v in extra.items():
            if key in p0 and not key.startswith("L"):
                p0[key] = tuple(v) if isinstance(v, list) else v
            elif key == "krylov" and "krylov" not in p0:
                p0["accel"], p0["restart"] = v
        r2 = coordinate_search(measure, ks, p0, rounds=rounds, rel_gain=rel_gain)
        trials = res.trials + r2.trials
        res = r2 if r2.cost < res.cost else res
        res = SearchResult(res.params, res.cost, trials)
    best_kw = solver_kwargs(res.params, tile_levels)
    best_eff = eff_of.get(json.dumps(res.params, sort_keys=True))
    default_eff = eff_of.get(json.dumps(res.trials[0][0], sort_keys=True)) if res.trials else None
    entry = {"params": best_kw, "ms": first_ms.get(best_eff, res.cost), "iters": iters.get(best_eff),
             "cost": res.cost, "problems": 1 + len(also or ()),
             "default_ms": first_ms.get(default_eff, res.trials[0][1]), "trials": len(res.trials),
             "seconds": round(time.perf_counter() - t_start, 2),
             "search": {k: (list(v) if isinstance(v, tuple) else v) for k, v in res.params.items()}}
    if db is not None:
        db.put(TuningDB.key(nx, ny, precision, device_name(device), _lib.version(), tag), entry)
    return entry


def tune_batch(shapes, eta_b, eta_p, rho_b, gxy, *, precision: Optional[int] = None, rtol: float = 1e-8,
               reps: int = 1, rounds: int = 2, rel_gain: float = 0.02, device=None,
               knobs: Optional[Sequence[Knob]] = None, log: Optional[Callable[[str], None]] = None) -> dict:
    """Tune the schedule of a batched solve (lists of per-problem device arrays).

    The batched kernels take no per-level plan, so the knobs are the
    schedule ones: Uzawa relaxation and steps, sweeps and restart length.
    The cost of a candidate is the median time of ``reps`` batched solves
    (after one untimed solve, which also captures the iteration graph).
    """
    import torch
    from . import MIXED, Batch

    precision = MIXED if precision is None else precision
    t_start = time.perf_counter()
    start: Params = {"alpha": 1.0, "uzawa_steps": 2, "nu_pre": 2, "nu_post": 2, "restart": 16}
    ks = knobs if knobs is not None else [Knob("uzawa_steps", [2, 3, 4, 6, 8, 12]), Knob("restart", [6, 8, 12, 16, 24]),
                                          Knob("alpha", [1.0, 1.5, 1.75, 2.0]), Knob("nu_pre", [1, 2, 3]),
                                          Knob("nu_post", [1, 2, 3])]

    def measure(p: Params) -> float:
        b = Batch(shapes, device=device, precision=precision, rtol=rtol, **p)
        try:
            b.set_coefficients(eta_b, eta_p, rho_b, gxy)
            outs = b.zeros(), b.zeros(), b.zeros()
            ts = []
            for r in range(reps + 1):
                for o in outs:
                    for t in o:
                        t.zero_()
                torch.cuda.synchronize(device)
                t0 = time.perf_counter()
                infos = b.solve(*outs)[3]
                torch.cuda.synchronize(device)
                if any(i.res_energy > rtol for i in infos):
                    return math.inf
                if r > 0:
                    ts.append(time.perf_counter() - t0)
            c = statistics.median(ts) * 1e3
            if log:
                log(f"[tune-batch] {p} -> {c:.1f} ms")
            return c
        finally:
            b.close()

    res = coordinate_search(measure, ks, start, rounds=rounds, rel_gain=rel_gain)
    return {"params": dict(res.params), "ms": res.cost, "default_ms": res.trials[0][1], "trials": len(res.trials),
            "seconds": round(time.perf_counter() - t_start, 2)}


def device_name(device=None) -> str:
    """Architecture and compute-unit count of the device (stable across tools)."""
    import torch
    pr = torch.cuda.get_device_properties(device)
    arch = getattr(pr, "gcnArchName", "") or pr.name
    return f"{arch.split(':')[0]}-{pr.multi_processor_count}cu"


def lookup(nx: int, ny: int, precision: int, db: Optional[TuningDB] = None, tag: str = "",
           device=None) -> Optional[dict]:
    """Tuned Solver keyword arguments for this grid and device, or None."""
    from . import _lib
    db = db or TuningDB()
    e = db.get(TuningDB.key(nx, ny, precision, device_name(device), _lib.version(), tag))
    return dict(e["params"]) if e else None
