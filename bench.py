#!/usr/bin/env python3
"""Throughput of the MI355X Stokes solver on its workloads.

One step = the whole hot path over one problem: coefficient setup
(viscosity restriction down the hierarchy, right-hand side, FP64 coarsest
factorisation) plus one solve from a zero initial guess to a relative energy
residual of 1e-8 (Krylov accelerator + V-cycle/Uzawa preconditioner).
Inputs are synthetic, seeded, and resident in HBM before timing starts.

Headline (``value``): the random-viscosity problem on 1024 x 1024 cells
(log10 viscosity a Gaussian random field, correlation length 0.05, contrast
1e4; density 1 - 0.01 log10(eta) + N(0, 0.01); free slip; g = (0, -1)), mixed
precision (FP32 V-cycle; FP64 residual, Krylov, coarsest solve and pressure
step), in cells per second, mean over --steps timed steps.  The solver's
schedule and kernel plan come from the autotuner run on a held-out instance
of the same recipe (other seeds), untimed; the FP64 solve is timed beside it.

Sections (``--only`` picks a subset; all but ``robust`` by default):
  headline  the 1024^2 random-viscosity problem, mixed and FP64, and the
            effective (cache-resident) bandwidth of its finest-level sweep
  config1   the 64^2 FP64 sinker (4-level V-cycle, FGMRES), FP64 and mixed
  large     4096^2 multi-inclusion problem (200 discs, viscosity 10^U(-3,3)),
            mixed (median of --large-reps solves) and FP64, the roofline of
            its dominant kernel (HIP-event time stamps inside the timed
            solves), and one viscosity-rescaling continuation solve
  batch     256 sinkers of sizes {64,...,512}, mixed and FP64 (medians)
  adjoint   misfit gradient on the 1024^2 field: forward solve, adjoint
            solve and gradient kernel, mixed and FP64
  accel     GCR and Anderson accelerators on the headline problem
  ras       RAS temporal-blocking smoother on the headline problem
  mic       marker-in-cell step (markers -> grid, solve, RK4)
  robust    1e8-contrast sinker, unaccelerated Uzawa + continuation
  cpu       the FP64 CPU oracle (assembled matrix + SuperLU) at --cpu-sizes,
            one single-threaded child process, with its peak memory

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only a,b,...]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import subprocess
import sys
import time

METRIC = "Stokes solve cells/s to 1e-8 rel. residual + HBM GB/s; mixed vs FP64 on 1 GPU"
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
SECTIONS = ("headline", "config1", "large", "batch", "adjoint", "accel", "ras", "mic", "robust", "cpu")
DEFAULT_SECTIONS = tuple(s for s in SECTIONS if s != "robust")

# Schedule of the 4096^2 multi-inclusion solve: the autotuner's schedule
# search (autotune.schedule_knobs) on a held-out instance of the recipe
# (seed 13) at 4096^2; `python bench.py --only large --tune-large` repeats
# that search and uses its result instead.
LARGE_PARAMS = {
    "mixed": {"nu_pre": 1, "nu_post": 2, "uzawa_steps": 16, "restart": 40, "alpha": 1.75, "accel": "gcr"},
    "fp64": {"nu_pre": 1, "nu_post": 2, "uzawa_steps": 12, "restart": 64, "alpha": 1.75, "accel": "gcr"},
}
LARGE_TUNE_SEED = 13
# Schedule of the 256-problem batch: autotune.tune_batch on a held-out batch
# of the recipe (seed 14); `--tune-batch` repeats that search.
BATCH_PARAMS = {"alpha": 1.5, "uzawa_steps": 8, "nu_pre": 2, "nu_post": 2, "restart": 16}
BATCH_TUNE_SEED = 14
# GRF and noise seeds of the held-out tuning instances: a candidate's cost is
# its mean solve time over all of them, so that the schedule is not picked for the
# iteration count of one instance
HEADLINE_TUNE_SEEDS = ((12, 32), (13, 33), (14, 34))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def median(xs):
    return statistics.median(xs) if xs else None


def eta_from_logvisc(m, n):
    """eta_p = 10**m at cell centres, eta_b = 10**(mean of m over the touching
    cells) at basic nodes, from a (n, n) torch tensor (differentiable)."""
    import torch
    ep = torch.ones((n + 2, n + 2), dtype=torch.float64, device=m.device)
    ep = ep.index_put((torch.arange(1, n + 1, device=m.device)[:, None],
                       torch.arange(1, n + 1, device=m.device)[None, :]), 10.0 ** m)
    mp = torch.nn.functional.pad(m, (1, 1, 1, 1))
    one = torch.nn.functional.pad(torch.ones_like(m), (1, 1, 1, 1))
    s = mp[:-1, :-1] + mp[1:, :-1] + mp[:-1, 1:] + mp[1:, 1:]
    c = one[:-1, :-1] + one[1:, :-1] + one[:-1, 1:] + one[1:, 1:]
    eb = torch.nn.functional.pad(10.0 ** (s / c), (0, 1, 0, 1), value=1.0)
    return eb, ep


def fd_check(n, base, m, cells, m_true, dev, log):
    """The adjoint workload's finite-difference check: dJ/dm (m = log10 eta_p
    per cell) from the adjoint path (StokesFunction) against central
    differences with h = 1e-3 on the given cells, two perturbed solves per
    cell (mixed, 1e-11).  Each perturbed solution is v0 + d with
    A(m +- h) d = b - A(m +- h) v0, so the solver error is relative to the
    small correction.  Returns the wall time of the perturbed solves and the
    largest relative error."""
    import numpy as np
    import torch
    import paper_2603_14040_amd as tph
    import workloads as wl
    s = tph.Solver(n, n, precision=tph.MIXED, rtol=1e-11, max_iters=3000, device=dev)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    rho = T(base.rho_b)
    gx, gy = base.gx, base.gy
    eb_t, ep_t = wl.logvisc_to_eta(m_true, n, n)
    s.set_coefficients(T(eb_t), T(ep_t), rho, gx, gy)
    target = s.solve()[0][n, 1:n].clone()

    def J_of_v(vx):
        return 0.5 * (1.0 / n) * torch.sum((vx[n, 1:n] - target) ** 2)

    mt = T(m).requires_grad_(True)
    eb, ep = eta_from_logvisc(mt, n)
    vx, _, _ = tph.StokesFunction.apply(eb, ep, rho, s, gx, gy)
    J_of_v(vx).backward()
    grad = mt.grad.detach().cpu().numpy()
    gmax = float(np.abs(grad).max())
    with torch.no_grad():
        eb0, ep0 = eta_from_logvisc(T(m), n)
        s.set_coefficients(eb0, ep0, rho, gx, gy)
        vx0, vy0, p0, _ = s.solve()
        bx, by = torch.zeros_like(rho), torch.zeros_like(rho)
        bx[1:n + 1, 1:n] = -gx * 0.5 * (rho[0:n, 1:n] + rho[1:n + 1, 1:n])
        by[1:n, 1:n + 1] = -gy * 0.5 * (rho[1:n, 0:n] + rho[1:n, 1:n + 1])

        def J_pert(mm):
            ebp, epp = eta_from_logvisc(mm, n)
            s.set_coefficients(ebp, epp, rho, gx, gy)
            ax, ay, ap = s.apply(vx0, vy0, p0)
            dvx, _, _, info = s.solve_rhs(bx - ax, by - ay, -ap)
            if info.res_energy > 1e-9:
                raise RuntimeError(f"finite-difference solve stopped at {info.res_energy:.2e}")
            return float(J_of_v(vx0 + dvx))

        h = 1e-3
        errs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (ci, cj) in cells:
            i, j = int(ci) - 1, int(cj) - 1
            mp_, mm_ = T(m), T(m)
            mp_[i, j] += h
            mm_[i, j] -= h
            fd = (J_pert(mp_) - J_pert(mm_)) / (2 * h)
            errs.append(abs(grad[i, j] - fd) / max(abs(fd), 1e-3 * gmax))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    s.close()
    res = {"cells": len(cells), "solves": 2 * len(cells), "seconds": round(dt, 3),
           "ms_per_solve": 1e3 * dt / (2 * len(cells)), "max_rel_err": float(max(errs)),
           "median_rel_err": float(np.median(errs)), "passed": bool(max(errs) <= 1e-4)}
    log(f"[bench] adjoint finite-difference check: {2 * len(cells)} solves in {dt:.2f} s, max rel err "
        f"{res['max_rel_err']:.2e}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default=",".join(DEFAULT_SECTIONS),
                    help=f"comma-separated sections out of {','.join(SECTIONS)}")
    ap.add_argument("--n", type=int, default=1024, help="cells per side of the headline problem")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 headline steps (default: --steps)")
    ap.add_argument("--no-tune", action="store_true", help="library defaults instead of autotuned parameters")
    ap.add_argument("--tune-reps", type=int, default=2, help="timed solves per autotuner candidate")
    ap.add_argument("--tuning-db", default=None, help="JSON tuning database to store (and with --reuse-tuning, "
                                                      "to read) the headline's tuned parameters")
    ap.add_argument("--reuse-tuning", action="store_true", help="take tuned parameters from --tuning-db if present")
    ap.add_argument("--large", type=int, default=4096, help="cells per side of the multi-inclusion problem")
    ap.add_argument("--large-reps", type=int, default=5, help="timed mixed solves of the large problem (median)")
    ap.add_argument("--large-fp64-reps", type=int, default=3, help="timed FP64 solves of the large problem (median)")
    ap.add_argument("--tune-large", action="store_true",
                    help="tune the large problem's schedule on its held-out instance instead of LARGE_PARAMS")
    ap.add_argument("--roofline-kernel", choices=("link", "smooth"), default="link",
                    help="kernel class of the roofline entry (timed inside the large mixed solves)")
    ap.add_argument("--skip-continuation", action="store_true", help="no continuation solve in the large section")
    ap.add_argument("--tune-batch", action="store_true",
                    help="tune the batch schedule on its held-out instance instead of BATCH_PARAMS")
    ap.add_argument("--batch", type=int, default=256, help="problems in the batched workload")
    ap.add_argument("--batch-reps", type=int, default=5, help="timed batched solves per precision (median)")
    ap.add_argument("--batch-precisions", default="mixed,fp64", help="precisions of the batched runs")
    ap.add_argument("--adjoint-reps", type=int, default=5)
    ap.add_argument("--adjoint-precisions", default="mixed,fp64", help="precisions of the adjoint runs")
    ap.add_argument("--fd-cells", type=int, default=64,
                    help="cells of the adjoint finite-difference check (two perturbed solves each; 0: skip)")
    ap.add_argument("--config1-steps", type=int, default=20)
    ap.add_argument("--accel-steps", type=int, default=5)
    ap.add_argument("--ras-steps", type=int, default=5)
    ap.add_argument("--mic-steps", type=int, default=3)
    ap.add_argument("--markers-per-cell", type=int, default=16)
    ap.add_argument("--robust-iters", type=int, default=1000, help="Uzawa iterations of the robustness runs")
    ap.add_argument("--cpu-sizes", default="64,128,256", help="oracle sample sizes (cells per side)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="same as leaving 'cpu' out of --only")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU; multi-GPU runs (--gpus > 1) are not supported "
                                   "(a sharded solve would split the grid into row bands, one per GPU, with "
                                   "halo exchanges per sweep and all-reduces for the Krylov dot products)"}))
        sys.exit(2)
    only = [s.strip() for s in args.only.split(",") if s.strip()]
    bad = [s for s in only if s not in SECTIONS]
    if bad:
        ap.error(f"unknown sections {bad}; choose from {SECTIONS}")
    if args.no_cpu_baseline and "cpu" in only:
        only.remove("cpu")

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import paper_2603_14040_amd as tph
    from paper_2603_14040_amd import _lib, autotune
    import workloads as wl

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sync = torch.cuda.synchronize
    out = {"metric": METRIC, "value": None, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 V-cycle + f64 Krylov/residual/coarsest/pressure (mixed)",
           "data": "synthetic", "config": None}

    def solve_stats(infos):
        return {"iters": infos[-1].iters, "vcycles": infos[-1].vcycles, "res_energy": infos[-1].res_energy,
                "res_l2": infos[-1].res_l2}

    def check_ok(infos, tag):
        for inf in infos:
            if inf.status != "TPH_OK":
                raise RuntimeError(f"{tag} solve did not converge: {inf}")

    # device-to-device copy bandwidth in the same run (context for the rooflines; also the calibration
    # copy of the counter runs: 1 GiB read and 1 GiB written per copy)
    def copy_probe():
        buf = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(buf)
        dst.copy_(buf)
        sync()
        t0 = time.perf_counter()
        for _ in range(20):
            dst.copy_(buf)
        sync()
        gbs = 2 * buf.numel() * 4 * 20 / (time.perf_counter() - t0) / 1e9
        del buf, dst
        torch.cuda.empty_cache()
        return gbs

    if "headline" in only or "large" in only or "batch" in only:
        out["copy_GBps"] = round(copy_probe(), 1)
        log(f"[bench] device copy {out['copy_GBps']:.0f} GB/s")

    n = args.n
    cells = n * n
    pr = eb = ep = rho = None
    heldout = None  # (eta_b, eta_p, rho, gx, gy, also): the first held-out instance and the others
    tuned = {"mixed": {"params": {}}, "fp64": {"params": {}}}
    if any(s in only for s in ("headline", "adjoint", "accel", "ras", "mic")):
        log(f"[bench] building the random-viscosity workload {n}x{n}")
        pr = wl.random_viscosity(n)
        eb, ep, rho = to(pr.eta_b), to(pr.eta_p), to(pr.rho_b)
        # schedule and kernel plan tuned on held-out instances of the recipe (untimed; the answer does not
        # depend on them)
        held = [wl.random_viscosity(n, seed_field=a, seed_noise=b) for a, b in HEADLINE_TUNE_SEEDS]
        ph = held[0]
        ebh, eph, rhoh = to(ph.eta_b), to(ph.eta_p), to(ph.rho_b)
        also = [(to(q.eta_b), to(q.eta_p), to(q.rho_b), q.gx, q.gy) for q in held[1:]]
        for prec, tag in ((tph.MIXED, "mixed"), (tph.FP64, "fp64")):
            if args.no_tune or (prec == tph.FP64 and args.fp64_steps == 0):
                tuned[tag] = {"params": {}, "ms": None, "default_ms": None, "trials": 0, "seconds": 0.0}
                continue
            db = autotune.TuningDB(args.tuning_db) if args.tuning_db else None
            key = autotune.TuningDB.key(n, n, prec, autotune.device_name(dev), _lib.version(), "grf-heldout") \
                if db else None
            if db is not None and args.reuse_tuning and db.get(key):
                tuned[tag] = db.get(key)
                log(f"[bench] {tag}: parameters from {args.tuning_db}")
                continue
            log(f"[bench] autotuning the {tag} solve on the held-out instances")
            tuned[tag] = autotune.tune(ebh, eph, rhoh, ph.gx, ph.gy, precision=prec, reps=args.tune_reps, device=dev,
                                       db=db, tag="grf-heldout", starts=[autotune.ALT_START], also=also)
            log(f"[bench] {tag}: tuned {tuned[tag]['params']} {tuned[tag]['ms']:.2f} ms on the first held-out "
                f"instance (defaults {tuned[tag]['default_ms']:.2f} ms, {tuned[tag]['trials']} trials, "
                f"{tuned[tag]['seconds']:.1f} s)")
        heldout = (ebh, eph, rhoh, ph.gx, ph.gy, also)
        del ebh, eph, rhoh, also

    # ---------------------------------------------------------------- headline
    if "headline" in only:
        live = {}

        def run(precision, steps, warmup, tag):
            s = tph.Solver(n, n, precision=precision, device=dev, **tuned[tag]["params"])
            vx, vy, p = s.zeros(), s.zeros(), s.zeros()

            def step():
                vx.zero_(); vy.zero_(); p.zero_()
                s.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
                return s.solve(vx, vy, p)[3]

            for _ in range(warmup):
                step()
            if precision == tph.MIXED:
                # kernel time stamps of every 17th finest-level smoothing launch of the timed solves (a
                # stride prime to the launch pattern samples every sweep mode)
                s.kernel_timing(17, target=_lib.KERNEL_SMOOTH)
                s.kernel_timing_read()
            sync()
            t0 = time.perf_counter()
            infos = [step() for _ in range(steps)]
            sync()
            dt = time.perf_counter() - t0
            if precision == tph.MIXED:
                live["smooth"] = s.kernel_timing_read()
                s.kernel_timing(0)
            check_ok(infos, tag)
            ms = 1e3 * dt / steps
            log(f"[bench] {tag}: {ms:.2f} ms/step, iters {infos[-1].iters}, vcycles {infos[-1].vcycles}, res "
                f"{infos[-1].res_energy:.2e}, setup {infos[-1].t_setup_ms:.2f} ms")
            return s, ms, infos

        s_mix, ms_mix, inf_mix = run(tph.MIXED, args.steps, args.warmup, "mixed")
        fp64_steps = args.steps if args.fp64_steps is None else args.fp64_steps
        ms_64 = inf_64 = None
        if fp64_steps > 0:
            s64, ms_64, inf_64 = run(tph.FP64, fp64_steps, 1, "fp64")
            s64.close()
        nk, msk, byk, drk = live["smooth"]
        if nk == 0:
            raise RuntimeError("no finest-level smoothing launch was timed")
        plan0 = s_mix.level_plan(0)
        out.update({
            "value": cells / (ms_mix * 1e-3), "ms_per_step": ms_mix,
            "config": {"workload": f"random-viscosity {n}x{n} cells, log10 eta Gaussian random field (corr. length "
                                   f"0.05, contrast 1e4, seeds 2/22), free slip, "
                                   f"{['FGMRES', 'GCR', 'Anderson'][s_mix.desc.accel]}({s_mix.desc.restart}) + "
                                   f"{s_mix.levels}-level V-cycle, relative energy residual 1e-8",
                       "cells": cells, "levels": s_mix.levels, "precision": "mixed", "global_batch": 1},
            "setup_ms": inf_mix[-1].t_setup_ms, "solve_ms": inf_mix[-1].t_solve_ms,
            "tuned": {"instance": "held-out random-viscosity instances (seeds " +
                                  ", ".join(f"{a}/{b}" for a, b in HEADLINE_TUNE_SEEDS) +
                                  "; cost = mean solve time over them; ms = the first)", **tuned},
            # the 1024^2 FP32 working set (~30 MB) sits in the 256 MB Infinity Cache: effective bandwidth, no
            # HBM fraction
            "cache_effective": {"kernel": f"finest-level Gauss-Seidel sweep ({plan0[0]}, tile shape {plan0[1]}), "
                                          f"every 17th launch inside the timed mixed solves",
                                "launches": nk, "dropped": drk, "us_per_launch": round(1e3 * msk / nk, 3),
                                "algorithmic_bytes_per_launch": byk / nk,
                                "GBps": round(byk / (msk * 1e-3) / 1e9, 1)},
        })
        out["configs"] = out.get("configs", {})
        out["configs"]["2_random_viscosity_1024"] = {
            "mixed": {"value": cells / (ms_mix * 1e-3), "ms": ms_mix, **solve_stats(inf_mix),
                      "vcycle_cells_per_s": cells * inf_mix[-1].vcycles / (ms_mix * 1e-3)},
            "fp64": ({"value": cells / (ms_64 * 1e-3), "ms": ms_64, **solve_stats(inf_64)} if inf_64 else None),
            "mixed_speedup_vs_fp64": (ms_64 / ms_mix) if ms_64 else None}
        s_mix.close()

    # ---------------------------------------------------------------- config 1
    if "config1" in only:
        p1 = wl.sinker(64)
        e1b, e1p, r1 = to(p1.eta_b), to(p1.eta_p), to(p1.rho_b)
        res1 = {}
        for prec, tag in ((tph.FP64, "fp64"), (tph.MIXED, "mixed")):
            s1 = tph.Solver(64, 64, precision=prec, levels=4, accel="fgmres", device=dev)
            ts, infs = [], []
            for k in range(args.config1_steps + 2):
                sync()
                t0 = time.perf_counter()
                s1.set_coefficients(e1b, e1p, r1, p1.gx, p1.gy)
                infs.append(s1.solve()[3])
                sync()
                if k >= 2:
                    ts.append(time.perf_counter() - t0)
            check_ok(infs, f"config1 {tag}")
            ms = 1e3 * median(ts)
            res1[tag] = {"value": 64 * 64 / (ms * 1e-3), "ms": ms, **solve_stats(infs)}
            log(f"[bench] config1 {tag}: {ms:.2f} ms, iters {infs[-1].iters}")
            s1.close()
        out.setdefault("configs", {})["1_sinker_64"] = {
            "workload": "64x64 sinker (disc r 0.1, eta 1e3, rho 1), free slip, FGMRES(20) + 4-level V-cycle, "
                        "defaults otherwise, median of the timed steps", **res1}

    # ---------------------------------------------------------------- large (config 3)
    if "large" in only:
        nl_ = args.large
        pl = wl.multi_inclusion(nl_)
        log(f"[bench] multi-inclusion workload {nl_}x{nl_}")
        lparams = {k: dict(v) for k, v in LARGE_PARAMS.items()}
        ltune = None
        if args.tune_large:
            ph_ = wl.multi_inclusion(nl_, seed=LARGE_TUNE_SEED)
            ltune = {}
            for prec, tag in ((tph.MIXED, "mixed"), (tph.FP64, "fp64")):
                r_ = autotune.tune(to(ph_.eta_b), to(ph_.eta_p), to(ph_.rho_b), ph_.gx, ph_.gy, precision=prec,
                                   reps=1, rounds=1, device=dev, knobs=autotune.schedule_knobs(),
                                   start=lparams[tag], max_iters=2000, log=log)
                lparams[tag] = {k: r_["params"][k] for k in LARGE_PARAMS[tag]}
                ltune[tag] = {"params": lparams[tag], "ms": r_["ms"], "trials": r_["trials"],
                              "seconds": r_["seconds"]}
                log(f"[bench] large {tag}: tuned on seed {LARGE_TUNE_SEED}: {lparams[tag]} {r_['ms']:.0f} ms "
                    f"({r_['trials']} trials)")
            del ph_
        leb, lep, lrho = to(pl.eta_b), to(pl.eta_p), to(pl.rho_b)
        large = {"workload": f"{nl_}x{nl_} cells, 200 discs (seed 3) radius U(0.005,0.03), eta 10^U(-3,3), rho "
                             f"U(-1,1), background eta 1 rho 0, free slip", "cells": nl_ * nl_,
                 "params": lparams, "schedule_source": ("tuned in this run" if ltune else
                                                        f"LARGE_PARAMS (tuned on seed {LARGE_TUNE_SEED})"),
                 "tuning": ltune}
        roof_target = _lib.KERNEL_LINK if args.roofline_kernel == "link" else _lib.KERNEL_SMOOTH
        for prec, tag, reps in ((tph.MIXED, "mixed", args.large_reps), (tph.FP64, "fp64", args.large_fp64_reps)):
            if reps <= 0:
                continue
            sl = tph.Solver(nl_, nl_, precision=prec, device=dev, max_iters=3000, **lparams[tag])
            vx, vy, p = sl.zeros(), sl.zeros(), sl.zeros()
            ts, infs = [], []
            for k in range(reps + 1):
                if k == 1 and prec == tph.MIXED:
                    # kernel time stamps of every 13th launch of the roofline kernel in the timed solves
                    sl.kernel_timing(13, target=roof_target)
                    sl.kernel_timing_read()
                vx.zero_(); vy.zero_(); p.zero_()
                sync()
                t0 = time.perf_counter()
                sl.set_coefficients(leb, lep, lrho, pl.gx, pl.gy)
                infs.append(sl.solve(vx, vy, p)[3])
                sync()
                if k >= 1:
                    ts.append(time.perf_counter() - t0)
            check_ok(infs, f"large {tag}")
            ms = 1e3 * median(ts)
            large[tag] = {"value": nl_ * nl_ / (ms * 1e-3), "ms": ms, "ms_all": [round(1e3 * t, 1) for t in ts],
                          **solve_stats(infs)}
            log(f"[bench] large {tag}: median {ms:.0f} ms over {len(ts)}, iters {infs[-1].iters}, vcycles "
                f"{infs[-1].vcycles}, res {infs[-1].res_energy:.1e}")
            if prec == tph.MIXED:
                nk, msk, byk, drk = sl.kernel_timing_read()
                sl.kernel_timing(0)
                if nk == 0:
                    raise RuntimeError("no launch of the roofline kernel was timed")
                achieved = byk / (msk * 1e-3) / 1e9
                from paper_2603_14040_amd import profiling
                traffic = None
                tfile = os.path.join(ROOT, "profiles", f"{args.roofline_kernel}_traffic_multi{nl_}_mixed.json")
                if os.path.exists(tfile):
                    with open(tfile) as fh:
                        tj = json.load(fh)
                    if tj.get("sources_sha256") == profiling.sources_hash(profiling.KERNEL_SOURCES[args.roofline_kernel]):
                        traffic = tj["bytes_per_launch"]
                what = ("Uzawa link pass (z += e with the pressure update, then the next step's FP64 residual or "
                        "the Krylov apply; FP32 correction, FP64 z, r, eta)" if args.roofline_kernel == "link" else
                        "finest-level Gauss-Seidel sweep on LDS tiles (FP32)")
                out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                                   "kernel": what, "workload": f"multi-inclusion {nl_}x{nl_}, mixed",
                                   "launches": nk, "dropped": drk, "us_per_launch": round(1e3 * msk / nk, 3),
                                   "algorithmic_bytes_per_launch": byk / nk,
                                   "frac_of_copy": round(achieved / out["copy_GBps"], 4)
                                   if out.get("copy_GBps") else None}
                log(f"[bench] roofline ({args.roofline_kernel}): {1e3 * msk / nk:.1f} us/launch, "
                    f"{achieved:.0f} GB/s = {achieved / HBM_PEAK_GBS:.3f} of HBM peak")
            if prec == tph.MIXED and not args.skip_continuation:
                # the same problem as a viscosity-rescaling continuation from the lithostatic pressure (next
                # row N1), one solve
                sync()
                t0 = time.perf_counter()
                cinf = sl.solve_continuation(leb, lep, lrho, pl.gx, pl.gy, thetas=(0.0, 0.25, 0.5, 0.75, 1.0),
                                             stage_rtol=1e-3, lithostatic=True)[3]
                sync()
                cdt = time.perf_counter() - t0
                large["continuation"] = {"thetas": [0.0, 0.25, 0.5, 0.75, 1.0], "stage_rtol": 1e-3,
                                         "lithostatic": True, "ms": 1e3 * cdt, "iters": cinf.iters,
                                         "res_energy": cinf.res_energy, "status": cinf.status,
                                         "value": nl_ * nl_ / cdt}
                log(f"[bench] large continuation: {1e3 * cdt:.0f} ms, {cinf.iters} iterations")
            sl.close()
            del sl, vx, vy, p
            torch.cuda.empty_cache()
        if large.get("mixed") and large.get("fp64"):
            large["mixed_speedup_vs_fp64"] = large["fp64"]["ms"] / large["mixed"]["ms"]
        out.setdefault("configs", {})["3_multi_inclusion_4096"] = large
        del leb, lep, lrho

    # ---------------------------------------------------------------- batch (config 4)
    if "batch" in only and args.batch > 0:
        probs = wl.batch_sinkers(args.batch, seed=4)
        bcells = sum(p.cells for p in probs)
        log(f"[bench] batched workload: {len(probs)} problems, {bcells} cells")
        ebs = [to(p.eta_b) for p in probs]
        eps = [to(p.eta_p) for p in probs]
        rhs_ = [to(p.rho_b) for p in probs]
        gxy = [(p.gx, p.gy) for p in probs]
        shapes = [(p.nx, p.ny) for p in probs]
        btuned = {"params": dict(BATCH_PARAMS), "source": f"BATCH_PARAMS (tuned on seed {BATCH_TUNE_SEED})"}
        if args.tune_batch:
            hp = wl.batch_sinkers(args.batch, seed=BATCH_TUNE_SEED)
            log(f"[bench] autotuning the batched schedule on the held-out batch (seed {BATCH_TUNE_SEED})")
            btuned = autotune.tune_batch([(p.nx, p.ny) for p in hp], [to(p.eta_b) for p in hp],
                                         [to(p.eta_p) for p in hp], [to(p.rho_b) for p in hp],
                                         [(p.gx, p.gy) for p in hp], precision=tph.MIXED, device=dev, log=log)
            btuned["source"] = f"tuned in this run on seed {BATCH_TUNE_SEED}"
            log(f"[bench] batch: tuned {btuned['params']} {btuned['ms']:.1f} ms (defaults "
                f"{btuned['default_ms']:.1f} ms, {btuned['trials']} trials, {btuned['seconds']:.1f} s)")
            del hp
            torch.cuda.empty_cache()
        batch = {"workload": f"{len(probs)} centred sinkers, sizes 64..512 (seed 4), radius U(0.05,0.2), contrast "
                             f"10^U(1,4), free slip", "cells": bcells, "tuned": btuned}
        for prec, tag in ((tph.MIXED, "mixed"), (tph.FP64, "fp64")):
            if tag not in args.batch_precisions.split(","):
                continue
            t0 = time.perf_counter()
            bat = tph.Batch(shapes, device=dev, precision=prec, **btuned["params"])
            t_create = time.perf_counter() - t0
            log(f"[bench] batch {tag}: created in {t_create:.1f} s")
            outs = bat.zeros(), bat.zeros(), bat.zeros()

            def bstep():
                for o in outs:
                    for t in o:
                        t.zero_()
                bat.set_coefficients(ebs, eps, rhs_, gxy)
                return bat.solve(*outs)[3]

            bstep()
            log(f"[bench] batch {tag}: warm-up solve done")
            ts, binf = [], None
            for _ in range(args.batch_reps):
                sync()
                t0 = time.perf_counter()
                binf = bstep()
                sync()
                ts.append(time.perf_counter() - t0)
            bdt = median(ts)
            its = [i.iters for i in binf]
            # lockstep fill: useful problem-iterations (weighted by cells) over what a
            # lockstep run to the slowest problem would cost with every problem active
            cell_its = sum(p.cells * i.iters for p, i in zip(probs, binf))
            vc_cells = sum(p.cells * i.vcycles for p, i in zip(probs, binf))
            batch[tag] = {"value": bcells / bdt, "ms": 1e3 * bdt, "ms_all": [round(1e3 * t, 1) for t in ts],
                          "iters_max": max(its), "iters_mean": sum(its) / len(its),
                          "lockstep_fill": cell_its / (bcells * max(its)),
                          "vcycle_cells_per_s": vc_cells / bdt,
                          "converged": sum(1 for i in binf if i.status == "TPH_OK"), "create_s": round(t_create, 2)}
            log(f"[bench] batch {tag}: median {1e3 * bdt:.1f} ms, {bcells / bdt:.3e} cells/s, iterations max "
                f"{max(its)} mean {sum(its) / len(its):.1f}")
            bat.close()
            del bat, outs
        if batch.get("mixed") and batch.get("fp64"):
            batch["mixed_speedup_vs_fp64"] = batch["fp64"]["ms"] / batch["mixed"]["ms"]
        out.setdefault("configs", {})["4_batch_256"] = batch
        del ebs, eps, rhs_
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- adjoint (config 5)
    if "adjoint" in only:
        base, m, m_true, cells_ = wl.adjoint_problem(n)
        eb_t, ep_t = wl.logvisc_to_eta(m_true, n, n)
        adj = {"workload": f"gradient of the surface-velocity misfit w.r.t. viscosity, {n}x{n} random field, "
                           f"target from the perturbed field (seed 5); forward solve, adjoint solve and gradient "
                           f"kernel each timed (median), plus the autograd step (StokesFunction)"}
        for prec, tag in ((tph.MIXED, "mixed"), (tph.FP64, "fp64")):
            if tag not in args.adjoint_precisions.split(","):
                continue
            sa = tph.Solver(n, n, precision=prec, device=dev, **tuned[tag]["params"])
            sa.set_coefficients(to(eb_t), to(ep_t), rho, pr.gx, pr.gy)
            target = sa.solve()[0][n, 1:n].clone()
            gvx = sa.zeros()
            tf, tad, tg, tt = [], [], [], []
            for k in range(args.adjoint_reps + 1):
                sync()
                t0 = time.perf_counter()
                sa.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
                vx_, vy_, p_, fi = sa.solve()
                sync()
                t1 = time.perf_counter()
                gvx.zero_()
                gvx[n, 1:n] = (1.0 / n) * (vx_[n, 1:n] - target)
                lvx, lvy, lp, ai = sa.solve_adjoint(gvx)
                sync()
                t2 = time.perf_counter()
                sa.coeff_gradient(vx_, vy_, p_, lvx, lvy, lp)
                sync()
                t3 = time.perf_counter()
                check_ok([fi, ai], f"adjoint {tag}")
                if k >= 1:
                    tf.append(t1 - t0); tad.append(t2 - t1); tg.append(t3 - t2)
            ebg = eb.clone().requires_grad_(True)
            epg = ep.clone().requires_grad_(True)
            for k in range(3):
                ebg.grad = None
                epg.grad = None
                sync()
                t0 = time.perf_counter()
                vx_, vy_, p_ = tph.StokesFunction.apply(ebg, epg, rho, sa, pr.gx, pr.gy)
                J = 0.5 * (1.0 / n) * torch.sum((vx_[n, 1:n] - target) ** 2)
                J.backward()
                sync()
                if k >= 1:
                    tt.append(time.perf_counter() - t0)
            fwd, adm, grd = 1e3 * median(tf), 1e3 * median(tad), 1e3 * median(tg)
            adj[tag] = {"forward_ms": fwd, "adjoint_ms": adm, "gradient_ms": grd, "autograd_step_ms": 1e3 * median(tt),
                        "value": 2 * cells / ((fwd + adm) * 1e-3), "unit": "cells/s (forward + adjoint solves)",
                        "forward_iters": fi.iters, "adjoint_iters": ai.iters}
            log(f"[bench] adjoint {tag}: forward {fwd:.1f} ms, adjoint {adm:.1f} ms, gradient {grd:.2f} ms, "
                f"autograd step {adj[tag]['autograd_step_ms']:.1f} ms")
            sa.close()
        if args.fd_cells > 0:
            adj["fd_check"] = fd_check(n, base, m, cells_[:args.fd_cells], m_true, dev, log)
        out.setdefault("configs", {})["5_adjoint_1024"] = adj

    # ---------------------------------------------------------------- accelerators (next row N2)
    if "accel" in only and args.accel_steps > 0:
        from paper_2603_14040_amd.autotune import Knob
        accels = {}
        base = dict(tuned["mixed"]["params"])
        space = {"gcr": [Knob("restart", [5, 8, 10, 15, 20, 30])],
                 "anderson": [Knob("restart", [3, 5, 8, 10, 15, 20]), Knob("beta", [0.5, 0.7, 0.85, 1.0])]}
        first = {"gcr": {"restart": int(base.get("restart", 20))}, "anderson": {"restart": 10, "beta": 1.0}}
        for name in ("gcr", "anderson"):
            params = dict(base, accel=name, **first[name])
            at_ = None
            if not args.no_tune:
                hb, hp, hr, hgx, hgy, hal = heldout
                at_ = autotune.tune(hb, hp, hr, hgx, hgy, precision=tph.MIXED, reps=1, rounds=1, device=dev,
                                    knobs=space[name], start=params, also=hal)
                params = at_["params"]
            sa_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, **params)
            ax_, ay_, ap_ = sa_.zeros(), sa_.zeros(), sa_.zeros()

            def astep_():
                ax_.zero_(); ay_.zero_(); ap_.zero_()
                sa_.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
                return sa_.solve(ax_, ay_, ap_)[3]

            astep_()
            sync()
            t0 = time.perf_counter()
            ainf = [astep_() for _ in range(args.accel_steps)]
            sync()
            ams = 1e3 * (time.perf_counter() - t0) / args.accel_steps
            check_ok(ainf, name)
            kind = _lib.KERNEL_GCR_STEP if name == "gcr" else _lib.KERNEL_AA_MIX
            kms, kby = sa_.time_kernel(kind, 100)
            kgbs = kby / (kms * 1e-3) / 1e9
            accels[name] = {"ms_per_step": ams, "value": cells / (ams * 1e-3), "unit": "cells/s",
                            "iters": ainf[-1].iters, "res_energy": ainf[-1].res_energy,
                            "restart": params["restart"], "beta": params["beta"] if name == "anderson" else None,
                            "tuning_trials": at_["trials"] if at_ else 0,
                            "tuned_on": "held-out instances" if at_ else None,
                            "kernel": {"name": "k_gcr_step" if name == "gcr" else "k_mix",
                                       "what": ("GCR step update with restart/2 earlier directions" if name == "gcr"
                                                else "Anderson mixing over restart + 1 stored pairs"),
                                       "us": round(kms * 1e3, 2), "bytes": kby, "effective_GBps": round(kgbs, 1)}}
            log(f"[bench] {name}: {ams:.2f} ms/step, iters {ainf[-1].iters}; {accels[name]['kernel']['name']} "
                f"{kgbs:.0f} GB/s effective")
            sa_.close()
        out["accelerators"] = accels

    # ---------------------------------------------------------------- RAS smoother (next row N3)
    if "ras" in only and args.ras_steps > 0:
        from paper_2603_14040_amd.autotune import Knob
        base = {k: v for k, v in tuned["mixed"]["params"].items() if k not in ("msweep", "tile_shape", "coarse_level")}
        params = dict(base, smoother=tph.SMOOTH_RAS, ras_tile=16, ras_inner=4, nu_pre=4, nu_post=4, omega=0.6)
        rt_ = None
        if not args.no_tune:
            hb, hp, hr, hgx, hgy, hal = heldout
            rt_ = autotune.tune(hb, hp, hr, hgx, hgy, precision=tph.MIXED, reps=1, rounds=2, device=dev, also=hal,
                                knobs=[Knob("smoother", [tph.SMOOTH_RAS, tph.SMOOTH_RAS_MIXED]),
                                       Knob("ras_tile", [8, 16, 32]), Knob("ras_inner", [1, 2, 4, 8]),
                                       Knob("nu_pre", [2, 4, 8]), Knob("nu_post", [2, 4, 8]),
                                       Knob("omega", [0.5, 0.6, 0.7])], start=params)
            params = {k: v for k, v in rt_["params"].items() if k not in ("msweep", "tile_shape", "coarse_level")}
        sr_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, **params)
        rx_, ry_, rp_ = sr_.zeros(), sr_.zeros(), sr_.zeros()

        def rstep_():
            rx_.zero_(); ry_.zero_(); rp_.zero_()
            sr_.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
            return sr_.solve(rx_, ry_, rp_)[3]

        rstep_()
        sync()
        t0 = time.perf_counter()
        rinf = [rstep_() for _ in range(args.ras_steps)]
        sync()
        rms = 1e3 * (time.perf_counter() - t0) / args.ras_steps
        check_ok(rinf, "RAS")
        sr_.close()
        kr_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, smoother=tph.SMOOTH_RAS,
                         ras_tile=params["ras_tile"], ras_inner=params["ras_inner"], omega=params["omega"])
        kr_.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
        kms, kby = kr_.time_kernel(_lib.KERNEL_SMOOTH, 100)
        kr_.close()
        kgbs = kby / (kms * 1e-3) / 1e9
        out["ras"] = {"ms_per_step": rms, "value": cells / (rms * 1e-3), "unit": "cells/s", "iters": rinf[-1].iters,
                      "res_energy": rinf[-1].res_energy,
                      "params": {k: params[k] for k in ("smoother", "ras_tile", "ras_inner", "nu_pre", "nu_post",
                                                        "omega", "accel", "restart", "uzawa_steps", "alpha")},
                      "tuning_trials": rt_["trials"] if rt_ else 0,
                      "tuned_on": "held-out instances" if rt_ else None,
                      "kernel": {"name": "k_ras_tile",
                                 "what": (f"one outer iteration ({params['ras_inner']} Jacobi sweeps) on "
                                          f"{params['ras_tile']}^2 tiles, finest level"),
                                 "us": round(kms * 1e3, 2), "bytes": kby, "effective_GBps": round(kgbs, 1)}}
        log(f"[bench] ras: {rms:.2f} ms/step, iters {rinf[-1].iters}; k_ras_tile {kms * 1e3:.1f} us per launch")

    # ---------------------------------------------------------------- marker-in-cell (next row N4)
    if "mic" in only and args.mic_steps > 0:
        xm_, ym_, meta_, mrho_ = wl.markers(pr, per_cell=args.markers_per_cell, seed=13)
        nm = xm_.size
        X_, Y_, E_, R_ = to(xm_), to(ym_), to(meta_), to(mrho_)
        mk_ = tph.Markers(n, n, capacity=nm, device=dev)
        sm_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, **tuned["mixed"]["params"])
        mvx, mvy, mp = sm_.zeros(), sm_.zeros(), sm_.zeros()
        stages = {"to_grid": 0.0, "solve": 0.0, "advect": 0.0}

        def mic_step(timed):
            t0 = time.perf_counter()
            eb_, rb_ = mk_.to_grid("basic", X_, Y_, [E_, R_])
            ep_ = mk_.to_grid("cell", X_, Y_, [E_])[0]
            ep_[0, :] = 1.0; ep_[-1, :] = 1.0; ep_[:, 0] = 1.0; ep_[:, -1] = 1.0   # unused entries
            eb_[-1, :] = 1.0; eb_[:, -1] = 1.0
            sync()
            t1 = time.perf_counter()
            mvx.zero_(); mvy.zero_(); mp.zero_()
            sm_.set_coefficients(eb_, ep_, rb_, pr.gx, pr.gy)
            inf_ = sm_.solve(mvx, mvy, mp)[3]
            sync()
            t2 = time.perf_counter()
            vmax = max(mvx.abs().max().item(), mvy.abs().max().item())
            mk_.advect_rk4(X_, Y_, mvx, mvy, 0.5 / n / max(vmax, 1e-300))
            sync()
            t3 = time.perf_counter()
            if timed:
                stages["to_grid"] += t1 - t0
                stages["solve"] += t2 - t1
                stages["advect"] += t3 - t2
            return inf_

        mic_step(False)
        t0 = time.perf_counter()
        minf = [mic_step(True) for _ in range(args.mic_steps)]
        mdt = (time.perf_counter() - t0) / args.mic_steps
        check_ok(minf, "marker-in-cell")
        Xa, Ya = X_.clone(), Y_.clone()
        mk_.advect_rk4(Xa, Ya, mvx, mvy, 1e-9)
        sync()
        t0 = time.perf_counter()
        for _ in range(20):
            mk_.advect_rk4(Xa, Ya, mvx, mvy, 1e-9)
        sync()
        rk_ms = 1e3 * (time.perf_counter() - t0) / 20
        per = {k: 1e3 * v / args.mic_steps for k, v in stages.items()}
        out["marker_in_cell"] = {
            "workload": f"{nm} markers ({args.markers_per_cell} per cell, seed 13) on the {n}x{n} random-viscosity "
                        f"grid, eta and rho per marker; step = marker -> grid (3 fields, 2 binnings) + mixed solve "
                        f"+ RK4", "markers": nm, "ms_per_step": 1e3 * mdt, "stages_ms": per,
            "iters": minf[-1].iters, "markers_to_grid_per_s": 3 * nm / (per["to_grid"] * 1e-3),
            "rk4": {"ms": rk_ms, "markers_per_s": nm / (rk_ms * 1e-3),
                    "effective_GBps": round(32.0 * nm / (rk_ms * 1e-3) / 1e9, 1),
                    "what": "positions 2 x 8 B read + written per marker; grid reads through the caches"}}
        log(f"[bench] marker-in-cell: {1e3 * mdt:.1f} ms/step (to_grid {per['to_grid']:.1f}, solve "
            f"{per['solve']:.1f}, advect {per['advect']:.2f} ms)")
        mk_.close()
        sm_.close()

    # ---------------------------------------------------------------- robustness (paper's sinker test set-up)
    if "robust" in only and args.robust_iters > 125:
        ps_ = wl.sinker(500, ny=600, ly=1.2, center=(0.5, 0.6), radius=0.2, eta_in=1e8, rho_in=33.0, eta_out=1.0,
                        rho_out=32.0)
        ebs_, eps_, rhos_ = to(ps_.eta_b), to(ps_.eta_p), to(ps_.rho_b)
        robust = {"workload": ("sinker 500x600 cells (501 x 601 nodes) on 1 x 1.2, contrast 1e8, densities 33 / 32, "
                               "free slip, unaccelerated Uzawa (one V-cycle per iteration, 4 levels coarsened by "
                               "2.5, 5+5 sweeps x2.5 per level, omega 0.3, alpha 0.6), continuation theta 0..1 in "
                               "steps of 0.25 every 25 iterations from the lithostatic pressure, FP64"),
                  "smoothers": {}}
        for name_, sm_ in (("rbgs", tph.SMOOTH_GS), ("jacobi", tph.SMOOTH_JACOBI), ("ras", tph.SMOOTH_RAS),
                           ("mixed", tph.SMOOTH_RAS_MIXED)):
            kw_ = dict(precision=tph.FP64, levels=4, coarsen=2.5, fused=False, smoother=sm_, nu_pre=5, nu_post=5,
                       nu_growth=2.5, omega=0.3, alpha=0.6, accel="anderson", restart=0, beta=1.0, uzawa_steps=1,
                       rtol=1e-14, ras_tile=32, ras_inner=4, ly=1.2)
            sync()
            t0 = time.perf_counter()
            s1_ = tph.Solver(500, 600, device=dev, max_iters=25, **kw_)
            vxs, vys, pps, i1_ = s1_.solve_continuation(ebs_, eps_, rhos_, ps_.gx, ps_.gy,
                                                        thetas=(0.0, 0.25, 0.5, 0.75, 1.0), stage_rtol=1e-14,
                                                        lithostatic=True, history=125)
            s2_ = tph.Solver(500, 600, device=dev, max_iters=args.robust_iters - i1_.iters, **kw_)
            s2_.set_coefficients(ebs_, eps_, rhos_, ps_.gx, ps_.gy)
            vxs, vys, pps, i2_ = s2_.solve(vxs, vys, pps, history=args.robust_iters)
            sync()
            rdt = time.perf_counter() - t0
            h_ = list(i1_.history) + list(i2_.history)
            first = {f"{t:.0e}": next((k + 1 for k, v in enumerate(h_) if k >= 100 and v <= t), None)
                     for t in (1e-6, 1e-8, 1e-10)}
            robust["smoothers"][name_] = {"iters": i1_.iters + i2_.iters, "seconds": round(rdt, 3),
                                          "res_final": i2_.res_energy, "first_iter_below": first}
            log(f"[bench] robustness {name_}: {i1_.iters + i2_.iters} iterations in {rdt:.2f} s")
            s1_.close()
            s2_.close()
        out["robustness"] = robust

    # ---------------------------------------------------------------- CPU baseline (the oracle)
    if "cpu" in only:
        sizes = [int(x) for x in args.cpu_sizes.split(",") if x.strip()]
        log(f"[bench] CPU oracle at {sizes} (one single-threaded child process)")
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        res = subprocess.run([sys.executable, "-m", "oracle.timing", *map(str, sizes)], cwd=ROOT, env=env,
                             capture_output=True, text=True, timeout=1200)
        if res.returncode != 0:
            raise RuntimeError(f"oracle timing failed:\n{res.stderr[-2000:]}")
        rows = [json.loads(ln) for ln in res.stdout.splitlines() if ln.startswith("{")]
        last = rows[-1]
        out["cpu_baseline"] = {
            "value": last["cells_per_s"], "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": (f"random-viscosity recipe (correlation length 0.05, contrast 1e4) at "
                       f"{', '.join(str(r['n']) + '^2' for r in rows)} cells: one FP64 assembled-matrix SuperLU "
                       f"solve each in a child process with one thread; value = the {last['n']}^2 solve "
                       f"({last['seconds']:.1f} s)"),
            "host_cores_available": len(os.sched_getaffinity(0)),
            "sizes": {str(r["n"]): {"cells_per_s": r["cells_per_s"], "seconds": r["seconds"],
                                    "peak_rss_mb": r["peak_rss_mb"], "res_energy": r["res_energy"]} for r in rows}}
        log(f"[bench] CPU oracle: " + ", ".join(f"{r['n']}^2 {r['seconds']:.1f} s" for r in rows))

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
