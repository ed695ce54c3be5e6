#!/usr/bin/env python3
"""Throughput of the MI355X Stokes solver on its headline workload.

One step = the whole hot path over one problem: coefficient setup
(viscosity restriction down the hierarchy, right-hand side, FP64 coarsest
factorisation) plus one solve from a zero initial guess to a relative energy
residual of 1e-8 (FGMRES + V-cycle/Uzawa preconditioner).  Workload: the
random-viscosity problem on a 1024 x 1024-cell grid (log10 viscosity a
Gaussian random field, correlation length 0.05, contrast 1e4; density
1 - 0.01 log10(eta) + N(0, 0.01); free slip; g = (0, -1)).  Inputs are
synthetic, seeded, and resident in HBM before timing starts.

Before timing, the autotuner (paper_2603_14040_amd.autotune) measures whole
solves of this problem and picks the per-level kernel plan, the sweeps, the
Uzawa steps and the restart length, for each precision (untimed; the answer
does not depend on these choices).  `tuned` reports the choice, its time and
the library defaults' time.

`value` is the mixed-precision throughput (FP32 V-cycle, FP64 outer Krylov,
residual, refinement and coarsest solve) in cells per second; the plain FP64
solve is timed beside it (`fp64`).  The roofline entry describes the dominant
kernel, the finest-level smoother, timed with HIP events on the solver's own
stream.  The CPU baseline is the FP64 oracle (assembled matrix + SuperLU) on
a bounded sample of the same recipe.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "Stokes solve cells/s to 1e-8 rel. residual + HBM GB/s; mixed vs FP64 on 1 GPU"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024, help="cells per side")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: --steps)")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-n", type=int, default=384, help="oracle sample size (cells per side)")
    ap.add_argument("--no-tune", action="store_true", help="library defaults instead of autotuned parameters")
    ap.add_argument("--tune-reps", type=int, default=2, help="timed solves per autotuner candidate")
    ap.add_argument("--tuning-db", default=None, help="JSON tuning database to store (and with --reuse-tuning, "
                                                       "read) the tuned parameters")
    ap.add_argument("--reuse-tuning", action="store_true", help="take tuned parameters from --tuning-db if present")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="problems in the batched workload (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-gradient workload")
    ap.add_argument("--large", type=int, default=4096, help="cells per side of the multi-inclusion workload (0: skip)")
    ap.add_argument("--accel-steps", type=int, default=5,
                    help="timed steps of the GCR and Anderson solves of the main workload (0: skip)")
    ap.add_argument("--ras-steps", type=int, default=5,
                    help="timed steps of the RAS-smoother solve of the main workload (0: skip)")
    ap.add_argument("--mic-steps", type=int, default=3,
                    help="timed marker-in-cell steps on the main grid (0: skip)")
    ap.add_argument("--markers-per-cell", type=int, default=16)
    ap.add_argument("--robust-iters", type=int, default=1000,
                    help="Uzawa iterations of the 1e8-contrast sinker robustness runs (0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU; multi-GPU runs (--gpus > 1) are not supported "
                                   "(a sharded solve would split the grid into row bands, one per GPU, with "
                                   "halo exchanges per sweep and all-reduces for the Krylov dot products)"}))
        sys.exit(2)

    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_2603_14040_amd as tph
    import workloads as wl

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = args.n
    cells = n * n
    log(f"[bench] building the random-viscosity workload {n}x{n}")
    pr = wl.random_viscosity(n)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    eb, ep, rho = to(pr.eta_b), to(pr.eta_p), to(pr.rho_b)

    # autotuned kernel plan and schedule (untimed; the answer does not depend on it)
    from paper_2603_14040_amd import autotune
    tuned = {}
    for prec, tag in ((tph.MIXED, "mixed"), (tph.FP64, "fp64")):
        if args.no_tune or (prec == tph.FP64 and args.fp64_steps == 0):
            tuned[tag] = {"params": {}, "ms": None, "default_ms": None, "trials": 0, "seconds": 0.0}
            continue
        db = autotune.TuningDB(args.tuning_db) if args.tuning_db else None
        key = autotune.TuningDB.key(n, n, prec, autotune.device_name(dev), tph._lib.version(), "grf") if db else None
        if db is not None and args.reuse_tuning and db.get(key):
            tuned[tag] = db.get(key)
            log(f"[bench] {tag}: parameters from {args.tuning_db}")
            continue
        log(f"[bench] autotuning the {tag} solve")
        tuned[tag] = autotune.tune(eb, ep, rho, pr.gx, pr.gy, precision=prec, reps=args.tune_reps, device=dev,
                                   db=db, tag="grf")
        log(f"[bench] {tag}: tuned {tuned[tag]['params']} {tuned[tag]['ms']:.2f} ms "
            f"(defaults {tuned[tag]['default_ms']:.2f} ms, {tuned[tag]['trials']} trials, "
            f"{tuned[tag]['seconds']:.1f} s)")

    def run(precision, steps, warmup, tag):
        s = tph.Solver(n, n, precision=precision, device=dev, **tuned[tag]["params"])
        vx, vy, p = s.zeros(), s.zeros(), s.zeros()

        def step():
            vx.zero_(); vy.zero_(); p.zero_()
            s.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
            return s.solve(vx, vy, p)[3]

        for _ in range(warmup):
            info = step()
        if precision == tph.MIXED:
            # kernel time stamps of every 17th finest-level smoothing launch of the timed solves
            # (a stride prime to the launch pattern samples every sweep mode)
            s.kernel_timing(17)
            s.kernel_timing_read()
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(step())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if precision == tph.MIXED:
            live[:] = s.kernel_timing_read()
            s.kernel_timing(0)
        for inf in infos:
            if inf.status != "TPH_OK":
                raise RuntimeError(f"{tag} solve did not converge: {inf}")
        ms = 1e3 * dt / steps
        log(f"[bench] {tag}: {ms:.2f} ms/step, iters {infos[-1].iters}, res {infos[-1].res_energy:.2e}, "
            f"setup {infos[-1].t_setup_ms:.2f} ms, solve {infos[-1].t_solve_ms:.2f} ms")
        return s, ms, infos

    live = [0, 0.0, 0.0, 0]
    s_mix, ms_mix, inf_mix = run(tph.MIXED, args.steps, args.warmup, "mixed")
    fp64_steps = args.steps if args.fp64_steps is None else args.fp64_steps
    s64 = None
    if fp64_steps > 0:
        s64, ms_64, inf_64 = run(tph.FP64, fp64_steps, 1, "fp64")
    plan0 = s_mix.level_plan(0)

    # the accelerators of Sec. "Accelerators" on the same workload, mixed precision, with the tuned schedule
    # and kernel plan: flexible GCR(m) (restart tuned) and Anderson AA(m, beta) (depth and mixing tuned);
    # the tuning is untimed, each timed step is set_coefficients + solve as above
    accels = {}
    if args.accel_steps > 0:
        from paper_2603_14040_amd.autotune import Knob
        base = dict(tuned["mixed"]["params"])
        space = {"gcr": [Knob("restart", [5, 8, 10, 15, 20, 30])],
                 "anderson": [Knob("restart", [3, 5, 8, 10, 15, 20]), Knob("beta", [0.5, 0.7, 0.85, 1.0])]}
        first = {"gcr": {"restart": int(base.get("restart", 20))}, "anderson": {"restart": 10, "beta": 1.0}}
        for name in ("gcr", "anderson"):
            params = dict(base, accel=name, **first[name])
            at_ = None
            if not args.no_tune:
                at_ = autotune.tune(eb, ep, rho, pr.gx, pr.gy, precision=tph.MIXED, reps=1, rounds=1, device=dev,
                                    knobs=space[name], start=params)
                params = at_["params"]
                log(f"[bench] {name}: tuned restart {params['restart']} beta {params['beta']} ({at_['trials']} trials)")
            sa_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, **params)
            ax_, ay_, ap_ = sa_.zeros(), sa_.zeros(), sa_.zeros()

            def astep_():
                ax_.zero_(); ay_.zero_(); ap_.zero_()
                sa_.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
                return sa_.solve(ax_, ay_, ap_)[3]

            astep_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ainf = [astep_() for _ in range(args.accel_steps)]
            torch.cuda.synchronize()
            ams = 1e3 * (time.perf_counter() - t0) / args.accel_steps
            if any(i.status != "TPH_OK" for i in ainf):
                raise RuntimeError(f"{name} solve did not converge: {ainf[-1]}")
            kind = tph._lib.KERNEL_GCR_STEP if name == "gcr" else tph._lib.KERNEL_AA_MIX
            kms, kby = sa_.time_kernel(kind, 100)
            kgbs = kby / (kms * 1e-3) / 1e9
            accels[name] = {"ms_per_step": ams, "value": cells / (ams * 1e-3), "unit": "cells/s",
                            "iters": ainf[-1].iters, "res_energy": ainf[-1].res_energy,
                            "restart": params["restart"], "beta": params["beta"] if name == "anderson" else None,
                            "tuning_trials": at_["trials"] if at_ else 0,
                            "kernel": {"name": "k_gcr_step" if name == "gcr" else "k_mix",
                                       "what": ("GCR step update with restart/2 earlier directions" if name == "gcr"
                                                else "Anderson mixing over restart + 1 stored pairs"),
                                       "us": round(kms * 1e3, 2), "bytes": kby, "GBps": round(kgbs, 1),
                                       "frac": round(kgbs / HBM_PEAK_GBS, 4)}}
            log(f"[bench] {name}: {ams:.2f} ms/step, iters {ainf[-1].iters}, res {ainf[-1].res_energy:.2e}; "
                f"{accels[name]['kernel']['name']} {kgbs:.0f} GB/s")
            sa_.close()
            del sa_

    # the RAS-type temporal-blocking smoother (every level, or below a Jacobi finest level) on the same
    # workload: smoother variant, tile side, inner sweeps, sweeps and damping tuned (untimed) around the
    # tuned accelerator schedule; the RAS kernel is timed on the finest level
    ras_out = None
    if args.ras_steps > 0:
        from paper_2603_14040_amd.autotune import Knob
        base = {k: v for k, v in tuned["mixed"]["params"].items() if k not in ("msweep", "tile_shape", "coarse_level")}
        params = dict(base, smoother=tph.SMOOTH_RAS, ras_tile=16, ras_inner=4, nu_pre=4, nu_post=4, omega=0.6)
        rt_ = None
        if not args.no_tune:
            rt_ = autotune.tune(eb, ep, rho, pr.gx, pr.gy, precision=tph.MIXED, reps=1, rounds=2, device=dev,
                                knobs=[Knob("smoother", [tph.SMOOTH_RAS, tph.SMOOTH_RAS_MIXED]),
                                       Knob("ras_tile", [8, 16, 32]), Knob("ras_inner", [1, 2, 4, 8]),
                                       Knob("nu_pre", [2, 4, 8]), Knob("nu_post", [2, 4, 8]),
                                       Knob("omega", [0.5, 0.6, 0.7])], start=params)
            params = {k: v for k, v in rt_["params"].items() if k not in ("msweep", "tile_shape", "coarse_level")}
            log(f"[bench] ras: tuned {params} ({rt_['trials']} trials, {rt_['seconds']:.1f} s)")
        sr_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, **params)
        rx_, ry_, rp_ = sr_.zeros(), sr_.zeros(), sr_.zeros()

        def rstep_():
            rx_.zero_(); ry_.zero_(); rp_.zero_()
            sr_.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
            return sr_.solve(rx_, ry_, rp_)[3]

        rstep_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rinf = [rstep_() for _ in range(args.ras_steps)]
        torch.cuda.synchronize()
        rms = 1e3 * (time.perf_counter() - t0) / args.ras_steps
        if any(i.status != "TPH_OK" for i in rinf):
            raise RuntimeError(f"RAS solve did not converge: {rinf[-1]}")
        sr_.close()
        # the RAS kernel on the finest level (one outer iteration of ras_inner sweeps)
        kr_ = tph.Solver(n, n, precision=tph.MIXED, device=dev, smoother=tph.SMOOTH_RAS,
                         ras_tile=params["ras_tile"], ras_inner=params["ras_inner"], omega=params["omega"])
        kr_.set_coefficients(eb, ep, rho, pr.gx, pr.gy)
        kms, kby = kr_.time_kernel(tph._lib.KERNEL_SMOOTH, 100)
        kr_.close()
        kgbs = kby / (kms * 1e-3) / 1e9
        ras_out = {"ms_per_step": rms, "value": cells / (rms * 1e-3), "unit": "cells/s", "iters": rinf[-1].iters,
                   "res_energy": rinf[-1].res_energy,
                   "params": {k: params[k] for k in ("smoother", "ras_tile", "ras_inner", "nu_pre", "nu_post",
                                                     "omega", "accel", "restart", "uzawa_steps", "alpha")},
                   "tuning_trials": rt_["trials"] if rt_ else 0,
                   "kernel": {"name": "k_ras_tile", "what": (f"one outer iteration ({params['ras_inner']} Jacobi "
                                                             f"sweeps) on {params['ras_tile']}^2 tiles, finest level"),
                              "us": round(kms * 1e3, 2), "bytes": kby, "GBps": round(kgbs, 1),
                              "frac": round(kgbs / HBM_PEAK_GBS, 4),
                              "sweeps_per_s": params["ras_inner"] / (kms * 1e-3)}}
        log(f"[bench] ras: {rms:.2f} ms/step, iters {rinf[-1].iters}, res {rinf[-1].res_energy:.2e}; k_ras_tile "
            f"{kms * 1e3:.1f} us per launch, {kgbs:.0f} GB/s")

    # dominant kernel: finest-level smoother of the mixed path, HIP events on the solver stream
    kern = {}
    names = {tph._lib.KERNEL_SMOOTH: "smooth_l0", tph._lib.KERNEL_APPLY: "apply_fp64",
             tph._lib.KERNEL_RESIDUAL: "residual_l0", tph._lib.KERNEL_RESTRICT: "restrict_l0",
             tph._lib.KERNEL_PROLONG: "prolong_l0"}
    for kind, name in names.items():
        if args.kernel_reps <= 0:
            break
        ms, by = s_mix.time_kernel(kind, args.kernel_reps)
        kern[name] = {"us": round(ms * 1e3, 3), "bytes": by, "GBps": round(by / (ms * 1e-3) / 1e9, 1)}
    # the roofline figure comes from the launches inside the timed solves
    n_l, ms_l, by_l, drop_l = live
    # HBM traffic per launch from the committed counter runs, valid only for these exact kernel sources
    traffic = None
    tfile = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "smooth_l0_traffic.json")
    if os.path.exists(tfile):
        from paper_2603_14040_amd import profiling
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("sources_sha256") == profiling.sources_hash():
            traffic = tj["bytes_per_launch"]
    if n_l == 0:
        raise RuntimeError("no finest-level smoothing launch was timed")
    us_live = 1e3 * ms_l / n_l
    achieved = by_l / (ms_l * 1e-3) / 1e9

    # device-to-device copy bandwidth in the same run (context for the roofline)
    buf = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(buf)
    dst.copy_(buf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        dst.copy_(buf)
    torch.cuda.synchronize()
    copy_gbs = 2 * buf.numel() * 4 * 20 / (time.perf_counter() - t0) / 1e9
    del buf, dst

    # batched workload: independent sinkers of sizes {64, 128, 256, 512}, one batched solve
    batch = None
    if args.batch > 0:
        s64 = None
        probs = wl.batch_sinkers(args.batch, seed=4)
        log(f"[bench] batched workload: {len(probs)} problems, {sum(p.cells for p in probs)} cells")
        ebs = [to(p.eta_b) for p in probs]
        eps = [to(p.eta_p) for p in probs]
        rhs_ = [to(p.rho_b) for p in probs]
        gxy = [(p.gx, p.gy) for p in probs]
        shapes = [(p.nx, p.ny) for p in probs]
        btuned = {"params": {"restart": 16}, "ms": None, "default_ms": None, "trials": 0, "seconds": 0.0}
        if not args.no_tune:
            log("[bench] autotuning the batched schedule")
            btuned = autotune.tune_batch(shapes, ebs, eps, rhs_, gxy, precision=tph.MIXED, device=dev)
            log(f"[bench] batch: tuned {btuned['params']} {btuned['ms']:.1f} ms (defaults "
                f"{btuned['default_ms']:.1f} ms, {btuned['trials']} trials, {btuned['seconds']:.1f} s)")
        t0 = time.perf_counter()
        bat = tph.Batch(shapes, device=dev, precision=tph.MIXED, **btuned["params"])
        t_create = time.perf_counter() - t0
        outs = bat.zeros(), bat.zeros(), bat.zeros()

        def bstep():
            for o in outs:
                for t in o:
                    t.zero_()
            bat.set_coefficients(ebs, eps, rhs_, gxy)
            return bat.solve(*outs)[3]

        bstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binf = bstep()
        torch.cuda.synchronize()
        bdt = time.perf_counter() - t0
        bcells = sum(p.cells for p in probs)
        its = [i.iters for i in binf]
        batch = {"workload": f"{len(probs)} centred sinkers, sizes 64..512 (seed 4), contrast 10^U(1,4), mixed",
                 "cells": bcells, "value": bcells / bdt, "unit": "cells/s", "ms_per_step": 1e3 * bdt,
                 "iters_max": max(its), "iters_mean": sum(its) / len(its),
                 "converged": sum(1 for i in binf if i.res_energy <= 1e-8), "create_s": round(t_create, 2),
                 "tuned": btuned}
        log(f"[bench] batch: {1e3 * bdt:.1f} ms, {bcells / bdt:.3e} cells/s, iterations max {max(its)}")
        bat.close()
        del bat, outs, ebs, eps, rhs_

    # adjoint workload: gradient of the surface-velocity misfit on the 1024^2 field
    adjoint = None
    if not args.no_adjoint:
        base, m, m_true, cells_ = wl.adjoint_problem(n)
        eb_t, ep_t = wl.logvisc_to_eta(m_true, n, n)
        sa = tph.Solver(n, n, precision=tph.MIXED, device=dev, **tuned["mixed"]["params"])
        sa.set_coefficients(to(eb_t), to(ep_t), rho, pr.gx, pr.gy)
        vxt = sa.solve()[0]
        target = vxt[n, 1:n].clone()
        ebg = to(pr.eta_b).requires_grad_(True)
        epg = to(pr.eta_p).requires_grad_(True)

        def astep():
            vx_, vy_, p_ = tph.StokesFunction.apply(ebg, epg, rho, sa, pr.gx, pr.gy)
            J = 0.5 * (1.0 / n) * torch.sum((vx_[n, 1:n] - target) ** 2)
            J.backward()
            return J

        astep()
        ebg.grad = None
        epg.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        astep()
        torch.cuda.synchronize()
        adt = time.perf_counter() - t0
        adjoint = {"workload": f"misfit gradient w.r.t. viscosity, {n}x{n} random field, mixed, forward + adjoint "
                               f"solve + gradient kernel", "ms_per_step": 1e3 * adt,
                   "cells_per_s": 2 * cells / adt}
        log(f"[bench] adjoint gradient: {1e3 * adt:.1f} ms")
        sa.close()

    # large multi-inclusion workload: 200 sharp discs, viscosity 10^U(-3,3); one mixed solve with the tuned
    # schedule and a longer restart (the 1e6 contrast needs it), the finest-level sweep timed inside it
    large = None
    if args.large > 0:
        nl_ = args.large
        pl = wl.multi_inclusion(nl_)
        log(f"[bench] multi-inclusion workload {nl_}x{nl_}")
        ltuned = {"params": {"restart": 30}, "ms": None, "trials": 0, "seconds": 0.0}
        if not args.no_tune:
            # the schedule (not the per-level plan) tuned on the same recipe at 1024^2, untimed
            ps = wl.multi_inclusion(1024)
            ltuned = autotune.tune(to(ps.eta_b), to(ps.eta_p), to(ps.rho_b), ps.gx, ps.gy, precision=tph.MIXED,
                                   reps=1, rounds=1, device=dev, knobs=autotune.schedule_knobs())
            log(f"[bench] large: schedule tuned at 1024^2 {ltuned['params']} ({ltuned['trials']} trials, "
                f"{ltuned['seconds']:.1f} s)")
        kw = dict(ltuned["params"])
        for key in ("msweep", "tile_shape", "coarse_level"):
            kw.pop(key, None)                        # the per-level plan belongs to the tuning grid
        sl = tph.Solver(nl_, nl_, precision=tph.MIXED, device=dev, max_iters=2000, **kw)
        sl.set_coefficients(to(pl.eta_b), to(pl.eta_p), to(pl.rho_b), pl.gx, pl.gy)
        sl.kernel_timing(17)
        sl.kernel_timing_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        linf = sl.solve()[3]
        torch.cuda.synchronize()
        ldt = time.perf_counter() - t0
        nk, msk, byk, _ = sl.kernel_timing_read()
        large = {"workload": f"{nl_}x{nl_} cells, 200 discs (seed 3) radius U(0.005,0.03), eta 10^U(-3,3), rho "
                             f"U(-1,1), mixed, schedule tuned on the 1024^2 instance", "cells": nl_ * nl_,
                 "tuned": ltuned,
                 "value": nl_ * nl_ / ldt, "unit": "cells/s", "ms": 1e3 * ldt, "iters": linf.iters,
                 "res_energy": linf.res_energy, "status": linf.status,
                 "smooth_l0": {"launches": nk, "us_per_launch": 1e3 * msk / max(nk, 1),
                               "GBps": byk / max(msk * 1e-3, 1e-30) / 1e9,
                               "frac": byk / max(msk * 1e-3, 1e-30) / 1e9 / HBM_PEAK_GBS}}
        log(f"[bench] large: {1e3 * ldt:.0f} ms, {linf.iters} iterations, res {linf.res_energy:.1e}, finest sweep "
            f"{large['smooth_l0']['GBps']:.0f} GB/s")
        # the same solve as a viscosity-rescaling continuation from the lithostatic pressure
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cinf = sl.solve_continuation(to(pl.eta_b), to(pl.eta_p), to(pl.rho_b), pl.gx, pl.gy,
                                     thetas=(0.0, 0.25, 0.5, 0.75, 1.0), stage_rtol=1e-3, lithostatic=True)[3]
        torch.cuda.synchronize()
        cdt = time.perf_counter() - t0
        large["continuation"] = {"thetas": [0.0, 0.25, 0.5, 0.75, 1.0], "stage_rtol": 1e-3, "lithostatic": True,
                                 "ms": 1e3 * cdt, "iters": cinf.iters, "res_energy": cinf.res_energy,
                                 "status": cinf.status, "value": nl_ * nl_ / cdt}
        log(f"[bench] large, continuation: {1e3 * cdt:.0f} ms, {cinf.iters} iterations, res {cinf.res_energy:.1e}")
        sl.close()
        del sl

    # robustness runs after the paper's sinker test (Ch. "Robustness" set-up): a centred inclusion of radius
    # 0.2 with viscosity contrast 1e8 and density 33 in a host of density 32 (the 3300 / 3200 kg/m^3 of the
    # test, scaled), free-slip walls (zero normal velocity on every wall), g = (0, -1), 512 x 608 cells on
    # the unit square (the test's 501 x 601 nodes; factor-2 coarsening over 5 levels gives the coarsest
    # 32 x 38 grid that 4 levels coarsened by 2.5 give there); unaccelerated Uzawa iterations (Anderson depth
    # 0, beta 1), one V-cycle each, 5 + 5 sweeps growing by 2.5 per level, omega_v = 0.3, alpha = 0.6,
    # continuation theta = 0, 0.25, ..., 1 switched every 25 iterations from the lithostatic pressure, then
    # theta = 1 up to --robust-iters iterations or until the residual stops falling; the four smoother
    # configurations of the test, FP64
    robust = None
    if args.robust_iters > 125:
        ps_ = wl.sinker(512, ny=608, radius=0.2, eta_in=1e8, rho_in=33.0, eta_out=1.0, rho_out=32.0)
        ebs_, eps_, rhos_ = to(ps_.eta_b), to(ps_.eta_p), to(ps_.rho_b)
        robust = {"workload": ("sinker 512x608 cells, contrast 1e8, densities 33 / 32, free slip, unaccelerated "
                               "Uzawa (one V-cycle per iteration, 5 levels, 5+5 sweeps x2.5 per level, omega 0.3, "
                               "alpha 0.6), continuation theta 0..1 in steps of 0.25 every 25 iterations from the "
                               "lithostatic pressure, FP64"), "smoothers": {}}
        for name_, sm_ in (("rbgs", tph.SMOOTH_GS), ("jacobi", tph.SMOOTH_JACOBI), ("ras", tph.SMOOTH_RAS),
                           ("mixed", tph.SMOOTH_RAS_MIXED)):
            kw_ = dict(precision=tph.FP64, levels=5, smoother=sm_, nu_pre=5, nu_post=5, nu_growth=2.5, omega=0.3,
                       alpha=0.6, accel="anderson", restart=0, beta=1.0, uzawa_steps=1, rtol=1e-14, ras_tile=32,
                       ras_inner=4)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1_ = tph.Solver(512, 608, device=dev, max_iters=25, **kw_)
            vxs, vys, pps, i1_ = s1_.solve_continuation(ebs_, eps_, rhos_, ps_.gx, ps_.gy,
                                                        thetas=(0.0, 0.25, 0.5, 0.75, 1.0), stage_rtol=1e-14,
                                                        lithostatic=True, history=125)
            s2_ = tph.Solver(512, 608, device=dev, max_iters=args.robust_iters - i1_.iters, **kw_)
            s2_.set_coefficients(ebs_, eps_, rhos_, ps_.gx, ps_.gy)
            vxs, vys, pps, i2_ = s2_.solve(vxs, vys, pps, history=args.robust_iters)
            torch.cuda.synchronize()
            rdt = time.perf_counter() - t0
            h_ = list(i1_.history) + list(i2_.history)
            first = {f"{t:.0e}": next((k + 1 for k, v in enumerate(h_) if k >= 100 and v <= t), None)
                     for t in (1e-6, 1e-8, 1e-10)}
            robust["smoothers"][name_] = {
                "iters": i1_.iters + i2_.iters, "seconds": round(rdt, 3), "res_final": i2_.res_energy,
                "res_at": {str(k): h_[k - 1] for k in (1, 25, 50, 75, 100, 125, 150, 200, 250) if k <= len(h_)},
                "first_iter_below": first}
            log(f"[bench] robustness {name_}: {i1_.iters + i2_.iters} iterations in {rdt:.2f} s, final residual "
                f"{i2_.res_energy:.2e}, first below 1e-8 at {first['1e-08']}")
            s1_.close()
            s2_.close()
        del ebs_, eps_, rhos_

    # marker-in-cell step (Sec. "The Marker-in-Cell Method"): markers carry viscosity and density; one step =
    # marker -> grid (eta_b, rho_b on basic nodes, eta_p on cells), the Stokes solve with the tuned schedule
    # (mixed), grid -> marker RK4 advection with dt = half a cell at the largest speed
    mic = None
    if args.mic_steps > 0:
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
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            mvx.zero_(); mvy.zero_(); mp.zero_()
            sm_.set_coefficients(eb_, ep_, rb_, pr.gx, pr.gy)
            inf_ = sm_.solve(mvx, mvy, mp)[3]
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            vmax = max(mvx.abs().max().item(), mvy.abs().max().item())
            mk_.advect_rk4(X_, Y_, mvx, mvy, 0.5 / n / max(vmax, 1e-300))
            torch.cuda.synchronize()
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
        if any(i.status != "TPH_OK" for i in minf):
            raise RuntimeError(f"marker-in-cell solve did not converge: {minf[-1]}")
        # the RK4 kernel alone: positions read and written once (32 B per marker), grids through the caches
        Xa, Ya = X_.clone(), Y_.clone()
        mk_.advect_rk4(Xa, Ya, mvx, mvy, 1e-9)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            mk_.advect_rk4(Xa, Ya, mvx, mvy, 1e-9)
        torch.cuda.synchronize()
        rk_ms = 1e3 * (time.perf_counter() - t0) / 20
        rk_gbs = 32.0 * nm / (rk_ms * 1e-3) / 1e9
        per = {k: 1e3 * v / args.mic_steps for k, v in stages.items()}
        mic = {"workload": f"{nm} markers ({args.markers_per_cell} per cell, seed 13) on the {n}x{n} random-viscosity "
                           f"grid, eta and rho per marker; step = marker -> grid (3 fields, 2 binnings) + mixed "
                           f"solve + RK4", "markers": nm, "ms_per_step": 1e3 * mdt,
               "stages_ms": per, "iters": minf[-1].iters, "res_energy": minf[-1].res_energy,
               "markers_to_grid_per_s": 3 * nm / (per["to_grid"] * 1e-3),
               "rk4": {"ms": rk_ms, "markers_per_s": nm / (rk_ms * 1e-3), "GBps": round(rk_gbs, 1),
                       "frac": round(rk_gbs / HBM_PEAK_GBS, 4),
                       "what": "positions 2 x 8 B read + written per marker; 64 grid reads per marker from cache"}}
        log(f"[bench] marker-in-cell: {1e3 * mdt:.1f} ms/step (to_grid {per['to_grid']:.1f}, solve "
            f"{per['solve']:.1f}, advect {per['advect']:.2f} ms), RK4 kernel {rk_ms:.2f} ms = {rk_gbs:.0f} GB/s")
        mk_.close()
        sm_.close()
        del mk_, sm_, X_, Y_, E_, R_

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import stokes as ost
        m = args.cpu_n
        log(f"[bench] CPU oracle on the {m}x{m} sample")
        sp_ = wl.random_viscosity(m)
        g = ost.Grid(m, m)
        t0 = time.perf_counter()
        sol = ost.solve(g, sp_.eta_b, sp_.eta_p, sp_.rho_b, sp_.gx, sp_.gy)
        dt = time.perf_counter() - t0
        cpu = {"value": m * m / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
               "sample": f"random-viscosity recipe at {m}x{m} cells (same correlation length 0.05 and "
                         f"contrast 1e4), one FP64 assembled-matrix SuperLU solve ({dt:.1f} s, energy "
                         f"residual {sol.residual_energy:.1e}); SuperLU is single-threaded",
               "seconds": round(dt, 2)}

    out = {
        "metric": METRIC,
        "value": cells / (ms_mix * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mix,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle + f64 Krylov/residual (mixed)",
        "data": "synthetic",
        "config": {"workload": f"random-viscosity {n}x{n} cells, log10 eta Gaussian random field "
                               f"(corr. length 0.05, contrast 1e4), free slip, "
                               f"{['FGMRES', 'GCR', 'Anderson'][s_mix.desc.accel]}({s_mix.desc.restart}) + "
                               f"{s_mix.levels}-level V-cycle, relative energy residual 1e-8",
                   "cells": cells, "levels": s_mix.levels, "precision": "mixed", "global_batch": 1},
        "iters": inf_mix[-1].iters,
        "res_energy": inf_mix[-1].res_energy,
        "setup_ms": inf_mix[-1].t_setup_ms,
        "solve_ms": inf_mix[-1].t_solve_ms,
        "fp64": ({"value": cells / (ms_64 * 1e-3), "ms_per_step": ms_64, "iters": inf_64[-1].iters,
                  "res_energy": inf_64[-1].res_energy} if fp64_steps > 0 else None),
        "mixed_speedup_vs_fp64": ms_64 / ms_mix if fp64_steps > 0 else None,
        "accelerators": accels or None,
        "ras": ras_out,
        "marker_in_cell": mic,
        "robustness": robust,
        "tuned": tuned,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": ("finest-level Gauss-Seidel on LDS tiles (FP32, " +
                                ("multi-sweep passes with fused residual-restriction / prolongation"
                                 if plan0[0] == "multisweep" else "one sweep per launch") +
                                f", tile shape {plan0[1]}), kernel time stamps (HIP events) of every 17th launch on "
                                "the solver stream inside the timed solves"),
                     "launches": n_l, "dropped": drop_l, "us_per_launch": round(us_live, 3),
                     "algorithmic_bytes_per_launch": by_l / n_l},
        "kernels": kern,
        "copy_GBps": round(copy_gbs, 1),
        "batched": batch,
        "adjoint": adjoint,
        "large": large,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
