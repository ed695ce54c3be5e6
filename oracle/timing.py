"""Wall time of one oracle solve (test infrastructure: the CPU baseline).

    python -m oracle.timing N [N ...]

For each N, builds the random-viscosity problem on N x N cells (the seeded
recipe of ``workloads.random_viscosity``), assembles the FP64 operator and
solves it with the oracle's direct sparse solve (``stokes.solve``: SuperLU,
one refinement step), and prints one JSON line per size: cells, seconds
(assembly + solve), cells per second, the oracle's energy residual and the
process's peak resident memory so far.  Run it as a child process with one
BLAS/OpenMP thread (the caller sets the environment) so that the peak memory
and the thread count are its own; SuperLU itself is single-threaded.

Only bench.py's cpu_baseline leg runs this module; nothing in the product
path imports it.
"""
from __future__ import annotations

import json
import os
import resource
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import workloads as wl  # noqa: E402

from oracle import stokes as ost  # noqa: E402


def main(argv=None) -> int:
    sizes = [int(a) for a in (argv if argv is not None else sys.argv[1:])]
    for m in sizes:
        pr = wl.random_viscosity(m)
        g = ost.Grid(m, m)
        t0 = time.perf_counter()
        sol = ost.solve(g, pr.eta_b, pr.eta_p, pr.rho_b, pr.gx, pr.gy)
        dt = time.perf_counter() - t0
        peak_mb = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1024.0
        print(json.dumps({"n": m, "cells": m * m, "seconds": round(dt, 3), "cells_per_s": m * m / dt,
                          "res_energy": sol.residual_energy, "peak_rss_mb": round(peak_mb, 1)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
