"""FP64 CPU oracle of the variable-viscosity Stokes solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the GPU path; the only module both sides read is ``workloads`` (seeded input
generators holding none of the method's arithmetic).

Contents
--------
``stokes``    assembled sparse saddle-point operator (stress-conservative
              staggered finite differences), right-hand side from density and
              gravity, bordered direct solve, energy residual.
``multigrid`` plain references of the multigrid pieces: normalised bilinear
              restriction computed from node coordinates, bilinear
              prolongation, coarse-grid viscosities, damped Jacobi and
              coloured Gauss-Seidel sweeps, the V-cycle and the Uzawa
              preconditioner.
``adjoint``   surface-velocity misfit, adjoint solve and the gradient with
              respect to the viscosity and density fields obtained by
              differentiating the assembled operator term by term.
``continuation`` viscosity-rescaling blend and lithostatic pressure.
``accelerators`` flexible GCR(m) and Anderson acceleration AA(m, beta)
              around the Uzawa fixed-point map.
``ras``       RAS-type temporal-blocking Jacobi smoother and its SplitMix64
              tile shifts.
``markers``   marker <-> grid bilinear interpolation and RK4 marker advection.
"""
from . import stokes, multigrid, adjoint, continuation, accelerators, ras, markers  # noqa: F401
