"""FP64 CPU oracle for the rain-augmented shallow water DG scheme.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised NumPy implementation of what the GPU library computes.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does, and it shares no code, headers,
tables or constants with the HIP library.

What it follows (Wichitrnithed et al., "A Discontinuous Galerkin Finite
Element Model for Compound Flood Simulations"):
  * Sec. 2.1, Eq. SWE and Eq. river_bc: the rain-augmented shallow water
    equations and the ocean / land / river boundary partition;
  * Sec. 2.2, Eq. elem_weak_form, Eq. dubiner, Eq. RKSSP: element weak form,
    orthogonal Dubiner modal basis with diagonal mass, SSP Runge-Kutta;
  * Sec. 2.3: edge integrals first, then area integrals; Roe or LLF flux;
    optional slope limiter; Eq. rain (nodal rain averaged per element, added
    in every element, wet or dry);
  * Sec. 2.4: the positive-depth operator split into a depth part and a
    discharge part, applied after every Runge-Kutta stage, and wet/dry
    element flags;
  * Sec. 2.5: parametric (storm-centred radial) and gridded rain;
  * Sec. 2.1 (the momentum sources F_x, F_y) with Sec. 2.3 and Sec. 3.3
    (parametric hurricane wind and pressure): :mod:`oracle.met`, a symmetric
    parametric vortex standing in for GAHM, whose expressions are not given;
  * Sec. 3: Manning friction, p = 1, Roe flux and two-stage second-order
    SSPRK as the common set-up; LLF for the large mesh; quadratic friction
    0.001 for the bathtub.

Where the paper is silent or garbled, the readings adopted are listed at the
top of :mod:`oracle.solver` and in the design notes of the repository.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force on tiny meshes, an independent
first-order finite-volume code and the numbers the paper prints for the
bathtub experiment (Sec. 3.1).  Equality with the authors' own DG-SWEM code
is *parity unpinned*: that code and its data are not available.
"""
from . import basis, mesh, physics, forcing, wetdry, limiter  # noqa: F401
from .solver import OracleSolver, ssp_rk2_step  # noqa: F401
