"""Seeded synthetic workloads for the rain-augmented shallow water DG solver.

This package only *describes* inputs: node coordinates, triangles, boundary
edge lists with their types, nodal bathymetry and friction, initial nodal
states and forcing descriptions (rain tracks, rain lattices, tides, river
series).  It holds none of the solver's arithmetic, so both the FP64 oracle
and the GPU library can consume it without sharing any method code.

Conventions (the same on every consumer):
  * coordinates in metres (Cartesian), bathymetry ``hb`` positive downward
    (problem statement, Sec. 2.1, Eq. SWE), free surface ``zeta`` positive
    upward, discharges ``qx = H u``, ``qy = H v`` in m^2/s;
  * boundary edge types: LAND (zero normal flow), OCEAN (specified
    elevation), RIVER (specified normal flux), OUTFLOW (transmissive) --
    the boundary partition of Sec. 2.1 plus a free outflow;
  * rain rates in m/s.
"""
from .generators import (  # noqa: F401
    LAND, OCEAN, RIVER, OUTFLOW,
    Mesh, Scenario,
    rect_grid, channel_c1, bathtub, basin, basin_window, small_mixed, lake_at_rest,
    parametric_track, gridded_field, seed_for, dam_break, inclined_plane,
    log_uniform_sizes, basin_member, ensemble_plan, request_trace, serving_pool_sizes,
)
from .graded import graded_coast, graded_small  # noqa: F401,E402
