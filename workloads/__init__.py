"""Seeded synthetic workloads: level geometry and initial data.

This package is shared input generation only.  It describes *which* problem
is solved (the refinement geometry of each configuration and the initial
fields on it) and holds none of the method's arithmetic: no stencils, no
Runge-Kutta, no dense output, no prolongation, no block splitting.  Both the
CPU reference implementation and the GPU library receive what it produces.
"""
from .geometry import (HierarchySpec, single_level, two_level_cube, tower_family, config_z4c_small,
                       config_c1, config_c2, config_c3, config_c5, config_e1, ensemble_c1,
                       grown_for_buffer_zones)
from .data import (SplitMix64Stream, canonical_coords, standing_wave, periodic_gaussian,
                   pulse_params, pulses_on_spec, standing_wave_on_spec,
                   gaussian_on_spec, ensemble_params, ensemble_on_spec, brill_lindquist,
                   brill_lindquist_on_spec, spherical_gaussian, spherical_gaussian_on_spec,
                   E1_AMPLITUDE, E1_SIGMA)

__all__ = [n for n in dir() if not n.startswith("_")]
