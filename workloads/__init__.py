"""Seeded synthetic inputs (density fields, grids, workload mixes) shared by the
HIP path's tests, the CPU oracle's tests and the benchmark.  Holds no part of
the multipole method itself."""
from . import mixes  # noqa: F401
from .fields import (  # noqa: F401
    FLOOR, Field, Star, Polytropes, UniformSphere, binary_polytrope, binary_polytrope_128,
    single_polytrope, cell_centres, uniform_grid, noisy_sphere_16, leaf_density,
    uniform_leaves, grid_to_leaves, leaves_to_grid, lane_emden_table, lane_emden_theta, OrbitalRate, noisy_rate, scf_initial_binary,
)
