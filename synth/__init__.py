"""Seeded synthetic inputs: icosahedral grids, vertical reference columns, initial states.

This package is shared by the oracle and the GPU path and holds none of the
time step's arithmetic.
"""
from .grid import make_grid, expected_counts, EARTH_RADIUS
from .state import add_cold_pools, initial_state, vertical, reference
from .workloads import WORKLOADS, build_workload, ensemble_member
