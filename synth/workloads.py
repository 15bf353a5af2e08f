"""Named synthetic workloads (grid, levels, time step, initial-state recipe).

Each entry stands in for the production NWP runs of the paper (R2B08-R2B10,
120 levels): same structure of grid and column, synthetic seeded fields.
"""
from __future__ import annotations

from .grid import make_grid
from .state import initial_state

WORKLOADS = {
    # Plain FP64 parity case: isothermal rest state plus vn noise (sigma 1 m/s).
    "r2b2_k30": dict(n=2, k=2, n_lev=30, z_top=30.0e3, dt=600.0, nsub=5, steps=10,
                     state=dict(seed=0, vn_sigma=1.0)),
    # Same grid, no noise: the resting isothermal atmosphere.
    "r2b2_k30_rest": dict(n=2, k=2, n_lev=30, z_top=30.0e3, dt=600.0, nsub=5, steps=10,
                          state=dict(seed=0)),
    # FP64 vs mixed: balanced zonal jet plus 20 temperature bumps.
    "r2b5_k65": dict(n=2, k=5, n_lev=65, z_top=75.0e3, dt=180.0, nsub=5, steps=100,
                     state=dict(seed=1, jet_u0=35.0, n_bumps=20)),
    # One GPU's production-scale share, space-filling-curve ordered.
    "r2b8_k90": dict(n=2, k=8, n_lev=90, z_top=75.0e3, dt=30.0, nsub=5, steps=20, sfc=1,
                     state=dict(seed=2, jet_u0=35.0, n_bumps=20)),
    # Surrogate training / evaluation grid.
    "r2b6_k65": dict(n=2, k=6, n_lev=65, z_top=75.0e3, dt=90.0, nsub=5, steps=200,
                     state=dict(seed=3, jet_u0=35.0, n_bumps=20)),
    # Longer stability run of the jet on a mid-size grid.
    "r2b4_k65": dict(n=2, k=4, n_lev=65, z_top=75.0e3, dt=180.0, nsub=5, steps=200,
                     state=dict(seed=1, jet_u0=35.0, n_bumps=20)),
    # Tiny grids for brute-force and ragged-tail cases.
    "r1b0_k4": dict(n=1, k=0, n_lev=4, z_top=10.0e3, dt=600.0, nsub=2, steps=2,
                    state=dict(seed=7, vn_sigma=1.0, n_bumps=3, bump_radius=3000.0e3)),
    "r2b0_k1": dict(n=2, k=0, n_lev=1, z_top=5.0e3, dt=600.0, nsub=2, steps=2,
                    state=dict(seed=8, vn_sigma=1.0)),
    "r2b1_k7": dict(n=2, k=1, n_lev=7, z_top=20.0e3, dt=600.0, nsub=3, steps=3,
                    state=dict(seed=9, vn_sigma=2.0, jet_u0=35.0, n_bumps=4, bump_radius=2000.0e3)),
}


def ensemble_member(m: int):
    """Member m (0..23) of the uneven ensemble: 12 x R2B4 then 12 x R2B5, 65 levels."""
    k = 4 if m < 12 else 5
    return dict(n=2, k=k, n_lev=65, z_top=75.0e3, dt=180.0, nsub=5, steps=20,
                state=dict(seed=1000 + m, jet_u0=35.0, vn_sigma=0.5, t_sigma=0.2))


def build_workload(spec, grid=None):
    """Return (grid, state, vert, spec) for a workload name or spec dict."""
    if isinstance(spec, str):
        spec = WORKLOADS[spec]
    if grid is None:
        grid = make_grid(spec["n"], spec["k"])
    state, vert = initial_state(grid, spec["n_lev"], spec["z_top"], **spec["state"])
    return grid, state, vert, spec
