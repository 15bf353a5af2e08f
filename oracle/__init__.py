"""Plain FP64 CPU oracle of the ICON-style non-hydrostatic dynamical-core step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library: the only common dependency is the seeded-input package ``synth``.

What it computes follows the paper's description of the time step
(Section 4.1 and Fig. 1 caption: nested time step, predictor-corrector
substeps starting with the advective tendencies, horizontal momentum update,
divergence damping only in the corrector, vertically implicit solver, and a
diffusion granule called once per time step; Section 5.1 "Experimental setup"
for the nh_solve / nh_diff split and the icosahedral grid).  The paper prints
no equations; every numerical detail is a written-out reading, stated in
the docstring of the function that implements it.

Modules:
  constants  -- physical constants and scheme parameters
  grid       -- canonical/derived connectivity, orientation, SFC renumbering
  operators  -- C-grid operators on the triangular grid
  dycore     -- velocity advection, predictor, corrector, column solver,
                diffusion, step, conservation diagnostics
  mlp        -- FP64 reference of the surrogate MLP (forward, backward, Adam)

Parity status: grid tables, operators, column solver and step invariants are
pinned by tests against closed forms, brute force and invariants.  Agreement
with ICON itself is "parity unpinned" (no ICON code or data is available).
"""
