"""Perturbed-ensemble verification in the manner of probtest (the paper's
Section 4.4): tolerances come from the spread that tiny perturbations of the
initial state grow to, not from a fixed threshold.

The R2B2 / 30-level workload (10 steps of 600 s, 5 substeps).  Seven members
perturb theta_v by a relative amount eps (seeded, uniform in [-eps, eps]); the
members run together through the ensemble runner (one graph launch per
step).  The tolerance of a field is FACTOR times the largest relative L2
distance of a member from the unperturbed run.

- eps = 1e-14 (rounding level): the GPU FP64 step against the FP64 oracle
  must lie within the tolerance: the two differ by no more than rounding
  noise grows to in 10 steps.
- eps = 1e-8: the mixed-precision step against the GPU FP64 step must lie
  within the tolerance: FP32 horizontal arithmetic perturbs the solution no
  more than a relative 1e-8 perturbation of theta_v does.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from oracle import dycore as O  # noqa: E402
from oracle.constants import default_params  # noqa: E402
from oracle.grid import Grid as OGrid  # noqa: E402
from synth import build_workload  # noqa: E402

FIELDS = ("vn", "w", "rho", "exner", "theta_v")
FACTOR = 5.0
MEMBERS = 7


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def r2b2_case():
    g0, S, vert, spec = build_workload("r2b2_k30")
    G = D.Grid(g0, vert)
    yield g0, S, vert, spec, G
    G.close()


def run(G, states, spec, precision="fp64"):
    sts = []
    for s in states:
        st = D.State(G, precision=precision)
        st.write(s)
        sts.append(st)
    E = D.Ensemble(sts)
    for _ in range(spec["steps"]):
        E.step(spec["dt"], spec["nsub"])
    out = [st.read() for st in sts]
    E.close()
    for st in sts:
        st.close()
    return out


def tolerances(G, S, spec, eps):
    members = [S]
    for m in range(1, MEMBERS + 1):
        rng = np.random.default_rng(100 + m)
        Sm = dict(S)
        Sm["theta_v"] = S["theta_v"] * (1.0 + eps * rng.uniform(-1.0, 1.0, S["theta_v"].shape))
        members.append(Sm)
    out = run(G, members, spec)
    spread = {f: max(rel(o[f], out[0][f]) for o in out[1:]) for f in FIELDS}
    return out[0], {f: FACTOR * v for f, v in spread.items()}


def test_gpu_fp64_within_rounding_ensemble_spread_of_oracle(r2b2_case):
    g0, S, vert, spec, G = r2b2_case
    gpu, tol = tolerances(G, S, spec, 1e-14)
    og = OGrid(g0, vert)
    wts = O.vertex_lsq_weights(og)
    ref = S
    for _ in range(spec["steps"]):
        ref = O.step(og, ref, spec["dt"], spec["nsub"], default_params(), diffuse=True, wts=wts)
    err = {f: rel(gpu[f], ref[f]) for f in FIELDS}
    print("tolerance (eps 1e-14):", tol)
    print("GPU FP64 vs oracle:   ", err)
    for f in FIELDS:
        assert err[f] <= tol[f], (f, err[f], tol[f])


def test_mixed_within_1e8_ensemble_spread_of_fp64(r2b2_case):
    g0, S, vert, spec, G = r2b2_case
    fp64, tol = tolerances(G, S, spec, 1e-8)
    mixed = run(G, [S], spec, precision="mixed")[0]
    err = {f: rel(mixed[f], fp64[f]) for f in FIELDS}
    print("tolerance (eps 1e-8):", tol)
    print("mixed vs FP64:       ", err)
    for f in FIELDS:
        assert err[f] <= tol[f], (f, err[f], tol[f])
