"""The allocation-free ensemble step (dc_ensemble_step_noalloc): its work
tables live in the library's static device array instead of memory
allocated per call.  Two calls in a row, the second with a smaller
ensemble (smaller tables), each against dc_ensemble_step_eager on identical
members, bit for bit; a step whose tables exceed the array is refused
without touching the members."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from synth import initial_state, make_grid  # noqa: E402

FIELDS = ("vn", "w", "rho", "exner", "theta_v")
K = 7
DT, NSUB = 600.0, 3


def _members(spec, precision):
    out = []
    for (n, k), seed in spec:
        g = make_grid(n, k)
        S, vert = initial_state(g, K, 20e3, seed=seed, vn_sigma=1.0, t_sigma=0.2, jet_u0=30.0)
        G = D.Grid(g, vert)
        st = D.State(G, precision=precision)
        st.write(S)
        out.append((G, st))
    return out


def _close(items):
    for G, st in items:
        st.close()
        G.close()


def _compare(spec, precision, steps):
    a = _members(spec, precision)
    b = _members(spec, precision)
    Ea = D.Ensemble([st for _, st in a])
    Eb = D.Ensemble([st for _, st in b])
    for _ in range(steps):
        Ea.step_noalloc(DT, NSUB)
        Eb.step(DT, NSUB, eager=True)
    for (_, x), (_, y) in zip(a, b):
        rx, ry = x.read(), y.read()
        for f in FIELDS:
            assert np.array_equal(rx[f], ry[f]), (precision, f)
        assert x.current() == y.current()
    Ea.close()
    Eb.close()
    _close(a)
    _close(b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_step_equals_eager_step(precision):
    # first call: four uneven members; second call: two small ones, whose
    # tables are smaller than what the array holds from the first call
    _compare([((2, 0), 11), ((2, 2), 12), ((2, 1), 13), ((1, 0), 14)], precision, 2)
    _compare([((1, 0), 21), ((2, 0), 22)], precision, 1)


def test_noalloc_step_refuses_oversized_tables():
    items = _members([((2, 1), 31), ((2, 0), 32), ((1, 0), 33)], "fp64")
    E = D.Ensemble([st for _, st in items])
    before = [st.read() for _, st in items]
    cur = [st.current() for _, st in items]
    with pytest.raises(D.DycoreError) as ei:
        E.step_noalloc(DT, 1000)  # 6005 phases of three members: far beyond the array
    assert ei.value.code == D.DC_EINVAL
    torch.cuda.synchronize()
    for (_, st), S0, c in zip(items, before, cur):
        assert st.current() == c
        S1 = st.read()
        for f in FIELDS:
            assert np.array_equal(S0[f], S1[f]), f
    E.step_noalloc(DT, NSUB)  # a step that fits still runs
    E.close()
    _close(items)
