"""Batched ensemble on the persistent path: every phase runs on a grid of a
fixed number of blocks per compute unit, so each block walks many
(member, tile) work items in turn (the path a tuned schedule of uneven
R2B4/R2B5 members takes).  Each member must stay bit-identical to stepping
it alone, after several steps and on every graph replay."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from synth import ensemble_member, initial_state, make_grid  # noqa: E402

FIELDS = ("vn", "w", "rho", "exner", "theta_v")
# two R2B4 and two R2B5 members of the uneven ensemble, 65 levels
MEMBERS = (0, 1, 12, 13)


def _states(precision, grids):
    out = []
    for m in MEMBERS:
        sp = ensemble_member(m)
        g, G = grids[sp["k"]]
        S, _ = initial_state(g, sp["n_lev"], sp["z_top"], **sp["state"])
        st = D.State(G, precision=precision)
        st.write(S)
        out.append(st)
    return out


@pytest.fixture(scope="module")
def grids():
    out = {}
    for k in (4, 5):
        g = make_grid(2, k)
        _, vert = initial_state(g, 65, 75.0e3, seed=0)
        out[k] = (g, D.Grid(g, vert))
    yield out
    for _, G in out.values():
        G.close()


@pytest.mark.parametrize("precision,gfac", [("mixed", 1), ("mixed", 8), ("fp64", 1)])
def test_persistent_walk_bitwise_equal_solo(precision, gfac, grids, tmp_path):
    sp = ensemble_member(0)
    dt, nsub = sp["dt"], sp["nsub"]
    ens = _states(precision, grids)
    solo = _states(precision, grids)
    E = D.Ensemble(ens)
    # a cached schedule: default-like tiles, gfac blocks per compute unit in
    # every phase (persistent grids), loaded without timing
    cells = sorted(grids[ensemble_member(m)["k"]][0]["n_cells"] for m in MEMBERS)
    key = f"prec={0 if precision == 'fp64' else 1};K=65;diff=0;cells=" + ",".join(str(c) for c in cells)
    sched = "256x11 64x33 256x22 256x6 128x13 | " + " ".join([str(gfac)] * len(D.KERNELS))
    cache = tmp_path / "sched.txt"
    cache.write_text(f"{key}\t{sched}\n")
    E.autotune(dt, nsub, str(cache))
    assert E.schedule().split("|")[1].split() == [str(gfac)] * len(D.KERNELS)
    # the persistent grids are much smaller than the work tables: every block
    # walks several column tiles (64 columns each) and stencil tiles
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    col_tiles = sum((c + 63) // 64 for c in cells)
    assert col_tiles >= 4 * gfac * n_cu or gfac == 8 and col_tiles > gfac * n_cu
    for rep in range(3):
        E.step(dt, nsub)
        for st in solo:
            st.step(dt, nsub)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ens, solo)):
            ra, rb = a.read(), b.read()
            for f in FIELDS:
                assert np.array_equal(ra[f], rb[f]), (precision, gfac, rep, MEMBERS[i], f)
    E.close()
    for st in ens + solo:
        st.close()
