"""GPU tests of the learned diffusion surrogate, through the C ABI.

- Network: the BF16-MFMA forward pass and gradients against the FP64 oracle
  evaluated on the same BF16-rounded weights and inputs (relative L2 <= 2e-2:
  the kernels also round the hidden activations and the backward products'
  operands to BF16, 8 significant bits).
- Sampler: features and targets of the collected pairs against the oracle's
  features and plain diffusion at the reported (edge, level) points.
- Step: threshold 0 flags every column, so every column runs the plain
  diffusion and the run must equal the plain run bit for bit; a column with
  a feature outside the normalisation range falls back on its own.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from oracle import dycore as O  # noqa: E402
from oracle import mlp as M  # noqa: E402
from oracle.constants import default_params  # noqa: E402
from oracle.grid import Grid as OGrid  # noqa: E402
from synth import initial_state, make_grid  # noqa: E402

FIELDS = ("vn", "w", "rho", "exner", "theta_v")
K = 7
DT, NSUB = 600.0, 3


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def small_state(seed=11, n=2, k=1, **kw):
    g0 = make_grid(n, k)
    args = dict(vn_sigma=1.0, t_sigma=0.2, jet_u0=30.0)
    args.update(kw)
    S, vert = initial_state(g0, K, 20e3, seed=seed, **args)
    return g0, S, vert


def test_forward_matches_oracle_on_bf16_data():
    rng = np.random.default_rng(3)
    p = M.init_params(5)
    p["b1"] = rng.normal(scale=0.1, size=64)
    p["b2"] = rng.normal(scale=0.1, size=64)
    p["b3"] = np.array([0.05])
    n = 300  # ragged: not a multiple of the 128-row block
    x = rng.normal(size=(n, 18)) * 3.0 + 1.0
    mean = rng.normal(size=18).astype(np.float32)
    std = rng.uniform(1.0, 4.0, size=18).astype(np.float32)
    tstd = np.float32(2.5)
    net = D.Mlp(0)
    net.set_params(D.mlp_pack(p))
    net.set_norm(mean, std, np.full(18, -np.inf, np.float32), np.full(18, np.inf, np.float32), tstd)
    y = net.forward(x)
    pb = {k: bf16(v) if k in ("w1", "w2") else np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    xs = bf16((x.astype(np.float32) - mean) * (np.float32(1.0) / std))
    want, _ = M.forward(pb, xs)
    want = want * float(tstd)
    err = rel_l2(y, want)
    print("forward rel L2", err)
    assert err <= 2e-2
    net.close()


def test_gradients_match_oracle_on_bf16_data():
    rng = np.random.default_rng(4)
    p = M.init_params(6)
    p["b1"] = rng.normal(scale=0.1, size=64)
    p["b2"] = rng.normal(scale=0.1, size=64)
    n = 256
    x = rng.normal(size=(n, 18))
    t = rng.normal(size=n)
    net = D.Mlp(0)
    net.set_params(D.mlp_pack(p))
    g, loss = net.grad(x, t)
    pb = {k: bf16(v) if k in ("w1", "w2") else np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    want_loss, want = M.loss_and_grads(pb, bf16(x), np.asarray(t, np.float32).astype(np.float64))
    got = D.mlp_unpack(g)
    errs = {k: rel_l2(got[k], want[k]) for k in want}
    print("grad rel L2", errs, "loss", loss, want_loss)
    assert abs(loss - want_loss) <= 1e-2 * want_loss
    for k, e in errs.items():
        assert e <= 2e-2, (k, e)
    net.close()


@pytest.mark.parametrize("nsub", [0, 2])
def test_collect_matches_oracle_features_and_target(nsub):
    g0, S, vert = small_state(seed=12)
    G = D.Grid(g0, vert)
    st = D.State(G, diffusion="surrogate")
    st.write(S)
    ne = G.info["n_edges"]
    n = K * ne  # every point: the permutation must cover each exactly once
    buf = torch.zeros((19, n + 64), dtype=torch.float32, device="cuda")
    idx = st.collect(DT, nsub, seed=4, n_samples=n, buf=buf, offset=32, return_index=True)
    torch.cuda.synchronize()
    assert np.array_equal(np.sort(idx), np.arange(n))
    got = buf.cpu().numpy()[:, 32:32 + n]
    assert np.all(buf.cpu().numpy()[:, :32] == 0) and np.all(buf.cpu().numpy()[:, 32 + n:] == 0)
    # oracle: the state before the diffusion, its features and the plain tendency
    g = OGrid(g0, vert)
    pr = default_params()
    pre = S
    if nsub > 0:
        for _ in range(nsub):
            pre = O.substep(g, pr, pre, DT / nsub)
    f = M.features(g, pre["vn"])
    T = M.diffusion_tendency(g, pr, pre, DT, O.diffusion)
    k, e = idx // ne, idx % ne
    for j in range(18):
        ref = f[k, e, j]
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got[j] - ref)) <= 1e-6 * scale + 1e-30, j
    ref = T[k, e]
    assert np.max(np.abs(got[18] - ref)) <= 1e-5 * np.max(np.abs(ref))
    # the step itself is the plain step: compare with a plain state
    after = st.read()
    st2 = D.State(G)
    st2.write(S)
    if nsub > 0:
        st2.step(DT, nsub)
        for name in FIELDS:
            assert np.array_equal(after[name], st2.read()[name]), name
    st2.close()
    st.close()
    G.close()


def test_collect_partial_sample_is_without_replacement():
    g0, S, vert = small_state(seed=13)
    G = D.Grid(g0, vert)
    st = D.State(G, diffusion="surrogate")
    st.write(S)
    ne = G.info["n_edges"]
    buf = torch.zeros((19, 1000), dtype=torch.float32, device="cuda")
    a = st.collect(DT, 1, seed=9, n_samples=1000, buf=buf, return_index=True)
    assert len(np.unique(a)) == 1000 and a.min() >= 0 and a.max() < K * ne
    b = st.collect(DT, 1, seed=10, n_samples=1000, buf=buf, return_index=True)
    assert not np.array_equal(a, b)
    st.close()
    G.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_threshold_zero_equals_plain_run(precision):
    g0, S, vert = small_state(seed=14)
    G = D.Grid(g0, vert)
    net = D.Mlp(1)
    sur = D.State(G, precision=precision, diffusion="surrogate")
    plain = D.State(G, precision=precision)
    sur.write(S)
    plain.write(S)
    sur.set_mlp(net, threshold=0.0, judge_every=3)
    for i in range(5):
        sur.step(DT, NSUB)
        plain.step(DT, NSUB)
        a, b = sur.read(), plain.read()
        for name in FIELDS:
            assert np.array_equal(a[name], b[name]), (i, name, np.max(np.abs(a[name] - b[name])))
    info = sur.surrogate_stats()
    assert info["steps"] == 5 and info["judge_steps"] == 2
    assert info["judge_flagged"] == G.info["n_edges"] and info["fallback"] == G.info["n_edges"]
    assert info["fallback_total"] == 3 * G.info["n_edges"]
    assert sur.diag()["fallback_fraction"] == 1.0
    sur.close()
    plain.close()
    net.close()
    G.close()


def test_out_of_range_column_falls_back():
    g0, S, vert = small_state(seed=15, jet_u0=0.0)
    g = OGrid(g0, vert)
    f = M.features(g, S["vn"])
    amax = np.max(np.abs(f.reshape(-1, 18)), axis=0)
    lo = np.concatenate([-3.0 * amax[:16], [0.0, 0.0]]).astype(np.float32)
    hi = np.concatenate([3.0 * amax[:16], [10.0, 10.0]]).astype(np.float32)
    spike = 57
    S = dict(S)
    S["vn"] = S["vn"].copy()
    S["vn"][:, spike] = 20.0 * amax[0]
    G = D.Grid(g0, vert)
    net = D.Mlp(2)
    net.set_norm(np.zeros(18), np.ones(18), lo, hi, 1e-3)
    sur = D.State(G, diffusion="surrogate")
    plain = D.State(G)
    sur.write(S)
    plain.write(S)
    sur.set_mlp(net, threshold=1e30, judge_every=100)
    for _ in range(2):  # a judge (plain) step, then a surrogate step
        sur.step(DT, NSUB)
        plain.step(DT, NSUB)
    info = sur.surrogate_stats()
    a, b = sur.read()["vn"], plain.read()["vn"]
    print(info)
    assert info["judge_flagged"] == 0
    assert 1 <= info["range_flagged"] == info["fallback"] < G.info["n_edges"] // 2
    assert np.array_equal(a[:, spike], b[:, spike])
    assert rel_l2(a, b) > 1e-8  # the other columns used the (untrained) network
    sur.close()
    plain.close()
    net.close()
    G.close()


def test_autotune_leaves_surrogate_state_alone():
    """The tuner's trial steps use the plain diffusion and restore the fields:
    the surrogate's judge flags and counters, and every later step, are those
    of an untuned state."""
    g0, S, vert = small_state(seed=16)
    G = D.Grid(g0, vert)
    net = D.Mlp(3)
    a = D.State(G, diffusion="surrogate")
    b = D.State(G, diffusion="surrogate")
    for st in (a, b):
        st.write(S)
        st.set_mlp(net, threshold=1e-3, judge_every=2)
        st.step(DT, NSUB)  # a judge step: sets the per-column flags
    a.autotune(DT, NSUB)
    assert a.surrogate_stats() == b.surrogate_stats()
    for _ in range(3):
        a.step(DT, NSUB)
        b.step(DT, NSUB)
    x, y = a.read(), b.read()
    for name in FIELDS:
        assert np.array_equal(x[name], y[name]), name
    assert a.surrogate_stats() == b.surrogate_stats()
    a.close()
    b.close()
    net.close()
    G.close()


def test_fit_norm_keeps_tiny_scales():
    """Feature scales span many orders of magnitude (div L1 ~ 1e-17 on a
    global grid): each gets its own scale, flow features and the target a
    zero mean and the symmetric range."""
    rng = np.random.default_rng(21)
    n = 5000
    scales = 10.0 ** np.linspace(-24, 2, 19)
    h = rng.normal(size=(19, n)) * scales[:, None]
    h[16:18] = 1.0 + 0.1 * rng.normal(size=(2, n))  # geometric ratios
    buf = torch.tensor(h, dtype=torch.float32, device="cuda")
    net = D.Mlp(0)
    net.fit_norm(buf, n)
    nrm = net.norm()
    hf = h.astype(np.float32).astype(np.float64)
    for i in range(16):
        rms = np.sqrt(np.mean(hf[i] ** 2))
        assert nrm["mean"][i] == 0.0 and abs(nrm["std"][i] / rms - 1) < 1e-5, i
        amax = np.max(np.abs(hf[i]))
        assert nrm["min"][i] == np.float32(-amax) and nrm["max"][i] == np.float32(amax), i
    for i in (16, 17):
        assert abs(nrm["mean"][i] - hf[i].mean()) < 1e-6 and abs(nrm["std"][i] / hf[i].std() - 1) < 1e-4
        assert nrm["min"][i] == np.float32(hf[i].min()) and nrm["max"][i] == np.float32(hf[i].max())
    assert abs(nrm["target_std"] / np.sqrt(np.mean(hf[18] ** 2)) - 1) < 1e-5
    net.close()


def test_training_reduces_loss_and_fits():
    g0, S, vert = small_state(seed=16, n=2, k=2)
    G = D.Grid(g0, vert)
    st = D.State(G, diffusion="surrogate")
    st.write(S)
    ne = G.info["n_edges"]
    per = 4096
    steps = 8
    buf = torch.zeros((19, per * steps), dtype=torch.float32, device="cuda")
    for i in range(steps):
        st.collect(DT, NSUB, seed=100 + i, n_samples=per, buf=buf, offset=i * per)
    held = torch.zeros((19, per), dtype=torch.float32, device="cuda")
    st.collect(DT, NSUB, seed=999, n_samples=per, buf=held)
    torch.cuda.synchronize()
    assert per <= K * ne
    net = D.Mlp(3)
    net.fit_norm(buf, per * steps)
    nrm = net.norm()
    assert nrm["target_std"] > 0 and np.all(nrm["std"] > 0)
    trace = net.train(buf, per * steps, batch=512, epochs=12, lr0=3e-3, lr1=1e-5, seed=1)
    assert trace.shape == ((per * steps) // 512 * 12,)
    first, last = float(np.mean(trace[:16])), float(np.mean(trace[-16:]))
    h = held.cpu().numpy()
    y = net.forward(h[:18].T.copy())
    r2 = 1.0 - np.sum((y - h[18]) ** 2) / np.sum((h[18] - h[18].mean()) ** 2)
    print("loss", first, "->", last, "held-out R2", r2)
    assert last < 0.3 * first
    assert r2 > 0.5
    st.close()
    net.close()
    G.close()


def test_surrogate_errors():
    g0, S, vert = small_state(seed=17)
    G = D.Grid(g0, vert)
    sur = D.State(G, diffusion="surrogate")
    plain = D.State(G)
    net = D.Mlp(0)
    with pytest.raises(D.DycoreError) as ei:
        sur.step(DT, NSUB)  # no network attached
    assert ei.value.code == D.DC_ESTATE
    with pytest.raises(D.DycoreError) as ei:
        plain.set_mlp(net)
    assert ei.value.code == D.DC_ESTATE
    buf = torch.zeros((19, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(D.DycoreError) as ei:
        plain.collect(DT, 1, 0, 10, buf)
    assert ei.value.code == D.DC_ESTATE
    with pytest.raises(D.DycoreError) as ei:
        sur.collect(DT, 1, 0, 300, buf)  # more than the buffer holds
    assert ei.value.code == D.DC_EINVAL
    with pytest.raises(D.DycoreError) as ei:
        net.grad(np.zeros((100, 18)), np.zeros(100))
    assert ei.value.code == D.DC_EINVAL
    with pytest.raises(D.DycoreError) as ei:
        net.train(buf, 256, batch=100)
    assert ei.value.code == D.DC_EINVAL
    with pytest.raises(D.DycoreError) as ei:
        net.set_norm(np.zeros(18), np.zeros(18), np.zeros(18), np.ones(18), 1.0)
    assert ei.value.code == D.DC_EINVAL
    with pytest.raises(D.DycoreError) as ei:
        sur.set_mlp(net, threshold=-1.0)
    assert ei.value.code == D.DC_EINVAL
    sur.close()
    plain.close()
    net.close()
    G.close()


def test_surrogate_step_matches_oracle_network_on_oracle_features():
    """One network step of the surrogate against the oracle: the state
    before the diffusion from the oracle's plain step and substeps, the
    oracle's 18 features of it, the oracle network on the same BF16-rounded
    weights and normalised BF16 inputs (times the target scale) for the vn
    increment dt T_mlp (relative L2 <= 2e-2, the BF16 bound of the network
    tests), and the plain diffusion's w and the untouched rho, exner,
    theta_v (<= 1e-11).  This checks the wiring inside the step: feature
    order, normalisation, target scale and the update vn += dt T_mlp."""
    g0, S, vert = small_state(seed=18)
    og = OGrid(g0, vert)
    pr = default_params()
    wts = O.vertex_lsq_weights(og)
    # step 1 is a judge step (plain diffusion); step 2 uses the network
    S1 = O.step(og, S, DT, NSUB, pr, wts=wts)
    pre = S1
    for _ in range(NSUB):
        pre = O.substep(og, pr, pre, DT / NSUB)
    f = M.features(og, pre["vn"], wts).reshape(-1, 18)
    T_plain = M.diffusion_tendency(og, pr, pre, DT, O.diffusion)
    rng = np.random.default_rng(19)
    p = M.init_params(7)
    p["b1"] = rng.normal(scale=0.1, size=64)
    p["b2"] = rng.normal(scale=0.1, size=64)
    p["b3"] = np.array([0.02])
    mean = np.zeros(18, np.float32)
    std = np.sqrt(np.mean(f ** 2, axis=0)).astype(np.float32)
    mean[16:] = f[:, 16:].mean(axis=0)
    std[16:] = f[:, 16:].std(axis=0)
    tstd = np.float32(np.sqrt(np.mean(T_plain ** 2)))
    inf = np.full(18, np.inf, np.float32)
    net = D.Mlp(0)
    net.set_params(D.mlp_pack(p))
    net.set_norm(mean, std, -inf, inf, tstd)
    G = D.Grid(g0, vert)
    st = D.State(G, diffusion="surrogate")
    st.write(S)
    st.set_mlp(net, threshold=np.inf, judge_every=1 << 30)
    st.step(DT, NSUB)
    st.step(DT, NSUB)
    out = st.read()
    info = st.surrogate_stats()
    assert info["judge_steps"] == 1 and info["fallback"] == 0 and info["range_flagged"] == 0
    pb = {k: bf16(v) if k in ("w1", "w2") else np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    istd = (np.float32(1.0) / std).astype(np.float32)
    xs = bf16((f.astype(np.float32) - mean) * istd)
    y, _ = M.forward(pb, xs)
    inc_want = DT * (y * float(tstd)).reshape(pre["vn"].shape)
    inc_got = out["vn"] - pre["vn"]
    err = rel_l2(inc_got, inc_want)
    print("surrogate increment rel L2 vs oracle network", err)
    assert err <= 2e-2
    # the network's increment is not the plain one (it is untrained): the
    # comparison above is not passed by the plain diffusion
    assert rel_l2(DT * T_plain, inc_want) > 0.1
    after = O.diffusion(og, pr, pre, DT, wts)
    for name in ("w", "rho", "exner", "theta_v"):
        e = rel_l2(out[name], after[name])
        assert e <= 1e-11, (name, e)
    st.close()
    net.close()
    G.close()


def test_trained_network_gains_over_no_diffusion_and_untrained():
    """The gain test at reduced size (R2B4, 65 levels, 50 steps): a network
    trained on pairs from plain FP64 steps of one state, evaluated from a
    held-out state with its per-column fallback, stays closer to the plain
    run than no vn diffusion at all (a zero network) and than the untrained
    network (both without judge steps)."""
    from synth import build_workload

    g0, S_tr, vert, spec = build_workload("r2b4_k65")
    S_ev, _ = initial_state(g0, spec["n_lev"], spec["z_top"], **dict(spec["state"], seed=5))
    dt, nsub = spec["dt"], spec["nsub"]
    G = D.Grid(g0, vert)
    n_tr, per = 40, 50_000
    buf = torch.empty((19, n_tr * per), dtype=torch.float32, device="cuda")
    st = D.State(G, diffusion="surrogate")
    st.write(S_tr)
    for i in range(n_tr):
        st.collect(dt, nsub, seed=(4 << 32) + i, n_samples=per, buf=buf, offset=i * per)
    st.close()
    net = D.Mlp(seed=3)
    net.fit_norm(buf, n_tr * per)
    trace = net.train(buf, n_tr * per, batch=4096, epochs=2, lr0=1e-3, lr1=1e-5, seed=4)
    print("loss", float(trace[:20].mean()), "->", float(trace[-20:].mean()))
    del buf
    nrm = net.norm()
    untrained = D.Mlp(seed=3)
    untrained.set_norm(nrm["mean"], nrm["std"], nrm["min"], nrm["max"], nrm["target_std"])
    zero = D.Mlp(seed=0)
    zero.set_params(np.zeros(D.MLP_NPARAMS, dtype=np.float32))
    steps, inf = 50, float("inf")

    def run(mlp=None, thr=None, judge=None):
        s = D.State(G, diffusion="surrogate" if mlp is not None else "plain")
        s.write(S_ev)
        if mlp is not None:
            s.set_mlp(mlp, thr, judge)
        for _ in range(steps):
            s.step(dt, nsub)
        out, info = s.read(), (s.surrogate_stats() if mlp is not None else None)
        s.close()
        return out, info

    ref, _ = run()
    err = {}
    for name, args in (("trained", (net, 1e-3, 10)), ("no_vn_diffusion", (zero, inf, 1 << 30)),
                       ("untrained", (untrained, inf, 1 << 30))):
        out, info = run(*args)
        err[name] = rel_l2(out["vn"], ref["vn"])
        print(name, "vn rel L2 vs plain", err[name], info)
        assert np.all(np.isfinite(out["vn"]))
    assert err["trained"] < err["no_vn_diffusion"]
    assert err["trained"] < err["untrained"]
    for m in (net, untrained, zero):
        m.close()
    G.close()
