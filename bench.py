"""Throughput of the dycore time step on one MI355X (plus the oracle on the host).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload r2b8_k90]

A step is one dc_dycore_step: nsub predictor-corrector substeps and one
diffusion step over the whole grid.  Inputs are resident in HBM when the
timed region starts.  Prints one JSON line (rank 0, N = 1).

The default workload is the largest single-GPU one: R2B8 (5,242,880 cells,
7,864,320 edges), 90 levels, curve-ordered, dt 30 s, 5 substeps, FP64, with
the mixed form measured beside it on the same steps.  The R2B5 / 65-level
jet workload follows as a secondary block: its rate, and the error of the
mixed form against FP64 per field after its 100 steps.  The oracle is timed
on one host core on a sample of the R2B5 workload (an R2B8 step is out of the
host's reach).

Sequence per precision: dc_state_autotune (launch tiles; fields restored),
W warm-up steps, K steps with events around every launch (the per-kernel
table), then the K timed steps with events around the dominant kernel's
launches only: `value` and the roofline's launch duration both come from
that timed region, which the per-launch events of the other kernels would
otherwise slow down.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dycore cell·level·steps/s, % HBM peak; mixed/surrogate vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0
FIELDS = ("vn", "w", "rho", "exner", "theta_v")


def kernel_bytes(C, E, V, K, r):
    """Algorithmic bytes of one launch of each kernel: every array the kernel
    reads or writes counted once per (entity, level); r = bytes of vn and of
    the horizontal intermediates (8 FP64, 4 mixed); cell prognostics are 8.
    gw is the edge term of the horizontal advection of w ([K+1][E], r bytes),
    tw0 the substep-start T_w ([K+1][C], r bytes).  The edge passes are the
    fused ones (a grid numbered with locality): vt, K_e and the vorticity
    stay in LDS, the vorticity pass is not launched and the corrector's cell
    pass forms only the damping field D2."""
    KE, KV, KC, K1C, K1E = K * E, K * V, K * C, (K + 1) * C, (K + 1) * E
    return {
        # reads vn, w, exner, theta; writes Y = vn + dtau (a0 T_vn0 - PGF), vn*, gw
        "edge_pred": r * KE + 8 * K1C + 8 * 2 * KC + r * 3 * KE,
        # reads gw, vn*, w, rho, exner, theta; writes w*, tw0, D = div vn*
        "column_pred": r * K1E + r * KE + 8 * K1C + 8 * 3 * KC + 8 * K1C + r * K1C + r * KC,
        # reads D; writes D2
        "vort_ke_corr": 2 * r * KC,
        # reads vn*, Y, D2, w*; writes vn', gw
        "edge_corr": r * 2 * KE + r * KC + 8 * K1C + r * 2 * KE,
        # reads gw, vn', w, w*, tw0, rho, exner, theta; writes w, rho, exner, theta
        "column_corr": r * K1E + r * KE + 8 * 2 * K1C + r * K1C + 8 * 3 * KC + 8 * (K1C + 3 * KC),
        "diff_vertex": r * KE + r * 4 * KV,
        "diff_div": r * KE + r * KC,
        "diff_edge1": r * KC + r * 4 * KV + r * 2 * KE,
        "diff_cell_vertex2": r * 2 * KE + 8 * 2 * K1C + r * (KC + KV),
        "diff_edge2": r * 3 * KE + r * KC + r * KV + r * KE,
        # option: reads vn, vt, rho and theta_v of the upwind cell and its neighbours; writes rho_e, theta_e (FP64)
        "edge_upwind": 2 * r * KE + 8 * 2 * KC + 8 * 2 * KE,
    }


def mixed_bound(workload, field):
    """The relative L2 error of the mixed form against FP64 stated per field:
    1e-4, except w on the R2B8 grid, where vn's FP32 storage alone drives
    w's error above it (5e-3 stated)."""
    return 5e-3 if (field == "w" and workload.startswith("r2b8")) else 1e-4


def step_algorithmic_bytes(C, E, K, nsub, r):
    """Compulsory HBM traffic of a whole step with perfect fusion, as the
    scope table's measurement section counts it: each substep's predictor
    reads the state S^n and writes the predicted state S* (all five fields),
    the corrector reads S^n and the predicted vn*, w* and writes S^{n+1};
    diffusion reads and writes vn and w once.  FP64 (r = 8): 1,020 B per
    cell and level at nsub = 5 with E = 1.5 C; mixed (vn in FP32): 858 B."""
    state = r * K * E + 8 * ((K + 1) * C + 3 * K * C)
    pred = 2 * state                                       # read S^n, write S*
    corr = state + r * K * E + 8 * (K + 1) * C + state    # read S^n, vn*, w*, write S^{n+1}
    diff = 2 * (r * K * E + 8 * (K + 1) * C)
    return nsub * (pred + corr) + diff


def step_algorithmic_bytes_r15(C, E, K, nsub, r):
    """The same with the predictor writing only vn* and w*: the corrector
    reuses the predictor's pressure gradient and column coefficients, all of
    which depend on S^n only, so the predicted rho, exner, theta_v are never
    needed (903 B per cell and level in FP64)."""
    state = r * K * E + 8 * ((K + 1) * C + 3 * K * C)
    pred = state + r * K * E + 8 * (K + 1) * C
    corr = state + r * K * E + 8 * (K + 1) * C + state
    diff = 2 * (r * K * E + 8 * (K + 1) * C)
    return nsub * (pred + corr) + diff


def kernel_compulsory_bytes(kid, C, E, K, r):
    """A column kernel's share of the compulsory traffic (the per-phase words
    of the scope table's measurement section): column_corr reads w, rho,
    exner, theta_v of S^n, the predicted w* and the new vn whose fluxes it
    forms, and writes w, rho, exner, theta_v of S^{n+1}; column_pred reads
    S^n's w, rho, exner, theta_v and vn*, and writes w*.  None for kernels
    without a natural share (the horizontal passes split the edge fields
    between them)."""
    cells = 8 * ((K + 1) * C + 3 * K * C)
    if kid == "column_corr":
        return 2 * cells + 8 * (K + 1) * C + r * K * E
    if kid == "column_pred":
        return cells + r * K * E + 8 * (K + 1) * C
    return None


# kernels of the step as rocprofv3 names them -> the ids used above
_BODY_IDS = {("BVc", "false"): "vort_ke_pred", ("BVc", "true"): "vort_ke_corr",
             ("BEdge", "false"): "edge_pred", ("BEdge", "true"): "edge_corr",
             ("BCol", "false"): "column_pred", ("BCol", "true"): "column_corr",
             ("BDvert", None): "diff_vertex", ("BDiv", None): "diff_div", ("BDedge1", None): "diff_edge1",
             ("BDcv2", None): "diff_cell_vertex2", ("BDedge2", None): "diff_edge2"}


def kernel_id(name):
    """Step-kernel id of a rocprofv3 kernel name (None for other kernels)."""
    import re

    m = re.search(r"k_one<dc::bodies::(B\w+)<(?:double|float)(?:, (true|false))?", name)
    if not m:
        return None
    return _BODY_IDS.get((m.group(1), m.group(2)))


def sources_sha256():
    """Hash of the kernel sources: counter figures taken with other sources are stale."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2608_21150_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def summarize_profile(trace_dir, fetch_dir, write_dir, cfetch_dir, cwrite_dir, out, command, workload, precision):
    """Markdown summary of a rocprofv3 kernel-trace run and two counter runs
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), scaled by what the same
    counters read for a 1 GiB device copy; the last line carries the scaled
    bytes per launch of every step kernel and the kernel-source hash."""
    import collections
    import csv

    def short(n):
        return n.replace("dc::bodies::", "").replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")

    def counters(d):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in agg.items()}

    rows = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    F, W, cF, cW = counters(fetch_dir), counters(write_dir), counters(cfetch_dir), counters(cwrite_dir)
    copy = [k for k in cF if "copyBuffer" in k][0]
    kib = 1024 * 1024  # the copy moves 1 GiB each way
    sf, sw = kib / cF[copy], kib / cW[[k for k in cW if "copyBuffer" in k][0]]
    lines = [f"command: `{command}`", "",
             f"counter calibration (`python bench.py --calibrate-copy 1024`, a 1 GiB device-to-device copy): "
             f"FETCH_SIZE reads {cF[copy]:.0f} KiB and WRITE_SIZE {cW[[k for k in cW if 'copyBuffer' in k][0]]:.0f} "
             f"KiB per {kib} KiB moved -> scale fetch x{sf:.3f}, write x{sw:.3f}", "",
             "| kernel | id | calls | avg us | share % | FETCH KiB raw | WRITE KiB raw | HBM MB/launch (scaled) "
             "| HBM GB/s (counters) | algorithmic MB/launch | algorithmic GB/s |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    from synth import WORKLOADS, expected_counts

    wl = WORKLOADS[workload]
    C, E, V = expected_counts(wl["n"], wl["k"])
    alg = kernel_bytes(C, E, V, wl["n_lev"], 4 if precision == "mixed" else 8)
    per = {}
    for r in rows:
        name = r["Name"]
        f, w = F.get(name), W.get(name)
        mb = (f * sf + w * sw) * 1024 / 1e6 if f is not None and w is not None else None
        kid = kernel_id(name)
        if kid and mb is not None:
            per[kid] = {"bytes": mb * 1e6, "avg_us": float(r["AverageNs"]) / 1e3}
        us = float(r["AverageNs"]) / 1e3
        gbs = "-" if mb is None or us <= 0 else f"{mb / us * 1e3:.0f}"
        amb = alg.get(kid) / 1e6 if kid in alg else None
        ags = "-" if amb is None or us <= 0 else f"{amb / us * 1e3:.0f}"
        lines.append(f"| {short(name)[:90]} | {kid or '-'} | {r['Calls']} | {us:.1f} | "
                     f"{float(r['Percentage']):.2f} | {f if f is None else round(f, 1)} | "
                     f"{w if w is None else round(w, 1)} | {'-' if mb is None else round(mb, 1)} | {gbs} | "
                     f"{'-' if amb is None else round(amb, 1)} | {ags} |")
    meta = {"workload": workload, "precision": precision, "sources_sha256": sources_sha256(),
            "fetch_scale": sf, "write_scale": sw, "kernels": per}
    lines += ["", "<!-- traffic " + json.dumps(meta) + " -->"]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profiled_traffic(workload, precision, kid):
    """HBM bytes per launch of kernel kid from the committed counter summary
    of this workload, or None if there is none or its sources differ."""
    path = os.path.join(ROOT, "profiles", f"step_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("<!-- traffic "):
            meta = json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
            if meta.get("sources_sha256") != sources_sha256() or kid not in meta["kernels"]:
                return None
            return meta["kernels"][kid]["bytes"]
    return None


def cpu_baseline(spec, g0, S, vert, budget_s=25.0):
    """The oracle, as it stands, on one host core for a bounded sample."""
    import numpy as np

    from oracle import dycore as O
    from oracle.constants import default_params
    from oracle.grid import Grid as OGrid

    try:
        old = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(old)})
    except (AttributeError, OSError):
        old = None
    try:
        og = OGrid(g0, vert)
        wts = O.vertex_lsq_weights(og)
        p = default_params()
        t0 = time.perf_counter()
        steps = 0
        Sx = S
        while True:
            Sx = O.step(og, Sx, spec["dt"], spec["nsub"], p, wts=wts)
            steps += 1
            if time.perf_counter() - t0 > budget_s * 0.5 or steps >= 3:
                break
        el = time.perf_counter() - t0
    finally:
        if old is not None:
            os.sched_setaffinity(0, old)
    units = og.nc * og.n_lev * steps
    return {"value": units / el, "unit": "cell·level·steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} full step(s) of the same workload ({og.nc} cells x {og.n_lev} levels, nsub "
                      f"{spec['nsub']}), NumPy FP64 oracle pinned to one core, {el:.1f} s; host os.cpu_count()="
                      f"{os.cpu_count()}"}


def bench_r2b5(args, D, torch, dev):
    """The R2B5 / 65-level jet workload (81,920 cells, dt 180 s, 5
    substeps): FP64 and mixed rates (tuned tiles, warm-up, timed steps), and
    the mixed form's error against FP64 per field after the workload's 100
    steps from the same initial state, with the mass drift of both."""
    import numpy as np

    from synth import build_workload

    name = "r2b5_k65"
    print(f"[bench] secondary workload {name}", file=sys.stderr, flush=True)
    g0, S, vert, spec = build_workload(name)
    C, K = g0["n_cells"], spec["n_lev"]
    G = D.Grid(g0, vert, sfc=bool(spec.get("sfc", 0)))
    stream = torch.cuda.current_stream(dev)
    res = {"workload": f"{name}: R2B5 icosahedral grid, {C} cells, {K} levels, dt {spec['dt']} s, "
                       f"{spec['nsub']} substeps, generator-ordered"}
    for prec in ("fp64", "mixed"):
        st = D.State(G, precision=prec, device=dev)
        st.write(S)
        if not args.no_autotune:
            st.autotune(spec["dt"], spec["nsub"])
        for _ in range(args.warmup):
            st.step(spec["dt"], spec["nsub"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            st.step(spec["dt"], spec["nsub"])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        st.close()
        b = step_algorithmic_bytes(C, g0["n_edges"], K, spec["nsub"], 8 if prec == "fp64" else 4)
        res[prec] = {"value": C * K / (ms * 1e-3), "ms_per_step": ms,
                     "step_hbm_effective_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    res["mixed"]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    # errors after the workload's steps, both runs from the initial state
    outs, diags = {}, {}
    for prec in ("fp64", "mixed"):
        st = D.State(G, precision=prec, device=dev)
        st.write(S)
        d0 = st.diag()
        for _ in range(spec["steps"]):
            st.step(spec["dt"], spec["nsub"])
        outs[prec], d1 = st.read(), st.diag()
        diags[prec] = {"mass_rel_drift": d1["mass"] / d0["mass"] - 1.0,
                       "theta_mass_rel_drift": d1["theta_mass"] / d0["theta_mass"] - 1.0,
                       "n_nonfinite": d1["n_nonfinite"]}
        st.close()
    G.close()
    res["mixed_rel_l2_vs_fp64"] = {k: float(np.linalg.norm(outs["mixed"][k] - outs["fp64"][k])
                                         / np.linalg.norm(outs["fp64"][k])) for k in FIELDS}
    res["mixed_within_1e-4"] = all(v <= 1e-4 for v in res["mixed_rel_l2_vs_fp64"].values())
    res["after_steps"] = spec["steps"]
    res["diag"] = diags
    return res


def bench_ensemble(args, D, torch):
    """24 uneven members (12 x R2B4 + 12 x R2B5, 65 levels, mixed precision):
    one graph launch per step against a loop of per-member steps."""
    from synth import ensemble_member, initial_state, make_grid

    grids, states, cells = {}, [], 0
    spec = ensemble_member(0)
    for m in range(24):
        sp = ensemble_member(m)
        if sp["k"] not in grids:
            g = make_grid(sp["n"], sp["k"])
            _, vert = initial_state(g, sp["n_lev"], sp["z_top"], seed=0)
            grids[sp["k"]] = (g, D.Grid(g, vert))
        g, G = grids[sp["k"]]
        S, _ = initial_state(g, sp["n_lev"], sp["z_top"], **sp["state"])
        st = D.State(G, precision="mixed")
        st.write(S)
        states.append(st)
        cells += g["n_cells"] * sp["n_lev"]
    dt, nsub = spec["dt"], spec["nsub"]
    E = D.Ensemble(states)
    cache = os.environ.get("DC_SCHEDULE_CACHE", "/tmp/dycore_schedules.txt")
    t0 = time.perf_counter()
    E.autotune(dt, nsub, cache)
    tune_s = time.perf_counter() - t0
    sched = E.schedule()
    stream = torch.cuda.current_stream()
    # every member of the batched run equals its run alone: two steps of the
    # ensemble against solo states of four members (two of each grid)
    import numpy as np

    for _ in range(2):
        E.step(dt, nsub)
    check = (0, 11, 12, 23)
    member_equal = True
    for m in check:
        sp = ensemble_member(m)
        g, G = grids[sp["k"]]
        S, _ = initial_state(g, sp["n_lev"], sp["z_top"], **sp["state"])
        solo = D.State(G, precision="mixed")
        solo.write(S)
        for _ in range(2):
            solo.step(dt, nsub)
        a, b = states[m].read(), solo.read()
        solo.close()
        member_equal &= all(np.array_equal(a[f], b[f]) for f in FIELDS)
    print(f"[bench] ensemble members {check} bitwise equal to their solo runs: {member_equal}", file=sys.stderr,
          flush=True)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_graph = timed(lambda: E.step(dt, nsub), args.steps)
    E.close()

    def loop():
        for st in states:
            st.step(dt, nsub)

    ms_loop = timed(loop, args.steps)
    line = {"metric": METRIC, "value": cells / (ms_graph * 1e-3), "unit": "cell·level·steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "ensemble: 12 x R2B4 + 12 x R2B5 members, 65 levels, mixed precision, "
                                   f"dt {dt} s, {nsub} substeps, one graph launch per step",
                       "members": 24, "cell_levels": cells},
            "per_member_loop": {"ms_per_step": ms_loop, "value": cells / (ms_loop * 1e-3)},
            "speedup_vs_loop": ms_loop / ms_graph, "schedule": sched,
            "members_bitwise_equal_solo": {"members": list(check), "after_steps": 2, "equal": bool(member_equal)},
            "autotune_s": tune_s}
    for st in states:
        st.close()
    for _, G in grids.values():
        G.close()
    line["small_members"] = bench_ensemble_small(args, D, torch, timed)
    print(json.dumps(line), flush=True)


def bench_ensemble_small(args, D, torch, timed, n_members=64):
    """Where batching pays: many small members (R2B2, 30 levels, mixed), whose
    per-member launches are short enough that the launch cost of a loop over
    them shows (the paper's Section 4.3.3 hides it behind asynchronous
    dispatch); one graph launch per step against the per-member loop."""
    from synth import initial_state, make_grid

    g = make_grid(2, 2)
    _, vert = initial_state(g, 30, 30e3, seed=0)
    G = D.Grid(g, vert)
    states = []
    for m in range(n_members):
        S, _ = initial_state(g, 30, 30e3, seed=2000 + m, vn_sigma=1.0, t_sigma=0.2, jet_u0=35.0)
        st = D.State(G, precision="mixed")
        st.write(S)
        states.append(st)
    dt, nsub = 600.0, 5
    E = D.Ensemble(states)
    ms_graph = timed(lambda: E.step(dt, nsub), args.steps)
    E.close()

    def loop():
        for st in states:
            st.step(dt, nsub)

    ms_loop = timed(loop, args.steps)
    for st in states:
        st.close()
    G.close()
    cells = n_members * g["n_cells"] * 30
    return {"members": n_members, "workload": "R2B2 (1280 cells), 30 levels, mixed, dt 600 s, 5 substeps, "
                                              "default schedule",
            "ms_per_step": ms_graph, "value": cells / (ms_graph * 1e-3),
            "per_member_loop_ms_per_step": ms_loop, "speedup_vs_loop": ms_loop / ms_graph}


def bench_surrogate(args, D, torch):
    """The learned diffusion on R2B6 / 65 levels: collect training pairs from
    plain FP64 steps, fit and train the network, then run the same number of
    steps from a held-out initial state with (i) the plain diffusion, (ii) the
    network with per-column fallback, (ii') the network without judge steps,
    (iii) no vn diffusion (a zero network) and (iv) an untrained network;
    report each run's error against (i) and its time per step."""
    import numpy as np

    from synth import build_workload, initial_state

    name = "r2b6_k65"
    g0, S_tr, vert, spec = build_workload(name)
    S_ev, _ = initial_state(g0, spec["n_lev"], spec["z_top"], **dict(spec["state"], seed=5))
    C, E, K = g0["n_cells"], g0["n_edges"], spec["n_lev"]
    dt, nsub = spec["dt"], spec["nsub"]
    G = D.Grid(g0, vert)
    n_tr, per = args.train_steps, args.train_per_step
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    buf = torch.empty((19, n_tr * per), dtype=torch.float32, device="cuda")
    st = D.State(G, diffusion="surrogate")
    st.write(S_tr)
    t0 = time.perf_counter()
    for i in range(n_tr):
        st.collect(dt, nsub, seed=(4 << 32) + i, n_samples=per, buf=buf, offset=i * per)
        if (i + 1) % 50 == 0 or i + 1 == n_tr:
            torch.cuda.synchronize()
            log(f"collected {i + 1}/{n_tr} steps")
    t_collect = time.perf_counter() - t0
    st.close()
    n = n_tr * per
    net = D.Mlp(seed=3)
    net.fit_norm(buf, n)
    t0 = time.perf_counter()
    trace = net.train(buf, n, batch=4096, epochs=2, lr0=1e-3, lr1=1e-5, seed=4)
    t_train = time.perf_counter() - t0
    log(f"trained {len(trace)} Adam steps in {t_train:.1f} s, loss {trace[:100].mean():.4g} -> {trace[-100:].mean():.4g}")
    del buf
    torch.cuda.empty_cache()
    nrm = net.norm()
    untrained = D.Mlp(seed=3)
    untrained.set_norm(nrm["mean"], nrm["std"], nrm["min"], nrm["max"], nrm["target_std"])
    zero = D.Mlp(seed=0)
    zero.set_params(np.zeros(D.MLP_NPARAMS, dtype=np.float32))
    inf = float("inf")

    def run(label, mlp=None, thr=None, judge=None, steps=args.eval_steps):
        s = D.State(G, diffusion="surrogate" if mlp is not None else "plain")
        s.write(S_ev)
        if mlp is not None:
            s.set_mlp(mlp, thr, judge)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            s.step(dt, nsub)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out = s.read()
        info = s.surrogate_stats() if mlp is not None else None
        s.close()
        log(f"{label}: {steps} steps, {ms:.3f} ms/step")
        return ms, out, info

    run("warm-up", net, 1e-3, 10, steps=3)
    runs = {"plain": run("plain"),
            "mlp_fallback": run("mlp_fallback", net, 1e-3, 10),
            "mlp_no_judge": run("mlp_no_judge", net, inf, 1 << 30),
            "no_vn_diffusion": run("no_vn_diffusion", zero, inf, 1 << 30),
            "untrained_mlp": run("untrained_mlp", untrained, inf, 1 << 30)}
    ref = runs["plain"][1]
    res = {}
    for k, (ms, out, info) in runs.items():
        r = {"ms_per_step": ms, "rel_l2_vs_plain": {f: float(np.linalg.norm(out[f] - ref[f]) / np.linalg.norm(ref[f]))
                                                    for f in FIELDS}}
        if info is not None:
            apply_steps = info["steps"] - info["judge_steps"]
            r["judge_steps"] = info["judge_steps"]
            r["mean_fallback_fraction"] = info["fallback_total"] / max(1, apply_steps * info["n_columns"])
        res[k] = r
    err = {k: res[k]["rel_l2_vs_plain"]["vn"] for k in res}
    ms_sur, ms_plain = res["mlp_fallback"]["ms_per_step"], res["plain"]["ms_per_step"]
    line = {"metric": METRIC, "value": C * K / (ms_sur * 1e-3), "unit": "cell·level·steps/s", "n_gpus": 1,
            "steps": args.eval_steps, "warmup": 0, "ms_per_step": ms_sur, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
            "config": {"workload": f"surrogate: R2B6 icosahedral grid, {C} cells, {E} edges, {K} levels, dt {dt} s, "
                                   f"{nsub} substeps, FP64 dycore; network trained on {n} pairs from {n_tr} plain "
                                   f"steps (seed 3), evaluated over {args.eval_steps} steps from a held-out state "
                                   f"(seed 5), threshold 1e-3, judge every 10 steps"},
            "surrogate": {"runs": res, "speedup_vs_plain": ms_plain / ms_sur,
                          "gain_test_pass": bool(err["mlp_fallback"] < err["no_vn_diffusion"]
                                                 and err["mlp_fallback"] < err["untrained_mlp"]),
                          "train": {"pairs": n, "adam_steps": len(trace), "collect_s": t_collect,
                                    "train_s": t_train, "loss_first100": float(trace[:100].mean()),
                                    "loss_last100": float(trace[-100:].mean())}}}
    for m in (net, untrained, zero):
        m.close()
    G.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="r2b8_k90")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--sfc", type=int, default=-1, help="1/0 force the space-filling-curve renumbering; -1 workload default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--train-steps", type=int, default=200, help="surrogate: plain steps that collect pairs")
    ap.add_argument("--train-per-step", type=int, default=1_000_000, help="surrogate: pairs per collected step")
    ap.add_argument("--eval-steps", type=int, default=500, help="surrogate: steps of every evaluation run")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch tiles")
    ap.add_argument("--theta", action="store_true", help="also time the step with the theta_v diffusion on")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the R2B5 block (rate and mixed-vs-FP64 errors after 100 steps)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--stream-probe", type=int, default=0, metavar="MIB",
                    help="only time plain streams over MIB MiB (read, write, copy; torch kernels) and exit")
    ap.add_argument("--summarize-profile", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write a profile summary from rocprofv3 output folders and exit")
    ap.add_argument("--profile-out", default=None)
    ap.add_argument("--profile-command", default="")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(*args.summarize_profile, args.profile_out, args.profile_command, args.workload,
                          args.precision)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return

    if args.stream_probe:
        # what plain streaming reaches on this GPU: the practical side of the
        # HBM roofline (best of 5 after a warm-up, events on the current stream)
        n = args.stream_probe * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        res = {}
        for name, fn, moved in (("read (sum)", lambda: x.sum(), n * 8), ("write (fill)", lambda: y.fill_(2.0), n * 8),
                                ("copy", lambda: y.copy_(x), 2 * n * 8)):
            fn()
            best = 1e30
            for _ in range(5):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                torch.cuda.synchronize()
                best = min(best, a.elapsed_time(b))
            res[name] = {"ms": round(best, 4), "GB/s": round(moved / best / 1e6, 1)}
        print(json.dumps({"stream_probe_bytes": n * 8, "results": res}))
        return

    from paper_2608_21150_amd import dycore as D
    from synth import WORKLOADS, build_workload

    if args.workload == "ensemble":
        return bench_ensemble(args, D, torch)
    if args.workload == "surrogate":
        return bench_surrogate(args, D, torch)
    spec = WORKLOADS[args.workload]
    sfc = bool(spec.get("sfc", 0)) if args.sfc < 0 else bool(args.sfc)
    print(f"[bench] building workload {args.workload}", file=sys.stderr, flush=True)
    g0, S, vert, spec = build_workload(args.workload)
    S0 = S
    C, E, V, K = g0["n_cells"], g0["n_edges"], g0["n_verts"], spec["n_lev"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    G = D.Grid(g0, vert, sfc=sfc)

    def run(precision, steps, warmup, tune, params=None):
        """Tune (outside every timed region), warm up, then two passes of
        `steps` steps: the first records events around every launch (the
        per-kernel table), the second is the timed one and records events
        around the launches of the dominant kernel only."""
        st = D.State(G, precision=precision, device=dev, params=params)
        st.write(S)
        tune_s = None
        if tune:
            t0 = time.perf_counter()
            st.autotune(spec["dt"], spec["nsub"])
            tune_s = time.perf_counter() - t0
        for _ in range(warmup):
            st.step(spec["dt"], spec["nsub"])
        torch.cuda.synchronize()
        st.profile(True)
        for _ in range(steps):
            st.step(spec["dt"], spec["nsub"])
        prof = st.profile_read()
        dom = max(prof, key=lambda n: prof[n][1])
        st.profile_select([dom])
        st.profile(True)
        stream = torch.cuda.current_stream(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            st.step(spec["dt"], spec["nsub"])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        prof_dom = st.profile_read()[dom]
        st.profile(False)
        st.profile_select(None)
        out = st.read()
        d = st.diag()
        tiles = st.tiles()
        st.close()
        return {"ms": ms, "prof": prof, "dom": dom, "dom_timed": prof_dom, "out": out, "diag": d, "tiles": tiles,
                "tune_s": tune_s}

    tune = not args.no_autotune
    print(f"[bench] {args.precision}: {'autotune, ' if tune else ''}{args.warmup} warmup + {args.steps} profiled "
          f"+ {args.steps} timed steps", file=sys.stderr, flush=True)
    R1 = run(args.precision, args.steps, args.warmup, tune)
    ms, prof, out, diag = R1["ms"], R1["prof"], R1["out"], R1["diag"]
    ms_step = ms / args.steps
    value = C * K * args.steps / (ms / 1e3)
    r = 4 if args.precision == "mixed" else 8
    kb = kernel_bytes(C, E, V, K, r)
    kernels = {}
    for name, (calls, tot) in prof.items():
        if calls:
            avg = tot / calls
            kernels[name] = {"calls": calls, "avg_us": avg * 1e3, "GBps": kb[name] / (avg * 1e-3) / 1e9,
                             "share": tot / sum(t for _, t in prof.values())}
    dom = R1["dom"]
    calls, tot = R1["dom_timed"]
    avg_ms = tot / calls
    # algorithmic bytes of the dominant kernel: its share of the compulsory
    # traffic where it has one, else every array it reads or writes once
    comp = kernel_compulsory_bytes(dom, C, E, K, r)
    alg_bytes = comp if comp is not None else kb[dom]
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic(args.workload, args.precision, dom),
            "bytes_per_launch": alg_bytes,
            "bytes_basis": "compulsory share" if comp is not None else "kernel arrays",
            "kernel_arrays_bytes_per_launch": kb[dom],
            "kernel_arrays_GBps": round(kb[dom] / (avg_ms * 1e-3) / 1e9, 1),
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches_timed": calls}
    b_step = step_algorithmic_bytes(C, E, K, spec["nsub"], r)
    line = {
        "metric": METRIC, "value": value, "unit": "cell·level·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: R{g0['n']}B{g0['k']} icosahedral grid, {C} cells, {E} edges, "
                               f"{V} vertices, {K} levels, dt {spec['dt']} s, {spec['nsub']} substeps, "
                               f"{'curve-ordered' if sfc else 'generator-ordered'}, {args.precision}",
                   "cells": C, "levels": K, "dt": spec["dt"], "nsub": spec["nsub"], "precision": args.precision,
                   "tiles": {k: f"{t}x{l}" for k, (t, l) in R1["tiles"].items()},
                   "autotune_s": None if R1["tune_s"] is None else round(R1["tune_s"], 2)},
        "roofline": roof,
        "step_hbm_effective_frac": round(b_step / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_algorithmic_bytes_per_cell_level": round(b_step / (C * K), 1),
        "step_hbm_effective_frac_predictor_vn_w_only": round(
            step_algorithmic_bytes_r15(C, E, K, spec["nsub"], r) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": {n: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}
                    for n, d in kernels.items()},
        "diag": {"mass": diag["mass"], "n_nonfinite": diag["n_nonfinite"]},
    }
    if args.precision == "fp64" and not args.no_mixed:
        print("[bench] mixed precision run", file=sys.stderr, flush=True)
        R2 = run("mixed", args.steps, args.warmup, tune)
        ms2, out2, d2 = R2["ms"], R2["out"], R2["diag"]
        errs = {k: float(np.linalg.norm(out2[k] - out[k]) / np.linalg.norm(out[k])) for k in FIELDS}
        b_mix = step_algorithmic_bytes(C, E, K, spec["nsub"], 4)
        line["mixed"] = {"value": C * K * args.steps / (ms2 / 1e3), "ms_per_step": ms2 / args.steps,
                         "step_hbm_effective_frac": round(b_mix / (ms2 / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "speedup_vs_fp64": ms / ms2, "rel_l2_vs_fp64": errs,
                         "after_steps": 2 * args.steps + args.warmup,
                         "stated_bound": {k: mixed_bound(args.workload, k) for k in FIELDS},
                         "within_stated_bound": all(errs[k] <= mixed_bound(args.workload, k) for k in FIELDS),
                         "mass_rel_diff_vs_fp64": d2["mass"] / diag["mass"] - 1.0,
                         "tiles": {k: f"{t}x{l}" for k, (t, l) in R2["tiles"].items()},
                         "kernels": {n: round(1e3 * t / c, 2) for n, (c, t) in R2["prof"].items() if c}}
    if args.theta:
        # the optional theta_v/exner diffusion, same timing: what it adds to a step
        print("[bench] theta_v diffusion run", file=sys.stderr, flush=True)
        R3 = run(args.precision, args.steps, args.warmup, tune, params=D.default_params(diffuse_theta=1))
        line["theta_diffusion"] = {"ms_per_step": R3["ms"] / args.steps, "cost_vs_plain": R3["ms"] / ms,
                                   "diff_cell_vertex2_us": round(1e3 * R3["prof"]["diff_cell_vertex2"][1]
                                                                 / R3["prof"]["diff_cell_vertex2"][0], 2)}
    G.close()
    secondary = "r2b5_k65" if args.workload != "r2b5_k65" else None
    cpu_case = (spec, g0, S0, vert) if secondary is None else None
    # the headline's host copies are no longer needed (R2B8: ~21 GB each)
    del S, S0, out, R1
    if "R2" in locals():
        del R2, out2
    if secondary is not None and not args.no_secondary:
        line["r2b5_k65"] = bench_r2b5(args, D, torch, dev)
    if not args.no_cpu_baseline:
        print("[bench] oracle on the host", file=sys.stderr, flush=True)
        if cpu_case is not None:
            line["cpu_baseline"] = cpu_baseline(*cpu_case)
        else:
            # the oracle on the R2B5 workload: an R2B8 step is beyond the host
            gb, Sb, vb, sb = build_workload(secondary)
            line["cpu_baseline"] = cpu_baseline(sb, gb, Sb, vb)
            line["cpu_baseline"]["sample"] = "R2B5 / 65-level workload (the R2B8 grid is beyond the host): " + \
                line["cpu_baseline"]["sample"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
