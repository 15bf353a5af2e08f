"""Thin ctypes binding of libdycore.so (argument marshalling only).

Every step of the time step runs in the library's HIP kernels; PyTorch only
provides device memory (the borrowed field buffers and the workspace) and the
current HIP stream.  Importing this module fails loudly when the library is
not built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdycore.so")

DC_OK, DC_EINVAL, DC_EGRID, DC_EHIP, DC_ENOMEM, DC_ENONFINITE, DC_EBUSY, DC_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
PREC = {"fp64": 0, "mixed": 1}
DIFF = {"plain": 0, "surrogate": 1, "none": 2}
FIELDS = ("vn", "w", "rho", "exner", "theta_v")
# parts of a step (dc_dycore_part) and the predictor's workspace fields (dc_state_read_work)
PARTS = {"predictor": 0, "corrector": 1, "diffusion": 2}
WORK = {"vn_pred": 0, "y": 1, "w_pred": 2, "t_w": 3, "div": 4}
# kernel ids of the per-kernel profile, and the five launch-tile families
KERNELS = ("vort_ke_pred", "edge_pred", "column_pred", "vort_ke_corr", "edge_corr", "column_corr", "diff_vertex",
           "diff_div", "diff_edge1", "diff_cell_vertex2", "diff_edge2", "edge_upwind")
TILE_FAMILIES = ("vort_ke", "edge", "diff_vertex", "diff_cell", "diff_edge")
TABLES = ("e2c", "c2e", "e2v", "c2e2c", "c2v", "v2e", "v2c", "e2c2e", "e2c2v", "perm_cell", "perm_edge", "perm_vert")

_p = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
MLP_NPARAMS = 5441
MLP_NFEATURES = 18


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int32), ("n_edges", ctypes.c_int32), ("n_verts", ctypes.c_int32), ("n_lev", ctypes.c_int32),
        ("e2c", _i32p), ("c2e", _i32p), ("e2v", _i32p), ("c2e2c", _i32p),
        ("vert_xyz", _f64p), ("cell_xyz", _f64p), ("edge_xyz", _f64p),
        ("edge_length", _f64p), ("dual_edge_length", _f64p),
        ("cell_area", _f64p), ("dual_area", _f64p),
        ("edge_normal_xyz", _f64p),
        ("z_half", _f64p),
        ("exner_ref_full", _f64p), ("theta_ref_full", _f64p),
        ("theta_ref_half", _f64p), ("dexner_dz_ref_half", _f64p),
        ("radius", ctypes.c_double),
        ("sfc_reorder", ctypes.c_int32),
    ]


class GridInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("n_cells", "n_edges", "n_verts", "n_lev", "cell_stride", "edge_stride", "vert_stride",
                 "fused_edge_pass")]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("eta", "adv_w0", "adv_w1", "divdamp_c4", "rayleigh_tau0", "rayleigh_zfrac", "smag_cs",
                 "smag_cap", "hdiff_k4", "rd", "cpd", "cvd", "omega")] + [
        ("diffuse_w", ctypes.c_int32), ("check_finite", ctypes.c_int32), ("diffuse_theta", ctypes.c_int32),
        ("theta_enh_nlev", ctypes.c_int32), ("theta_enh_thresh", ctypes.c_double),
        ("miura", ctypes.c_int32), ("vt_rbf", ctypes.c_int32)]


class Fields(ctypes.Structure):
    _fields_ = [(n, _p) for n in FIELDS]


class Diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("theta_mass", ctypes.c_double), ("max_abs_w", ctypes.c_double),
                ("max_abs_vn", ctypes.c_double), ("n_nonfinite", ctypes.c_int64),
                ("fallback_fraction", ctypes.c_double)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("epochs", ctypes.c_int32), ("lr0", ctypes.c_double),
                ("lr1", ctypes.c_double), ("seed", ctypes.c_uint64), ("shuffle", ctypes.c_int32),
                ("augment", ctypes.c_int32)]


class SurrogateInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("judge_steps", ctypes.c_int64), ("judge_flagged", ctypes.c_int64),
                ("range_flagged", ctypes.c_int64), ("fallback", ctypes.c_int64), ("fallback_total", ctypes.c_int64),
                ("n_columns", ctypes.c_int64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("calls", ctypes.c_int64), ("total_ms", ctypes.c_double)]


def _hip_runtimes() -> set:
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return set()


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or python -m paper_2608_21150_amd.build")
    # PyTorch ships its own HIP runtime with the same soname as the system
    # one.  Loading torch first makes this library bind to that copy, so the
    # process holds a single runtime; two runtimes cannot share the device.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise RuntimeError("two HIP runtimes are loaded (%s): import torch before any other HIP library"
                           % ", ".join(sorted(rts)))
    sig = {
        "dc_last_error": (ctypes.c_char_p, []),
        "dc_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
        "dc_grid_create": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(_p)]),
        "dc_grid_info_get": (ctypes.c_int, [_p, ctypes.POINTER(GridInfo)]),
        "dc_grid_table": (ctypes.c_int, [_p, ctypes.c_int32, _i32p, ctypes.c_size_t]),
        "dc_grid_destroy": (ctypes.c_int, [_p]),
        "dc_field_bytes": (ctypes.c_int, [_p, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
        "dc_state_workspace_bytes": (ctypes.c_int, [_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
        "dc_state_workspace_bytes_params": (ctypes.c_int, [_p, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int,
                                                           ctypes.POINTER(ctypes.c_size_t)]),
        "dc_state_create": (ctypes.c_int, [_p, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int, Fields, Fields, _p,
                                           ctypes.c_size_t, _p, ctypes.POINTER(_p)]),
        "dc_state_current": (ctypes.c_int, [_p, ctypes.POINTER(ctypes.c_int32)]),
        "dc_state_read": (ctypes.c_int, [_p, ctypes.c_int32, _f64p, ctypes.c_size_t]),
        "dc_state_write": (ctypes.c_int, [_p, ctypes.c_int32, _f64p, ctypes.c_size_t]),
        "dc_dycore_step": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32]),
        "dc_dycore_part": (ctypes.c_int, [_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32]),
        "dc_state_read_work": (ctypes.c_int, [_p, ctypes.c_int32, _f64p, ctypes.c_size_t]),
        "dc_diag_conservation": (ctypes.c_int, [_p, ctypes.POINTER(Diag)]),
        "dc_state_destroy": (ctypes.c_int, [_p]),
        "dc_state_profile": (ctypes.c_int, [_p, ctypes.c_int32]),
        "dc_state_profile_select": (ctypes.c_int, [_p, ctypes.c_uint32]),
        "dc_state_autotune": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32]),
        "dc_state_tiles": (ctypes.c_int, [_p, _i32p, ctypes.c_int32]),
        "dc_state_profile_read": (ctypes.c_int, [_p, ctypes.POINTER(KernelStat), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_int32)]),
        "dc_ensemble_create": (ctypes.c_int, [ctypes.POINTER(_p), ctypes.c_int32, ctypes.POINTER(_p)]),
        "dc_ensemble_step": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32]),
        "dc_ensemble_destroy": (ctypes.c_int, [_p]),
        "dc_ensemble_step_eager": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32]),
        "dc_ensemble_step_noalloc": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32]),
        "dc_ensemble_autotune": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32, ctypes.c_char_p]),
        "dc_ensemble_schedule": (ctypes.c_int, [_p, ctypes.c_char_p, ctypes.c_size_t]),
        "dc_mlp_create": (ctypes.c_int, [ctypes.c_uint64, ctypes.POINTER(_p)]),
        "dc_mlp_destroy": (ctypes.c_int, [_p]),
        "dc_mlp_get_params": (ctypes.c_int, [_p, _f32p, ctypes.c_int64]),
        "dc_mlp_set_params": (ctypes.c_int, [_p, _f32p, ctypes.c_int64]),
        "dc_mlp_set_norm": (ctypes.c_int, [_p, _f32p, _f32p, _f32p, _f32p, ctypes.c_float]),
        "dc_mlp_get_norm": (ctypes.c_int, [_p, _f32p, ctypes.c_int64]),
        "dc_mlp_fit_norm": (ctypes.c_int, [_p, _p, ctypes.c_int64, ctypes.c_int64]),
        "dc_mlp_train": (ctypes.c_int, [_p, _p, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(TrainCfg)]),
        "dc_mlp_loss_trace": (ctypes.c_int, [_p, _f32p, ctypes.c_int64, _i64p]),
        "dc_mlp_forward": (ctypes.c_int, [_p, _f32p, ctypes.c_int64, _f32p]),
        "dc_mlp_grad": (ctypes.c_int, [_p, _f32p, _f32p, ctypes.c_int64, _f32p, _f32p]),
        "dc_state_set_mlp": (ctypes.c_int, [_p, _p, ctypes.c_double, ctypes.c_int32]),
        "dc_surrogate_stats": (ctypes.c_int, [_p, ctypes.POINTER(SurrogateInfo)]),
        "dc_surrogate_collect": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                                _p, ctypes.c_int64, ctypes.c_int64, _i64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class DycoreError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dycore error {code}: {msg}")
        self.code = code


def check(rc):
    if rc != DC_OK:
        raise DycoreError(rc, lib.dc_last_error().decode())


def default_params(**overrides) -> Params:
    p = Params()
    check(lib.dc_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


class Grid:
    """Host description of an icosahedral grid plus its vertical column."""

    def __init__(self, grid: dict, vert: dict, sfc: bool = False):
        keep = []

        def I(name):
            a, p = _i32(grid[name])
            keep.append(a)
            return p

        def F(arr):
            a, p = _f64(arr)
            keep.append(a)
            return p

        d = GridDesc()
        d.n_cells, d.n_edges, d.n_verts = grid["n_cells"], grid["n_edges"], grid["n_verts"]
        d.n_lev = len(vert["z_half"]) - 1
        d.e2c, d.c2e, d.e2v, d.c2e2c = I("e2c"), I("c2e"), I("e2v"), I("c2e2c")
        for name in ("vert_xyz", "cell_xyz", "edge_xyz", "edge_length", "dual_edge_length", "cell_area",
                     "dual_area", "edge_normal_xyz"):
            setattr(d, name, F(grid[name]))
        for name in ("z_half", "exner_ref_full", "theta_ref_full", "theta_ref_half", "dexner_dz_ref_half"):
            setattr(d, name, F(vert[name]))
        d.radius = grid["radius"]
        d.sfc_reorder = 1 if sfc else 0
        h = _p()
        check(lib.dc_grid_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        info = GridInfo()
        check(lib.dc_grid_info_get(h, ctypes.byref(info)))
        self.info = {n: getattr(info, n) for n, _ in GridInfo._fields_}

    def table(self, name: str) -> np.ndarray:
        i = self.info
        shape = {"e2c": (i["n_edges"], 2), "c2e": (i["n_cells"], 3), "e2v": (i["n_edges"], 2),
                 "c2e2c": (i["n_cells"], 3), "c2v": (i["n_cells"], 3), "v2e": (i["n_verts"], 6),
                 "v2c": (i["n_verts"], 6), "e2c2e": (i["n_edges"], 4), "e2c2v": (i["n_edges"], 4),
                 "perm_cell": (i["n_cells"],), "perm_edge": (i["n_edges"],), "perm_vert": (i["n_verts"],)}[name]
        out = np.empty(shape, dtype=np.int32)
        check(lib.dc_grid_table(self.handle, TABLES.index(name), out.ctypes.data_as(_i32p), out.size))
        return out

    def close(self):
        if self.handle:
            check(lib.dc_grid_destroy(self.handle))
            self.handle = None


class State:
    """A prognostic state on the GPU over torch-owned device buffers."""

    def __init__(self, grid: Grid, precision: str = "fp64", diffusion: str = "plain", params: Params | None = None,
                 device=None, stream=None):
        import torch

        self.torch = torch
        self.grid = grid
        self.precision = precision
        self.diffusion = diffusion
        dev = torch.device(device if device is not None else "cuda")
        self.device = dev
        prec = PREC[precision]
        self.bufs = []
        for _ in range(2):
            b = {}
            for fi, name in enumerate(FIELDS):
                nb = ctypes.c_size_t()
                check(lib.dc_field_bytes(grid.handle, prec, fi, ctypes.byref(nb)))
                b[name] = torch.zeros(nb.value, dtype=torch.uint8, device=dev)
            self.bufs.append(b)
        self.params = params if params is not None else default_params()
        nb = ctypes.c_size_t()
        check(lib.dc_state_workspace_bytes_params(grid.handle, ctypes.byref(self.params), prec, DIFF[diffusion],
                                                  ctypes.byref(nb)))
        self.workspace = torch.zeros(nb.value, dtype=torch.uint8, device=dev)
        fa = Fields(*[self.bufs[0][n].data_ptr() for n in FIELDS])
        fb = Fields(*[self.bufs[1][n].data_ptr() for n in FIELDS])
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        h = _p()
        check(lib.dc_state_create(grid.handle, ctypes.byref(self.params), prec, DIFF[diffusion], fa, fb,
                                  self.workspace.data_ptr(), self.workspace.numel(), _p(stream.cuda_stream),
                                  ctypes.byref(h)))
        self.handle = h

    def write(self, state: dict):
        for fi, name in enumerate(FIELDS):
            a, p = _f64(state[name])
            check(lib.dc_state_write(self.handle, fi, p, a.size))

    def read(self) -> dict:
        K = self.grid.info["n_lev"]
        nc, ne = self.grid.info["n_cells"], self.grid.info["n_edges"]
        shapes = {"vn": (K, ne), "w": (K + 1, nc), "rho": (K, nc), "exner": (K, nc), "theta_v": (K, nc)}
        out = {}
        for fi, name in enumerate(FIELDS):
            a = np.empty(shapes[name], dtype=np.float64)
            check(lib.dc_state_read(self.handle, fi, a.ctypes.data_as(_f64p), a.size))
            out[name] = a
        return out

    def step(self, dt: float, nsub: int):
        check(lib.dc_dycore_step(self.handle, float(dt), int(nsub)))

    def part(self, name: str, dt: float, nsub: int):
        """One part of a step: "predictor", "corrector" or "diffusion"."""
        check(lib.dc_dycore_part(self.handle, PARTS[name], float(dt), int(nsub)))

    def read_work(self, name: str) -> np.ndarray:
        """A workspace field of the last predictor part: "vn_pred", "y",
        "w_pred", "t_w" or "div" (FP64, unpadded, original numbering)."""
        K = self.grid.info["n_lev"]
        nc, ne = self.grid.info["n_cells"], self.grid.info["n_edges"]
        shape = {"vn_pred": (K, ne), "y": (K, ne), "w_pred": (K + 1, nc), "t_w": (K + 1, nc), "div": (K, nc)}[name]
        a = np.empty(shape, dtype=np.float64)
        check(lib.dc_state_read_work(self.handle, WORK[name], a.ctypes.data_as(_f64p), a.size))
        return a

    def current(self) -> int:
        w = ctypes.c_int32()
        check(lib.dc_state_current(self.handle, ctypes.byref(w)))
        return w.value

    def diag(self) -> dict:
        d = Diag()
        check(lib.dc_diag_conservation(self.handle, ctypes.byref(d)))
        return {n: getattr(d, n) for n, _ in Diag._fields_}

    def set_mlp(self, mlp: "Mlp", threshold: float = 1e-3, judge_every: int = 10):
        check(lib.dc_state_set_mlp(self.handle, mlp.handle, float(threshold), int(judge_every)))
        self._mlp = mlp  # keep the network alive while the state uses it

    def surrogate_stats(self) -> dict:
        info = SurrogateInfo()
        check(lib.dc_surrogate_stats(self.handle, ctypes.byref(info)))
        return {n: getattr(info, n) for n, _ in SurrogateInfo._fields_}

    def collect(self, dt: float, nsub: int, seed: int, n_samples: int, buf, offset: int = 0,
                return_index: bool = False):
        """One plain step recording n_samples (features, tendency) pairs into
        columns offset.. of buf, a float32 device tensor of shape (19, stride)."""
        assert buf.dtype == self.torch.float32 and buf.dim() == 2 and buf.shape[0] == 19 and buf.is_contiguous()
        idx = np.empty(n_samples, dtype=np.int64) if return_index else None
        check(lib.dc_surrogate_collect(self.handle, float(dt), int(nsub), int(seed), int(n_samples), buf.data_ptr(),
                                       buf.shape[1], int(offset),
                                       idx.ctypes.data_as(_i64p) if idx is not None else None))
        return idx

    def profile(self, enable: bool):
        check(lib.dc_state_profile(self.handle, 1 if enable else 0))

    def profile_select(self, kernels=None):
        """Record only the named kernels (names as profile_read reports them); None: all."""
        mask = 0
        if kernels is not None:
            for k in kernels:
                mask |= 1 << KERNELS.index(k)
        check(lib.dc_state_profile_select(self.handle, mask))

    def autotune(self, dt: float, nsub: int):
        """Time candidate launch tiles with trial steps; the state's fields are restored."""
        check(lib.dc_state_autotune(self.handle, dt, nsub))

    def tiles(self) -> dict:
        out = np.zeros(10, dtype=np.int32)
        check(lib.dc_state_tiles(self.handle, out.ctypes.data_as(_i32p), out.size))
        return {name: (int(out[2 * i]), int(out[2 * i + 1])) for i, name in enumerate(TILE_FAMILIES)}

    def profile_read(self) -> dict:
        arr = (KernelStat * 32)()
        n = ctypes.c_int32()
        check(lib.dc_state_profile_read(self.handle, arr, 32, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].calls, arr[i].total_ms) for i in range(n.value)}

    def close(self):
        if self.handle:
            check(lib.dc_state_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Members stepped together by one graph launch per step (batched kernels)."""

    def __init__(self, members):
        self.members = list(members)
        arr = (_p * len(self.members))(*[m.handle for m in self.members])
        h = _p()
        check(lib.dc_ensemble_create(arr, len(self.members), ctypes.byref(h)))
        self.handle = h

    def step(self, dt: float, nsub: int, eager: bool = False):
        fn = lib.dc_ensemble_step_eager if eager else lib.dc_ensemble_step
        check(fn(self.handle, float(dt), int(nsub)))

    def step_noalloc(self, dt: float, nsub: int):
        """The eager step with its work tables in the library's static device
        array (no device allocation; synchronising)."""
        check(lib.dc_ensemble_step_noalloc(self.handle, float(dt), int(nsub)))

    def autotune(self, dt: float, nsub: int, cache_path: str | None = None):
        check(lib.dc_ensemble_autotune(self.handle, float(dt), int(nsub),
                                       cache_path.encode() if cache_path else None))

    def schedule(self) -> str:
        buf = ctypes.create_string_buffer(512)
        check(lib.dc_ensemble_schedule(self.handle, buf, 512))
        return buf.value.decode()

    def close(self):
        if self.handle:
            check(lib.dc_ensemble_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The diffusion surrogate network: FP32 master weights on the GPU."""

    def __init__(self, seed: int = 0):
        h = _p()
        check(lib.dc_mlp_create(int(seed), ctypes.byref(h)))
        self.handle = h

    def params(self) -> np.ndarray:
        a = np.empty(MLP_NPARAMS, dtype=np.float32)
        check(lib.dc_mlp_get_params(self.handle, a.ctypes.data_as(_f32p), a.size))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        check(lib.dc_mlp_set_params(self.handle, a.ctypes.data_as(_f32p), a.size))

    def set_norm(self, mean, std, fmin, fmax, target_std: float):
        arrs = [np.ascontiguousarray(x, dtype=np.float32) for x in (mean, std, fmin, fmax)]
        check(lib.dc_mlp_set_norm(self.handle, *[x.ctypes.data_as(_f32p) for x in arrs], float(target_std)))

    def norm(self) -> dict:
        a = np.empty(4 * MLP_NFEATURES + 1, dtype=np.float32)
        check(lib.dc_mlp_get_norm(self.handle, a.ctypes.data_as(_f32p), a.size))
        F = MLP_NFEATURES
        return {"mean": a[:F], "std": a[F:2 * F], "min": a[2 * F:3 * F], "max": a[3 * F:4 * F], "target_std": a[4 * F]}

    def fit_norm(self, buf, n: int):
        check(lib.dc_mlp_fit_norm(self.handle, buf.data_ptr(), buf.shape[1], int(n)))

    def train(self, buf, n: int, batch: int = 4096, epochs: int = 2, lr0: float = 1e-3, lr1: float = 1e-5,
              seed: int = 0, shuffle: bool = True, augment: bool = True) -> np.ndarray:
        cfg = TrainCfg(batch, epochs, lr0, lr1, seed, 1 if shuffle else 0, 1 if augment else 0)
        check(lib.dc_mlp_train(self.handle, buf.data_ptr(), buf.shape[1], int(n), ctypes.byref(cfg)))
        cnt = ctypes.c_int64()
        check(lib.dc_mlp_loss_trace(self.handle, None, 0, ctypes.byref(cnt)))
        tr = np.empty(cnt.value, dtype=np.float32)
        check(lib.dc_mlp_loss_trace(self.handle, tr.ctypes.data_as(_f32p), tr.size, ctypes.byref(cnt)))
        return tr

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty(x.shape[0], dtype=np.float32)
        check(lib.dc_mlp_forward(self.handle, x.ctypes.data_as(_f32p), x.shape[0], y.ctypes.data_as(_f32p)))
        return y

    def grad(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.empty(MLP_NPARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        check(lib.dc_mlp_grad(self.handle, x.ctypes.data_as(_f32p), t.ctypes.data_as(_f32p), x.shape[0],
                              g.ctypes.data_as(_f32p), ctypes.byref(loss)))
        return g, loss.value

    def close(self):
        if self.handle:
            check(lib.dc_mlp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_pack(p: dict) -> np.ndarray:
    """Flatten a parameter dict (w1, b1, w2, b2, w3, b3) in the library's order."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1)
                           for k in ("w1", "b1", "w2", "b2", "w3", "b3")]).astype(np.float32)


def mlp_unpack(a) -> dict:
    a = np.asarray(a)
    F, H = MLP_NFEATURES, 64
    o = np.cumsum([0, F * H, H, H * H, H, H, 1])
    return {"w1": a[o[0]:o[1]].reshape(F, H), "b1": a[o[1]:o[2]], "w2": a[o[2]:o[3]].reshape(H, H),
            "b2": a[o[3]:o[4]], "w3": a[o[4]:o[5]], "b3": a[o[5]:o[6]]}
