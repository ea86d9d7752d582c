"""ctypes binding of libaiwc_rf.so (the C ABI in include/aiwc_rf.h).

Argument marshalling only: every step runs in the library's HIP kernels.  Device
arrays are torch tensors on the current HIP device (torch supplies memory and
streams); the default stream argument is torch's current stream.  The function
names are those of the C ABI.  Importing this module fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaiwc_rf.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -4, -5
FIT_FUSED, FIT_PLAIN, FIT_ASYNC, FIT_TUNE = 0, 1, 2, 4
LEAF = 255
MAX_ROWS = 1 << 18

# torch first: the library must bind to the HIP runtime torch already loaded, so
# that device pointers and stream handles mean the same thing on both sides.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")

_L = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i32, _i64, _u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32


class Params(ctypes.Structure):
    """aiwc_rf_params: num.trees, mtry, min.node.size (Sec. III-B), bootstrap, seed."""

    _fields_ = [("num_trees", ctypes.c_int32), ("mtry", ctypes.c_int32), ("min_node_size", ctypes.c_int32),
                ("bootstrap", ctypes.c_int32), ("seed", ctypes.c_uint64)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_L, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("aiwc_rf_bin", [_P, _P, _i64, _i32, _i32, _i32, _P, _P, _P])
_sig("aiwc_rf_binner_from_counts", [_P, _i32, _P])
_sig("aiwc_rf_binner_export_host", [_P, _P, _P, _P, _P])
_sig("aiwc_rf_binner_free", [_P], None)
_sig("aiwc_rf_fit", [_P, _i64, _i32, _P, _P, _P, _P, _P, _i32, _u32, _P, _P])
_sig("aiwc_rf_forest_wait", [_P])
_sig("aiwc_rf_forest_info", [_P, _i32, _P, _P, _P, _P])
_sig("aiwc_rf_forest_tree_sizes", [_P, _i32, _i32, _i32, _P])
_sig("aiwc_rf_forest_stats", [_P, _i32, _P, _P])
_sig("aiwc_rf_forest_launch", [_P, _P])
_sig("aiwc_rf_forest_export_host", [_P, _i32, _i32, _i32, _P, _P, _P, _P, _P])
_sig("aiwc_rf_forest_free", [_P], None)
_sig("aiwc_rf_predict", [_P, _i32, _P, _i64, _P, _P])
_sig("aiwc_rf_predict_noalloc", [_P, _i32, _P, _i64, _P, _P])
_sig("aiwc_rf_predict_sum", [_P, _i32, _i32, _i32, _P, _i64, _P, _P])
_sig("aiwc_rf_select_device", [_P, _i32, _P, _i64, _P, _P, _P])
_sig("aiwc_rf_rank_accuracy", [_P, _P, _i64, _i32, _P, _P, _P, _P])
_sig("aiwc_rf_oob_error", [_P, _i32, _i32, _P, _P, _P, _P, _P, _P, _P, _P])
_sig("aiwc_rf_fit_groups", [_P, _i64, _i32, _P, _P, _P, _P, _P, _i32, _u32, _P, _P])
_sig("aiwc_rf_heldout_error", [_P, _i32, _i32, _P, _P, _P, _P, _P, _P, _P])
_sig("aiwc_rf_heldout_rows", [_P, _i32, _P, _P])
_sig("aiwc_rf_tune_sa", [_P, _i64, _i32, _P, _P, _P, _P, _P, _P, _P])
_sig("aiwc_rf_server_create", [_P, _i32, _i64, _i32, _i32, _P])
_sig("aiwc_rf_server_submit", [_P, _P, _i64, _P, _P])
_sig("aiwc_rf_server_poll", [_P, _P, _P, _i32, _P])
_sig("aiwc_rf_server_drain", [_P])
_sig("aiwc_rf_server_stats", [_P, _P, _P, _P, _P])
_sig("aiwc_rf_server_free", [_P], None)
_sig("aiwc_rf_last_error", [], ctypes.c_char_p)

SYMBOLS = ("aiwc_rf_bin", "aiwc_rf_binner_from_counts", "aiwc_rf_binner_export_host", "aiwc_rf_binner_free",
           "aiwc_rf_fit", "aiwc_rf_forest_wait", "aiwc_rf_forest_info", "aiwc_rf_forest_stats", "aiwc_rf_forest_launch",
           "aiwc_rf_forest_tree_sizes",
           "aiwc_rf_forest_export_host", "aiwc_rf_forest_free", "aiwc_rf_predict", "aiwc_rf_predict_noalloc",
           "aiwc_rf_predict_sum",
           "aiwc_rf_select_device", "aiwc_rf_rank_accuracy", "aiwc_rf_oob_error", "aiwc_rf_fit_groups", "aiwc_rf_heldout_error",
           "aiwc_rf_heldout_rows", "aiwc_rf_tune_sa", "aiwc_rf_server_create", "aiwc_rf_server_submit", "aiwc_rf_server_poll", "aiwc_rf_server_drain",
           "aiwc_rf_server_stats", "aiwc_rf_server_free", "aiwc_rf_last_error")


class LaunchInfo(ctypes.Structure):
    """aiwc_rf_launch_info: the grow kernel's launch shape a fit used."""

    _fields_ = [("block", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("wide_limit", ctypes.c_int32),
                ("big_cols", ctypes.c_int32), ("grid", ctypes.c_int32), ("wide_phase", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("graph_reused", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("task_groups", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class RFError(RuntimeError):
    def __init__(self, rc: int, what: str):
        msg = _L.aiwc_rf_last_error().decode()
        super().__init__(f"{what} failed ({rc}): {msg}")
        self.rc = rc


def _check(rc: int, what: str):
    if rc != OK:
        raise RFError(rc, what)


def _stream(stream):
    import torch

    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, what):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _release(obj, free_name: str):
    """Free a handle from __del__; at interpreter shutdown the library and this
    module's globals may already be gone, and then there is nothing to do."""
    h = getattr(obj, "handle", None)
    if not h:
        return
    obj.handle = None
    try:
        getattr(_L, free_name)(h)
    except Exception:  # shutdown: module globals torn down
        pass


def _host(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Binner:
    """Handle of a fitted binning (thresholds per feature column + bin counts)."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle

    def export(self):
        p, d = ctypes.c_int32(), ctypes.c_int32()
        _check(_L.aiwc_rf_binner_export_host(self.handle, ctypes.byref(p), ctypes.byref(d), None, None),
               "aiwc_rf_binner_export_host")
        nb = np.zeros(p.value + 1, np.int32)
        thr = np.zeros((p.value, 255), np.float32)
        rc = _L.aiwc_rf_binner_export_host(self.handle, None, None, _host(nb), _host(thr))
        if rc != OK:  # counts-only binner
            _check(_L.aiwc_rf_binner_export_host(self.handle, None, None, _host(nb), None),
                   "aiwc_rf_binner_export_host")
            thr = None
        return nb, thr

    @property
    def n_bins(self) -> np.ndarray:
        return self.export()[0]

    def __del__(self, _release=_release):  # (bound now: module globals may be gone at shutdown)
        _release(self, "aiwc_rf_binner_free")


def aiwc_rf_bin(X, device_id, n_devices: int, max_bins: int = 256, binner: Binner | None = None, codes=None,
                stream=None):
    """Bin features X (n x p float32) and device ids (n int32) to codes (n x (p+1) uint8).

    Fits a new binner unless one is given.  Returns (codes, binner)."""
    import torch

    n, p = X.shape
    if codes is None:
        codes = torch.empty((n, p + 1), dtype=torch.uint8, device=X.device)
    h = ctypes.c_void_p(binner.handle.value if binner is not None else None)
    _check(_L.aiwc_rf_bin(_dev(X, torch.float32, "X"), _dev(device_id, torch.int32, "device_id"), n, p, n_devices,
                          max_bins, ctypes.byref(h), _dev(codes, torch.uint8, "codes"), _stream(stream)),
           "aiwc_rf_bin")
    return codes, (binner if binner is not None else Binner(h))


def aiwc_rf_binner_from_counts(n_bins) -> Binner:
    nb = np.ascontiguousarray(n_bins, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(_L.aiwc_rf_binner_from_counts(_host(nb), nb.shape[0], ctypes.byref(h)), "aiwc_rf_binner_from_counts")
    return Binner(h)


class Forest:
    """Handle of one or many fitted forests (device resident)."""

    def __init__(self, handle: ctypes.c_void_p, n_forests: int):
        self.handle = handle
        self.n_forests = n_forests

    def wait(self) -> int:
        return _L.aiwc_rf_forest_wait(self.handle)

    def num_trees(self, forest_index: int = 0) -> int:
        nt = ctypes.c_int32()
        _check(_L.aiwc_rf_forest_info(self.handle, forest_index, None, None, ctypes.byref(nt), None),
               "aiwc_rf_forest_info")
        return nt.value

    def total_nodes(self, forest_index: int = 0) -> int:
        tot = ctypes.c_int64()
        _check(_L.aiwc_rf_forest_info(self.handle, forest_index, None, None, None, ctypes.byref(tot)),
               "aiwc_rf_forest_info")
        return tot.value

    def stats(self, forest_index: int = 0):
        """(work, grow_ms): work = [searched rows, searched nodes, partitioned rows, max levels,
        LDS histogram bin adds]."""
        w = np.zeros(5, np.int64)
        ms = ctypes.c_float()
        _check(_L.aiwc_rf_forest_stats(self.handle, forest_index, _host(w), ctypes.byref(ms)), "aiwc_rf_forest_stats")
        return w, ms.value

    def launch(self) -> dict:
        """The grow kernel's launch shape this fit used (aiwc_rf_forest_launch)."""
        info = LaunchInfo()
        _check(_L.aiwc_rf_forest_launch(self.handle, ctypes.byref(info)), "aiwc_rf_forest_launch")
        return info.as_dict()

    def tree_sizes(self, forest_index: int = 0, tree_begin: int = 0, tree_end: int | None = None) -> np.ndarray:
        if tree_end is None:
            tree_end = self.num_trees(forest_index)
        out = np.zeros(tree_end - tree_begin, np.int64)
        _check(_L.aiwc_rf_forest_tree_sizes(self.handle, forest_index, tree_begin, tree_end, _host(out)),
               "aiwc_rf_forest_tree_sizes")
        return out

    def export(self, forest_index: int = 0, tree_begin: int = 0, tree_end: int | None = None) -> list[dict]:
        """Node arrays (col, bin, left, q, N) of each tree in [tree_begin, tree_end)."""
        if tree_end is None:
            tree_end = self.num_trees(forest_index)
        sizes = self.tree_sizes(forest_index, tree_begin, tree_end)
        tot = int(sizes.sum())
        col = np.zeros(tot, np.uint8)
        bn = np.zeros(tot, np.uint8)
        left = np.zeros(tot, np.int32)
        q = np.zeros(tot, np.int64)
        N = np.zeros(tot, np.int32)
        _check(_L.aiwc_rf_forest_export_host(self.handle, forest_index, tree_begin, tree_end, _host(col), _host(bn),
                                             _host(left), _host(q), _host(N)), "aiwc_rf_forest_export_host")
        out, s = [], 0
        for k in sizes:
            k = int(k)
            out.append({"col": col[s:s + k], "bin": bn[s:s + k], "left": left[s:s + k], "q": q[s:s + k],
                        "N": N[s:s + k]})
            s += k
        return out

    def __del__(self, _release=_release):  # (bound now: module globals may be gone at shutdown)
        _release(self, "aiwc_rf_forest_free")


def make_params(num_trees: int, mtry: int, min_node_size: int, bootstrap: bool = True, seed: int = 1) -> Params:
    return Params(num_trees, mtry, min_node_size, 1 if bootstrap else 0, seed)


def aiwc_rf_fit(codes, binner: Binner, y_log10, params, fold_id=None, heldout_fold=None, flags: int = FIT_FUSED,
                stream=None) -> Forest:
    """Fit one forest (params: a Params) or a grid (params: a sequence of Params, with
    heldout_fold giving each forest's held-out fold id or -1)."""
    import torch

    n, C = codes.shape
    plist = [params] if isinstance(params, Params) else list(params)
    arr = (Params * len(plist))(*plist)
    hf = None
    if heldout_fold is not None:
        hf = np.ascontiguousarray(heldout_fold, dtype=np.int32)
        assert hf.shape[0] == len(plist)
    fp = _dev(fold_id, torch.int8, "fold_id") if fold_id is not None else None
    h = ctypes.c_void_p()
    _check(_L.aiwc_rf_fit(_dev(codes, torch.uint8, "codes"), n, C, binner.handle, _dev(y_log10, torch.float64, "y"),
                          fp, arr, None if hf is None else _host(hf), len(plist), flags, ctypes.byref(h),
                          _stream(stream)), "aiwc_rf_fit")
    return Forest(h, len(plist))


def aiwc_rf_fit_groups(codes, binner: Binner, y_log10, params, group_id, train_mask, flags: int = FIT_FUSED,
                       stream=None) -> Forest:
    """A grid whose forest k trains on the rows whose group (int8 device tensor, -1 =
    always trained on) has its bit set in train_mask[k] (uint64)."""
    import torch

    n, C = codes.shape
    plist = [params] if isinstance(params, Params) else list(params)
    arr = (Params * len(plist))(*plist)
    masks = np.ascontiguousarray(np.asarray(train_mask, dtype=np.uint64))
    assert masks.shape[0] == len(plist)
    h = ctypes.c_void_p()
    _check(_L.aiwc_rf_fit_groups(_dev(codes, torch.uint8, "codes"), n, C, binner.handle,
                                 _dev(y_log10, torch.float64, "y"), _dev(group_id, torch.int8, "group_id"), _host(masks),
                                 arr, len(plist), flags, ctypes.byref(h), _stream(stream)), "aiwc_rf_fit_groups")
    return Forest(h, len(plist))


def aiwc_rf_heldout_rows(forest: Forest, forest_index: int = 0) -> np.ndarray:
    """Row indices (ascending) that forest forest_index holds out."""
    cnt = ctypes.c_int32()
    _check(_L.aiwc_rf_heldout_rows(forest.handle, forest_index, None, ctypes.byref(cnt)), "aiwc_rf_heldout_rows")
    rows = np.zeros(cnt.value, np.int32)
    if cnt.value:
        _check(_L.aiwc_rf_heldout_rows(forest.handle, forest_index, _host(rows), ctypes.byref(cnt)),
               "aiwc_rf_heldout_rows")
    return rows


@dataclass
class HeldoutResult:
    sums: object  # int64 device tensor: leaf sums per held-out row (forests in turn), or None
    mse: np.ndarray  # per forest
    mae: np.ndarray
    rows: np.ndarray


def aiwc_rf_heldout_error(forest: Forest, codes, y_log10, forest_begin: int = 0, forest_end: int | None = None,
                          n_heldout=None, stream=None) -> HeldoutResult:
    """Held-out predictions and errors of forests [forest_begin, forest_end).

    n_heldout: total held-out rows of those forests (sizes the per-row sums); when
    omitted the sums are not returned."""
    import torch

    if forest_end is None:
        forest_end = forest.n_forests
    nf = forest_end - forest_begin
    mse = np.zeros(nf)
    mae = np.zeros(nf)
    rows = np.zeros(nf, np.int64)
    sums = None
    if n_heldout is not None:
        sums = torch.empty(max(int(n_heldout), 1), dtype=torch.int64, device=codes.device)
    _check(_L.aiwc_rf_heldout_error(forest.handle, forest_begin, forest_end, _dev(codes, torch.uint8, "codes"),
                                    _dev(y_log10, torch.float64, "y"),
                                    None if sums is None else _dev(sums, torch.int64, "sums"),
                                    _host(mse), _host(mae), _host(rows), _stream(stream)), "aiwc_rf_heldout_error")
    if sums is not None:
        sums = sums[:int(n_heldout)]
    return HeldoutResult(sums, mse, mae, rows)


class SAConfig(ctypes.Structure):
    _fields_ = [("lower", ctypes.c_int32 * 3), ("upper", ctypes.c_int32 * 3), ("start", ctypes.c_int32 * 3),
                ("levels", ctypes.c_int32), ("proposals", ctypes.c_int32), ("t0", ctypes.c_double),
                ("cooling", ctypes.c_double), ("step_frac", ctypes.c_double), ("seed", ctypes.c_uint64)]


class SAStep(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("index", ctypes.c_int32), ("params", ctypes.c_int32 * 3),
                ("accepted", ctypes.c_int32), ("current", ctypes.c_int32 * 3), ("oob_rows", ctypes.c_int64),
                ("objective", ctypes.c_double)]


def sa_config(lower, upper, start, levels: int, proposals: int, t0: float, cooling: float, step_frac: float,
              seed: int = 1) -> SAConfig:
    c = SAConfig()
    c.lower[:] = list(lower)
    c.upper[:] = list(upper)
    c.start[:] = list(start)
    c.levels, c.proposals, c.t0, c.cooling, c.step_frac, c.seed = levels, proposals, t0, cooling, step_frac, seed
    return c


def aiwc_rf_tune_sa(codes, binner: Binner, y_log10, cfg: SAConfig, stream=None):
    """Annealing search of (num.trees, mtry, min.node.size) by out-of-bag MSE:
    (best triple, best objective, list of trace dicts in evaluation order)."""
    import torch

    n, C = codes.shape
    best = (ctypes.c_int32 * 3)()
    best_f = ctypes.c_double()
    trace = (SAStep * (1 + cfg.levels * cfg.proposals))()
    _check(_L.aiwc_rf_tune_sa(_dev(codes, torch.uint8, "codes"), n, C, binner.handle, _dev(y_log10, torch.float64, "y"),
                              ctypes.byref(cfg), best, ctypes.byref(best_f), trace, _stream(stream)), "aiwc_rf_tune_sa")
    steps = [{"level": t.level, "index": t.index, "params": tuple(t.params), "accepted": bool(t.accepted),
              "current": tuple(t.current), "oob_rows": t.oob_rows, "objective": t.objective} for t in trace]
    return tuple(best), best_f.value, steps


def aiwc_rf_predict(forest: Forest, codes, forest_index: int = 0, out=None, stream=None):
    """Predicted log10 execution time of each row of codes (float64 device tensor)."""
    import torch

    n = codes.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=codes.device)
    _check(_L.aiwc_rf_predict(forest.handle, forest_index, _dev(codes, torch.uint8, "codes"), n,
                              _dev(out, torch.float64, "out"), _stream(stream)), "aiwc_rf_predict")
    return out


def aiwc_rf_predict_noalloc(forest: Forest, codes, out, forest_index: int = 0, stream=None):
    """aiwc_rf_predict without any device allocation (n <= 2^20 rows; out is a
    caller-owned float64 device tensor).  Overlapping calls on one GPU race."""
    import torch

    n = codes.shape[0]
    assert out.shape[0] == n
    _check(_L.aiwc_rf_predict_noalloc(forest.handle, forest_index, _dev(codes, torch.uint8, "codes"), n,
                                      _dev(out, torch.float64, "out"), _stream(stream)), "aiwc_rf_predict_noalloc")
    return out


def aiwc_rf_predict_sum(forest: Forest, codes, tree_begin: int, tree_end: int, forest_index: int = 0, out=None,
                        stream=None):
    """Exact int64 sums of leaf values over trees [tree_begin, tree_end)."""
    import torch

    n = codes.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=codes.device)
    _check(_L.aiwc_rf_predict_sum(forest.handle, forest_index, tree_begin, tree_end,
                                  _dev(codes, torch.uint8, "codes"), n, _dev(out, torch.int64, "out"),
                                  _stream(stream)), "aiwc_rf_predict_sum")
    return out


@dataclass
class OobResult:
    sums: object  # int64 device tensor: out-of-bag leaf sums per training row (forests in turn)
    counts: object  # int32 device tensor: out-of-bag trees per training row
    mse: np.ndarray  # per forest
    mae: np.ndarray
    rows: np.ndarray


def aiwc_rf_oob_error(forest: Forest, codes, y_log10, forest_begin: int = 0, forest_end: int | None = None,
                      n_train=None, stream=None) -> OobResult:
    """Out-of-bag predictions and errors of forests [forest_begin, forest_end).

    n_train: total training rows of those forests (sizes the per-row outputs); when
    omitted the per-row outputs are not returned."""
    import torch

    if forest_end is None:
        forest_end = forest.n_forests
    nf = forest_end - forest_begin
    mse = np.zeros(nf)
    mae = np.zeros(nf)
    rows = np.zeros(nf, np.int64)
    sums = counts = None
    if n_train is not None:
        sums = torch.empty(n_train, dtype=torch.int64, device=codes.device)
        counts = torch.empty(n_train, dtype=torch.int32, device=codes.device)
    _check(_L.aiwc_rf_oob_error(forest.handle, forest_begin, forest_end, _dev(codes, torch.uint8, "codes"),
                                _dev(y_log10, torch.float64, "y"),
                                None if sums is None else _dev(sums, torch.int64, "sums"),
                                None if counts is None else _dev(counts, torch.int32, "counts"),
                                _host(mse), _host(mae), _host(rows), _stream(stream)), "aiwc_rf_oob_error")
    return OobResult(sums, counts, mse, mae, rows)


def aiwc_rf_select_device(forest: Forest, feature_codes, forest_index: int = 0, n_devices: int | None = None,
                          times=None, best=None, stream=None):
    """Fastest device per kernel from its feature codes alone: (best int32[m], times float64[m, D])."""
    import torch

    m = feature_codes.shape[0]
    if n_devices is None:
        raise ValueError("n_devices (the device column's bin count) is required to size the outputs")
    if times is None:
        times = torch.empty((m, n_devices), dtype=torch.float64, device=feature_codes.device)
    if best is None:
        best = torch.empty(m, dtype=torch.int32, device=feature_codes.device)
    _check(_L.aiwc_rf_select_device(forest.handle, forest_index, _dev(feature_codes, torch.uint8, "feature_codes"), m,
                                    _dev(times, torch.float64, "times"), _dev(best, torch.int32, "best"),
                                    _stream(stream)), "aiwc_rf_select_device")
    return best, times


@dataclass
class RankAccuracy:
    correct: object  # int32 device tensor [m]: device pairs ranked right per kernel
    counted: object  # int32 device tensor [m]: pairs with different true times
    hit: object  # int32 device tensor [m]: 1 when the predicted fastest device is a truly fastest one

    @property
    def pairwise(self) -> float:
        """Share of all counted device pairs, over every kernel, ranked right."""
        return float(self.correct.sum().item()) / max(1, int(self.counted.sum().item()))

    @property
    def top1(self) -> float:
        """Share of kernels whose fastest device was predicted."""
        return float(self.hit.double().mean().item()) if self.hit.numel() else 0.0


def aiwc_rf_rank_accuracy(times, truth, stream=None) -> RankAccuracy:
    """Sec. VI's pairwise device-ranking accuracy of predicted times (m x D float64
    device tensor) against true times of the same shape."""
    import torch

    m, D = times.shape
    assert tuple(truth.shape) == (m, D)
    out = [torch.empty(m, dtype=torch.int32, device=times.device) for _ in range(3)]
    _check(_L.aiwc_rf_rank_accuracy(_dev(times, torch.float64, "times"), _dev(truth, torch.float64, "truth"), m, D,
                                    *[_dev(o, torch.int32, "out") for o in out], _stream(stream)),
           "aiwc_rf_rank_accuracy")
    return RankAccuracy(*out)


@dataclass
class ServerStats:
    rows: int
    batches: int
    peak_bytes: int
    memory_waits: int


class Server:
    """aiwc_rf_server_*: continuous-batching prediction server over a resident forest."""

    def __init__(self, forest: Forest, forest_index: int = 0, memory_budget_bytes: int = 1 << 28,
                 max_batch_rows: int = 1 << 16, n_streams: int = 4):
        self.forest = forest  # keeps the forest alive
        self.handle = ctypes.c_void_p()
        _check(_L.aiwc_rf_server_create(forest.handle, forest_index, memory_budget_bytes, max_batch_rows, n_streams,
                                        ctypes.byref(self.handle)), "aiwc_rf_server_create")
        self._keep = {}

    def submit(self, codes: np.ndarray, out: np.ndarray) -> int:
        """Queue rows (uint8 n x C host array); results land in out (float64[n])."""
        assert codes.dtype == np.uint8 and codes.flags.c_contiguous
        assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape[0] == codes.shape[0]
        t = ctypes.c_int64()
        _check(_L.aiwc_rf_server_submit(self.handle, _host(codes), codes.shape[0], _host(out), ctypes.byref(t)),
               "aiwc_rf_server_submit")
        self._keep[t.value] = (codes, out)
        return t.value

    def poll(self, max_tickets: int = 4096):
        tk = np.zeros(max_tickets, np.int64)
        lat = np.zeros(max_tickets, np.float64)
        nd = ctypes.c_int32()
        _check(_L.aiwc_rf_server_poll(self.handle, _host(tk), _host(lat), max_tickets, ctypes.byref(nd)),
               "aiwc_rf_server_poll")
        k = nd.value
        for t in tk[:k]:
            self._keep.pop(int(t), None)
        return tk[:k].copy(), lat[:k].copy()

    def drain(self):
        _check(_L.aiwc_rf_server_drain(self.handle), "aiwc_rf_server_drain")

    def stats(self) -> ServerStats:
        r, b, p, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_L.aiwc_rf_server_stats(self.handle, ctypes.byref(r), ctypes.byref(b), ctypes.byref(p),
                                       ctypes.byref(w)), "aiwc_rf_server_stats")
        return ServerStats(r.value, b.value, p.value, w.value)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _L.aiwc_rf_server_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals torn down
            pass
