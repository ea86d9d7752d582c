"""Python access to the CPU oracle (liboracle_rf.so): TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
import this module.  It compiles ``oracle_rf.c`` with gcc on first use (no GPU,
no HIP, nothing shared with the library under test) and wraps its functions with
NumPy arrays.  Every function follows the readings documented in
``oracle_rf.c``; see that file for the method's steps and citations.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle_rf.c")
LIB = os.path.join(HERE, "liboracle_rf.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]

OK, EINVAL, ERANGE, ENOMEM = 0, -1, -2, -3
LEAF = 255


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what} failed with code {rc}")
        self.rc = rc


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (idempotent unless forced)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "oracle_rf.h"))):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def configure(L):
    """Declare the C signatures on a loaded oracle library and return it."""
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.oracle_philox4x64_10.argtypes = [P, P, P]
    L.oracle_philox4x64_10.restype = None
    L.oracle_rf_bin.argtypes = [P, P, i64, i32, i32, i32, P, P, P]
    L.oracle_rf_bin_apply.argtypes = [P, P, i64, i32, i32, P, P, P]
    L.oracle_rf_y_fixed.argtypes = [P, i64, P]
    L.oracle_rf_fit.argtypes = [P, i64, i32, P, P, P, i64, P, i32, i32, i64, P, P, P, P, P, P, i32]
    L.oracle_rf_predict.argtypes = [P, i64, i32, i32, i64, P, P, P, P, P, P]
    L.oracle_rf_oob.argtypes = [P, i32, P, P, i64, P, i32, i64, P, P, P, P, P, P, P, P, P]
    for f in ("oracle_rf_bin", "oracle_rf_bin_apply", "oracle_rf_y_fixed", "oracle_rf_fit",
              "oracle_rf_predict", "oracle_rf_oob"):
        getattr(L, f).restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = configure(ctypes.CDLL(LIB))
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


class Params(ctypes.Structure):
    _fields_ = [("num_trees", ctypes.c_int32), ("mtry", ctypes.c_int32), ("min_node_size", ctypes.c_int32),
                ("bootstrap", ctypes.c_int32), ("seed", ctypes.c_uint64)]


def philox(counter, key) -> np.ndarray:
    """One Philox4x64-10 block for a 4-word counter and a 2-word key."""
    c = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(_p(c), _p(k), _p(out))
    return out


@dataclass
class Binning:
    thresholds: np.ndarray  # float32 [p, 255]
    n_bins: np.ndarray  # int32 [p + 1]
    codes: np.ndarray  # uint8 [n, p + 1]

    def column_thresholds(self, j: int) -> np.ndarray:
        return self.thresholds[j, : self.n_bins[j] - 1]


def bin(X: np.ndarray, device: np.ndarray, n_devices: int, max_bins: int) -> Binning:
    X = np.ascontiguousarray(X, dtype=np.float32)
    device = np.ascontiguousarray(device, dtype=np.int32)
    n, p = X.shape
    thr = np.zeros((p, 255), dtype=np.float32)
    nb = np.zeros(p + 1, dtype=np.int32)
    codes = np.zeros((n, p + 1), dtype=np.uint8)
    _check(lib().oracle_rf_bin(_p(X), _p(device), n, p, n_devices, max_bins, _p(thr), _p(nb), _p(codes)),
           "oracle_rf_bin")
    return Binning(thr, nb, codes)


def bin_apply(b: Binning, X: np.ndarray, device: np.ndarray, n_devices: int) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    device = np.ascontiguousarray(device, dtype=np.int32)
    n, p = X.shape
    codes = np.zeros((n, p + 1), dtype=np.uint8)
    _check(lib().oracle_rf_bin_apply(_p(X), _p(device), n, p, n_devices, _p(b.thresholds), _p(b.n_bins),
                                     _p(codes)), "oracle_rf_bin_apply")
    return codes


def y_fixed(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(y.shape[0], dtype=np.int64)
    _check(lib().oracle_rf_y_fixed(_p(y), y.shape[0], _p(out)), "oracle_rf_y_fixed")
    return out


@dataclass
class Forest:
    """Trees [tree_begin, tree_end) of one forest, each in a slot of `capacity` nodes."""

    num_trees: int
    tree_begin: int
    capacity: int
    col: np.ndarray
    bin: np.ndarray
    left: np.ndarray
    q: np.ndarray
    N: np.ndarray
    n_nodes: np.ndarray

    def tree(self, t: int) -> dict:
        """Node arrays of tree t (breadth-first order), trimmed to its node count."""
        s = (t - self.tree_begin) * self.capacity
        k = int(self.n_nodes[t - self.tree_begin])
        return {"col": self.col[s:s + k], "bin": self.bin[s:s + k], "left": self.left[s:s + k],
                "q": self.q[s:s + k], "N": self.N[s:s + k]}


def fit(codes: np.ndarray, n_bins: np.ndarray, y: np.ndarray, num_trees: int, mtry: int, min_node_size: int,
        seed: int = 1, bootstrap: bool = True, train_rows: np.ndarray | None = None, trees=None,
        n_threads: int = 0) -> Forest:
    """Grow trees `trees` (a range; default all) of a forest on the given code matrix."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    n, C = codes.shape
    n_bins = np.ascontiguousarray(n_bins, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    tr = None if train_rows is None else np.ascontiguousarray(train_rows, dtype=np.int64)
    n_train = n if tr is None else tr.shape[0]
    if trees is None:
        trees = range(num_trees)
    t0, t1 = trees.start, trees.stop
    cap = max(1, 2 * n_train - 1)
    k = t1 - t0
    col = np.zeros(k * cap, np.uint8)
    bn = np.zeros(k * cap, np.uint8)
    left = np.zeros(k * cap, np.int32)
    q = np.zeros(k * cap, np.int64)
    N = np.zeros(k * cap, np.int32)
    nn = np.zeros(k, np.int64)
    prm = Params(num_trees, mtry, min_node_size, 1 if bootstrap else 0, seed)
    _check(lib().oracle_rf_fit(_p(codes), n, C, _p(n_bins), _p(y), _p(tr), n_train, ctypes.byref(prm), t0, t1,
                               cap, _p(col), _p(bn), _p(left), _p(q), _p(N), _p(nn), n_threads),
           "oracle_rf_fit")
    return Forest(num_trees, t0, cap, col, bn, left, q, N, nn)


def predict(forest: Forest, codes: np.ndarray):
    """(P, yhat): int64 leaf sums over the forest's trees and the forest mean.

    The mean divides by the number of trees held (the whole forest when all trees
    were grown)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    m, C = codes.shape
    k = forest.n_nodes.shape[0]
    P = np.zeros(m, np.int64)
    yhat = np.zeros(m, np.float64)
    _check(lib().oracle_rf_predict(_p(codes), m, C, k, forest.capacity, _p(forest.col), _p(forest.bin),
                                   _p(forest.left), _p(forest.q), _p(P), _p(yhat)), "oracle_rf_predict")
    return P, yhat


def oob(forest: Forest, codes: np.ndarray, y: np.ndarray, mtry: int, min_node_size: int, seed: int = 1,
        bootstrap: bool = True, train_rows: np.ndarray | None = None):
    """Out-of-bag sums, counts and (mse, mae, rows) of a forest grown by fit() over all its trees."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    n, C = codes.shape
    y = np.ascontiguousarray(y, dtype=np.float64)
    tr = None if train_rows is None else np.ascontiguousarray(train_rows, dtype=np.int64)
    n_train = n if tr is None else tr.shape[0]
    assert forest.tree_begin == 0
    k = forest.n_nodes.shape[0]
    P = np.zeros(n_train, np.int64)
    cnt = np.zeros(n_train, np.int32)
    mse, mae, m = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    prm = Params(forest.num_trees, mtry, min_node_size, 1 if bootstrap else 0, seed)
    _check(lib().oracle_rf_oob(_p(codes), C, _p(y), _p(tr), n_train, ctypes.byref(prm), k, forest.capacity,
                               _p(forest.col), _p(forest.bin), _p(forest.left), _p(forest.q), _p(P), _p(cnt),
                               ctypes.byref(mse), ctypes.byref(mae), ctypes.byref(m)), "oracle_rf_oob")
    return P, cnt, (mse.value, mae.value, m.value)


def select_device(forest: Forest, feature_codes: np.ndarray, n_devices: int):
    """Predicted log10 time of every kernel on every device, and the fastest device
    (lowest id on ties): each kernel's feature codes with device code d appended."""
    fc = np.ascontiguousarray(feature_codes, dtype=np.uint8)
    m = fc.shape[0]
    expanded = np.concatenate([np.repeat(fc, n_devices, axis=0),
                               np.tile(np.arange(n_devices, dtype=np.uint8), m)[:, None]], axis=1)
    _, yhat = predict(forest, expanded)
    times = yhat.reshape(m, n_devices)
    return np.argmin(times, axis=1).astype(np.int32), times


def heldout(forest: Forest, codes: np.ndarray, y: np.ndarray, rows: np.ndarray):
    """Held-out leaf sums of the given rows (every tree of the forest) and
    (mse, mae, rows): the mean squared and absolute difference between the
    forest mean and y, accumulated in row order."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.shape[0] == 0:
        return np.zeros(0, np.int64), (0.0, 0.0, 0)
    P, yhat = predict(forest, np.ascontiguousarray(codes[rows]))
    sq = ab = 0.0
    for i in range(rows.shape[0]):
        e = float(yhat[i]) - float(y[rows[i]])
        sq += e * e
        ab += abs(e)
    m = rows.shape[0]
    return P, (sq / m, ab / m, m)


def anneal(objective, lower, upper, start, levels: int, proposals: int, t0: float, cooling: float,
           step_frac: float, seed: int):
    """Simulated annealing over integer triples (num.trees, mtry, min.node.size).

    objective(list of triples) -> list of (value, oob_rows).  The start is scored
    first.  Level l (temperature t0 * cooling^l) draws `proposals` triples around
    the state it starts from, proposal j from Philox block (0, 2, l, j) with key
    (seed, 0): word c moves coordinate c by floor(word * (2h_c + 1) / 2^64) - h_c
    with h_c = max(1, floor(step_frac * (upper_c - lower_c))), clamped to the
    bounds; word 3 gives u = (word >> 11) * 2^-53.  All proposals are scored, then
    taken in order: accepted if not worse than the current value, or if
    u < exp(-(worse by) / T).  Returns (best triple, best value, trace), the best
    being the first evaluation with the lowest value."""
    half = [max(1, math.floor(step_frac * (upper[c] - lower[c]))) for c in range(3)]
    cur = tuple(start)
    f_cur, rows = objective([cur])[0]
    trace = [dict(level=-1, index=0, params=cur, accepted=True, current=cur, oob_rows=rows, objective=f_cur)]
    best, f_best = cur, f_cur
    T = t0
    for level in range(levels):
        base = cur
        props, us = [], []
        for j in range(proposals):
            w = [int(v) for v in philox([0, 2, level, j], [seed, 0])]
            p = []
            for c in range(3):
                step = (w[c] * (2 * half[c] + 1)) >> 64
                p.append(min(upper[c], max(lower[c], base[c] + step - half[c])))
            props.append(tuple(p))
            us.append((w[3] >> 11) * 2.0 ** -53)
        scores = objective(props)
        for j, (p, (f, r)) in enumerate(zip(props, scores)):
            d = f - f_cur
            if T > 0.0:
                accept = d <= 0.0 or us[j] < math.exp(-d / T)
            else:
                accept = d <= 0.0
            if accept:
                cur, f_cur = p, f
            if f < f_best:
                best, f_best = p, f
            trace.append(dict(level=level, index=j, params=p, accepted=accept, current=cur, oob_rows=r, objective=f))
        T *= cooling
    return best, f_best, trace


def oob_objective(codes: np.ndarray, n_bins: np.ndarray, y: np.ndarray, seed: int):
    """The annealing objective: out-of-bag MSE of the forest grown with a triple on all rows."""
    def score(triples):
        out = []
        for nt, mt, mn in triples:
            f = fit(codes, n_bins, y, nt, mt, mn, seed=seed)
            _, _, (mse, _, rows) = oob(f, codes, y, mt, mn, seed=seed)
            out.append((mse, rows))
        return out
    return score


def ranking_accuracy(times: np.ndarray, truth: np.ndarray):
    """How well predicted times rank the devices of each kernel (Sec. VI).

    Sec. VI judges the model as a scheduler would use it: for any pair of devices
    it should name the one on which the kernel runs faster.  For kernel k and
    devices i < j the prediction chooses i when times[k, i] <= times[k, j] (the
    lowest id on a tie, as the device-selection query does) and j otherwise; the
    choice is correct when its true time is strictly the smaller one.  Pairs whose
    true times are equal have no wrong choice and are not counted.  The fastest
    device is hit when the predicted best (the smallest prediction, lowest id on
    ties) has the smallest true time.

    Returns per kernel (int32 correct pairs, int32 counted pairs, int32 top-1 hit)."""
    times = np.asarray(times, dtype=np.float64)
    truth = np.asarray(truth, dtype=np.float64)
    m, D = times.shape
    correct = np.zeros(m, np.int32)
    counted = np.zeros(m, np.int32)
    hit = np.zeros(m, np.int32)
    for k in range(m):
        for i in range(D):
            for j in range(i + 1, D):
                if truth[k, i] == truth[k, j]:
                    continue
                counted[k] += 1
                chosen, other = (i, j) if times[k, i] <= times[k, j] else (j, i)
                if truth[k, chosen] < truth[k, other]:
                    correct[k] += 1
        best = 0
        for d in range(1, D):
            if times[k, d] < times[k, best]:
                best = d
        hit[k] = 1 if truth[k, best] == min(truth[k, d] for d in range(D)) else 0
    return correct, counted, hit
