"""Benchmark of the random-forest performance model on one MI355X.

python bench.py [--steps K] [--warmup W] [--workload c4|c1|c2|c3|c5|studies|tune|lds|copy]

The default workload is the tuning grid (c4), on which the headline metric is
quoted: one step fits all 1700 forests in one fused graph launch (the timed
value) and then again as one launch sequence per forest (the plain comparison).
For the single-forest workloads one step is one pass of the whole hot path over
one batch of synthetic input that is already resident in device memory:
quantile binning of the feature matrix, the forest fit (fixed-point response,
bootstrap, per-node mtry draw, histogram and split search, partition, leaves)
and the prediction of every row.  Launch shapes are the library's defaults
(reproducible, and the ones the committed profiles were taken with); --tune
lets the autotuner pick them in the warmup instead.

Workloads (synthetic, shaped like the paper's frame: 37 kernels x 4 sizes x 15
devices, 34 features; see paper_1811_00156_amd/synth.py):
  c1  2220 rows, 64 bins, 100 trees, mtry 6, min.node.size 5
  c2  2220 rows, 256 bins, 2000 trees, mtry 12, min.node.size 1
  c3  200000 rows x 64 features + 32 devices, 256 bins, 500 trees, mtry 16, min.node.size 5
  c4  2220 rows, 64 bins, 10 folds x mtry 1..34 x min.node.size {1,3,5,7,9} = 1700 forests x 256 trees,
      fused single launch vs one launch sequence per forest   (default; the line also carries the
      200000-row forest's grow-kernel roofline and the serving p50/p99 at 2000 QPS)
  c5  serving: the c3 forest answers Poisson request streams of 1..4096 rows
  studies  the kernel studies of Sec. III-C on 2220 rows, 256 bins, num.trees 505, mtry 30,
      min.node.size 9: leave-one-kernel-out (37 forests) and training on i = 1..36 random
      kernels (--repeats forests per i), each forest's held-out kernels predicted on the device
  tune  the annealing search of Sec. III-B on 2220 rows, 256 bins: num.trees 10..1000, mtry 1..35,
      min.node.size 1..50 from (500, 17, 5), 10 levels x 32 proposals fitted together per level

  lds  LDS atomic add throughput (the probe library): the second ceiling of the grow kernel
  copy  a plain device copy (calibrates rocprofv3's FETCH_SIZE / WRITE_SIZE)

Prints ONE JSON line.  `value` is whole-step throughput in rows x trees per
second (c5: rows per second).  `roofline` describes the tree-growing kernel:
algorithmic bytes per launch (the per-row model of the tree-growing steps:
mtry candidate codes + 8 bytes of response + 1 of weight + 4 of row index per
searched row and level, 10 bytes per partitioned row and level) over its
event-timed duration; `lds_roofline` sets its LDS histogram adds against the
probe's measured rate.  `cpu_baseline` is the CPU oracle timed on the host
cores, at all of them and at one, on a bounded sample of the same work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    "c1": dict(data="d1", bins=64, num_trees=100, mtry=6, min_node=5),
    "c2": dict(data="d1", bins=256, num_trees=2000, mtry=12, min_node=1),
    "c3": dict(data="d3", bins=256, num_trees=500, mtry=16, min_node=5),
    "c4": dict(data="d1", bins=64, num_trees=256),
    "c5": dict(data="d3", bins=256, num_trees=500, mtry=16, min_node=5),
    "studies": dict(data="d1", bins=256, num_trees=505, mtry=30, min_node=9),
    "tune": dict(data="d1", bins=256, lower=(10, 1, 1), upper=(1000, 35, 50), start=(500, 17, 5), levels=10,
                 proposals=32, t0=0.02, cooling=0.7, step_frac=0.15),
}

METRIC = "forest fit rows·trees/s (fused grid vs plain); predict rows/s + p99 latency"


TUNE = False


def tune_flag():
    """FIT_TUNE when --tune asks the autotuner to pick the launch shape, else the
    library's default shape (or the one the environment names)."""
    from paper_1811_00156_amd import rf

    return rf.FIT_TUNE if TUNE else 0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def grow_bytes(work, mtry):
    """Algorithmic bytes of the tree-growing kernel, per the method's own row
    counts: every in-bag row of a node whose split is searched costs its code in
    each of the mtry candidate columns, its 8-byte fixed-point response, its
    1-byte bootstrap weight and its 4-byte row index (mtry + 13 bytes); every row
    of a node that splits costs 10 bytes to route into a child (its code in the
    split column, index and weight read, index written)."""
    searched_rows, part_rows = int(work[0]), int(work[2])
    return searched_rows * (mtry + 13) + part_rows * 10


TRAFFIC_SOURCES = ["paper_1811_00156_amd/csrc/fit.hip", "paper_1811_00156_amd/csrc/fit_grouped.hip",
                   "paper_1811_00156_amd/csrc/device.h", "paper_1811_00156_amd/csrc/api.cpp",
                   "paper_1811_00156_amd/csrc/internal.h"]


def profiled_record(kernel_key):
    """The rocprofv3 counter figures of a grow-kernel instantiation summarised in
    profiles/ (traffic.json: HBM bytes per launch from the byte-exact L2 request
    counters, VALU wave-instructions per launch), or None when the kernel, or the
    host code that picks its launch shape, has changed since they were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel_key)
    if not rec:
        return None
    if rec.get("kernel_sources") != TRAFFIC_SOURCES:
        return None
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest()[:16] != rec["kernel_sha256_16"]:
        return None
    return rec


def measured_traffic(kernel_key):
    """HBM bytes per launch (profiles/k_grow_traffic.txt), or None (see profiled_record)."""
    rec = profiled_record(kernel_key)
    return rec["traffic_bytes"] if rec else None


# wave64 VALU instructions per second of the MI355X: 256 CUs x 4 SIMDs, each
# issuing one VALU instruction per cycle at 2.4 GHz, a wave64 instruction
# holding its 16-lane SIMD for 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def issue_roofline(kernel_key, ms):
    """The grow kernel's VALU instruction issue rate against the chip's: the
    profiled wave-instructions per launch (SQ_INSTS_VALU, profiles/
    k_grow_shader_counters.txt) over this run's launch time; None when the
    profile is stale."""
    rec = profiled_record(kernel_key)
    if not rec or "valu_wave_instructions" not in rec:
        return None
    n = float(rec["valu_wave_instructions"])
    achieved = n / (ms / 1000.0)
    return {"kernel": "k_grow", "bound": "valu_issue", "achieved": achieved, "unit": "wave64 VALU instructions/s",
            "peak": VALU_ISSUE_PEAK, "frac": achieved / VALU_ISSUE_PEAK, "instructions_per_launch": n,
            "source": "SQ_INSTS_VALU, profiles/k_grow_shader_counters.txt"}


def lds_peak():
    """The probe's LDS atomic add rates (lane-adds/s): ds_add_u64 with the lanes
    of an instruction on distinct consecutive bins (the conflict-free peak) and
    on pseudo-random bins (the histogram build's pattern)."""
    import ctypes

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1811_00156_amd", "libaiwc_rf_probe.so"))
    lib.aiwc_rf_probe_lds_add.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_void_p] * 3
    lib.aiwc_rf_probe_last_error.restype = ctypes.c_char_p
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for width in (64, 32):
        for pattern, name in ((0, "distinct"), (1, "random")):
            r, ms = ctypes.c_double(), ctypes.c_double()
            rc = lib.aiwc_rf_probe_lds_add(width, pattern, 8 * cus, 2000, ctypes.byref(r), ctypes.byref(ms), None)
            if rc != 0:
                raise RuntimeError(f"LDS probe failed ({rc}): {lib.aiwc_rf_probe_last_error().decode()}")
            out[f"u{width}_{name}"] = r.value
    return out


def lds_roofline(work_hist, ms, peaks):
    """The grow kernel's LDS histogram adds per second against the probe."""
    achieved = float(work_hist) / (ms / 1000.0)
    return {"kernel": "k_grow", "bound": "lds_atomic", "achieved": achieved, "unit": "adds/s",
            "peak": peaks["u64_distinct"], "frac": achieved / peaks["u64_distinct"],
            "peak_random_bins": peaks["u64_random"], "frac_random_bins": achieved / peaks["u64_random"],
            "adds_per_launch": int(work_hist),
            "peak_source": "ds_add_u64 probe (libaiwc_rf_probe.so), 8 workgroups of 256 threads per CU"}


# ---------------------------------------------------------------------------- CPU baseline
CPU_TARGET_S = 10.0  # seconds of oracle work per thread count


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_legs(leg, unit):
    """leg(n_threads) -> (rate, sample description), timed at every host thread
    and at one; the all-threads rate is the baseline's value."""
    cores = host_threads()
    v, smp = leg(cores)
    v1, smp1 = leg(1)
    return {"value": v, "unit": unit, "cores": cores, "kind": "oracle", "sample": smp,
            "value_1thread": v1, "sample_1thread": smp1, "cpu_model": cpu_model()}


def forest_cpu_leg(wl, ds, probe_trees):
    """The oracle's whole-step throughput: bin once, then fit and predict trees of
    the same forest (repeating the whole forest when it takes less) until about
    CPU_TARGET_S seconds of work; a first pass of probe_trees trees sizes the
    sample."""
    from oracle import oracle as O

    def leg(threads):
        t0 = time.perf_counter()
        b = O.bin(ds.X, ds.device, ds.n_devices, wl["bins"])
        t_bin = time.perf_counter() - t0
        nt = wl["num_trees"]

        def fit_predict(k):
            f = O.fit(b.codes, b.n_bins, ds.y, nt, wl["mtry"], wl["min_node"], seed=1, trees=range(k),
                      n_threads=threads)
            O.predict(f, b.codes)

        probe = min(max(1, probe_trees * threads // host_threads()), nt)
        t0 = time.perf_counter()
        fit_predict(probe)
        per_tree = (time.perf_counter() - t0) / probe
        want = max(probe, int(CPU_TARGET_S / max(per_tree, 1e-9)))
        # in pieces of about an eighth of the estimate, stopping once the target
        # time is spent (the probe can misjudge the host's sustained rate)
        piece = max(probe, want // 8)
        t0 = time.perf_counter()
        done = 0
        el = 0.0
        while done < want and (done == 0 or el < CPU_TARGET_S):
            k = min(nt, want - done, piece)
            fit_predict(k)
            done += k
            el = time.perf_counter() - t0
        # one step = bin + fit and predict the whole forest; fit and predict are linear in trees
        step_s = t_bin + el * nt / done
        return ds.n * nt / step_s, (f"{threads} thread(s): bin all {ds.n} rows ({t_bin:.2f} s) + fit and predict "
                                    f"{done} trees of the {nt}-tree forest ({el:.1f} s), scaled to one step")

    return leg


# ---------------------------------------------------------------------------- single forests
def fit_forest_steps(wl, ds, steps, warmup, tag, predict_all=True):
    """Timed bin + fit (+ predict) steps of one forest workload.  Returns the
    step wall time and medians of each part, the last forest and its work."""
    import torch

    from paper_1811_00156_amd import rf

    dev = torch.device("cuda:0")
    X = torch.from_numpy(ds.X).to(dev)
    did = torch.from_numpy(ds.device).to(dev)
    y = torch.from_numpy(ds.y).to(dev)
    prm = rf.make_params(wl["num_trees"], wl["mtry"], wl["min_node"], True, 1)
    out = torch.empty(ds.n, dtype=torch.float64, device=dev)

    def step():
        codes, binner = rf.aiwc_rf_bin(X, did, ds.n_devices, wl["bins"])
        forest = rf.aiwc_rf_fit(codes, binner, y, prm, flags=tune_flag())
        if predict_all:
            rf.aiwc_rf_predict(forest, codes, out=out)
        return forest, binner

    for i in range(warmup):
        log(f"{tag} warmup {i}")
        keep = step()
    torch.cuda.synchronize()
    keep = None
    grow_ms, bin_ms, fit_ms, pred_ms = [], [], [], []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    forests = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[0].record()
        codes, binner = rf.aiwc_rf_bin(X, did, ds.n_devices, wl["bins"])
        ev[1].record()
        forest = rf.aiwc_rf_fit(codes, binner, y, prm, flags=tune_flag())
        ev[2].record()
        if predict_all:
            rf.aiwc_rf_predict(forest, codes, out=out)
        ev[3].record()
        ev[3].synchronize()
        bin_ms.append(ev[0].elapsed_time(ev[1]))
        fit_ms.append(ev[1].elapsed_time(ev[2]))
        pred_ms.append(ev[2].elapsed_time(ev[3]))
        grow_ms.append(forest.stats()[1])
        if forests:
            forests.pop()  # release the previous step's forest
        forests.append((forest, binner, codes))
        log(f"{tag} step {i}: bin {bin_ms[-1]:.2f} ms fit {fit_ms[-1]:.2f} ms (grow {grow_ms[-1]:.2f}) "
            f"predict {pred_ms[-1]:.3f} ms")
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / steps
    forest, binner, codes = forests[-1]
    work, _ = forest.stats()
    return dict(ms_step=ms_step, bin=float(np.median(bin_ms)), fit=float(np.median(fit_ms)),
                grow=float(np.mean(grow_ms)), predict=float(np.median(pred_ms)), forest=forest, binner=binner,
                codes=codes, work=work, launch=forest.launch())


def grow_roofline(work, mtry, g_ms, key, peaks=None):
    gbytes = grow_bytes(work, mtry)
    achieved = gbytes / (g_ms / 1000.0) / 1e9
    r = {"kernel": "k_grow", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(key),
         "algorithmic_bytes_per_launch": int(gbytes), "avg_launch_ms": g_ms}
    return r


def bench_forest(args, wl_name):
    from paper_1811_00156_amd import synth

    wl = WORKLOADS[wl_name]
    ds = synth.d1() if wl["data"] == "d1" else synth.d3()
    r = fit_forest_steps(wl, ds, args.steps, args.warmup, wl_name)
    work = r["work"]
    rows_trees = ds.n * wl["num_trees"]
    res = {
        "metric": METRIC, "value": rows_trees / (r["ms_step"] / 1000.0), "unit": "rows·trees/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": f"{wl_name}: {ds.n} rows x {ds.p} features + device ({ds.n_devices} levels), "
                               f"{wl['bins']} bins, num.trees {wl['num_trees']}, mtry {wl['mtry']}, "
                               f"min.node.size {wl['min_node']}; bin + fit + predict all rows",
                   "rows": ds.n, "num_trees": wl["num_trees"], "bins": wl["bins"], "mtry": wl["mtry"],
                   "min_node_size": wl["min_node"], "launch": r["launch"]},
        "breakdown_ms": {"bin": r["bin"], "fit": r["fit"], "grow_kernel": r["grow"], "predict": r["predict"]},
        "fit_rows_trees_per_s": rows_trees / (r["fit"] / 1000.0),
        "predict_rows_per_s": ds.n / (r["predict"] / 1000.0),
        "tree_stats": {"total_nodes": int(r["forest"].total_nodes()), "searched_rows": int(work[0]),
                       "searched_nodes": int(work[1]), "partitioned_rows": int(work[2]), "max_levels": int(work[3]),
                       "lds_bin_adds": int(work[4])},
        "roofline": grow_roofline(work, wl["mtry"], r["grow"], f"k_grow@{wl_name}"),
    }
    if not args.no_lds:
        res["lds_roofline"] = lds_roofline(work[4], r["grow"], lds_peak())
    res["issue_roofline"] = issue_roofline(f"k_grow@{wl_name}", r["grow"])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        sample = {"c1": 100, "c2": 200, "c3": 16}.get(wl_name, 16)
        res["cpu_baseline"] = cpu_legs(forest_cpu_leg(wl, ds, sample), "rows·trees/s")
    return res


# ---------------------------------------------------------------------------- the tuning grid
def bench_grid(args):
    import torch

    from paper_1811_00156_amd import rf, synth

    ds = synth.d1()
    dev = torch.device("cuda:0")
    folds = synth.cv_folds()
    combos = synth.grid_forests()
    params = [rf.make_params(256, m, mn, True, 1) for _, m, mn in combos]
    held = [f for f, _, _ in combos]
    X = torch.from_numpy(ds.X).to(dev)
    did = torch.from_numpy(ds.device).to(dev)
    y = torch.from_numpy(ds.y).to(dev)
    fd = torch.from_numpy(folds).to(dev)
    codes, binner = rf.aiwc_rf_bin(X, did, ds.n_devices, 64)
    n_train = np.array([ds.n - int((folds == f).sum()) for f in held])
    rows_trees = int(n_train.sum()) * 256

    def run(flags):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = rf.aiwc_rf_fit(codes, binner, y, params, fold_id=fd, heldout_fold=held, flags=flags)
        torch.cuda.synchronize()
        return g, (time.perf_counter() - t0) * 1000.0

    # the warmup runs both paths (and tunes each one's launch shape under --tune)
    for i in range(args.warmup):
        log(f"grid warmup {i}")
        g, _ = run(rf.FIT_FUSED | tune_flag())
        del g
        if not args.no_plain:
            g, _ = run(rf.FIT_PLAIN | tune_flag())
            del g
    fused_ms, plain_ms, grow_ms = [], [], []
    for i in range(args.steps):
        g, ms = run(rf.FIT_FUSED | tune_flag())
        fused_ms.append(ms)
        grow_ms.append(g.stats(0)[1])
        log(f"grid fused step {i}: {ms:.1f} ms (graph {grow_ms[-1]:.1f} ms)")
        if i + 1 < args.steps:
            del g
        else:
            fused = g
        if args.no_plain:
            continue
        gp, ms = run(rf.FIT_PLAIN | tune_flag())
        plain_ms.append(ms)
        log(f"grid plain step {i}: {ms:.1f} ms")
        del gp
    f_ms = float(np.median(fused_ms))
    p_ms = float(np.median(plain_ms)) if plain_ms else float("nan")
    # the kernel's work: per forest (its own mtry in the byte model)
    gbytes = 0
    work = np.zeros(5, np.int64)
    for k, (_, m, _) in enumerate(combos):
        w, _ = fused.stats(k)
        gbytes += grow_bytes(w, m)
        work += w
    g_ms = float(np.mean(grow_ms))
    achieved = gbytes / (g_ms / 1000.0) / 1e9
    launch = fused.launch()
    # out-of-bag scoring of every forest of the grid (the tuning objective), after the fit
    oob_ms = []
    for i in range(max(args.steps, 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = rf.aiwc_rf_oob_error(fused, codes, y)
        oob_ms.append((time.perf_counter() - t0) * 1000.0)
    best = int(np.argmin(o.mse))
    log(f"grid oob: {float(np.median(oob_ms)):.1f} ms; lowest OOB MSE {o.mse[best]:.4f} at forest {best} "
        f"(fold {combos[best][0]}, mtry {combos[best][1]}, min.node.size {combos[best][2]})")
    del fused
    res = {
        "metric": METRIC, "value": rows_trees / (f_ms / 1000.0), "unit": "rows·trees/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": "c4: 2220 rows x 34 features + device (15 levels), 64 bins, 10 CV folds x "
                               "mtry 1..34 x min.node.size {1,3,5,7,9} = 1700 forests x 256 trees, "
                               "one fused graph launch per step (value); the same forests as 1700 plain "
                               "launch sequences (plain_ms)",
                   "forests": len(params), "trees": 256 * len(params), "rows_trees": rows_trees, "launch": launch},
        "fused_ms": f_ms, "plain_ms": p_ms, "plain_rows_trees_per_s": rows_trees / (p_ms / 1000.0),
        "fused_speedup": p_ms / f_ms, "fused_ms_runs": fused_ms, "plain_ms_runs": plain_ms,
        "roofline": {"kernel": "k_grow", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("k_grow@c4"),
                     "algorithmic_bytes_per_launch": int(gbytes), "avg_launch_ms": g_ms},
        "tree_stats": {"searched_rows": int(work[0]), "searched_nodes": int(work[1]), "partitioned_rows": int(work[2]),
                       "lds_bin_adds": int(work[4])},
        "oob_ms": float(np.median(oob_ms)), "oob_rows_trees_per_s": rows_trees / (float(np.median(oob_ms)) / 1000.0),
    }
    if not args.no_lds:
        res["lds_roofline"] = lds_roofline(work[4], g_ms, lds_peak())
    res["issue_roofline"] = issue_roofline("k_grow@c4", g_ms)
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        ob = O.bin(ds.X, ds.device, ds.n_devices, 64)

        def leg(threads):
            # random forests of the grid, whole, until about CPU_TARGET_S seconds of work
            pick = np.random.default_rng(0).permutation(len(combos))
            t0 = time.perf_counter()
            rt = used = 0
            for k in pick:
                f, m, mn = combos[k]
                train = np.nonzero(folds != f)[0]
                O.fit(ob.codes, ob.n_bins, ds.y, 256, m, mn, seed=1, train_rows=train, n_threads=threads)
                rt += train.shape[0] * 256
                used += 1
                if time.perf_counter() - t0 >= CPU_TARGET_S:
                    break
            el = time.perf_counter() - t0
            return rt / el, f"{threads} thread(s): {used} random forests of the grid (256 trees each), {el:.1f} s"

        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_legs(leg, "rows·trees/s")
    if not args.no_extras:
        res.update(extra_legs(args))
    return res


def extra_legs(args):
    """The 200000-row forest's grow-kernel roofline and the serving latency of
    that forest at 2000 QPS, beside the grid's line."""
    from paper_1811_00156_amd import synth

    wl = WORKLOADS["c3"]
    ds = synth.d3()
    r = fit_forest_steps(wl, ds, 3, 1, "c3", predict_all=False)
    rows_trees = ds.n * wl["num_trees"]
    c3 = {"workload": "c3: 200000 rows x 64 features + device (32 levels), 256 bins, num.trees 500, mtry 16, "
                      "min.node.size 5; bin + fit", "launch": r["launch"],
          "ms_per_step": r["ms_step"], "fit_ms": r["fit"], "fit_rows_trees_per_s": rows_trees / (r["fit"] / 1000.0),
          "roofline": grow_roofline(r["work"], wl["mtry"], r["grow"], "k_grow@c3"),
          "lds_bin_adds": int(r["work"][4])}
    if not args.no_lds:
        c3["lds_roofline"] = lds_roofline(r["work"][4], r["grow"], lds_peak())
    c3["issue_roofline"] = issue_roofline("k_grow@c3", r["grow"])
    log(f"c3: fit {r['fit']:.1f} ms, grow {r['grow']:.1f} ms, frac {c3['roofline']['frac']:.3f}")
    sv = serve_points(r["forest"], r["codes"].cpu().numpy(), ds.n, args.requests, load_fracs=(),
                      fixed_qps=(2000.0,))
    c5 = {"workload": "c5: serving the c3 forest; Poisson arrivals at 2000 QPS, 1..4096 rows per request "
                      "(log-uniform); arrival to answer in host memory",
          "saturated_rows_per_s": sv["saturated"]["rows_per_s"], "at_2000qps": sv["points"]["2000qps"]}
    log(f"c5: saturated {c5['saturated_rows_per_s']:.3g} rows/s; 2000 QPS p50 {c5['at_2000qps']['p50_ms']:.3f} ms "
        f"p99 {c5['at_2000qps']['p99_ms']:.3f} ms")
    return {"c3": c3, "c5": c5}


# ---------------------------------------------------------------------------- serving
def serve_points(forest, host_codes, n_rows, n_req, load_fracs=(0.25, 0.5, 0.8), fixed_qps=(2000.0,)):
    """Saturated rows/s (median of three closed-loop passes after a warmup pass)
    and open-loop p50/p99 latency at fractions of it and at fixed rates."""
    from paper_1811_00156_amd import rf, synth

    def stream(qps, seed_shift=0):
        arrivals, sizes, row_seed = synth.request_stream(n_req, qps)
        rng = np.random.default_rng(row_seed + seed_shift)
        reqs = [np.ascontiguousarray(host_codes[rng.integers(0, n_rows, size=int(s))]) for s in sizes]
        return arrivals, reqs

    def serve(arrivals, reqs, open_loop=True):
        srv = rf.Server(forest, memory_budget_bytes=1 << 26, max_batch_rows=16384, n_streams=4)
        outs = [np.empty(r.shape[0]) for r in reqs]
        t0 = time.perf_counter()
        for a, r, o in zip(arrivals, reqs, outs):
            if open_loop:
                while time.perf_counter() - t0 < a:
                    pass
            srv.submit(r, o)
        srv.drain()
        el = time.perf_counter() - t0
        _, lat = srv.poll(len(reqs) + 1)
        st = srv.stats()
        srv.close()
        rows = sum(r.shape[0] for r in reqs)
        return {"rows_per_s": rows / el, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "batches": st.batches, "requests": len(reqs),
                "memory_waits": st.memory_waits}

    arr, reqs = stream(1000.0)
    log("serve warmup")
    serve(arr, reqs, open_loop=False)
    # saturated: the median of three closed-loop passes (one pass is short, and
    # its host-side submission varies from run to run)
    sats = []
    for i in range(3):
        log(f"serve saturated {i}")
        sats.append(serve(arr, reqs, open_loop=False))
    sat = sorted(sats, key=lambda d: d["rows_per_s"])[1]
    mean_rows = np.mean([r.shape[0] for r in reqs])
    points = {}
    for frac in load_fracs:
        qps = frac * sat["rows_per_s"] / mean_rows
        a, r = stream(qps, 1)
        log(f"serve {frac:.0%} load ({qps:.0f} QPS)")
        points[f"{int(frac * 100)}%"] = dict(qps=qps, **serve(a, r))
    for qps in fixed_qps:
        a, r = stream(qps, 2)
        log(f"serve {qps:.0f} QPS")
        points[f"{int(qps)}qps"] = dict(qps=qps, **serve(a, r))
    return {"saturated": sat, "saturated_runs": [d["rows_per_s"] for d in sats], "points": points}


def bench_serve(args):
    import torch

    from paper_1811_00156_amd import rf, synth

    wl = WORKLOADS["c5"]
    ds = synth.d3()
    dev = torch.device("cuda:0")
    codes, binner = rf.aiwc_rf_bin(torch.from_numpy(ds.X).to(dev), torch.from_numpy(ds.device).to(dev),
                                   ds.n_devices, wl["bins"])
    forest = rf.aiwc_rf_fit(codes, binner, torch.from_numpy(ds.y).to(dev),
                            rf.make_params(wl["num_trees"], wl["mtry"], wl["min_node"], True, 1))
    sv = serve_points(forest, codes.cpu().numpy(), ds.n, args.requests)
    return {
        "metric": METRIC, "value": sv["saturated"]["rows_per_s"], "unit": "rows/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": "c5: serving the c3 forest (500 trees, 65 columns); Poisson arrivals, "
                               "1..4096 rows per request (log-uniform)", "requests": args.requests},
        "saturated": sv["saturated"], "saturated_rows_per_s_runs": sv["saturated_runs"],
        "load_points": sv["points"],
    }


def bench_studies(args):
    """Algorithm 1 (leave one kernel out) and Algorithm 2 (train on i random kernels,
    test on the rest) of Sec. III-C as fused group grids, with held-out scoring."""
    import torch

    from paper_1811_00156_amd import rf, synth

    wl = WORKLOADS["studies"]
    ds = synth.d1()
    dev = torch.device("cuda:0")
    X = torch.from_numpy(ds.X).to(dev)
    did = torch.from_numpy(ds.device).to(dev)
    y = torch.from_numpy(ds.y).to(dev)
    g = synth.kernel_groups(ds)
    gd = torch.from_numpy(g).to(dev)
    codes, binner = rf.aiwc_rf_bin(X, did, ds.n_devices, wl["bins"])
    prm = rf.make_params(wl["num_trees"], wl["mtry"], wl["min_node"], True, 1)
    per_group = np.bincount(g, minlength=37)
    loo = synth.leave_one_kernel_out_masks()
    counts, masks = synth.kernel_subset_masks(repeats=args.repeats, counts=range(1, 37))

    def n_rows(m):
        return int(sum(per_group[k] for k in range(37) if (int(m) >> k) & 1))

    def run_grid(mask_list):
        t0 = time.perf_counter()
        f = rf.aiwc_rf_fit_groups(codes, binner, y, [prm] * len(mask_list), gd, mask_list, flags=tune_flag())
        t1 = time.perf_counter()
        h = rf.aiwc_rf_heldout_error(f, codes, y)
        t2 = time.perf_counter()
        del f
        return (t1 - t0) * 1000.0, (t2 - t1) * 1000.0, h

    def run_study(quiet):
        fit_ms = score_ms = 0.0
        rows_trees = 0
        ms1, hs1, h1 = run_grid(loo)
        fit_ms += ms1
        score_ms += hs1
        rows_trees += sum(n_rows(m) for m in loo) * wl["num_trees"]
        alg1 = float(np.sum(h1.mae * h1.rows) / np.sum(h1.rows))
        if not quiet:
            log(f"algorithm 1: 37 forests, fit {ms1:.1f} ms, held-out scoring {hs1:.1f} ms, held-out MAE {alg1:.4f}")
        maes = []
        for i in range(1, 37):
            sel = masks[counts == i]
            ms, hs, h = run_grid(sel)
            fit_ms += ms
            score_ms += hs
            rows_trees += sum(n_rows(m) for m in sel) * wl["num_trees"]
            maes.append(float(np.sum(h.mae * h.rows) / np.sum(h.rows)))
            if not quiet:
                log(f"algorithm 2: i={i}, {len(sel)} forests, fit {ms:.1f} ms, scoring {hs:.1f} ms, MAE {maes[-1]:.4f}")
        return fit_ms, score_ms, rows_trees, alg1, maes

    # the warmup runs the whole study once, so that every problem shape's launch
    # shape is tuned before the timed pass
    for i in range(min(args.warmup, 1)):
        log("studies warmup: the whole study once")
        run_study(True)
    torch.cuda.synchronize()
    fit_ms, score_ms, rows_trees, alg1_mae, mae_by_count = run_study(False)
    # Sec. VI on Algorithm 1's forests (untimed): each forest that never saw kernel
    # k ranks the devices of k's four size vectors against the noiseless truth
    f = rf.aiwc_rf_fit_groups(codes, binner, y, [prm] * len(loo), gd, loo, flags=tune_flag())
    vrows = synth.vector_rows(ds)
    rc = rn = rh = 0
    for k in range(37):
        vecs = np.arange(4 * k, 4 * k + 4)
        feats = codes[torch.from_numpy(vrows[vecs]).to(dev), :-1].contiguous()
        _, times = rf.aiwc_rf_select_device(f, feats, forest_index=k, n_devices=ds.n_devices)
        r = rf.aiwc_rf_rank_accuracy(times, torch.from_numpy(np.ascontiguousarray(ds.truth[vecs])).to(dev))
        rc += int(r.correct.sum().item())
        rn += int(r.counted.sum().item())
        rh += int(r.hit.sum().item())
    del f
    log(f"device ranking of unseen kernels: {rc}/{rn} pairs in the right order, fastest device {rh}/148")
    total_ms = fit_ms + score_ms
    n_forests = 37 + int(len(masks))
    res = {
        "metric": "kernel-study forest fit + held-out scoring rows·trees/s", "value": rows_trees / (total_ms / 1000.0),
        "unit": "rows·trees/s", "n_gpus": 1, "steps": 1, "warmup": min(args.warmup, 1), "ms_per_step": total_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": f"studies: 2220 rows, 256 bins, num.trees 505, mtry 30, min.node.size 9; "
                               f"37 leave-one-kernel-out forests + {len(masks)} kernel-subset forests "
                               f"(i = 1..36, {args.repeats} each)", "forests": n_forests},
        "fit_ms": fit_ms, "heldout_scoring_ms": score_ms, "alg1_heldout_mae": alg1_mae,
        "alg1_device_ranking": {"pairs_right": rc, "pairs_counted": rn, "pairwise_accuracy": rc / max(1, rn),
                                "fastest_device_hits": rh, "vectors": 148},
        "alg2_mae_by_kernel_count": mae_by_count,
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        ob = O.bin(ds.X, ds.device, ds.n_devices, wl["bins"])
        # one leave-one-kernel-out forest and every 25th kernel subset (all counts), 505 trees each
        step = max(1, len(masks) // 144)
        sample = list(loo[:1]) + list(masks[::step])
        t0 = time.perf_counter()
        rt = 0
        for m in sample:
            inside = np.array([(int(m) >> int(k)) & 1 for k in g], dtype=bool)
            train = np.nonzero(inside)[0]
            O.fit(ob.codes, ob.n_bins, ds.y, wl["num_trees"], wl["mtry"], wl["min_node"], seed=1, train_rows=train,
                  n_threads=cores)
            rt += train.shape[0] * wl["num_trees"]
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": rt / el, "unit": "rows·trees/s", "cores": cores, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"{len(sample)} study forests (one leave-one-kernel-out, every {step}th "
                                         f"kernel subset), 505 trees each, {el:.1f} s"}
    return res


def bench_tune(args):
    """The annealing parameter search: every level's proposals in one fused fit,
    scored by out-of-bag error on the device."""
    import torch

    from paper_1811_00156_amd import rf, synth

    wl = WORKLOADS["tune"]
    ds = synth.d1()
    dev = torch.device("cuda:0")
    codes, binner = rf.aiwc_rf_bin(torch.from_numpy(ds.X).to(dev), torch.from_numpy(ds.device).to(dev),
                                   ds.n_devices, wl["bins"])
    y = torch.from_numpy(ds.y).to(dev)
    cfg = rf.sa_config(wl["lower"], wl["upper"], wl["start"], wl["levels"], wl["proposals"], wl["t0"], wl["cooling"],
                       wl["step_frac"], seed=1)
    for i in range(min(args.warmup, 1)):
        log("tune warmup: the whole search once")
        rf.aiwc_rf_tune_sa(codes, binner, y, cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, fb, trace = rf.aiwc_rf_tune_sa(codes, binner, y, cfg)
    ms = (time.perf_counter() - t0) * 1000.0
    rows_trees = sum(ds.n * t["params"][0] for t in trace)
    log(f"tune: {len(trace)} forests in {ms:.1f} ms; best {best} OOB MSE {fb:.5f} "
        f"(start {trace[0]['params']} OOB MSE {trace[0]['objective']:.5f}); "
        f"accepted {sum(t['accepted'] for t in trace[1:])} of {len(trace) - 1}")
    res = {
        "metric": "annealing search forest fit + out-of-bag scoring rows·trees/s", "value": rows_trees / (ms / 1000.0),
        "unit": "rows·trees/s", "n_gpus": 1, "steps": 1, "warmup": min(args.warmup, 1), "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": "tune: 2220 rows, 256 bins; num.trees 10..1000, mtry 1..35, min.node.size 1..50 "
                               "from (500, 17, 5); 10 levels x 32 proposals", "forests": len(trace)},
        "best_params": list(best), "best_oob_mse": fb, "start_oob_mse": trace[0]["objective"],
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        ob = O.bin(ds.X, ds.device, ds.n_devices, wl["bins"])
        # the oracle's objective on every 10th triple the search evaluated
        sample = [t["params"] for t in trace[::10]]
        t0 = time.perf_counter()
        rt = 0
        for nt, mt, mn in sample:
            f = O.fit(ob.codes, ob.n_bins, ds.y, nt, mt, mn, seed=1, n_threads=cores)
            O.oob(f, ob.codes, ds.y, mt, mn, seed=1)
            rt += ds.n * nt
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": rt / el, "unit": "rows·trees/s", "cores": cores, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"fit + out-of-bag error of {len(sample)} of the search's triples, {el:.1f} s"}
    return res


def bench_copy(args):
    """A plain device-to-device copy of known size: the reference that scales
    rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch

    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    gbs = 2 * nbytes / (ms / 1000.0) / 1e9
    return {"metric": "device copy GB/s (counter calibration)", "value": gbs, "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"copy: {nbytes} bytes read + {nbytes} bytes written per step"}}


def bench_lds(args):
    """The probe's LDS atomic add rates on their own."""
    peaks = lds_peak()
    return {"metric": "LDS atomic adds/s (ceiling of the histogram build)", "value": peaks["u64_distinct"],
            "unit": "adds/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "lds: 8 workgroups of 256 threads per CU, 2000 x 8 adds per lane into a "
                                   "256-bin histogram per wave"}, "rates": peaks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS) + ["copy", "lds"])
    ap.add_argument("--requests", type=int, default=4000)
    ap.add_argument("--repeats", type=int, default=100, help="studies: kernel subsets per kernel count (paper: 500)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lds", action="store_true", help="skip the LDS atomic probe and the lds_roofline object")
    ap.add_argument("--no-extras", action="store_true", help="c4: skip the c3 roofline and c5 latency legs")
    ap.add_argument("--no-plain", action="store_true", help="c4: skip the per-forest plain launches (profiling runs)")
    ap.add_argument("--tune", action="store_true",
                    help="let the autotuner pick every fit's launch shape in the warmup (default: the library's "
                         "default shapes, or AIWC_RF_GROW_BLOCK / AIWC_RF_HUGE_MIN / AIWC_RF_GROW_OCC / "
                         "AIWC_RF_BIG_COLS)")
    args = ap.parse_args()
    global TUNE
    TUNE = args.tune
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                                   "(the forest shards by trees across GPUs; only the one-GPU path is built here)"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.workload == "copy":
        res = bench_copy(args)
    elif args.workload == "lds":
        res = bench_lds(args)
    elif args.workload == "c4":
        res = bench_grid(args)
    elif args.workload == "c5":
        res = bench_serve(args)
    elif args.workload == "studies":
        res = bench_studies(args)
    elif args.workload == "tune":
        res = bench_tune(args)
    else:
        res = bench_forest(args, args.workload)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
