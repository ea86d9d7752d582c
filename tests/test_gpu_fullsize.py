"""GPU parity at the benchmark's own sizes and launch shapes, against the CPU oracle.

* 200000 rows x 65 columns, 256 bins, num.trees 500, mtry 16, min.node.size 5:
  every tree's node arrays, at the untuned launch shape and at the autotuned
  one, and the whole forest's predictions of a seeded 20000-row subset.
* The tuning grid on 2220 rows, 64 bins: 10 folds x mtry 1..34 x min.node.size
  {1,3,5,7,9} = 1700 forests x 256 trees in one fused graph launch at its
  default shape (64 threads, 5 waves per SIMD, 4 columns per large-node task):
  a seeded subset of 50 forests tree for tree with their predictions, then
  every forest once.
* Serving the 500-tree forest above: a Poisson stream of log-uniform requests
  (1..4096 rows), continuously batched under a memory budget that makes
  requests wait, every answer equal to the oracle's prediction of its rows.

Tolerance zero throughout: node arrays, leaf sums and binary64 bit patterns.
"""
import numpy as np
import pytest

from paper_1811_00156_amd import synth
from tests._gpu import assert_tree_equal, log, to_dev

pytestmark = pytest.mark.gpu

C3 = dict(num_trees=500, mtry=16, min_node=5, bins=256)
POOL_ROWS = 20000


@pytest.fixture(scope="module")
def rf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_00156_amd import rf as _rf

    return _rf


@pytest.fixture(scope="module")
def c3(rf, oracle):
    """The 500-tree forest on D3 from the oracle (all host threads) and the codes it was fitted on."""
    d3 = synth.d3()
    log("c3: oracle bin + fit of 500 trees")
    ob = oracle.bin(d3.X, d3.device, d3.n_devices, C3["bins"])
    of = oracle.fit(ob.codes, ob.n_bins, d3.y, C3["num_trees"], C3["mtry"], C3["min_node"], seed=1, n_threads=0)
    pool = np.sort(np.random.default_rng(181100160).choice(d3.n, size=POOL_ROWS, replace=False))
    pool_codes = np.ascontiguousarray(ob.codes[pool])
    P, yhat = oracle.predict(of, pool_codes)
    log("c3: oracle done")
    return dict(ds=d3, ob=ob, of=of, pool_codes=pool_codes, P=P, yhat=yhat)


def compare_forest(forest, of, num_trees, what, forest_index=0):
    trees = forest.export(forest_index)
    assert len(trees) == num_trees
    for t in range(num_trees):
        assert_tree_equal(trees[t], of.tree(t), f"{what} tree {t}")


@pytest.mark.parametrize("tuned", [False, True], ids=["default-shape", "autotuned-shape"])
def test_c3_every_tree_and_predictions(rf, c3, tuned):
    ob, of = c3["ob"], c3["of"]
    log(f"c3 gpu fit, tuned={tuned}")
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    codes = to_dev(ob.codes)
    flags = rf.FIT_TUNE if tuned else 0
    forest = rf.aiwc_rf_fit(codes, binner, to_dev(c3["ds"].y),
                            rf.make_params(C3["num_trees"], C3["mtry"], C3["min_node"], True, 1), flags=flags)
    li = forest.launch()
    log(f"c3 launch shape {li}")
    assert li["wide_phase"] == 1 and li["task_groups"] == C3["num_trees"]
    if not tuned:
        assert li["block"] == 1024 and li["wide_limit"] == 512
    compare_forest(forest, of, C3["num_trees"], f"C3 ({'tuned' if tuned else 'default'} shape)")
    pc = to_dev(c3["pool_codes"])
    g = rf.aiwc_rf_predict(forest, pc).cpu().numpy()
    assert np.array_equal(g.view(np.uint64), c3["yhat"].view(np.uint64)), "C3 predictions differ"
    s = rf.aiwc_rf_predict_sum(forest, pc, 0, C3["num_trees"]).cpu().numpy()
    assert np.array_equal(s, c3["P"])


# ---------------------------------------------------------------------------- the tuning grid
@pytest.fixture(scope="module")
def grid(rf, oracle):
    d1 = synth.d1()
    ob = oracle.bin(d1.X, d1.device, d1.n_devices, 64)
    folds = synth.cv_folds()
    combos = synth.grid_forests()
    params = [rf.make_params(256, m, mn, True, 1) for _, m, mn in combos]
    held = [f for f, _, _ in combos]
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    codes = to_dev(ob.codes)
    log("grid: fused fit of 1700 forests x 256 trees")
    g = rf.aiwc_rf_fit(codes, binner, to_dev(d1.y), params, fold_id=to_dev(folds), heldout_fold=held,
                       flags=rf.FIT_FUSED)
    return dict(ds=d1, ob=ob, folds=folds, combos=combos, forest=g, codes=codes)


def oracle_grid_forest(oracle, grid, k):
    f, m, mn = grid["combos"][k]
    ds, ob = grid["ds"], grid["ob"]
    train = np.nonzero(grid["folds"] != f)[0]
    return oracle.fit(ob.codes, ob.n_bins, ds.y, 256, m, mn, seed=1, train_rows=train, n_threads=0)


def test_grid_default_shape(grid):
    li = grid["forest"].launch()
    log(f"grid launch shape {li}")
    # 87040 task groups on 2000-row training sets: the shape of a grid whose
    # queue holds at least 64 work items per CU (and the one the fused
    # benchmark times unless it is tuned)
    assert (li["block"], li["waves_per_simd"], li["big_cols"], li["wide_phase"], li["graph"]) == (64, 5, 4, 0, 1)
    # tree t of the five forests of each (fold, mtry) is one task group
    assert li["task_groups"] == 10 * 34 * 256


def test_grid_seeded_subset(rf, oracle, grid):
    """50 seeded forests of the fused launch, tree for tree, with their predictions of all rows."""
    pick = np.sort(np.random.default_rng(181100161).choice(len(grid["combos"]), size=50, replace=False))
    ob = grid["ob"]
    for k in pick:
        k = int(k)
        of = oracle_grid_forest(oracle, grid, k)
        compare_forest(grid["forest"], of, 256, f"grid forest {k} {grid['combos'][k]}", forest_index=k)
        _, yhat = oracle.predict(of, ob.codes)
        g = rf.aiwc_rf_predict(grid["forest"], grid["codes"], forest_index=k).cpu().numpy()
        assert np.array_equal(g.view(np.uint64), yhat.view(np.uint64)), f"grid forest {k}: predictions differ"
    log(f"grid: 50 forests equal the oracle ({pick[:5].tolist()} ...)")


def test_grid_every_forest(oracle, grid):
    """All 1700 forests of the fused launch once, tree for tree."""
    n = len(grid["combos"])
    for k in range(n):
        of = oracle_grid_forest(oracle, grid, k)
        compare_forest(grid["forest"], of, 256, f"grid forest {k} {grid['combos'][k]}", forest_index=k)
        if k % 170 == 169:
            log(f"grid: forests 0..{k} equal the oracle")


# ---------------------------------------------------------------------------- serving
def test_serve_c3_forest_against_oracle(rf, c3):
    """Continuous batching of the 500-tree forest; every answer equals the oracle's."""
    ob, pool_codes, yhat = c3["ob"], c3["pool_codes"], c3["yhat"]
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    forest = rf.aiwc_rf_fit(to_dev(ob.codes), binner, to_dev(c3["ds"].y),
                            rf.make_params(C3["num_trees"], C3["mtry"], C3["min_node"], True, 1))
    _, sizes, row_seed = synth.request_stream(300, 2000.0)
    rng = np.random.default_rng(row_seed)
    idx = [rng.integers(0, POOL_ROWS, size=int(s)) for s in sizes]
    reqs = [np.ascontiguousarray(pool_codes[i]) for i in idx]
    outs = [np.full(r.shape[0], np.nan) for r in reqs]
    budget = 3 << 20  # a few large requests at a time: later ones wait for memory
    srv = rf.Server(forest, memory_budget_bytes=budget, max_batch_rows=16384, n_streams=4)
    log(f"serve: {len(reqs)} requests, {int(sizes.sum())} rows, budget {budget} bytes")
    tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]
    srv.drain()
    done, lat = srv.poll(len(reqs) + 1)
    st = srv.stats()
    srv.close()
    assert sorted(done.tolist()) == sorted(tickets)
    assert st.rows == int(sizes.sum())
    assert st.peak_bytes <= budget
    assert st.batches < len(reqs)
    assert st.memory_waits > 0  # the budget bound: some requests waited for memory
    log(f"serve: {st.batches} batches, peak {st.peak_bytes} bytes, {st.memory_waits} memory waits, "
        f"p50 {np.percentile(lat, 50) * 1e3:.2f} ms")
    for t, (i, o) in enumerate(zip(idx, outs)):
        assert np.array_equal(o.view(np.uint64), yhat[i].view(np.uint64)), f"request {t} differs from the oracle"
