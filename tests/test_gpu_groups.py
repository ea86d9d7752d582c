"""Fused fits whose forests differ only in min.node.size (task groups), against the oracle.

The grow kernel grows tree t of such forests once, down to the first level that
holds a node which is a leaf for some of them only, puts that level aside and
grows each forest's tree on from it.  The cases:

* ten values of min.node.size for one (fold, mtry), plus a repeated value: more
  forests than a group holds (groups of 8 and 3);
* forests without bootstrap (no in-bag bitmaps);
* forests that differ in tree count as well (separate groups);
* min.node.size above the root's weight next to 1: the trees part at the root.

Every tree of every forest, node for node, and the out-of-bag sums and counts of
every forest (each member's in-bag bitmap is written by its group).  The same
forests fitted with one launch per forest (no groups) must equal them too.
A larger training set (24000 rows, 256 bins) runs the groups in the kernel with
the workgroup-wide phase, parting where some nodes are still wide (their rows'
candidate codes are put aside and restored with the level).
Tolerance zero: node arrays, leaf sums and integer out-of-bag sums.
"""
import numpy as np
import pytest

from paper_1811_00156_amd import synth
from tests._gpu import assert_tree_equal, log, to_dev

pytestmark = pytest.mark.gpu

# (held-out fold or -1, trees, mtry, min.node.size, bootstrap, seed)
FORESTS = (
    [(2, 16, 5, mn, True, 7) for mn in (9, 1, 2, 3, 4, 5, 6, 7, 12, 20, 5)]
    + [(-1, 16, 12, mn, False, 3) for mn in (5, 1, 9)]
    + [(4, 12, 20, 3, True, 7), (4, 16, 20, 5, True, 7), (4, 12, 20, 9, True, 7)]
    + [(6, 8, 3, 100000, True, 2), (6, 8, 3, 1, True, 2)]
)
# groups of the fused launch: 11 forests of 16 trees in groups of 8 and 3, three
# without bootstrap, two and one of mtry 20 (different tree counts), and two of mtry 3
GROUPS = 2 * 16 + 16 + 12 + 16 + 8


@pytest.fixture(scope="module")
def rf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_00156_amd import rf as _rf

    return _rf


@pytest.fixture(scope="module")
def setup(rf, oracle):
    ds = synth.d1()
    ob = oracle.bin(ds.X, ds.device, ds.n_devices, 64)
    folds = synth.cv_folds()
    trains = [np.arange(ds.n) if f < 0 else np.nonzero(folds != f)[0] for f, *_ in FORESTS]
    log(f"groups: oracle fits of {len(FORESTS)} forests")
    ofs = [oracle.fit(ob.codes, ob.n_bins, ds.y, nt, m, mn, seed=sd, bootstrap=b, train_rows=trains[k], n_threads=0)
           for k, (_, nt, m, mn, b, sd) in enumerate(FORESTS)]
    return dict(ds=ds, ob=ob, folds=folds, trains=trains, ofs=ofs)


def fit(rf, setup, flags):
    ds, ob = setup["ds"], setup["ob"]
    params = [rf.make_params(nt, m, mn, b, sd) for _, nt, m, mn, b, sd in FORESTS]
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    return rf.aiwc_rf_fit(to_dev(ob.codes), binner, to_dev(ds.y), params, fold_id=to_dev(setup["folds"]),
                          heldout_fold=[f for f, *_ in FORESTS], flags=flags)


@pytest.mark.parametrize("plain", [False, True], ids=["fused-groups", "plain-per-forest"])
def test_groups_every_tree(rf, setup, plain):
    forest = fit(rf, setup, rf.FIT_PLAIN if plain else rf.FIT_FUSED)
    li = forest.launch()
    log(f"groups: plain={plain} launch {li}")
    n_tasks = sum(nt for _, nt, *_ in FORESTS)
    assert li["task_groups"] == (n_tasks if plain else GROUPS)
    for k, (f, nt, m, mn, b, sd) in enumerate(FORESTS):
        trees = forest.export(k)
        assert len(trees) == nt
        for t in range(nt):
            assert_tree_equal(trees[t], setup["ofs"][k].tree(t), f"forest {k} {FORESTS[k]} tree {t}")
    # min.node.size above the root's weight: every tree is one leaf
    assert all(tr["col"].shape[0] == 1 for tr in forest.export(len(FORESTS) - 2))


def test_groups_oob(rf, oracle, setup):
    """Out-of-bag sums and counts of every forest of the fused launch."""
    ds, ob, trains = setup["ds"], setup["ob"], setup["trains"]
    forest = fit(rf, setup, rf.FIT_FUSED)
    codes, y = to_dev(ob.codes), to_dev(ds.y)
    total = sum(t.shape[0] for t in trains)
    res = rf.aiwc_rf_oob_error(forest, codes, y, 0, len(FORESTS), n_train=total)
    sums, counts = res.sums.cpu().numpy(), res.counts.cpu().numpy()
    off = 0
    for k, (f, nt, m, mn, b, sd) in enumerate(FORESTS):
        P, cnt, (_, _, rows) = oracle.oob(setup["ofs"][k], ob.codes, ds.y, m, mn, seed=sd, bootstrap=b,
                                          train_rows=trains[k])
        n = trains[k].shape[0]
        assert np.array_equal(sums[off:off + n], P), f"forest {k} {FORESTS[k]}: out-of-bag sums"
        assert np.array_equal(counts[off:off + n], cnt), f"forest {k} {FORESTS[k]}: out-of-bag counts"
        assert res.rows[k] == rows
        off += n


# (trees, mtry, min.node.size): one group of four (min.node.size 700 parts the
# trees while other nodes of the level still have more than 512 rows) and a
# forest of another mtry, a group of its own
WIDE_FORESTS = [(6, 16, mn) for mn in (5, 1, 700, 60)] + [(6, 8, 5)]
WIDE_ROWS = 24000


def test_groups_wide_kernel(rf, oracle):
    d3 = synth.d3()
    rows = np.sort(np.random.default_rng(181100162).choice(d3.n, size=WIDE_ROWS, replace=False))
    X, dev_id, y = np.ascontiguousarray(d3.X[rows]), np.ascontiguousarray(d3.device[rows]), np.ascontiguousarray(d3.y[rows])
    ob = oracle.bin(X, dev_id, d3.n_devices, 256)
    params = [rf.make_params(nt, m, mn, True, 5) for nt, m, mn in WIDE_FORESTS]
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    log(f"groups wide: fused fit of {len(WIDE_FORESTS)} forests on {WIDE_ROWS} rows")
    forest = rf.aiwc_rf_fit(to_dev(ob.codes), binner, to_dev(y), params, heldout_fold=[-1] * len(WIDE_FORESTS),
                            flags=rf.FIT_FUSED)
    li = forest.launch()
    log(f"groups wide: launch {li}")
    assert li["wide_phase"] == 1 and li["block"] == 1024
    assert li["task_groups"] == 6 + 6
    for k, (nt, m, mn) in enumerate(WIDE_FORESTS):
        of = oracle.fit(ob.codes, ob.n_bins, y, nt, m, mn, seed=5, n_threads=0)
        trees = forest.export(k)
        for t in range(nt):
            assert_tree_equal(trees[t], of.tree(t), f"wide forest {k} {WIDE_FORESTS[k]} tree {t}")
