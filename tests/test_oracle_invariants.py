"""Invariants and special cases that pin the oracle's forest end to end."""
import numpy as np
import pytest

from paper_1811_00156_amd import synth


@pytest.fixture(scope="module")
def d1_binned(oracle):
    ds = synth.d1()
    return ds, oracle.bin(ds.X, ds.device, ds.n_devices, 64)


def test_weights_conserved(oracle, d1_binned):
    """Leaf weights sum to the bootstrap size; children's weights sum to the parent's."""
    ds, b = d1_binned
    f = oracle.fit(b.codes, b.n_bins, ds.y, 20, 6, 5, seed=3)
    for t in range(20):
        tr = f.tree(t)
        leaf = tr["col"] == 255
        assert tr["N"][leaf].sum() == ds.n
        internal = np.nonzero(~leaf)[0]
        l = tr["left"][internal]
        assert np.array_equal(tr["N"][l] + tr["N"][l + 1], tr["N"][internal])
        assert np.all(tr["N"] > 0)
        # min.node.size: every split node is heavier than it
        assert np.all(tr["N"][internal] > 5)


def test_constant_response_gives_single_leaf(oracle, d1_binned):
    ds, b = d1_binned
    y = np.full(ds.n, -2.3456789)
    f = oracle.fit(b.codes, b.n_bins, y, 10, 12, 1, seed=9)
    assert np.all(f.n_nodes == 1)
    y_fp = int(np.rint(-2.3456789 * 65536))
    P, yhat = oracle.predict(f, b.codes)
    assert np.all(yhat == y_fp / 65536.0)


def test_single_unbootstrapped_tree_reproduces_training_rows(oracle, d1_binned):
    """One tree, no bootstrap, min.node.size 1, mtry = all columns, distinct rows."""
    ds, b = d1_binned
    _, first = np.unique(b.codes, axis=0, return_index=True)
    rows = np.sort(first)
    codes, y = b.codes[rows], ds.y[rows]
    f = oracle.fit(codes, b.n_bins, y, 1, codes.shape[1], 1, seed=1, bootstrap=False)
    _, yhat = oracle.predict(f, codes)
    assert np.array_equal(yhat, np.rint(y * 65536.0) / 65536.0)


def test_matches_sklearn_tree_with_lossless_bins(oracle):
    """Same partition as a CART regression tree on raw values (black-box comparator).

    With lossless binning, no bootstrap and mtry = all columns, the forest's tree is
    CART with the squared-error criterion; on tie-free data its leaves hold exactly
    the same training rows as scikit-learn's DecisionTreeRegressor with
    min_samples_split = min.node.size + 1.
    """
    from sklearn.tree import DecisionTreeRegressor

    rng = np.random.default_rng(11)
    n, p = 180, 4
    X = rng.normal(size=(n, p)).astype(np.float32)
    dev = rng.integers(0, 3, size=n).astype(np.int32)
    y = rng.normal(size=n) + X[:, 0].astype(np.float64) * 2.0
    b = oracle.bin(X, dev, 3, 256)
    for min_node in (1, 4, 9):
        f = oracle.fit(b.codes, b.n_bins, y, 1, p + 1, min_node, bootstrap=False)
        tr = f.tree(0)
        # leaf id of each row in the oracle tree
        leaf_o = np.zeros(n, np.int64)
        for i in range(n):
            node = 0
            while tr["col"][node] != 255:
                c = tr["col"][node]
                node = tr["left"][node] + (0 if b.codes[i, c] <= tr["bin"][node] else 1)
            leaf_o[i] = node
        sk = DecisionTreeRegressor(min_samples_split=min_node + 1, random_state=0)
        Xd = np.concatenate([X.astype(np.float64), dev[:, None].astype(np.float64)], axis=1)
        sk.fit(Xd, np.rint(y * 65536.0))
        leaf_s = sk.apply(Xd)
        # same partition of the rows into leaves
        pairs = set(zip(leaf_o.tolist(), leaf_s.tolist()))
        assert len(pairs) == len(set(leaf_o.tolist())) == len(set(leaf_s.tolist()))
        assert sk.get_n_leaves() == int((tr["col"] == 255).sum())


def test_thread_count_and_run_invariance(oracle, d1_binned):
    ds, b = d1_binned
    f1 = oracle.fit(b.codes, b.n_bins, ds.y, 16, 6, 5, seed=5, n_threads=1)
    f8 = oracle.fit(b.codes, b.n_bins, ds.y, 16, 6, 5, seed=5, n_threads=8)
    f8b = oracle.fit(b.codes, b.n_bins, ds.y, 16, 6, 5, seed=5, n_threads=8)
    for a, c in ((f1, f8), (f8, f8b)):
        assert np.array_equal(a.n_nodes, c.n_nodes)
        for t in range(16):
            for k in ("col", "bin", "left", "q", "N"):
                assert np.array_equal(a.tree(t)[k], c.tree(t)[k])


def test_tree_range_is_independent_of_batch(oracle, d1_binned):
    """Tree t depends only on (seed, t): growing [5, 9) alone equals those trees of [0, 12)."""
    ds, b = d1_binned
    full = oracle.fit(b.codes, b.n_bins, ds.y, 12, 6, 5, seed=2)
    part = oracle.fit(b.codes, b.n_bins, ds.y, 12, 6, 5, seed=2, trees=range(5, 9))
    for t in range(5, 9):
        for k in ("col", "bin", "left", "q", "N"):
            assert np.array_equal(full.tree(t)[k], part.tree(t)[k])


def test_training_subset_equals_compacted_data(oracle, d1_binned):
    ds, b = d1_binned
    fold = synth.cv_folds()
    train = np.nonzero(fold != 3)[0]
    a = oracle.fit(b.codes, b.n_bins, ds.y, 6, 9, 3, seed=1, train_rows=train)
    c = oracle.fit(b.codes[train], b.n_bins, ds.y[train], 6, 9, 3, seed=1)
    for t in range(6):
        for k in ("col", "bin", "left", "q", "N"):
            assert np.array_equal(a.tree(t)[k], c.tree(t)[k])


def test_prediction_sum_and_mean(oracle, d1_binned):
    ds, b = d1_binned
    f = oracle.fit(b.codes, b.n_bins, ds.y, 8, 6, 5, seed=4)
    P, yhat = oracle.predict(f, b.codes)
    # the mean is the sum of leaf values scaled by 2^-32 and divided by the tree count
    assert np.array_equal(yhat, (P.astype(np.float64) * 2.0**-32) / 8.0)
    per_tree = np.zeros((8, ds.n), np.int64)
    for t in range(8):
        one = oracle.Forest(8, 0, f.capacity, f.col[t * f.capacity:(t + 1) * f.capacity],
                            f.bin[t * f.capacity:(t + 1) * f.capacity], f.left[t * f.capacity:(t + 1) * f.capacity],
                            f.q[t * f.capacity:(t + 1) * f.capacity], f.N[t * f.capacity:(t + 1) * f.capacity],
                            f.n_nodes[t:t + 1])
        per_tree[t] = oracle.predict(one, b.codes)[0]
    assert np.array_equal(per_tree.sum(axis=0), P)


def test_fit_argument_errors(oracle, d1_binned):
    ds, b = d1_binned
    with pytest.raises(oracle.OracleError):
        oracle.fit(b.codes, b.n_bins, ds.y, 1, 36, 1)  # mtry > columns
    with pytest.raises(oracle.OracleError):
        oracle.fit(b.codes, b.n_bins, ds.y, 1, 0, 1)
    with pytest.raises(oracle.OracleError):
        oracle.fit(b.codes, b.n_bins, ds.y, 1, 3, 0)
    bad = ds.y.copy()
    bad[7] = 70.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.fit(b.codes, b.n_bins, bad, 1, 3, 1)
    assert e.value.rc == oracle.ERANGE


def test_statistical_sanity_held_out(oracle):
    """Context only: held-out error on the synthetic frame is far below its spread."""
    ds = synth.d1()
    b = oracle.bin(ds.X, ds.device, ds.n_devices, 256)
    fold = synth.cv_folds()
    train = np.nonzero(fold != 0)[0]
    test = np.nonzero(fold == 0)[0]
    f = oracle.fit(b.codes, b.n_bins, ds.y, 64, 30, 9, seed=1, train_rows=train)
    _, yhat = oracle.predict(f, b.codes[test])
    mae = np.abs(yhat - ds.y[test]).mean()
    assert mae < 0.5 * np.abs(ds.y - ds.y.mean()).mean()


def test_last_code_column_splits_and_is_not_a_leaf(oracle):
    """With 255 code columns the last one (id 254) is an ordinary split column,
    distinct from the leaf marker; 256 columns are rejected."""
    n, C = 8, 255
    codes = np.zeros((n, C), np.uint8)
    codes[:, C - 1] = np.arange(n) % 2
    n_bins = np.full(C, 2, np.int32)
    y = np.where(codes[:, C - 1] == 1, 1.0, -1.0)
    f = oracle.fit(codes, n_bins, y, 1, C, 1, bootstrap=False)
    t = f.tree(0)
    assert t["col"][0] == C - 1 and t["col"][0] != oracle.LEAF
    assert list(t["col"][1:]) == [oracle.LEAF, oracle.LEAF]
    _, yhat = oracle.predict(f, codes)
    assert np.array_equal(yhat, y)
    wide = np.zeros((n, 256), np.uint8)
    with pytest.raises(oracle.OracleError) as e:
        oracle.fit(wide, np.full(256, 2, np.int32), y, 1, 1, 1)
    assert e.value.rc == oracle.EINVAL
