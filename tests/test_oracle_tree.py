"""Pin the oracle's tree growth against an exact, exhaustive re-derivation.

For tiny random inputs every node of every grown tree is checked by
``tests/_ref.verify_tree``: bootstrap weights and mtry candidate sets from NumPy's
Philox, node weights, leaf rules (min.node.size, purity, no improving split),
split optimality by exhaustive search over every (column, bin) with the exact
drop in sum of squared deviations, the first-strictly-greater tie rule, breadth
first child ids and exact leaf values.
"""
import numpy as np
import pytest

from tests._ref import verify_tree


def tiny_case(rng):
    n = int(rng.integers(1, 25))
    C = int(rng.integers(1, 5))
    n_bins = rng.integers(1, 9, size=C).astype(np.int32)
    codes = np.stack([rng.integers(0, nb, size=n) for nb in n_bins], axis=1).astype(np.uint8)
    if rng.random() < 0.5:
        y = rng.choice(np.array([-1.0, 0.0, 0.5, 2.0]), size=n)  # many ties and pure nodes
    else:
        y = rng.normal(0.0, 2.0, size=n)
    return codes, n_bins, y


@pytest.mark.parametrize("case", range(120))
def test_tiny_trees_exact(oracle, case):
    rng = np.random.default_rng(1000 + case)
    codes, n_bins, y = tiny_case(rng)
    n, C = codes.shape
    mtry = int(rng.integers(1, C + 1))
    min_node = int(rng.integers(1, 5))
    bootstrap = bool(rng.random() < 0.7)
    seed = int(rng.integers(0, 2**40))
    num_trees = 4
    f = oracle.fit(codes, n_bins, y, num_trees, mtry, min_node, seed=seed, bootstrap=bootstrap, n_threads=1)
    y_fp = np.rint(y * 65536.0).astype(np.int64)
    for t in range(num_trees):
        verify_tree(f.tree(t), codes, n_bins, y_fp, list(range(n)), seed, t, mtry, min_node, bootstrap)


@pytest.mark.parametrize("case", range(12))
def test_tiny_trees_with_training_subset(oracle, case):
    rng = np.random.default_rng(5000 + case)
    codes, n_bins, y = tiny_case(rng)
    n, C = codes.shape
    train = np.sort(rng.choice(n, size=max(1, n - int(rng.integers(0, n))), replace=False)).astype(np.int64)
    mtry = int(rng.integers(1, C + 1))
    f = oracle.fit(codes, n_bins, y, 3, mtry, 1, seed=7, train_rows=train, n_threads=1)
    y_fp = np.rint(y * 65536.0).astype(np.int64)
    y_train = y_fp[train]
    for t in range(3):
        # verify_tree indexes codes through train_rows and y through the local index
        verify_tree(f.tree(t), codes, n_bins, y_train, list(train), 7, t, mtry, 1, True)
