"""Pins of the oracle's out-of-bag error and device selection (Sec. III-B, III-C).

The out-of-bag sums are re-derived here from NumPy's own Philox stream and a
Python traversal of the exported trees; the errors are re-derived in exact
rational arithmetic.  Device selection is checked on hand-built trees whose
answer is known, and by brute force against per-row traversal."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1811_00156_amd import synth
from _ref import bootstrap_weights


def _leaf_q(tree, row):
    node = 0
    while tree["col"][node] != 255:
        c = tree["col"][node]
        node = tree["left"][node] + (0 if row[c] <= tree["bin"][node] else 1)
    return int(tree["q"][node])


@pytest.fixture(scope="module")
def d1_binned(oracle):
    ds = synth.d1()
    return ds, oracle.bin(ds.X, ds.device, ds.n_devices, 64)


@pytest.mark.parametrize("fold", [-1, 4])
def test_oob_matches_brute_force(oracle, d1_binned, fold):
    ds, b = d1_binned
    folds = synth.cv_folds()
    train = None if fold < 0 else np.nonzero(folds != fold)[0]
    rows = np.arange(ds.n) if train is None else train
    T, seed = 9, 17
    f = oracle.fit(b.codes, b.n_bins, ds.y, T, 5, 3, seed=seed, train_rows=train)
    P, cnt, (mse, mae, m) = oracle.oob(f, b.codes, ds.y, 5, 3, seed=seed, train_rows=train)
    n = rows.shape[0]
    ref_P = [0] * n
    ref_c = [0] * n
    for t in range(T):
        w = bootstrap_weights(seed, t, n)
        tree = f.tree(t)
        for i in range(n):
            if w[i] == 0:
                ref_P[i] += _leaf_q(tree, b.codes[rows[i]])
                ref_c[i] += 1
    assert P.tolist() == ref_P
    assert cnt.tolist() == ref_c
    used = [i for i in range(n) if ref_c[i] > 0]
    assert m == len(used)
    # per-row error as the method defines it (one rounding per operation), mean exactly
    errs = [(float(ref_P[i]) * 2.0 ** -32) / float(ref_c[i]) - float(ds.y[rows[i]]) for i in used]
    ex_mse = sum(Fraction(e) * Fraction(e) for e in errs) / len(errs)
    ex_mae = sum(abs(Fraction(e)) for e in errs) / len(errs)
    # row-order summation of n non-negative terms: relative error below n * 2^-53
    tol = 2 * len(errs) * 2.0 ** -53
    assert abs(Fraction(mse) - ex_mse) <= tol * ex_mse
    assert abs(Fraction(mae) - ex_mae) <= tol * ex_mae


def test_oob_fraction_near_e_inverse(oracle, d1_binned):
    """Each row is left out of a bootstrap sample with probability (1 - 1/n)^n ~ 1/e."""
    ds, b = d1_binned
    T = 40
    f = oracle.fit(b.codes, b.n_bins, ds.y, T, 8, 5, seed=5)
    _, cnt, (_, _, m) = oracle.oob(f, b.codes, ds.y, 8, 5, seed=5)
    p = (1 - 1 / ds.n) ** ds.n
    frac = cnt.mean() / T
    sd = np.sqrt(p * (1 - p) / (T * ds.n))
    assert abs(frac - p) < 6 * sd
    assert m == int((cnt > 0).sum())


def test_oob_without_bootstrap_has_no_rows(oracle, d1_binned):
    ds, b = d1_binned
    f = oracle.fit(b.codes, b.n_bins, ds.y, 4, 8, 5, seed=5, bootstrap=False)
    P, cnt, (mse, mae, m) = oracle.oob(f, b.codes, ds.y, 8, 5, seed=5, bootstrap=False)
    assert m == 0 and mse == 0.0 and mae == 0.0
    assert not cnt.any() and not P.any()


def _hand_forest(oracle, col, bin_, left, q):
    k = len(col)
    return oracle.Forest(num_trees=1, tree_begin=0, capacity=k, col=np.array(col, np.uint8),
                         bin=np.array(bin_, np.uint8), left=np.array(left, np.int32), q=np.array(q, np.int64),
                         N=np.ones(k, np.int32), n_nodes=np.array([k], np.int64))


def test_select_device_ties_go_to_lowest_id(oracle):
    """A tree that never splits on the device predicts the same time everywhere."""
    f = _hand_forest(oracle, [0, 255, 255], [3, 0, 0], [1, -1, -1], [0, 7 << 32, -(5 << 32)])
    feats = np.array([[2, 9], [4, 1], [3, 3]], np.uint8)  # device column appended as column 2
    best, times = oracle.select_device(f, feats, 6)
    assert best.tolist() == [0, 0, 0]
    assert times.tolist() == [[7.0] * 6, [-5.0] * 6, [7.0] * 6]


def test_select_device_splits_on_device(oracle):
    """Device ids <= 1 are slow, the rest fast except where feature 0 is large."""
    # node 0: device <= 1 ? node 1 (leaf 3.0) : node 2; node 2: feature 0 <= 4 ? leaf -1.0 : leaf 2.5
    f = _hand_forest(oracle, [1, 255, 0, 255, 255], [1, 0, 4, 0, 0], [1, -1, 3, -1, -1],
                     [0, 3 << 32, 0, -(1 << 32), 5 << 31])
    feats = np.array([[0], [4], [5], [255]], np.uint8)
    best, times = oracle.select_device(f, feats, 4)
    assert best.tolist() == [2, 2, 2, 2]
    assert times[0].tolist() == [3.0, 3.0, -1.0, -1.0]
    assert times[2].tolist() == [3.0, 3.0, 2.5, 2.5]
    # with only devices 0 and 1 there is a tie at 3.0: the lowest id wins
    best2, _ = oracle.select_device(f, feats, 2)
    assert best2.tolist() == [0, 0, 0, 0]


def test_select_device_brute_force(oracle, d1_binned):
    ds, b = d1_binned
    T = 6
    f = oracle.fit(b.codes, b.n_bins, ds.y, T, 10, 5, seed=2)
    feats = b.codes[::97, :-1]
    best, times = oracle.select_device(f, feats, ds.n_devices)
    trees = [f.tree(t) for t in range(T)]
    for i in range(feats.shape[0]):
        row_t = []
        for d in range(ds.n_devices):
            row = np.concatenate([feats[i], [d]]).astype(np.uint8)
            P = sum(_leaf_q(tr, row) for tr in trees)
            row_t.append((float(P) * 2.0 ** -32) / T)
        assert times[i].tolist() == row_t
        assert best[i] == min(range(ds.n_devices), key=lambda d: (row_t[d], d))


def test_kernel_groups_and_study_masks():
    """D1's rows form 37 kernels of 4 sizes x 15 devices; the study masks select
    exactly the stated number of kernels, every kernel but one, reproducibly."""
    ds = synth.d1()
    g = synth.kernel_groups(ds)
    assert g.dtype == np.int8 and g.min() == 0 and g.max() == 36
    assert np.all(np.bincount(g) == 60)
    loo = synth.leave_one_kernel_out_masks()
    assert [bin(int(m)).count("1") for m in loo] == [36] * 37
    assert all((int(m) >> k) & 1 == 0 for k, m in enumerate(loo))
    cnt, masks = synth.kernel_subset_masks(repeats=3, counts=[1, 5, 37])
    assert cnt.tolist() == [1] * 3 + [5] * 3 + [37] * 3
    assert [bin(int(m)).count("1") for m in masks] == cnt.tolist()
    assert all(int(m) < (1 << 37) for m in masks)
    cnt2, masks2 = synth.kernel_subset_masks(repeats=3, counts=[1, 5, 37])
    assert np.array_equal(masks, masks2)


def test_heldout_matches_brute_force(oracle, d1_binned):
    """Held-out leaf sums by Python traversal; errors as exact rational means."""
    ds, b = d1_binned
    g = synth.kernel_groups(ds)
    train = np.nonzero(g != 7)[0]
    test = np.nonzero(g == 7)[0]
    T = 5
    f = oracle.fit(b.codes, b.n_bins, ds.y, T, 9, 3, seed=2, train_rows=train)
    P, (mse, mae, m) = oracle.heldout(f, b.codes, ds.y, test)
    trees = [f.tree(t) for t in range(T)]
    ref = [sum(_leaf_q(tr, b.codes[r]) for tr in trees) for r in test]
    assert P.tolist() == ref and m == test.shape[0] == 60
    errs = [(float(p) * 2.0 ** -32) / T - float(ds.y[r]) for p, r in zip(ref, test)]
    ex_mse = sum(Fraction(e) * Fraction(e) for e in errs) / len(errs)
    ex_mae = sum(abs(Fraction(e)) for e in errs) / len(errs)
    tol = 2 * len(errs) * 2.0 ** -53
    assert abs(Fraction(mse) - ex_mse) <= tol * ex_mse
    assert abs(Fraction(mae) - ex_mae) <= tol * ex_mae
    # nothing held out: no rows, zero errors
    P0, (a, b0, m0) = oracle.heldout(f, b.codes, ds.y, np.zeros(0, np.int64))
    assert P0.shape == (0,) and (a, b0, m0) == (0.0, 0.0, 0)


# ---------------------------------------------------------------------------- annealing search
def _numpy_proposals(seed, level, proposals, base, lower, upper, step_frac):
    """Proposals and uniforms of one level from NumPy's own Philox4x64-10."""
    from _ref import numpy_block

    half = [max(1, int(step_frac * (upper[c] - lower[c]))) for c in range(3)]
    out = []
    for j in range(proposals):
        w = [int(v) for v in numpy_block([0, 2, level, j], [seed, 0])[0]]
        p = tuple(min(upper[c], max(lower[c], base[c] + ((w[c] * (2 * half[c] + 1)) >> 64) - half[c]))
                  for c in range(3))
        out.append((p, (w[3] >> 11) / 2.0 ** 53))
    return out


def test_anneal_proposals_follow_the_philox_stream(oracle):
    """A flat objective accepts every proposal, so each level starts from the
    previous level's last proposal; the proposals equal NumPy's Philox draws."""
    lower, upper, start = (1, 1, 1), (1000, 35, 50), (500, 17, 25)
    best, fb, trace = oracle.anneal(lambda ts: [(1.0, 7)] * len(ts), lower, upper, start, 3, 4, 1.0, 0.5, 0.1, 99)
    assert all(t["accepted"] for t in trace) and best == start and fb == 1.0
    base = start
    for level in range(3):
        expect = _numpy_proposals(99, level, 4, base, lower, upper, 0.1)
        got = [t["params"] for t in trace if t["level"] == level]
        assert got == [p for p, _ in expect]
        base = got[-1]


def test_anneal_greedy_reaches_the_optimum(oracle):
    """At zero temperature only non-worsening proposals are taken; with unit steps
    on a separable convex objective the search ends at its minimum, and the best
    is the lowest value met (first on ties)."""
    target = (40, 5, 7)
    obj = lambda ts: [(float(sum((a - b) ** 2 for a, b in zip(t, target))), 1) for t in ts]
    best, fb, trace = oracle.anneal(obj, (1, 1, 1), (64, 12, 16), (3, 11, 15), 60, 8, 0.0, 0.9, 0.0, 3)
    assert best == target and fb == 0.0
    f_cur = trace[0]["objective"]
    for t in trace[1:]:
        assert t["accepted"] == (t["objective"] <= f_cur)
        if t["accepted"]:
            f_cur = t["objective"]
    vals = [t["objective"] for t in trace]
    assert fb == min(vals) and trace[vals.index(min(vals))]["params"] == best


def test_anneal_hot_accepts_everything_and_respects_bounds(oracle):
    obj = lambda ts: [(float(t[0] * 7 % 13 + t[1] + t[2]), 1) for t in ts]
    lower, upper = (2, 1, 3), (9, 4, 8)
    best, fb, trace = oracle.anneal(obj, lower, upper, (5, 2, 3), 10, 6, 1e300, 1.0, 0.5, 11)
    assert all(t["accepted"] for t in trace)
    for t in trace:
        assert all(lower[c] <= t["params"][c] <= upper[c] for c in range(3))


def test_anneal_accepts_worse_by_metropolis(oracle):
    """A worse proposal is taken iff u < exp(-(f' - f) / T), u from the stream."""
    obj = lambda ts: [(float(t[0]), 1) for t in ts]  # lower num.trees is better
    lower, upper, start = (1, 1, 1), (100, 1, 1), (50, 1, 1)
    best, fb, trace = oracle.anneal(obj, lower, upper, start, 1, 16, 5.0, 1.0, 0.2, 5)
    draws = _numpy_proposals(5, 0, 16, start, lower, upper, 0.2)
    f_cur = 50.0
    import math

    for (p, u), t in zip(draws, trace[1:]):
        d = p[0] - f_cur
        assert t["accepted"] == (d <= 0 or u < math.exp(-d / 5.0))
        if t["accepted"]:
            f_cur = float(p[0])


# ---------------------------------------------------------------------------- device ranking accuracy (Sec. VI)
def test_ranking_accuracy_against_kendall_tau(oracle):
    """Without ties, the share of concordant device pairs is (1 + tau) / 2 for
    Kendall's tau (scipy), so a dropped pair, a flipped comparison or a wrong
    index in the pair loop shows."""
    from scipy.stats import kendalltau

    rng = np.random.default_rng(4)
    m, D = 40, 15
    truth = rng.normal(size=(m, D))
    times = truth + rng.normal(scale=0.7, size=(m, D))
    correct, counted, hit = oracle.ranking_accuracy(times, truth)
    assert np.all(counted == D * (D - 1) // 2)
    for k in range(m):
        tau = kendalltau(times[k], truth[k]).statistic
        assert abs(correct[k] / counted[k] - (1.0 + tau) / 2.0) < 1e-12
        assert hit[k] == int(np.argmin(times[k]) == np.argmin(truth[k]))


def test_ranking_accuracy_special_cases(oracle):
    truth = np.array([[3.0, 1.0, 2.0, 5.0]])
    # a prediction that is a monotone transform of the truth ranks every pair right
    c, n, h = oracle.ranking_accuracy(2.0 * truth + 7.0, truth)
    assert (c[0], n[0], h[0]) == (6, 6, 1)
    # the reversed ranking ranks every pair wrong and misses the fastest device
    c, n, h = oracle.ranking_accuracy(-truth, truth)
    assert (c[0], n[0], h[0]) == (0, 6, 0)
    # equal true times leave a pair uncounted; a predicted tie chooses the lower id
    truth = np.array([[1.0, 1.0, 2.0]])
    times = np.array([[0.5, 0.5, 0.5]])
    c, n, h = oracle.ranking_accuracy(times, truth)
    # pairs (0,2) and (1,2) count; the tie picks device 0 (resp. 1), both faster
    assert (c[0], n[0], h[0]) == (2, 2, 1)
    times = np.array([[0.7, 0.5, 0.5]])  # (1,2) tie -> device 1 (right); (0,2) picks 2 (wrong)
    c, n, h = oracle.ranking_accuracy(times, truth)
    assert (c[0], n[0], h[0]) == (1, 2, 1)
    # the best is hit when its true time equals the smallest, whichever device that is
    times = np.array([[0.6, 0.5, 0.9]])
    assert oracle.ranking_accuracy(times, truth)[2][0] == 1


def test_ranking_of_synthetic_truth(oracle):
    """The generator's noiseless truth ranks its own devices perfectly, and the
    noisy responses it drew rank most pairs right (the noise is small against
    the device offsets)."""
    from paper_1811_00156_amd import synth

    ds = synth.d1()
    c, n, h = oracle.ranking_accuracy(ds.truth, ds.truth)
    assert np.all(c == n) and np.all(h == 1)
    noisy = np.zeros_like(ds.truth)
    noisy[ds.kernel, ds.device] = ds.y
    c, n, h = oracle.ranking_accuracy(noisy, ds.truth)
    assert c.sum() / n.sum() > 0.95
