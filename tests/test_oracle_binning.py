"""Pin the oracle's quantile binning.

Binning is not described in the paper (ranger splits on raw values); the reading
taken is: per feature column, thresholds are the order statistics
s[floor(k n / B) - 1], k = 1..B-1, of the column's sorted values, with repeats and
values not below the column maximum dropped, unless the column has at most B
distinct values, in which case the thresholds are all distinct values but the
largest (lossless).  code(x) = number of thresholds strictly below x.  The device
id is its own column with code = id.  The pins below do not retype that rule:
they check the rank property, monotonicity, exact bin populations of tie-free data
(a closed form), and error handling.
"""
import numpy as np
import pytest

from paper_1811_00156_amd import synth


def test_lossless_codes_are_distinct_ranks(oracle):
    ds = synth.d1()  # 148 distinct vectors per column, so 256 bins are lossless
    b = oracle.bin(ds.X, ds.device, ds.n_devices, 256)
    for j in range(ds.p):
        _, inv = np.unique(ds.X[:, j], return_inverse=True)
        assert np.array_equal(b.codes[:, j], inv.astype(np.uint8))
        assert b.n_bins[j] == 148
    assert np.array_equal(b.codes[:, ds.p], ds.device.astype(np.uint8))
    assert b.n_bins[ds.p] == ds.n_devices


@pytest.mark.parametrize("n,B", [(1000, 64), (2220, 64), (997, 256), (5000, 7), (300, 2)])
def test_tie_free_bin_populations_closed_form(oracle, n, B):
    rng = np.random.default_rng(n + B)
    X = rng.permutation(np.arange(1, n + 1, dtype=np.float32) * 0.37)[:, None]
    X = np.concatenate([X, -X * 3.0], axis=1).astype(np.float32)
    dev = np.zeros(n, np.int32)
    b = oracle.bin(X, dev, 1, B)
    for j in range(2):
        counts = np.bincount(b.codes[:, j], minlength=B)
        k = np.arange(B)
        expect = (k + 1) * n // B - k * n // B
        assert np.array_equal(counts, expect)
        assert b.n_bins[j] == B


def test_monotone_thresholds_are_data_values(oracle):
    ds = synth.d3()
    sub = slice(0, 20000)
    X, dev = ds.X[sub], ds.device[sub]
    b = oracle.bin(X, dev, ds.n_devices, 256)
    for j in range(0, ds.p, 7):
        t = b.column_thresholds(j)
        assert np.all(np.diff(t) > 0)
        assert np.all(t < X[:, j].max())
        assert np.all(np.isin(t, X[:, j]))
        order = np.argsort(X[:, j], kind="stable")
        assert np.all(np.diff(b.codes[order, j].astype(int)) >= 0)
        # every code is used (thresholds are data values, so every bin holds its threshold)
        assert len(np.unique(b.codes[:, j])) == b.n_bins[j]


def test_heavy_ties_and_signed_zero(oracle):
    n = 500
    rng = np.random.default_rng(3)
    x = rng.choice(np.array([-0.0, 0.0, 1.5, 2.5, 2.5, 9.0], np.float32), size=n)
    X = np.stack([x, np.full(n, 4.0, np.float32)], axis=1)
    b = oracle.bin(X, np.zeros(n, np.int32), 1, 2)
    # -0.0 and +0.0 share a code; a constant column has one bin
    assert len(set(b.codes[X[:, 0] == 0.0, 0])) == 1
    assert b.n_bins[1] == 1 and np.all(b.codes[:, 1] == 0)
    assert b.n_bins[0] <= 2


def test_apply_matches_fit_and_clamps(oracle):
    ds = synth.d1()
    b = oracle.bin(ds.X, ds.device, ds.n_devices, 64)
    assert np.array_equal(oracle.bin_apply(b, ds.X, ds.device, ds.n_devices), b.codes)
    far = np.concatenate([np.full((1, ds.p), -1e30, np.float32), np.full((1, ds.p), 1e30, np.float32)])
    c = oracle.bin_apply(b, far, np.array([0, 14], np.int32), ds.n_devices)
    assert np.all(c[0, :ds.p] == 0)
    assert np.array_equal(c[1, :ds.p], (b.n_bins[:ds.p] - 1).astype(np.uint8))


def test_invalid_arguments(oracle):
    X = np.ones((4, 2), np.float32)
    dev = np.zeros(4, np.int32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.bin(np.where(np.eye(4, 2) > 0, np.nan, X).astype(np.float32), dev, 1, 8)
    assert e.value.rc == oracle.EINVAL
    with pytest.raises(oracle.OracleError):
        oracle.bin(X, np.array([0, 1, 2, 3], np.int32), 3, 8)  # device id out of range
    with pytest.raises(oracle.OracleError):
        oracle.bin(X, dev, 1, 1)  # max_bins < 2
    with pytest.raises(oracle.OracleError):
        oracle.bin(X, dev, 1, 257)
    with pytest.raises(oracle.OracleError) as e:
        oracle.y_fixed(np.array([0.0, 64.5]))
    assert e.value.rc == oracle.ERANGE
    with pytest.raises(oracle.OracleError):
        oracle.y_fixed(np.array([np.inf]))


def test_fixed_point_rounds_half_even(oracle):
    y = np.array([0.5 / 65536, 1.5 / 65536, -0.5 / 65536, -2.5 / 65536, 64.0, -64.0, 1.0 / 3.0])
    got = oracle.y_fixed(y)
    assert got.tolist() == [0, 2, 0, -2, 64 << 16, -(64 << 16), 21845]


def test_column_limit_below_leaf_marker(oracle):
    """Column ids must stay below the leaf marker 255: 254 features (255 code
    columns with the device) are accepted, 255 features are rejected."""
    rng = np.random.default_rng(3)
    dev = np.zeros(6, np.int32)
    b = oracle.bin(rng.normal(size=(6, 254)).astype(np.float32), dev, 1, 4)
    assert b.codes.shape == (6, 255)
    with pytest.raises(oracle.OracleError) as e:
        oracle.bin(rng.normal(size=(6, 255)).astype(np.float32), dev, 1, 4)
    assert e.value.rc == oracle.EINVAL
