"""The allocation-free prediction entry point against aiwc_rf_predict, bit for bit.

Two calls in a row (the second with fewer rows, so stale sums of the first sit
in the shared array), a call large enough that one tree chunk covers all trees
(sums written, not accumulated), argument limits, and the oracle's predictions.
"""
import numpy as np
import pytest

from paper_1811_00156_amd import synth
from tests._gpu import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fitted():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    ds = synth.small(n_vec=500, n_devices=12, p_ln=6, p_u=5, seed=21)
    ob = O.bin(ds.X, ds.device, ds.n_devices, 64)
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    forest = rf.aiwc_rf_fit(to_dev(ob.codes), binner, to_dev(ds.y), rf.make_params(96, 4, 3, True, 9))
    of = O.fit(ob.codes, ob.n_bins, ds.y, 96, 4, 3, seed=9)
    return rf, O, forest, of, ob.codes


def rows(codes, m, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(codes[rng.integers(0, codes.shape[0], size=m)])


@pytest.mark.parametrize("first,second", [(5000, 300), (300_000, 1)])
def test_noalloc_equals_predict(fitted, first, second):
    import torch

    rf, O, forest, of, codes = fitted
    for m, seed in ((first, 1), (second, 2)):
        log(f"predict_noalloc m={m}")
        c_host = rows(codes, m, seed + first)
        c = to_dev(c_host)
        want = rf.aiwc_rf_predict(forest, c).cpu().numpy()
        out = torch.full((m,), float("nan"), dtype=torch.float64, device=c.device)
        rf.aiwc_rf_predict_noalloc(forest, c, out)
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), f"m={m}: differs from aiwc_rf_predict"
        if m <= 5000:
            _, yhat = O.predict(of, c_host)
            assert np.array_equal(got.view(np.uint64), yhat.view(np.uint64)), f"m={m}: differs from the oracle"


def test_noalloc_limits(fitted):
    import torch

    rf, _, forest, _, codes = fitted
    c = to_dev(rows(codes, 4, 0))
    out = torch.empty(0, dtype=torch.float64, device=c.device)
    rf.aiwc_rf_predict_noalloc(forest, c[:0], out)  # n = 0: nothing to do
    big = (1 << 20) + 1
    cb = torch.zeros((big, codes.shape[1]), dtype=torch.uint8, device=c.device)
    ob = torch.empty(big, dtype=torch.float64, device=c.device)
    with pytest.raises(rf.RFError) as e:
        rf.aiwc_rf_predict_noalloc(forest, cb, ob)
    assert e.value.rc == rf.EINVAL and "2^20" in str(e.value)
    with pytest.raises(rf.RFError) as e:
        rf.aiwc_rf_predict_noalloc(forest, c, torch.empty(4, dtype=torch.float64, device=c.device), forest_index=1)
    assert e.value.rc == rf.EINVAL
