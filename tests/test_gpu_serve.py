"""Serving: each answer is the same alone and inside a mixed, continuously batched stream."""
import numpy as np
import pytest

from paper_1811_00156_amd import synth
from tests._gpu import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    ds = synth.small(n_vec=400, n_devices=16, p_ln=8, p_u=6, seed=3)
    ob = O.bin(ds.X, ds.device, ds.n_devices, 128)
    binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
    forest = rf.aiwc_rf_fit(to_dev(ob.codes), binner, to_dev(ds.y), rf.make_params(64, 5, 3, True, 2))
    return rf, forest, ob.codes


def test_alone_equals_mixed(served):
    rf, forest, codes = served
    rng = np.random.default_rng(5)
    sizes = [1, 7, 4096, 300, 1, 2, 999, 64, 65, 3000, 17, 1, 2048]
    reqs = [np.ascontiguousarray(codes[rng.integers(0, codes.shape[0], size=s)]) for s in sizes]
    alone = [rf.aiwc_rf_predict(forest, to_dev(r)).cpu().numpy() for r in reqs]
    log("serve mixed stream")
    # a row slot costs 2 * 15 + 24 = 54 bytes of the budget (device codes, sum and
    # answer; pinned codes and answer), so 280000 bytes hold about 5100 rows: the
    # 4096-row request fits, the whole stream (10495 rows) does not, and later
    # requests wait for retiring batches
    budget = 280_000
    srv = rf.Server(forest, memory_budget_bytes=budget, max_batch_rows=4096, n_streams=3)
    outs = [np.zeros(r.shape[0]) for r in reqs]
    tickets = [srv.submit(r, o) for r, o in zip(reqs, outs)]
    srv.drain()
    done, lat = srv.poll()
    assert sorted(done.tolist()) == sorted(tickets)
    assert np.all(lat > 0)
    for a, o in zip(alone, outs):
        assert np.array_equal(a.view(np.uint64), o.view(np.uint64))
    st = srv.stats()
    assert st.rows == sum(sizes)
    assert st.peak_bytes <= budget
    assert st.batches < len(sizes)  # requests were batched together
    assert st.memory_waits > 0  # and some waited for memory
    srv.close()


def test_admission_limits(served):
    rf, forest, codes = served
    srv = rf.Server(forest, memory_budget_bytes=10_000, max_batch_rows=100, n_streams=1)
    big = np.ascontiguousarray(codes[:200])
    with pytest.raises(rf.RFError) as e:
        srv.submit(big, np.zeros(200))
    assert e.value.rc == rf.ENOMEM
    assert "max_batch_rows" in str(e.value)
    srv.close()
    # a request larger than the whole budget can never be admitted
    srv = rf.Server(forest, memory_budget_bytes=10_000, max_batch_rows=1000, n_streams=1)
    with pytest.raises(rf.RFError) as e:
        srv.submit(big, np.zeros(200))
    assert e.value.rc == rf.ENOMEM
    assert "memory budget" in str(e.value)
    srv.close()
