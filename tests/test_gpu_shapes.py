"""Launch shapes never change results: every workgroup size and huge-node limit,
and the autotuned choice, grow the same forest bit for bit (and match the oracle)."""
import os

import numpy as np
import pytest

from paper_1811_00156_amd import synth
from tests._gpu import assert_tree_equal, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    ds = synth.small(n_vec=1500, n_devices=6, p_ln=6, p_u=4, seed=21)  # 9000 rows
    ob = O.bin(ds.X, ds.device, ds.n_devices, 256)
    of = O.fit(ob.codes, ob.n_bins, ds.y, 6, 4, 3, seed=9)
    return rf, ds, ob, of


def fit_with(rf, ds, ob, env, flags=0, params=None):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        binner = rf.aiwc_rf_binner_from_counts(ob.n_bins)
        prm = params if params is not None else rf.make_params(6, 4, 3, True, 9)
        return rf.aiwc_rf_fit(to_dev(ob.codes), binner, to_dev(ds.y), prm, flags=flags)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("block", ["192", "256", "512", "1024"])
@pytest.mark.parametrize("huge_min", ["64", "300", "2048", "4096", "100000"])
def test_shape_invariance(setup, block, huge_min):
    rf, ds, ob, of = setup
    log(f"shape block={block} huge_min={huge_min}")
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_HUGE_MIN": huge_min})
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"block {block} huge_min {huge_min} tree {t}")


@pytest.mark.parametrize("block", ["64", "128"])
@pytest.mark.parametrize("occ", ["4", "5", "6"])
def test_narrow_workgroup_invariance(setup, block, occ):
    """One- and two-wave workgroups (the shapes of deep grid queues) grow the
    same trees; they never take the workgroup-wide phase."""
    rf, ds, ob, of = setup
    log(f"shape block={block} occ={occ}")
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_GROW_OCC": occ, "AIWC_RF_HUGE_MIN": "100000"})
    li = f.launch()
    assert (li["block"], li["waves_per_simd"], li["wide_phase"]) == (int(block), int(occ), 0)
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"block {block} occ {occ} tree {t}")
    with pytest.raises(rf.RFError):
        fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_HUGE_MIN": "300"})


def test_autotuned_fit_matches(setup):
    rf, ds, ob, of = setup
    f = fit_with(rf, ds, ob, {}, flags=rf.FIT_TUNE)
    g = fit_with(rf, ds, ob, {}, flags=rf.FIT_TUNE)  # second call: cached shape
    for t in range(6):
        assert_tree_equal(f.export(0, t, t + 1)[0], of.tree(t), f"tuned tree {t}")
        assert_tree_equal(g.export(0, t, t + 1)[0], of.tree(t), f"cached tuned tree {t}")
    codes = to_dev(ob.codes)
    _, yhat = __import__("oracle.oracle", fromlist=["predict"]).predict(of, ob.codes)
    assert np.array_equal(rf.aiwc_rf_predict(f, codes).cpu().numpy().view(np.uint64), yhat.view(np.uint64))


@pytest.mark.parametrize("block", ["192", "256", "1024"])
def test_wide_batches_in_column_chunks(block):
    """Every node above 64 rows in workgroup-wide batches, with more candidate
    columns (35 of 35, 256 bins) than one batch's LDS holds at a 256-thread
    workgroup, so the columns are histogrammed in chunks."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    log(f"wide chunks block={block}")
    ds = synth.d1()
    ob = O.bin(ds.X, ds.device, ds.n_devices, 256)
    of = O.fit(ob.codes, ob.n_bins, ds.y, 4, 35, 1, seed=5)
    old = {k: os.environ.get(k) for k in ("AIWC_RF_GROW_BLOCK", "AIWC_RF_HUGE_MIN")}
    os.environ.update({"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_HUGE_MIN": "64"})
    try:
        f = rf.aiwc_rf_fit(to_dev(ob.codes), rf.aiwc_rf_binner_from_counts(ob.n_bins), to_dev(ds.y),
                           rf.make_params(4, 35, 1, True, 5))
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"wide chunks block {block} tree {t}")


@pytest.mark.parametrize("block,huge_min", [("256", "64"), ("1024", "64"), ("512", "100000")])
def test_wide_code_rows_and_many_candidates(block, huge_min):
    """100 features (code rows wider than 80 bytes, so the wide batches gather
    codes byte by byte) and mtry 90 (more candidates than one 64-column staging
    chunk of the small-node tasks), against the oracle."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    log(f"wide rows block={block} huge_min={huge_min}")
    ds = synth.small(n_vec=700, n_devices=5, p_ln=60, p_u=40, seed=41)  # 3500 rows, 101 code columns
    ob = O.bin(ds.X, ds.device, ds.n_devices, 256)
    of = O.fit(ob.codes, ob.n_bins, ds.y, 3, 90, 1, seed=6)
    old = {k: os.environ.get(k) for k in ("AIWC_RF_GROW_BLOCK", "AIWC_RF_HUGE_MIN")}
    os.environ.update({"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_HUGE_MIN": huge_min})
    try:
        f = rf.aiwc_rf_fit(to_dev(ob.codes), rf.aiwc_rf_binner_from_counts(ob.n_bins), to_dev(ds.y),
                           rf.make_params(3, 90, 1, True, 6))
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"wide rows block {block} huge_min {huge_min} tree {t}")


@pytest.mark.parametrize("block", ["192", "256", "512", "1024"])
@pytest.mark.parametrize("occ", ["5", "6"])
def test_occupancy_variants(setup, block, occ):
    """The kernel without the wide phase built for 5 and 6 waves per SIMD grows
    the same trees."""
    rf, ds, ob, of = setup
    log(f"occupancy block={block} occ={occ}")
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_HUGE_MIN": "100000", "AIWC_RF_GROW_OCC": occ})
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"block {block} occupancy {occ} tree {t}")


@pytest.mark.parametrize("block", ["192", "1024"])
@pytest.mark.parametrize("big_cols", ["1", "2", "3", "4"])
def test_large_node_columns_per_task(block, big_cols):
    """Large-node tasks taking 1 to 4 candidate columns each (mtry 7, so the
    last task of a node takes fewer) grow the oracle's trees."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    log(f"large-node columns block={block} big_cols={big_cols}")
    ds = synth.small(n_vec=700, n_devices=5, p_ln=8, p_u=6, seed=43)  # 3500 rows
    ob = O.bin(ds.X, ds.device, ds.n_devices, 100)
    of = O.fit(ob.codes, ob.n_bins, ds.y, 4, 7, 1, seed=8)
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_HUGE_MIN": "100000", "AIWC_RF_BIG_COLS": big_cols},
                 params=rf.make_params(4, 7, 1, True, 8))
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"block {block} big_cols {big_cols} tree {t}")


@pytest.mark.parametrize("big_cols", ["2", "4"])
def test_large_node_columns_with_256_bins(setup, big_cols):
    """With 256-bin columns a wave's LDS area holds two large-node histograms,
    so a request for four columns per task takes two; the trees still match."""
    rf, ds, ob, of = setup
    assert max(ob.n_bins) > 152
    log(f"large-node columns 256 bins big_cols={big_cols}")
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": "192", "AIWC_RF_HUGE_MIN": "100000", "AIWC_RF_BIG_COLS": big_cols})
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"256 bins big_cols {big_cols} tree {t}")


def test_partition_cursors_in_global_memory():
    """A level with more nodes than a 192-thread workgroup's LDS area holds
    cursors for (about 900) keeps its partition cursors in global memory; a deep
    tree on 60000 rows has such levels, and still matches the oracle."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    log("global partition cursors")
    ds = synth.small(n_vec=10000, n_devices=6, p_ln=6, p_u=4, seed=47)  # 60000 rows
    ob = O.bin(ds.X, ds.device, ds.n_devices, 64)
    of = O.fit(ob.codes, ob.n_bins, ds.y, 2, 5, 1, seed=12)
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": "192", "AIWC_RF_HUGE_MIN": "100000"},
                 params=rf.make_params(2, 5, 1, True, 12))
    # some level holds far more than 900 nodes (the widest about 10000)
    widest = 0
    for t in range(2):
        left, level = of.tree(t)["left"], [0]
        while level:
            widest = max(widest, len(level))
            level = [c for k in level if left[k] >= 0 for c in (left[k], left[k] + 1)]
    assert widest > 4 * 900, widest
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"global cursors tree {t}")


@pytest.mark.parametrize("p_ln,p_u,n_vec", [(40, 20, 4000), (60, 40, 2400)])
@pytest.mark.parametrize("huge_min", ["64", "100000"])
def test_line_aligned_code_rows(p_ln, p_u, n_vec, huge_min):
    """Training sets whose codes exceed 1 MB are gathered from the copy whose
    rows are padded to a cache-line divisor or multiple (64 bytes for 61
    columns, 128 for 101): the trees still match the oracle."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_1811_00156_amd import rf

    ds = synth.small(n_vec=n_vec, n_devices=5, p_ln=p_ln, p_u=p_u, seed=53)
    assert ds.n * (ds.X.shape[1] + 1) > 1 << 20
    log(f"line-aligned rows {ds.n} x {ds.X.shape[1] + 1} huge_min={huge_min}")
    ob = O.bin(ds.X, ds.device, ds.n_devices, 256)
    of = O.fit(ob.codes, ob.n_bins, ds.y, 2, 20, 2, seed=14)
    f = fit_with(rf, ds, ob, {"AIWC_RF_GROW_BLOCK": "512", "AIWC_RF_HUGE_MIN": huge_min},
                 params=rf.make_params(2, 20, 2, True, 14))
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"line-aligned rows huge_min {huge_min} tree {t}")


@pytest.mark.parametrize("wide_sums", ["0", "1"])
@pytest.mark.parametrize("block,occ", [("192", "6"), ("512", "4")])
def test_small_node_sums_byte_planes_and_64_bit(setup, wide_sums, block, occ):
    """The small-node searches' left sums from byte-plane dot products (weights
    below 256) and from 64-bit adds (forced) grow the same trees; no-bootstrap
    and bootstrap forests, with 64-row leaves so that every segment width occurs."""
    rf, ds, ob, of = setup
    env = {"AIWC_RF_WIDE_SUMS": wide_sums, "AIWC_RF_GROW_BLOCK": block, "AIWC_RF_GROW_OCC": occ,
           "AIWC_RF_HUGE_MIN": "100000"}
    log(f"small-node sums wide_sums={wide_sums} block={block}")
    f = fit_with(rf, ds, ob, env)
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, of.tree(t), f"wide_sums {wide_sums} tree {t}")
    from oracle import oracle as O

    ofn = O.fit(ob.codes, ob.n_bins, ds.y, 3, 7, 1, seed=4, bootstrap=False)
    g = fit_with(rf, ds, ob, env, params=rf.make_params(3, 7, 1, False, 4))
    for t, tree in enumerate(g.export()):
        assert_tree_equal(tree, ofn.tree(t), f"wide_sums {wide_sums} no bootstrap tree {t}")


@pytest.mark.parametrize("bins", [64, 256])
@pytest.mark.parametrize("block,occ", [("64", "5"), ("192", "6")])
def test_small_node_sums_wide_responses(setup, bins, block, occ):
    """Responses ten times wider (log10 times in [-59, -7]): with bootstrap
    weights of 3 and more, w y no longer fits 24 bits in many waves, so the
    small-node searches take both the four- and the five-plane byte sums (and,
    at 64 bins, the 7-bit code comparisons); the trees equal the oracle's."""
    rf, ds, ob, of = setup
    from oracle import oracle as O

    y10 = np.ascontiguousarray(ds.y * 10.0)
    assert np.abs(y10).max() < 64.0
    obb = O.bin(ds.X, ds.device, ds.n_devices, bins)
    ofb = O.fit(obb.codes, obb.n_bins, y10, 4, 5, 1, seed=23)
    env = {"AIWC_RF_GROW_BLOCK": block, "AIWC_RF_GROW_OCC": occ, "AIWC_RF_HUGE_MIN": "100000"}
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        binner = rf.aiwc_rf_binner_from_counts(obb.n_bins)
        f = rf.aiwc_rf_fit(to_dev(obb.codes), binner, to_dev(y10), rf.make_params(4, 5, 1, True, 23))
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    log(f"wide responses bins={bins} block={block}")
    for t, tree in enumerate(f.export()):
        assert_tree_equal(tree, ofb.tree(t), f"wide responses bins {bins} block {block} tree {t}")
