"""Hand-derived trees (tests/golden/hand_trees.json) reproduced by the oracle."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_trees.json")
CASES = json.load(open(GOLDEN))["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_tree(oracle, case):
    X = np.array(case["X"], np.float32)
    dev = np.array(case["device"], np.int32)
    b = oracle.bin(X, dev, case["n_devices"], case["max_bins"])
    p = case["params"]
    f = oracle.fit(b.codes, b.n_bins, np.array(case["y"]), p["num_trees"], p["mtry"], p["min_node_size"],
                   seed=p["seed"], bootstrap=bool(p["bootstrap"]))
    tr = f.tree(0)
    for k, v in case["tree"].items():
        assert tr[k].tolist() == v, k
    P, yhat = oracle.predict(f, b.codes)
    if "yhat" in case:
        assert yhat.tolist() == case["yhat"]
    else:
        assert np.all(P == case["tree"]["q"][0])
