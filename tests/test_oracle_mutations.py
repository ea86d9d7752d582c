"""The pins have teeth: plausible mistakes planted in a copy of the oracle fail them.

Each mutation edits one expression of ``oracle/oracle_rf.c`` in a temporary copy,
compiles it on the CPU, and runs the exact tree verifier and the hand-derived
trees against it.  The real oracle is never modified.
"""
import ctypes
import json
import os
import subprocess

import numpy as np
import pytest

from tests._ref import verify_tree
from tests.test_oracle_tree import tiny_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle_rf.c")

MUTATIONS = {
    "tie_keeps_last": ("if (!found || score > best)", "if (!found || score >= best)"),
    "transposed_divisor": ("dSR * dSR / (double)NR", "dSR * dSR / (double)NL"),
    "dropped_right_term": ("dSL * dSL / (double)NL + dSR * dSR / (double)NR", "dSL * dSL / (double)NL"),
    "partition_strict": ("if (codes[row * C + best_c] <= best_b && (rc", "if (codes[row * C + best_c] < best_b && (rc"),
    "accept_zero_gain": ("split = found && (best - parent > 0.0);", "split = found && (best - parent >= 0.0);"),
    "min_node_inclusive": ("if (N > prm->min_node_size &&", "if (N >= prm->min_node_size &&"),
    "leaf_truncates": ("int64_t mag = (a * 131072 + N) / (2 * N);", "int64_t mag = (a * 131072) / (2 * N);"),
    "fisher_yates_full_range": ("int32_t j = k + (int32_t)scale_draw(r, (uint64_t)(C - k));",
                                "int32_t j = (int32_t)scale_draw(r, (uint64_t)C);"),
    "bootstrap_modulo": ("w[scale_draw(r, (uint64_t)n_train)] += 1;", "w[r % (uint64_t)n_train] += 1;"),
    "mtry_key_uses_tree_for_node": ("philox_draw(prm->seed, TAG_MTRY, (uint64_t)node, (uint64_t)tree, (uint64_t)k)",
                                    "philox_draw(prm->seed, TAG_MTRY, (uint64_t)tree, (uint64_t)node, (uint64_t)k)"),
    "purity_ignored": ("(__int128)N * Q != (__int128)S * S", "1"),
    "prefix_skips_first_bin": ("NL += hN[b];\n          SL += hS[b];", "NL += hN[b + 1 < B ? b : b];\n          SL += hS[b] + (b == 0 ? hS[b] : 0);"),
}


def run_battery(O, L):
    """True if every pin passes with library L."""
    old = O._lib
    O._lib = L
    try:
        for case in range(60):
            rng = np.random.default_rng(1000 + case)
            codes, n_bins, y = tiny_case(rng)
            n, C = codes.shape
            mtry = int(rng.integers(1, C + 1))
            min_node = int(rng.integers(1, 5))
            bootstrap = bool(rng.random() < 0.7)
            seed = int(rng.integers(0, 2**40))
            f = O.fit(codes, n_bins, y, 3, mtry, min_node, seed=seed, bootstrap=bootstrap, n_threads=1)
            y_fp = np.rint(y * 65536.0).astype(np.int64)
            for t in range(3):
                verify_tree(f.tree(t), codes, n_bins, y_fp, list(range(n)), seed, t, mtry, min_node, bootstrap)
        gold = json.load(open(os.path.join(ROOT, "tests", "golden", "hand_trees.json")))["cases"]
        for c in gold:
            b = O.bin(np.array(c["X"], np.float32), np.array(c["device"], np.int32), c["n_devices"], c["max_bins"])
            p = c["params"]
            f = O.fit(b.codes, b.n_bins, np.array(c["y"]), 1, p["mtry"], p["min_node_size"], seed=p["seed"],
                      bootstrap=bool(p["bootstrap"]))
            for k, v in c["tree"].items():
                assert f.tree(0)[k].tolist() == v
        return True
    except (AssertionError, O.OracleError, IndexError, KeyError):
        return False
    finally:
        O._lib = old


def test_unmutated_oracle_passes(oracle):
    assert run_battery(oracle, oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(oracle, tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = tmp_path / "oracle_rf.c"
    mutated.write_text(src.replace(old, new, 1))
    (tmp_path / "oracle_rf.h").write_text(open(os.path.join(ROOT, "oracle", "oracle_rf.h")).read())
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           str(mutated), "-o", str(so), "-lm"])
    L = oracle.configure(ctypes.CDLL(str(so)))
    assert not run_battery(oracle, L), f"planted mistake {name} went unnoticed"
