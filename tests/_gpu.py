"""Helpers of the GPU parity tests: device upload, oracle comparison, progress."""
import sys

import numpy as np


def log(msg: str):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def dev():
    import torch

    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def assert_tree_equal(gpu_tree: dict, oracle_tree: dict, what: str):
    for k in ("col", "bin", "left", "q", "N"):
        g, o = gpu_tree[k], oracle_tree[k]
        assert g.shape == o.shape, f"{what}: {k} has {g.shape[0]} nodes on the GPU, {o.shape[0]} in the oracle"
        if not np.array_equal(g, o):
            i = int(np.nonzero(g != o)[0][0])
            raise AssertionError(f"{what}: {k} differs first at node {i}: gpu {g[i]} oracle {o[i]}")
