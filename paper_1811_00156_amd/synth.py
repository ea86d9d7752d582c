"""Seeded synthetic workloads shaped like the paper's data.

The paper's training frame pairs the AIWC feature vector of each OpenCL kernel
invocation (Table I; 34 predictor columns, Sec. III-B) with its execution time
measured on each of 15 devices (Table II), for 37 kernels at 4 problem sizes
(Sec. III-A).  Neither the feature vectors nor the timings are published, so this
module draws stand-ins with the same shape:

* one feature vector per (kernel, size) pair: the first ``p_ln`` columns are
  log-normal counts ``exp(8 + 3 z)``, the remaining ``p_u`` columns are uniform
  scores in ``[0, 32)``; all stored as float32;
* the vector is replicated across every device, because AIWC features do not
  depend on the device (Abstract, Sec. I);
* the response is a log10 time: a linear term and a few pairwise products of the
  standardised features, a per-device offset and small noise;
* rows are shuffled by a seeded permutation.

This module holds no arithmetic of the forest method itself (no binning, no
sampling, no fixed point): both the CPU oracle and the HIP library consume its
output, and neither is imported here.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Seeds of the five workloads (kept here so tests, bench and fixtures agree).
SEED_D1 = 181100156
SEED_D3 = 181100157
SEED_FOLDS = 181100158
SEED_REQUESTS = 181100159
SEED_SUBSETS = 181100160

# Held-out fold sizes of the 10-fold cross-validation grid (sum 2220).
FOLD_SIZES = (199, 245, 210, 233, 222, 215, 229, 204, 240, 223)


@dataclass
class Dataset:
    X: np.ndarray  # float32 [n, p] row-major feature matrix
    device: np.ndarray  # int32 [n] device id in [0, n_devices)
    y: np.ndarray  # float64 [n] log10 execution time (seconds)
    kernel: np.ndarray  # int32 [n] index of the (kernel, size) vector the row replicates
    n_devices: int
    # noiseless log10 time of every (vector, device): the response without its
    # per-row noise term, the "measured" ordering a device choice is judged by
    truth: np.ndarray | None = None  # float64 [n_vectors, n_devices]

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])


def generate(n_kernels: int, n_sizes: int, n_devices: int, p_ln: int, p_u: int,
             n_pairs: int, seed: int) -> Dataset:
    """Draw the synthetic frame described in the module docstring.

    The draws happen in a fixed order from ``numpy.random.Generator(PCG64(seed))``:
    z (log-normal normals), uniforms, linear weights a, pair indices, pair weights
    b, device offsets, per-row noise, row permutation.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n_vec = n_kernels * n_sizes
    p = p_ln + p_u
    z = rng.standard_normal((n_vec, p_ln))
    x_ln = np.exp(8.0 + 3.0 * z).astype(np.float32)
    x_u = rng.uniform(0.0, 32.0, size=(n_vec, p_u)).astype(np.float32)
    vec = np.concatenate([x_ln, x_u], axis=1)

    # standardised features, computed from the stored float32 values
    u = np.empty((n_vec, p), dtype=np.float64)
    u[:, :p_ln] = (np.log(vec[:, :p_ln].astype(np.float64)) - 8.0) / 3.0
    u[:, p_ln:] = vec[:, p_ln:].astype(np.float64) / 16.0 - 1.0

    a = rng.normal(0.0, 0.3, size=p)
    pairs = np.stack([rng.choice(p, size=2, replace=False) for _ in range(n_pairs)]) if n_pairs else np.zeros((0, 2), int)
    b = rng.normal(0.0, 0.2, size=n_pairs)
    dev_off = rng.normal(0.0, 1.0, size=n_devices)

    base = -3.0 + u @ a
    for (j, k), bjk in zip(pairs, b):
        base = base + bjk * u[:, j] * u[:, k]

    n = n_vec * n_devices
    kernel = np.repeat(np.arange(n_vec, dtype=np.int32), n_devices)
    device = np.tile(np.arange(n_devices, dtype=np.int32), n_vec)
    eps = rng.normal(0.0, 0.05, size=n)
    y = base[kernel] + dev_off[device] + eps

    perm = rng.permutation(n)
    X = np.ascontiguousarray(vec[kernel[perm]])
    truth = np.ascontiguousarray(base[:, None] + dev_off[None, :])
    ds = Dataset(X=X, device=np.ascontiguousarray(device[perm]), y=np.ascontiguousarray(y[perm]),
                 kernel=np.ascontiguousarray(kernel[perm]), n_devices=n_devices, truth=truth)
    assert np.all(np.abs(ds.y) <= 64.0), "synthetic response outside the fixed-point range"
    return ds


def d1() -> Dataset:
    """37 kernels x 4 sizes x 15 devices, 20 log-normal + 14 uniform features."""
    return generate(37, 4, 15, 20, 14, 16, SEED_D1)


def d3() -> Dataset:
    """6250 vectors x 32 devices = 200000 rows, 40 log-normal + 24 uniform features."""
    return generate(6250, 1, 32, 40, 24, 24, SEED_D3)


def vector_rows(ds: Dataset) -> np.ndarray:
    """For every (kernel, size) vector v, one row index of the frame that holds it
    (the first), so ds.X[vector_rows(ds)[v]] is vector v's features."""
    first = np.full(int(ds.kernel.max()) + 1, -1, dtype=np.int64)
    order = np.argsort(ds.kernel, kind="stable")
    ks = ds.kernel[order]
    starts = np.r_[0, np.nonzero(np.diff(ks))[0] + 1]
    first[ks[starts]] = order[starts]
    return first


def small(n_vec: int, n_devices: int, p_ln: int, p_u: int, seed: int, n_pairs: int = 4) -> Dataset:
    """A small frame of the same family, for parity cases that must run in seconds."""
    return generate(n_vec, 1, n_devices, p_ln, p_u, n_pairs, seed)


def cv_folds(n: int = 2220, sizes=FOLD_SIZES, seed: int = SEED_FOLDS) -> np.ndarray:
    """Fold id (int8) per row: a seeded permutation cut into the given fold sizes."""
    assert sum(sizes) == n
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(n)
    fold = np.empty(n, dtype=np.int8)
    start = 0
    for f, s in enumerate(sizes):
        fold[perm[start:start + s]] = f
        start += s
    return fold


def grid_forests(n_folds: int = 10, mtry_max: int = 34, min_node_sizes=(1, 3, 5, 7, 9)):
    """(held-out fold, mtry, min.node.size) of every forest in the tuning grid.

    Forest index = (fold * mtry_max + mtry - 1) * len(min_node_sizes) + min_node_idx.
    """
    out = []
    for f in range(n_folds):
        for m in range(1, mtry_max + 1):
            for mn in min_node_sizes:
                out.append((f, m, mn))
    return out


def kernel_groups(ds: Dataset, n_sizes: int = 4) -> np.ndarray:
    """Group id (int8) of every row: the kernel of its (kernel, size) vector, with
    vector v = kernel * n_sizes + size (37 groups of 4 x 15 = 60 rows in D1)."""
    return (ds.kernel // n_sizes).astype(np.int8)


def leave_one_kernel_out_masks(n_kernels: int = 37) -> np.ndarray:
    """Training masks of a leave-one-kernel-out study (Sec. III-C, Algorithm 1):
    forest k trains on every kernel but k."""
    full = (1 << n_kernels) - 1
    return np.array([full & ~(1 << k) for k in range(n_kernels)], dtype=np.uint64)


def kernel_subset_masks(n_kernels: int = 37, repeats: int = 500, counts=None, seed: int = SEED_SUBSETS):
    """Training masks of the kernel-count study (Sec. III-C, Algorithm 2): for each
    count i, `repeats` shuffles of the kernels, training on the first i.  Returns
    (counts per forest, masks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = list(range(1, n_kernels + 1)) if counts is None else list(counts)
    cnt, masks = [], []
    for i in counts:
        for _ in range(repeats):
            order = rng.permutation(n_kernels)
            m = 0
            for k in order[:i]:
                m |= 1 << int(k)
            cnt.append(i)
            masks.append(m)
    return np.array(cnt, dtype=np.int32), np.array(masks, dtype=np.uint64)


def request_stream(n_requests: int, qps: float, max_rows: int = 4096, seed: int = SEED_REQUESTS):
    """Poisson arrival times (seconds) and log-uniform request sizes in [1, max_rows]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arrivals = np.cumsum(gaps)
    sizes = np.minimum(max_rows, np.floor(np.exp(rng.uniform(0.0, np.log(max_rows + 1), size=n_requests)))).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    row_seed = int(rng.integers(0, 2**63 - 1))
    return arrivals, sizes, row_seed
