"""Independent helpers for pinning the oracle (no code shared with it).

* ``numpy_block`` draws Philox4x64-10 blocks from NumPy's own implementation.
* ``verify_tree`` re-derives, node by node and in exact rational arithmetic, what
  the forest method requires of a grown tree, and checks a tree against it.  It
  measures split quality by the direct definition -- the drop in weighted sum of
  squared deviations from the node mean -- rather than by the S^2/N shortcut the
  oracle evaluates, so an algebra slip in the oracle cannot cancel here.
"""
from fractions import Fraction

import numpy as np

M64 = (1 << 64) - 1


def numpy_block(counter, key, n_blocks=1):
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4 * n_blocks).reshape(n_blocks, 4)


def draws(seed, tag, node, tree, count):
    if count == 0:
        return []
    blocks = numpy_block([0, tag, node, tree], [seed, 0], n_blocks=(count + 3) // 4).reshape(-1)
    return [int(x) for x in blocks[:count]]


def scaled(r, m):
    return (r * m) >> 64


def bootstrap_weights(seed, tree, n_train, bootstrap=True):
    w = [0] * n_train
    if not bootstrap:
        return [1] * n_train
    for r in draws(seed, 0, 0, tree, n_train):
        w[scaled(r, n_train)] += 1
    return w


def candidates(seed, tree, node, C, mtry):
    perm = list(range(C))
    for k, r in enumerate(draws(seed, 1, node, tree, mtry)):
        j = k + scaled(r, C - k)
        perm[k], perm[j] = perm[j], perm[k]
    return sorted(perm[:mtry])


def sse(items):
    """Weighted sum of squared deviations from the weighted mean (exact)."""
    W = sum(w for w, _ in items)
    if W == 0:
        return Fraction(0)
    mean = Fraction(sum(w * y for w, y in items), W)
    return sum(w * (y - mean) ** 2 for w, y in items)


def round_half_away(fr: Fraction) -> int:
    a = abs(fr)
    v = int(a + Fraction(1, 2))  # floor(|x| + 1/2)
    return v if fr >= 0 else -v


def verify_tree(tree, codes, n_bins, y_fp, train_rows, seed, t, mtry, min_node, bootstrap=True, tol=Fraction(0)):
    """Check one grown tree (dict of node arrays) against the method, exactly."""
    C = codes.shape[1]
    n_train = len(train_rows)
    w = bootstrap_weights(seed, t, n_train, bootstrap)
    rows_of = {0: [i for i in range(n_train) if w[i] > 0]}
    col, bn, left, q, N = (tree[k] for k in ("col", "bin", "left", "q", "N"))
    n_nodes = len(col)
    next_id = 1
    for i in range(n_nodes):
        rows = rows_of.pop(i)
        items = [(w[r], int(y_fp[r])) for r in rows]
        Nn = sum(a for a, _ in items)
        Sn = sum(a * b for a, b in items)
        assert N[i] == Nn, f"node {i}: N {N[i]} != {Nn}"
        pure = len({b for _, b in items}) == 1
        if col[i] == 255:
            assert left[i] == -1
            assert q[i] == round_half_away(Fraction(Sn * 65536, Nn)), f"node {i}: leaf value"
            if Nn > min_node and not pure:
                cand = candidates(seed, t, i, C, mtry)
                best = Fraction(-1)
                base = sse(items)
                for c in cand:
                    for b in range(n_bins[c] - 1):
                        L = [it for r, it in zip(rows, items) if codes[train_rows[r], c] <= b]
                        R = [it for r, it in zip(rows, items) if codes[train_rows[r], c] > b]
                        if L and R:
                            best = max(best, base - sse(L) - sse(R))
                assert best <= tol * (1 + abs(Fraction(Sn * Sn, Nn))), f"node {i}: leaf although a split helps"
            continue
        assert Nn > min_node and not pure, f"node {i}: split a node that must be a leaf"
        cand = candidates(seed, t, i, C, mtry)
        c, b = int(col[i]), int(bn[i])
        assert c in cand, f"node {i}: column {c} not among candidates {cand}"
        base = sse(items)
        gains = {}
        lsets = {}
        for cc in cand:
            for bb in range(n_bins[cc] - 1):
                L = [(r, it) for r, it in zip(rows, items) if codes[train_rows[r], cc] <= bb]
                R = [it for r, it in zip(rows, items) if codes[train_rows[r], cc] > bb]
                if L and R:
                    gains[(cc, bb)] = base - sse([it for _, it in L]) - sse(R)
                    lsets[(cc, bb)] = (sum(it[0] for _, it in L), sum(it[0] * it[1] for _, it in L))
        assert (c, b) in gains, f"node {i}: split ({c},{b}) leaves a side empty"
        gmax = max(gains.values())
        assert gains[(c, b)] > 0
        assert gains[(c, b)] >= gmax - tol * (1 + gmax), f"node {i}: split not optimal"
        # first strictly greater wins: no earlier pair gives the same (N_L, S_L)
        for key, ls in lsets.items():
            if key < (c, b):
                assert ls != lsets[(c, b)], f"node {i}: earlier pair {key} has the same split"
        assert left[i] == next_id, f"node {i}: child id {left[i]} != {next_id}"
        rows_of[next_id] = [r for r in rows if codes[train_rows[r], c] <= b]
        rows_of[next_id + 1] = [r for r in rows if codes[train_rows[r], c] > b]
        next_id += 2
    assert next_id == n_nodes and not rows_of
