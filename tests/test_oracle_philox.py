"""Pin the oracle's Philox4x64-10 against NumPy's independent implementation.

NumPy's ``Philox`` bit generator is Philox4x64-10 (Salmon et al., SC'11).  It
increments its 256-bit counter before producing a block, so the block for
counter c is the first block NumPy yields when seeded with counter c - 1.
"""
import numpy as np
import pytest

M64 = (1 << 64) - 1


def numpy_block(counter, key, n_blocks=1):
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4 * n_blocks).reshape(n_blocks, 4)


@pytest.mark.parametrize("seed", [0, 1, 5, 181100156, M64])
def test_philox_matches_numpy(oracle, seed):
    rng = np.random.Generator(np.random.PCG64(seed & 0xFFFF))
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] = int(rng.integers(0, 1000))
        key = [seed, int(rng.integers(0, 2**63))]
        mine = oracle.philox(ctr, key)
        ref = numpy_block(ctr, key)[0]
        assert np.array_equal(mine, ref)


def test_philox_zero_counter_and_consecutive_blocks(oracle):
    key = [181100156, 0]
    ref = numpy_block([0, 1, 7, 3], key, n_blocks=6)
    for b in range(6):
        assert np.array_equal(oracle.philox([b, 1, 7, 3], key), ref[b])
    # all-zero counter and key is well defined too
    assert np.array_equal(oracle.philox([0, 0, 0, 0], [0, 0]), numpy_block([0, 0, 0, 0], [0, 0])[0])
