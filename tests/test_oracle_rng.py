"""Pins of the oracle's random numbers and random ordering against numpy's Philox.

numpy.random.Philox is an independent implementation of Philox4x64-10 (Salmon et
al., SC'11).  It increments its 256-bit counter before producing a block, so the
block at counter c is read after setting the counter to c - 1.
"""
import numpy as np
import pytest

import oracle as O

M64 = (1 << 64) - 1


def numpy_block(ctr, key):
    c = 0
    for i, w in enumerate(ctr):
        c |= int(w) << (64 * i)
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4)


def test_philox_known_answer_zero():
    # Philox4x64-10 at counter 0, key 0 (Random123 known-answer vector)
    out = O.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert [int(x) for x in out] == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                     0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_philox_matches_numpy_random_counters():
    rng = np.random.default_rng(1)
    for _ in range(300):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.int64)]
        ctr = [c * 2 + int(rng.integers(0, 2)) for c in ctr]  # full 64-bit words
        key = [int(x) * 2 + 1 for x in rng.integers(0, 2**63, 2, dtype=np.int64)]
        got = O.philox4x64_10(ctr, key)
        assert np.array_equal(got, numpy_block(ctr, key))


@pytest.mark.parametrize("ctr", [[M64, 0, 0, 0], [M64, M64, 5, 0], [0, 0, 0, M64], [7, 3, 2**40, 1]])
def test_philox_matches_numpy_edge_counters(ctr):
    key = [0xDEADBEEF, 0x12345678]
    assert np.array_equal(O.philox4x64_10(ctr, key), numpy_block(ctr, key))


def test_draw_layout():
    # draw t of walk w of row k = 32-bit word (t mod 8) of the block at counter
    # (t div 8, w, k, 0), low half of each 64-bit word first
    seed = 0xABCDEF0123
    for (k, w, t) in [(0, 0, 0), (5, 3, 7), (1023, 63, 8), (77, 200, 123), (2**21, 511, 99999)]:
        blk = numpy_block([t // 8, w, k, 0], [seed, 0])
        word = int(blk[(t % 8) // 2])
        want = word & 0xFFFFFFFF if t % 2 == 0 else word >> 32
        assert O.draw(seed, k, w, t) == want


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 5), (1000, 0), (4097, 123456789)])
def test_rank_is_sort_of_numpy_keys(n, seed):
    keys = np.array([numpy_block([0, 0, v, 1], [seed, 0])[0] for v in range(n)], dtype=np.uint64)
    order = np.lexsort((np.arange(n), keys))  # by key, ties by node id
    want = np.empty(n, np.int32)
    want[order] = np.arange(n, dtype=np.int32)
    assert np.array_equal(O.rank(n, seed), want)


def test_rank_is_uniform_permutation():
    # position of node 0 over many seeds is uniform on [0, n)
    n = 8
    pos = np.array([O.rank(n, s)[0] for s in range(4000)])
    counts = np.bincount(pos, minlength=n)
    chi2 = ((counts - 500.0) ** 2 / 500.0).sum()
    assert chi2 < 30.0  # 7 dof, p ~ 1e-4
