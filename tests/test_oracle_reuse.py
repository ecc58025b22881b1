"""Pins of the oracle's walk reuse (Section 5.3, Algorithm "reuse").

References independent of the stack algorithm: the paper's worked example (Figure
'sequence'), a brute-force extraction written from the text's definition of legal
sequences and its rules (no two overlapping walks from one start node, a walk starts
as early as possible, one-step walks are ignored), the plain walks of the same draws,
and the absorbing chain's limits (oracle/dense.py) that every counted walk of a row
must follow.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import dense
from paper_math_0609672_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
Z = 5.0


def as_record(seq):
    """(row, end, visits, length) of a legal sequence taken as one walk."""
    return (seq[0], seq[-1], sum(1 for x in seq[:-1] if x == seq[0]), len(seq) - 1)


def records(r: O.Records):
    return sorted(zip(r.row.tolist(), r.end.tolist(), r.visits.tolist(), r.length.tolist()))


def test_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "reuse_example.json")))
    seq = g["sequence"]
    got = records(O.reuse_sequence(seq, seq))
    want = sorted([as_record(seq)] + [as_record(x) for x in g["extracted"]])
    assert got == want
    for x in g["not_extracted"]:
        assert as_record(x) not in [as_record(y) for y in g["extracted"]]
    # the extracted sequences are segments of the walk
    for x in g["extracted"]:
        assert any(seq[i:i + len(x)] == x for i in range(len(seq)))


def brute_force(keys, nodes):
    """Extraction from the definition: the walk starting at position p ends at the first
    later position whose key is below key[p]; it is counted when it has at least two
    steps and does not overlap a walk already counted from the same node, deciding
    p = 1, 2, ... in order (earliest start)."""
    L = len(keys)
    out = []
    busy_until = {}  # node -> last position of its counted walk
    for p in range(L - 1):
        q = next(j for j in range(p + 1, L) if keys[j] < keys[p])
        if q - p < 2:
            continue
        if busy_until.get(nodes[p], -1) > p:
            continue
        busy_until[nodes[p]] = q
        vis = sum(1 for j in range(p, q) if nodes[j] == nodes[p])
        out.append((nodes[p], nodes[q], vis, q - p))
    return sorted(out)


def random_legal_sequence(rng, n=8):
    keys = rng.permutation(n)
    start = int(rng.integers(0, n))
    while keys[start] == 0:
        start = int(rng.integers(0, n))
    up = [v for v in range(n) if keys[v] >= keys[start]]
    seq = [start]
    for _ in range(int(rng.integers(1, 40))):
        nxt = int(rng.choice(up))
        if nxt != seq[-1]:
            seq.append(nxt)
    down = [v for v in range(n) if keys[v] < keys[start]]
    end = int(rng.choice(down)) if rng.random() < 0.8 else -1  # -1: ground
    seq.append(end)
    k = [int(keys[v]) if v >= 0 else -1 for v in seq]
    return k, seq


def test_matches_definition_on_random_sequences():
    rng = np.random.default_rng(5)
    total = 0
    for _ in range(400):
        k, seq = random_legal_sequence(rng)
        got = records(O.reuse_sequence(k, seq))
        assert got == brute_force(k, seq), (k, seq)
        total += len(got)
    assert total > 1200  # many extracted walks were compared


def test_one_step_and_minimal_sequences():
    # a one-step walk {3, 1} is ignored (handled exactly by Section 5.2)
    assert records(O.reuse_sequence([3, 1], [3, 1])) == []
    # two steps: only the walk itself
    assert records(O.reuse_sequence([3, 5, 1], [3, 5, 1])) == [(3, 1, 1, 2)]
    # ground as the lowest key ends every open walk there
    r = records(O.reuse_sequence([3, 5, 7, 6, -1], [3, 5, 7, 6, -1]))
    assert r == sorted([(3, -1, 1, 4), (5, -1, 1, 3)])


def small(n=9, edges=16, seed=3):
    return W.random_graph(n, edges, seed=seed)


def test_reuse_keeps_the_simulated_walks():
    """The walk itself is always counted: per row, the plain walks' records are a
    sub-multiset of the reuse records, and the rest were extracted from other walks."""
    A = small(12, 24, seed=4)
    rk = O.rank(A.n, 4)
    tb = O.table(A, rk)
    rows = np.arange(A.n)
    plain = O.walk_rows(A, rk, tb, 11, rows, 200)
    re = O.walk_rows_reuse(A, rk, tb, 11, rows, 200)
    extra = 0
    for r, k in enumerate(rows):
        s = slice(plain.rec_off[r], plain.rec_off[r + 1])
        a = sorted(zip(plain.end[s].tolist(), plain.visits[s].tolist(), plain.length[s].tolist()))
        m = re.row == k
        b = sorted(zip(re.end[m].tolist(), re.visits[m].tolist(), re.length[m].tolist()))
        rest = list(b)
        for x in a:
            rest.remove(x)  # raises if a plain walk is missing
        extra += len(rest)
        assert all(x[2] >= 2 for x in b)  # every counted walk has >= 2 steps
    assert extra > 0


@pytest.mark.parametrize("seed", [0, 7])
def test_counted_walks_follow_the_conditioned_game(seed):
    """Every walk counted for row k (simulated or extracted) is a sample of the walk
    game of row k with its first step among the motels: ends, stays and lengths match
    the absorbing chain's limits within 5 sigma."""
    A = small(9, 15, seed=seed)
    Ad = A.dense()
    rk = O.rank(A.n, seed + 100)
    tb = O.table(A, rk)
    rec = O.walk_rows_reuse(A, rk, tb, 99, np.arange(A.n), 6000)
    checked = 0
    for k in range(A.n):
        lim = dense.walk_limits(Ad, rk, k)
        m = rec.row == k
        if lim["p"] is None:
            assert not m.any()
            continue
        M = int(m.sum())
        end, vis, ln = rec.end[m], rec.visits[m].astype(float), rec.length[m].astype(float)
        for i in range(A.n):
            p = lim["p"][i]
            assert abs(np.mean(end == i) - p) <= Z * np.sqrt(max(p * (1 - p), 1e-12) / M) + 1e-12
        pg = lim["p_ground"]
        assert abs(np.mean(end == -1) - pg) <= Z * np.sqrt(max(pg * (1 - pg), 1e-12) / M) + 1e-12
        assert abs(vis.mean() - lim["visits_motel"]) <= Z * vis.std() / np.sqrt(M) + 1e-12
        assert abs(ln.mean() - lim["length_motel"]) <= Z * ln.std() / np.sqrt(M) + 1e-12
        checked += 1
    assert checked >= 4


def test_reuse_factor_converges_to_exact_ldl():
    A = small(10, 17, seed=2)
    Ad = A.dense()
    rk = O.rank(A.n, 2)
    F = O.build_factor(A, 20000, 0.0, 3, rk=rk, reuse=True)
    Ye, De = dense.exact_factor_schur(Ad, rk)
    Y = F.dense_y()
    tau = F.table.tau
    M = F.tallies.walks
    for k in range(A.n):
        lim = dense.walk_limits(Ad, rk, k)
        for i in range(A.n):
            if rk[i] >= rk[k]:
                assert Y[k, i] == (1.0 if i == k else 0.0)
                continue
            if M[k] == 0:
                assert np.isclose(Y[k, i], Ye[k, i], rtol=1e-14, atol=0)
                continue
            p = lim["p"][i]
            sd = tau[k] * np.sqrt(max(p * (1 - p), 1e-12) / M[k])
            assert abs(Y[k, i] - Ye[k, i]) <= Z * sd + 1e-13, (k, i)
    # reuse only adds walks: every row with walks has at least its budget
    assert np.all(M[tau > 0] >= 20000)
