"""Pins of the oracle's birth/death branching (the DMC weights of Eq. 1 as
walker counts; the paper leaves the control scheme open) against facts that
do not come from its code:

* integer weights make the multiplicities deterministic (floor(n + u) = n
  for u in [0, 1)), so whole layouts can be worked out by hand from the
  slot rule; three such layouts (same size, shrinking, growing) are written
  out below;
* on random weights, the new population holds walker j exactly M_j times,
  every destination is an empty or new slot below W', no source is a
  destination, and a walker with a copy below W' keeps its slot;
* M_j is floor(w_j) or floor(w_j) + 1 and unbiased: E[M_j] = w_j (the mean
  over many steps within five standard errors of the Bernoulli spread);
* flagged and non-finite weights get no copy; an empty or an over-capacity
  population is refused.
"""
import math

import numpy as np

import oracle


def _population(W, copies, pairs, w_new):
    """Slot -> source walker of the new population, from the pairs."""
    src = {j: j for j in range(W) if copies[j] > 0}
    for d, s in pairs:
        src[int(d)] = int(s)
    return [src.get(k, -1) for k in range(w_new)]


HAND = [
    # M = [0, 3, 1, 0, 0, 2]: walker 1's two extras fill the dead slots 0 and
    # 3, walker 5's extra the dead slot 4.
    ([0, 3, 1, 0, 0, 2], [1, 1, 2, 1, 5, 5]),
    # M = [0, 0, 2, 0, 1, 0, 1, 0]: W' = 4; walker 2's extra fills slot 0,
    # the walkers 4 and 6 (slots >= 4) move into the empty slots 1 and 3.
    ([0, 0, 2, 0, 1, 0, 1, 0], [2, 4, 2, 6]),
    # M = [2, 0, 3]: W' = 5; walker 0's extra fills slot 1, walker 2's two
    # extras the new slots 3 and 4.
    ([2, 0, 3], [0, 0, 2, 2, 2]),
]


def test_hand_worked_layouts():
    for M, expect in HAND:
        W = len(M)
        lw = np.array([math.log(m) if m > 0 else -np.inf for m in M])
        copies, pairs, wn, rc = oracle.branch(lw, seed=3, step=7, cap=32)
        assert rc == 0
        np.testing.assert_array_equal(copies, M)
        assert wn == len(expect)
        assert _population(W, copies, pairs, wn) == expect


def test_invariants_on_random_weights():
    rng = np.random.default_rng(11)
    for trial in range(200):
        W = int(rng.integers(1, 60))
        lw = rng.normal(0.0, 0.9, W)
        cap = 4 * W + 8
        copies, pairs, wn, rc = oracle.branch(lw, seed=trial, step=trial * 3, cap=cap)
        if wn < 1:
            assert rc == 5
            continue
        assert rc == 0
        w = np.exp(lw)
        assert np.all((copies == np.floor(w)) | (copies == np.floor(w) + 1))
        assert wn == copies.sum()
        dst = pairs[:, 0]
        assert len(set(dst.tolist())) == len(dst)
        assert np.all(dst < wn)
        assert not set(dst.tolist()) & set(pairs[:, 1].tolist())
        for d in dst:
            assert d >= W or copies[d] == 0
        for j in range(min(W, wn)):
            if copies[j] > 0:
                assert j not in dst
        pop = _population(W, copies, pairs, wn)
        assert -1 not in pop
        np.testing.assert_array_equal(np.bincount(pop, minlength=W), copies)


def test_unbiased_multiplicities():
    lw = np.log(np.array([0.05, 0.5, 0.93, 1.0, 1.37, 2.5, 3.999]))
    n = 4000
    tot = np.zeros(len(lw))
    for st in range(n):
        copies, _, _, rc = oracle.branch(lw, seed=21, step=st, cap=100)
        assert rc == 0
        tot += copies
    w = np.exp(lw)
    f = w - np.floor(w)
    se = np.sqrt(np.maximum(f * (1 - f), 1e-12) / n)
    print("[branch] mean copies", tot / n, "weights", w)
    assert np.all(np.abs(tot / n - w) <= 5 * se + 1e-12)


def test_flags_dead_and_capacity():
    lw = np.zeros(6)
    flags = np.array([0, 1, 0, 0, 2, 0], dtype=np.uint8)
    copies, pairs, wn, rc = oracle.branch(lw, 1, 0, 16, flags=flags)
    assert rc == 0
    np.testing.assert_array_equal(copies, [1, 0, 1, 1, 0, 1])
    assert wn == 4
    # slots 1 and 4 are empty; walker 5 (slot >= 4) moves into slot 1
    assert _population(6, copies, pairs, wn) == [0, 5, 2, 3]
    lw2 = np.array([0.0, np.nan, np.inf, -np.inf])
    copies, _, wn, rc = oracle.branch(lw2, 1, 0, 16)
    np.testing.assert_array_equal(copies, [1, 0, 0, 0])
    assert rc == 0 and wn == 1
    _, _, wn, rc = oracle.branch(np.full(4, -np.inf), 1, 0, 16)
    assert rc == 5 and wn == 0
    _, pairs, wn, rc = oracle.branch(np.full(4, math.log(5.0)), 1, 0, 16)
    assert rc == 5 and wn == 17 and pairs.shape[0] == 0
