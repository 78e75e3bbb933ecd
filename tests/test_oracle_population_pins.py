"""Pins of the oracle's population control (comb reconfiguration at fixed
population, applied to the DMC weights of Eq. 1) against facts that do not
come from the oracle's own loop.

* Brute force: every tooth is placed in the weight interval that contains it
  ([C_{j-1}, C_j)), by testing all (tooth, walker) pairs on the same IEEE
  doubles (Python floats: the same sequential sums and products).
* Closed forms: equal weights give one copy each for any offset; all weight
  on one walker gives it every copy; zero and non-finite weights get none.
* Properties of the comb: sum of copies = W, |n_j - W w_j / S| < 1, and the
  copies averaged over a uniform grid of offsets equal W w_j / S (unbiased).
* Slot rules: a walker with copies keeps its slot, every walker without one
  receives exactly one copy, extra copies go out in walker order to the
  lowest free slots.
* log of the mean weight against logsumexp.
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

import oracle


def _brute(log_w, u):
    W = len(log_w)
    fin = [x for x in log_w if math.isfinite(x)]
    m = max(fin)
    w = [math.exp(x - m) if math.isfinite(x) else 0.0 for x in log_w]
    C, acc = [], 0.0
    for x in w:
        acc += x
        C.append(acc)
    S = acc
    step = S / W
    n = [0] * W
    for k in range(W):
        t = (k + u) * step
        hits = [j for j in range(W) if (0.0 if j == 0 else C[j - 1]) <= t < C[j]]
        assert len(hits) <= 1
        if hits:
            n[hits[0]] += 1
        else:  # rounding past the last cumulative sum: last positive weight
            n[max(j for j in range(W) if w[j] > 0)] += 1
    return np.array(n), w, S


def _check_slots(copies, pairs):
    W = len(copies)
    dst = pairs[:, 0]
    src = pairs[:, 1]
    dead = np.flatnonzero(copies == 0)
    np.testing.assert_array_equal(dst, dead)           # every dead slot, lowest first, once
    assert np.all(np.diff(src) >= 0)                   # sources in walker order
    for j in range(W):
        assert np.count_nonzero(src == j) == max(copies[j] - 1, 0)
    assert not np.intersect1d(dst, np.flatnonzero(copies > 0)).size


@pytest.mark.parametrize("W,seed", [(1, 0), (7, 1), (64, 2), (300, 3)])
def test_brute_force_teeth(W, seed):
    rng = np.random.default_rng(seed)
    log_w = rng.normal(0.0, 1.5, W)
    for u in (0.0, 0.5, rng.uniform(), 0.999999):
        copies, pairs, lwbar, rc = oracle.reconfigure(log_w, u)
        assert rc == 0
        n, w, S = _brute(list(log_w), u)
        np.testing.assert_array_equal(copies, n)
        assert copies.sum() == W
        _check_slots(copies, pairs)
        # comb property: within one copy of the expectation
        expect = W * np.array(w) / S
        assert np.all(np.abs(copies - expect) < 1.0 + 1e-12)
        assert abs(lwbar - (logsumexp(log_w) - math.log(W))) <= 1e-13 * max(1.0, abs(lwbar))


def test_equal_weights_identity():
    for W in (1, 5, 128):
        for u in (0.0, 0.3, 0.75):
            copies, pairs, lwbar, rc = oracle.reconfigure(np.full(W, -2.5), u)
            assert rc == 0 and pairs.shape[0] == 0
            np.testing.assert_array_equal(copies, np.ones(W))
            assert abs(lwbar + 2.5) < 1e-15


def test_all_weight_on_one_walker():
    W = 9
    log_w = np.full(W, -np.inf)
    log_w[4] = 3.0
    copies, pairs, lwbar, rc = oracle.reconfigure(log_w, 0.4)
    assert rc == 0
    expect = np.zeros(W, dtype=int)
    expect[4] = W
    np.testing.assert_array_equal(copies, expect)
    np.testing.assert_array_equal(pairs, [[j, 4] for j in range(W) if j != 4])
    assert abs(lwbar - (3.0 - math.log(W))) < 1e-14


def test_zero_and_nonfinite_weights_get_no_copy():
    log_w = np.array([0.0, -np.inf, np.nan, 0.5, np.inf, -1000.0, 0.2])
    for u in np.linspace(0.0, 0.95, 20):
        copies, pairs, lwbar, rc = oracle.reconfigure(log_w, u)
        assert rc == 0
        assert copies[1] == 0 and copies[2] == 0 and copies[4] == 0
        assert copies[5] == 0  # exp(-1000.5) underflows to zero weight
        assert copies.sum() == len(log_w)
        _check_slots(copies, pairs)


def test_no_positive_weight_keeps_population():
    copies, pairs, lwbar, rc = oracle.reconfigure(np.array([np.nan, -np.inf]), 0.2)
    assert rc == 0 and pairs.shape[0] == 0 and math.isnan(lwbar)
    np.testing.assert_array_equal(copies, [1, 1])


def test_unbiased_over_offsets():
    rng = np.random.default_rng(11)
    W, M = 37, 4000
    log_w = rng.normal(0.0, 1.0, W)
    w = np.exp(log_w - log_w.max())
    expect = W * w / w.sum()
    mean = np.zeros(W)
    for i in range(M):
        mean += oracle.reconfigure(log_w, (i + 0.5) / M)[0]
    mean /= M
    assert np.max(np.abs(mean - expect)) <= 2.0 / M + 1e-12


def test_invalid_offset_rejected():
    for u in (-0.1, 1.0, np.nan):
        assert oracle.reconfigure(np.zeros(3), u)[3] == -1
