"""Pins of the oracle's weighted walker estimators (QMC section, Eq. 1: each
walker carries the weight exp(log w)) against facts that do not come from the
estimator code: equal weights reduce to numpy's plain mean and variance, two
walkers have a closed form, integer weights equal replicated walkers, the
log-sum-exp shift cancels, and excluded walkers change nothing."""
import math

import numpy as np

import oracle


def test_equal_weights_are_plain_mean_and_variance():
    e = np.random.default_rng(1).normal(-3.0, 2.0, 37)
    out = oracle.estimators(np.full(37, 0.25), e, n_accepted=30, n_proposed=40)
    assert out[0] == 37 and out[1] == 0.25
    assert abs(out[2] - 37) < 1e-12 and abs(out[5] - 37) < 1e-12
    assert abs(out[6] - np.mean(e)) < 1e-13
    assert abs(out[7] - np.var(e)) < 1e-12
    assert out[8] == 0.25
    assert out[9] == 0.75 and out[10] == 40


def test_two_walkers_closed_form():
    # weights 1 and 3: <E> = (e0 + 3 e1)/4, var = 3/16 (e0 - e1)^2
    e0, e1 = -1.5, 2.5
    out = oracle.estimators([0.0, math.log(3.0)], [e0, e1])
    assert abs(out[6] - (e0 + 3 * e1) / 4) < 1e-14
    assert abs(out[7] - 3.0 / 16.0 * (e0 - e1) ** 2) < 1e-13
    assert abs(out[2] - 4.0 / 3.0) < 1e-14  # shifted by m = log 3
    assert abs(out[5] - (1.0 / 9.0 + 1.0)) < 1e-14
    assert math.isnan(out[9]) and out[10] == 0


def test_integer_weights_equal_replicated_walkers():
    rng = np.random.default_rng(2)
    e = rng.normal(size=9)
    k = rng.integers(1, 6, size=9)
    a = oracle.estimators(np.log(k.astype(float)), e)
    b = oracle.estimators(np.zeros(k.sum()), np.repeat(e, k))
    assert abs(a[6] - b[6]) < 1e-13 and abs(a[7] - b[7]) < 1e-12


def test_shift_invariance_and_extreme_log_weights():
    rng = np.random.default_rng(3)
    lw = rng.normal(0.0, 3.0, 50)
    e = rng.normal(size=50)
    a = oracle.estimators(lw, e)
    b = oracle.estimators(lw + 700.0, e)
    assert abs(b[1] - a[1] - 700.0) < 1e-12
    np.testing.assert_allclose(b[2:8], a[2:8], rtol=1e-13)
    assert abs(b[8] - a[8] - 700.0) < 1e-12


def test_excluded_walkers_change_nothing():
    rng = np.random.default_rng(4)
    lw = rng.normal(size=12)
    e = rng.normal(size=12)
    ref = oracle.estimators(lw[3:], e[3:])
    lw2, e2 = lw.copy(), e.copy()
    lw2[0] = np.nan
    e2[1] = np.inf
    flags = np.zeros(12, dtype=np.uint8)
    flags[2] = 2
    out = oracle.estimators(lw2, e2, flags=flags)
    assert out[0] == 9
    np.testing.assert_array_equal(out[:9], ref[:9])
    none = oracle.estimators([np.nan], [1.0])
    assert none[0] == 0 and np.isnan(none[1:9]).all()
