"""The linear-method step (host logic) against closed forms, and a whole
optimisation on the oracle's samples of the exactly solvable case.

* Two-state problem: with S = I and H symmetric 2 x 2 the step is the
  lowest eigenvector's ratio, written out here from the 2 x 2 eigenproblem.
* Parameter subsets keep the chosen rows and columns only.
* The hydrogen-like 1s with the exact Pade e-n term at b = 0: starting from
  b = 0.4, VMC samples of the oracle, its derivatives and its linear-method
  matrices drive b to zero (the exact wavefunction; E_L = -Z^2/2 there)
  within six steps, the first ones held by the trust bound.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import optimize, synth


def test_two_state_closed_form():
    a, b, d = -1.3, 0.4, 0.9
    H = np.array([[a, b], [b, d]])
    dp, E = optimize.linear_method_update(np.eye(2), H, shift=0.0, max_change=None)
    lam = 0.5 * (a + d) - math.sqrt(0.25 * (a - d) ** 2 + b * b)
    # eigenvector (b, lam - a): c1 / c0 = (lam - a) / b
    assert abs(E - lam) < 1e-14
    assert abs(dp[0] - (lam - a) / b) < 1e-13


def test_shift_damps_and_subsets_select():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 4))
    S = np.eye(4)
    S[1:, 1:] = X[:, 1:].T @ X[:, 1:] / 40
    H = S.copy() * -2.0
    H[0, 1:] = H[1:, 0] = [0.3, -0.2, 0.1]
    H[0, 0] = -2.0
    dp0, _ = optimize.linear_method_update(S, H, shift=0.0, max_change=None)
    dp1, _ = optimize.linear_method_update(S, H, shift=1.0, max_change=None)
    assert np.linalg.norm(dp1) < np.linalg.norm(dp0)
    dps, _ = optimize.linear_method_update(S, H, params=[1], shift=0.0, max_change=None)
    dps_ref, _ = optimize.linear_method_update(S[np.ix_([0, 2], [0, 2])],
                                               H[np.ix_([0, 2], [0, 2])], shift=0.0,
                                               max_change=None)
    np.testing.assert_allclose(dps, dps_ref, rtol=1e-13)
    # the trust bound: the step's S-norm stays within max_change
    dpt, _ = optimize.linear_method_update(S, H, shift=0.0, max_change=0.05)
    assert math.sqrt(dpt @ S[1:, 1:] @ dpt) <= 0.05 + 1e-15


def _hydrogenic(b, Z=1.0):
    return synth.System("h1s", np.zeros((1, 3)), np.array([Z]), [0], [0], [1], [0.0], [1.0],
                        np.ones((1, 1)), 1, 0, jen_a=np.array([-Z]), jen_b=b)


def test_oracle_optimisation_reaches_the_exact_jastrow():
    b = 0.4
    W = 400
    R = np.random.default_rng(5).normal(0.0, 1.0, (W, 1, 3))
    for it in range(6):
        s = _hydrogenic(b)
        out = oracle.run(s, R, n_steps=30, mode=0, tau=0.1, seed=11 + it)
        R = out["R"]
        _, _, E, _ = oracle.evaluate_batch(s, R)
        O, D, rc = oracle.jastrow_param_grads_batch(s, R)
        assert rc == 0
        S, H = oracle.linear_method(np.zeros(W), E, O, D)
        dp, _ = optimize.linear_method_update(S, H, params=[1], shift=1e-4)
        print(f"[optimize] step {it}: b {b:.5f} -> {b + dp[0]:.5f}, <E> {E.mean():.6f}")
        b += dp[0]
    assert abs(b) < 0.02
