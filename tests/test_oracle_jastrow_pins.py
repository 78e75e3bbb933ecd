"""Pins of the oracle's Jastrow parameter derivatives and linear-method
matrices (the optimisation of the Jastrow factor of Eq. 2, QMC section)
against facts that do not come from that code:

* the Pade b derivatives of ln Psi and E_L against Richardson-extrapolated
  central differences of the oracle's own ln|Psi| and E_L with b moved;
* the one-electron hydrogen-like case at b = 0, where ln Psi = -Z r / (1 + b r)
  gives d ln Psi / db = Z r^2 and dE_L / db = 2 Z^2 r - 3 Z in closed form;
* the three-body sums F_k against a two-electron closed form, and their
  E_L derivatives -1/2 sum_i [lap_i F_k + 2 v_i . grad_i F_k] against
  Laplacians and gradients of F_k taken by central differences in the
  electron coordinates (v_i from the oracle's drift, pinned elsewhere);
* electron permutations leave every derivative unchanged;
* the linear-method matrices against the correlated-sampling energy of the
  linearised wavefunction Psi + sum_k d_k dPsi/dp_k, whose value and
  H Psi / Psi at every walker come from differences of the oracle's own
  Psi and E_L Psi in the parameters: E(d) = sum w a b / sum w a^2 must equal
  c^T H c / c^T S c with c = (1 + sum_k d_k <O_k>, d);
* walkers with a non-finite weight or energy, or a flag, drop out.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import synth

J3_LMN = [(1, 1, 0), (1, 0, 1), (1, 1, 1), (2, 1, 0), (2, 0, 1), (1, 0, 2)]


def _sys():
    return synth.small_random_system(31, n_atom=3, n_up=3, n_dn=2, shells=(0, 0, 1, 2), nprim=2)


def _fd(f, h):
    """Richardson extrapolation of central differences with steps 2h and h."""
    d2 = (f(2 * h) - f(-2 * h)) / (4 * h)
    d1 = (f(h) - f(-h)) / (2 * h)
    return (4 * d1 - d2) / 3


def _with_b(s, which, t):
    return dataclasses.replace(s, **{which: getattr(s, which) + t})


@pytest.mark.parametrize("p,which", [(0, "jee_b"), (1, "jen_b")])
def test_pade_b_derivatives_vs_fd(p, which):
    s = _sys()
    R = synth.make_walkers(s, 3, 17)
    for w in range(3):
        O, D, rc = oracle.jastrow_param_grads(s, R[w])
        assert rc == 0
        lp = lambda t: oracle.evaluate(_with_b(s, which, t), R[w])[0]
        el = lambda t: oracle.evaluate(_with_b(s, which, t), R[w])[2]
        o_fd, d_fd = _fd(lp, 1e-3), _fd(el, 1e-3)
        print(f"[jparam] {which} O {O[p]:.10f} fd {o_fd:.10f}  dEL {D[p]:.8f} fd {d_fd:.8f}")
        assert abs(O[p] - o_fd) < 1e-9 * max(1.0, abs(o_fd))
        assert abs(D[p] - d_fd) < 1e-6 * max(1.0, abs(d_fd))


@pytest.mark.parametrize("Z", [1.0, 2.5])
def test_hydrogenic_closed_form(Z):
    s = synth.System("one", np.zeros((1, 3)), np.array([Z]), [0], [0], [1], [0.0], [1.0],
                     np.ones((1, 1)), 1, 0, jen_a=np.array([-Z]), jen_b=0.0)
    rng = np.random.default_rng(3)
    for _ in range(6):
        r = rng.standard_normal(3) * rng.uniform(0.2, 2.0)
        rr = np.linalg.norm(r)
        O, D, rc = oracle.jastrow_param_grads(s, r[None, :])
        assert rc == 0
        assert abs(O[1] - Z * rr * rr) < 1e-13 * max(1.0, Z * rr * rr)
        assert abs(D[1] - (2 * Z * Z * rr - 3 * Z)) < 1e-12 * max(1.0, abs(2 * Z * Z * rr))
        assert np.all(O[[0, 2, 3, 4, 5, 6, 7]] == 0.0) and np.all(D[[0, 2, 3, 4, 5, 6, 7]] == 0.0)


def test_three_body_two_electron_closed_form():
    ion = np.array([[0.3, -0.2, 0.1]])
    s = synth.System("two", ion, np.array([2.0]), [0], [0], [1], [0.7], [1.0],
                     np.ones((1, 1)), 1, 1)
    R = np.array([[1.0, 0.5, -0.4], [-0.6, 0.2, 1.1]])
    x = np.linalg.norm(R[0] - ion[0])
    y = np.linalg.norm(R[1] - ion[0])
    z = np.linalg.norm(R[0] - R[1])
    sx, sy, sz = x / (1 + x), y / (1 + y), z / (1 + z)
    ref = [(sx ** l * sy ** m + sx ** m * sy ** l) * sz ** n for l, m, n in J3_LMN]
    np.testing.assert_allclose(oracle.j3_values(s, R), ref, rtol=1e-14)
    O, D, rc = oracle.jastrow_param_grads(s, R)
    assert rc == 0
    np.testing.assert_allclose(O[2:], ref, rtol=1e-14)


def _fd_grad_lap_F(s, R, h=2e-3):
    """grad_i F_k and lap_i F_k by Richardson central differences of the
    plain three-body sums: [ne][3][6] and [ne][6]."""
    ne = R.shape[0]
    g = np.zeros((ne, 3, 6))
    lap = np.zeros((ne, 6))
    F0 = oracle.j3_values(s, R)
    for i in range(ne):
        for x in range(3):
            def f(t):
                Rt = R.copy()
                Rt[i, x] += t
                return oracle.j3_values(s, Rt)
            g[i, x] = _fd(f, h)
            d1 = (f(h) - 2 * F0 + f(-h)) / (h * h)
            d2 = (f(2 * h) - 2 * F0 + f(-2 * h)) / (4 * h * h)
            lap[i] += (4 * d1 - d2) / 3
    return g, lap


def test_three_body_energy_derivatives_vs_fd():
    s = _sys()
    R = synth.make_walkers(s, 2, 23)
    for w in range(2):
        O, D, rc = oracle.jastrow_param_grads(s, R[w])
        assert rc == 0
        np.testing.assert_allclose(O[2:], oracle.j3_values(s, R[w]), rtol=1e-13)
        v = oracle.evaluate(s, R[w])[3]
        g, lap = _fd_grad_lap_F(s, R[w])
        ref = -0.5 * (lap.sum(axis=0) + 2 * np.einsum("ix,ixk->k", v, g))
        print(f"[jparam] three-body dEL {D[2:]} fd {ref}")
        np.testing.assert_allclose(D[2:], ref, rtol=2e-6, atol=2e-6)


def test_permutation_invariance():
    s = _sys()
    R = synth.make_walkers(s, 1, 5)[0]
    O, D, _ = oracle.jastrow_param_grads(s, R)
    Rp = R.copy()
    Rp[[0, 2]] = R[[2, 0]]       # two up electrons
    Rp[[3, 4]] = R[[4, 3]]       # the two down electrons
    O2, D2, _ = oracle.jastrow_param_grads(s, Rp)
    np.testing.assert_allclose(O2, O, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(D2, D, rtol=1e-10, atol=1e-10)


def test_batch_equals_single():
    s = _sys()
    R = synth.make_walkers(s, 5, 8)
    O, D, rc = oracle.jastrow_param_grads_batch(s, R)
    assert rc == 0
    for w in range(5):
        o1, d1, _ = oracle.jastrow_param_grads(s, R[w])
        np.testing.assert_array_equal(O[w], o1)
        np.testing.assert_array_equal(D[w], d1)


def _linearised_energy(s, R, log_w, d, h=1e-3):
    """Correlated-sampling energy of Psi + d0 dPsi/db_ee + d1 dPsi/db_en
    + sum_k d_{2+k} F_k Psi over the walkers, weights exp(log w) |Psi|^2:
    at walker w, a = (Psi + ...) / Psi and b = H(Psi + ...) / Psi, with
    dPsi/db / Psi and d(E_L Psi)/db / Psi from central differences of the
    oracle's Psi and E_L Psi in b, and H(F Psi) / Psi = F E_L
    - 1/2 sum_i [lap_i F + 2 v_i . grad_i F] from differences of F in the
    electron coordinates."""
    num = den = 0.0
    om = np.exp(log_w - log_w.max())
    for w in range(R.shape[0]):
        lp0, sg0, e0, v, _ = oracle.evaluate(s, R[w])
        a, b = 1.0, e0
        for p, which in ((0, "jee_b"), (1, "jen_b")):
            def psi_ratio(t):
                lp, sg, _, _, _ = oracle.evaluate(_with_b(s, which, t), R[w])
                return sg * sg0 * math.exp(lp - lp0)
            def elpsi_ratio(t):
                lp, sg, el, _, _ = oracle.evaluate(_with_b(s, which, t), R[w])
                return el * sg * sg0 * math.exp(lp - lp0)
            a += d[p] * _fd(psi_ratio, h)
            b += d[p] * _fd(elpsi_ratio, h)
        F = oracle.j3_values(s, R[w])
        g, lap = _fd_grad_lap_F(s, R[w])
        hF = F * e0 - 0.5 * (lap.sum(axis=0) + 2 * np.einsum("ix,ixk->k", v, g))
        a += d[2:] @ F
        b += d[2:] @ hF
        num += om[w] * a * b
        den += om[w] * a * a
    return num / den


def test_linear_method_matrices_vs_correlated_sampling():
    s = _sys()
    W = 6
    R = synth.make_walkers(s, W, 61)
    lw = np.random.default_rng(2).normal(0.0, 0.8, W)
    _, _, E, _ = oracle.evaluate_batch(s, R)
    O, D, rc = oracle.jastrow_param_grads_batch(s, R)
    assert rc == 0
    S, H = oracle.linear_method(lw, E, O, D)
    assert S.shape == (9, 9) and H.shape == (9, 9)
    assert np.all(np.linalg.eigvalsh(S) > -1e-12)
    rng = np.random.default_rng(4)
    for trial in range(3):
        d = rng.normal(0.0, 0.05, 8) * np.array([1, 1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1])
        c = np.concatenate(([1.0 + d @ _means(lw, O)], d))
        e_lin = c @ H @ c / (c @ S @ c)
        e_ref = _linearised_energy(s, R, lw, d)
        print(f"[jparam] linearised energy {e_lin:.12f} correlated sampling {e_ref:.12f}")
        assert abs(e_lin - e_ref) < 2e-7 * max(1.0, abs(e_ref))


def _means(lw, O):
    om = np.exp(lw - lw.max())
    return om @ O / om.sum()


def test_linear_method_exclusions():
    rng = np.random.default_rng(9)
    W = 12
    lw = rng.normal(0, 1, W)
    E = rng.normal(-3, 0.5, W)
    O = rng.normal(0, 1, (W, 8))
    D = rng.normal(0, 1, (W, 8))
    keep = np.ones(W, bool)
    lw2, E2 = lw.copy(), E.copy()
    lw2[1] = -np.inf
    E2[4] = np.nan
    flags = np.zeros(W, np.uint8)
    flags[7] = 2
    keep[[1, 4, 7]] = False
    S, H = oracle.linear_method(lw2, E2, O, D, flags=flags)
    S0, H0 = oracle.linear_method(lw[keep], E[keep], O[keep], D[keep])
    np.testing.assert_array_equal(S, S0)
    np.testing.assert_array_equal(H, H0)
    # equal weights, one parameter, two walkers: S = ((O0 - O1) / 2)^2
    S1, H1 = oracle.linear_method([0.0, 0.0], [1.0, 3.0], [[2.0], [6.0]], [[0.5], [1.5]])
    assert S1[1, 1] == 4.0 and H1[0, 0] == 2.0 and H1[1, 0] == 2.0 and H1[0, 1] == 3.0
    assert H1[1, 1] == 0.5 * (4.0 * 1.0 + (-2.0) * 0.5) + 0.5 * (4.0 * 3.0 + 2.0 * 1.5)
