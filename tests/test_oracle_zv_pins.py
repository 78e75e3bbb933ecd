"""Pins of the oracle's derivative of the local energy (Single Determinant QMC
Forces, Eq. 4: d tr(A^{-1}B) = tr(A^{-1} dB - X dA), X = A^{-1} B A^{-1}) and of
the space-warp transformation, against facts that do not come from that code:

* basis Hessians and gradients of the Laplacian against central differences
  of the (separately pinned) basis gradients and Laplacians;
* dE_L and d ln|Psi| along ion, electron, mixed and warped directions against
  Richardson-extrapolated central differences of the oracle's own E_L and
  log|Psi| (electrons and ions displaced explicitly);
* the zero-variance case (hydrogen-like 1s, exact exponent): E_L = -Z^2/2 for
  every configuration and ion position, so every derivative vanishes;
* rigid translation of ions and electrons changes nothing;
* the warp weights sum to one, so the warped derivatives over all atoms sum to
  the rigid translation, i.e. to zero; the Jacobian term sums to zero;
* the zero-variance force estimate of the exact wavefunction is zero.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import synth


def _sys():
    return synth.small_random_system(23, n_atom=3, n_up=3, n_dn=2, shells=(0, 0, 1, 2), nprim=2)


def _fd(f, h):
    """Richardson extrapolation of central differences with steps 2h and h."""
    d2 = (f(2 * h) - f(-2 * h)) / (4 * h)
    d1 = (f(h) - f(-h)) / (2 * h)
    return (4 * d1 - d2) / 3


def _moved(s, R, dion, del_, t):
    s2 = dataclasses.replace(s, ion_xyz=s.ion_xyz + t * dion)
    return s2, R + t * del_


def test_basis_third_derivatives_vs_fd():
    s = _sys()
    r = np.array([0.3, -0.2, 0.5])
    b = oracle.basis_d3(s, r)
    vgl = oracle.basis_vgl(s, r)
    np.testing.assert_allclose(b[:, [0, 1, 2, 3, 10]], vgl, rtol=1e-13, atol=1e-13)
    hess = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for x in range(3):
        e = np.zeros(3)
        e[x] = 1.0
        fd = _fd(lambda t: oracle.basis_vgl(s, r + t * e), 1e-3)
        for q, (a, c) in enumerate(hess):
            if c == x:
                np.testing.assert_allclose(b[:, 4 + q], fd[:, 1 + a], rtol=1e-7, atol=1e-7)
            elif a == x:
                np.testing.assert_allclose(b[:, 4 + q], fd[:, 1 + c], rtol=1e-7, atol=1e-7)
        np.testing.assert_allclose(b[:, 11 + x], fd[:, 4], rtol=1e-7, atol=1e-6)


@pytest.mark.parametrize("kind", ["ion", "electron", "mixed", "warp"])
def test_local_energy_direction_vs_fd(kind):
    s = _sys()
    R = synth.make_walkers(s, 3, 88)
    rng = np.random.default_rng({"ion": 1, "electron": 2, "mixed": 3, "warp": 4}[kind])
    for Rw in R:
        dion = np.zeros_like(s.ion_xyz)
        del_ = np.zeros_like(Rw)
        if kind in ("ion", "mixed"):
            dion[rng.integers(s.n_atom)] = rng.standard_normal(3)
        if kind in ("electron", "mixed"):
            del_ = rng.standard_normal(Rw.shape)
        if kind == "warp":
            a, x = rng.integers(s.n_atom), rng.integers(3)
            dion[a, x] = 1.0
            for i in range(s.n_elec):
                del_[i, x] = oracle.warp_weights(s, Rw[i])[0][a]
        de, dl, rc = oracle.local_energy_dir(s, Rw, dion, del_)
        assert rc == 0

        def ev(t, q):
            s2, R2 = _moved(s, Rw, dion, del_, t)
            return oracle.evaluate(s2, R2)[q]

        fd_e = _fd(lambda t: ev(t, 2), 1e-4)
        fd_l = _fd(lambda t: ev(t, 0), 1e-4)
        assert abs(de - fd_e) <= 1e-6 * max(1.0, abs(fd_e)), (kind, de, fd_e)
        assert abs(dl - fd_l) <= 1e-7 * max(1.0, abs(fd_l)), (kind, dl, fd_l)


def test_zero_variance_case_has_zero_derivatives():
    Z = 2.0
    s = synth.System("h1s", np.zeros((1, 3)), np.array([Z]), [0], [0], [1], [0.0], [1.0],
                     np.ones((1, 1)), 1, 0, jen_a=np.array([-Z]), jen_b=0.0)
    rng = np.random.default_rng(5)
    for _ in range(4):
        R = rng.standard_normal((1, 3))
        for dion, del_ in ((rng.standard_normal((1, 3)), np.zeros((1, 3))),
                           (np.zeros((1, 3)), rng.standard_normal((1, 3)))):
            de, dl, _ = oracle.local_energy_dir(s, R, dion, del_)
            assert abs(de) < 1e-12
        for warp in (False, True):
            dEL, dlp, dj, _ = oracle.zv_grads_batch(s, R[None], warp)
            assert np.abs(dEL).max() < 1e-12


def test_rigid_translation_changes_nothing():
    s = _sys()
    R = synth.make_walkers(s, 2, 89)
    for Rw in R:
        for x in range(3):
            dion = np.zeros_like(s.ion_xyz)
            dion[:, x] = 1.0
            del_ = np.zeros_like(Rw)
            del_[:, x] = 1.0
            de, dl, _ = oracle.local_energy_dir(s, Rw, dion, del_)
            e = oracle.evaluate(s, Rw)[2]
            assert abs(de) < 1e-10 * max(1.0, abs(e))
            assert abs(dl) < 1e-11


def test_warp_weights_and_sum_rules():
    s = _sys()
    R = synth.make_walkers(s, 2, 90)
    r = np.array([0.4, 0.1, -0.3])
    om, dom = oracle.warp_weights(s, r)
    assert abs(om.sum() - 1.0) < 1e-15
    for x in range(3):
        e = np.zeros(3)
        e[x] = 1.0
        fd = _fd(lambda t: oracle.warp_weights(s, r + t * e)[0], 1e-4)
        np.testing.assert_allclose(dom[:, x], fd, rtol=1e-7, atol=1e-9)
    dEL, dlp, dj, rc = oracle.zv_grads_batch(s, R, True)
    assert rc == 0
    e = np.array([oracle.evaluate(s, Rw)[2] for Rw in R])
    assert np.all(np.abs(dEL.sum(axis=1)) < 1e-10 * np.maximum(1.0, np.abs(e))[:, None])
    assert np.abs(dlp.sum(axis=1)).max() < 1e-11
    assert np.abs(dj.sum(axis=1)).max() < 1e-10
    # without the warp: the ion derivatives are the ion part of the translation,
    # sum_a dE_L/dR_a = -sum_i dE_L/dr_i
    dEL0, dlp0, dj0, _ = oracle.zv_grads_batch(s, R, False)
    assert np.all(dj0 == 0.0)
    for w, Rw in enumerate(R):
        for x in range(3):
            del_ = np.zeros_like(Rw)
            del_[:, x] = 1.0
            de, dl, _ = oracle.local_energy_dir(s, Rw, np.zeros_like(s.ion_xyz), del_)
            assert abs(dEL0[w, :, x].sum() + de) < 1e-10 * max(1.0, abs(e[w]))
            assert abs(dlp0[w, :, x].sum() + dl) < 1e-11


def test_zero_variance_force_of_exact_wavefunction_is_zero():
    Z = 1.0
    s = synth.System("h1s", np.zeros((1, 3)), np.array([Z]), [0], [0], [1], [0.0], [1.0],
                     np.ones((1, 1)), 1, 0, jen_a=np.array([-Z]), jen_b=0.0)
    R = np.random.default_rng(6).standard_normal((16, 1, 3))
    e = np.array([oracle.evaluate(s, Rw)[2] for Rw in R])
    for warp in (False, True):
        dEL, dlp, dj, _ = oracle.zv_grads_batch(s, R, warp)
        F = oracle.zv_force_estimator(np.zeros(16), e, dEL, dlp, dj)
        assert np.abs(F).max() < 1e-12


def test_without_warp_ion_log_derivative_matches_eq3_gradients():
    """d ln|Psi| along an ion coordinate equals the Eq. 3 ion gradient that the
    oracle computes by its own forward mode."""
    s = _sys()
    R = synth.make_walkers(s, 3, 91)
    dEL, dlp, dj, _ = oracle.zv_grads_batch(s, R, False)
    dl, dv, _ = oracle.ion_grads_batch(s, R)
    np.testing.assert_allclose(dlp, dl, rtol=1e-12, atol=1e-12)
