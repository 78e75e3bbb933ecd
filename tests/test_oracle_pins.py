"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Each test ties one oracle function to something the paper or the mathematics
fixes (arXiv 2504.07948, QMC section):
  * Philox4x32-10 against its published known-answer vectors;
  * the LU log-determinant / inverse against numpy.linalg;
  * basis and orbital gradients/Laplacians against central finite differences,
    and single-Gaussian local energies against their closed forms;
  * the zero-variance case: a hydrogen-like 1s with the exact exponent has
    E_L = -Z^2/2 at every sample;
  * E_L against a finite-difference kinetic energy of log|Psi| (Eq. 2 trial
    function), invariances of Psi, and Eq. 3 ion gradients against finite
    differences and translation sum rules;
  * one DMC sweep (Eq. 1, fixed node) against a brute-force re-evaluation of
    Psi at every proposal.
A plausible mistake (dropped term, sign, index, transposed operand) in any
oracle function fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _one_electron_system(l, comp, alpha, Z=1.0, jen_a=0.0, jen_b=0.0, nprim_coef=1.0):
    nc = synth.NCART[l]
    mo = np.zeros((nc, 1))
    mo[comp, 0] = 1.0
    return synth.System("one", np.zeros((1, 3)), np.array([Z]), [0], [l], [1], [alpha],
                        [nprim_coef], mo, 1, 0, jen_a=np.array([jen_a]), jen_b=jen_b)


# ------------------------------------------------------------------ Philox --
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_move_draws_moments():
    chis, us = [], []
    for w in range(40):
        for i in range(50):
            c, u = oracle.move_draws(12345, 3, w, i)
            chis.append(c)
            us.append(u)
    chis = np.array(chis)
    us = np.array(us)
    n = len(us)
    assert abs(chis.mean()) < 4.0 / math.sqrt(3 * n)
    assert abs(chis.var() - 1.0) < 6.0 * math.sqrt(2.0 / (3 * n))
    assert abs(us.mean() - 0.5) < 4.0 * math.sqrt(1 / 12 / n)
    assert us.min() >= 0.0 and us.max() < 1.0
    # counter-based: same counter -> same draw, different counter -> different
    assert oracle.move_draws(1, 2, 3, 4)[1] == oracle.move_draws(1, 2, 3, 4)[1]
    assert oracle.move_draws(1, 2, 3, 4)[1] != oracle.move_draws(1, 2, 3, 5)[1]


# --------------------------------------------------------------------- LU --
@pytest.mark.parametrize("n", [1, 2, 5, 17, 56])
def test_lu_against_numpy(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    if n > 1:
        A[0, 0] = 0.0  # forces a row exchange
    sg, ld, inv, rc = oracle.lu_slogdet_inv(A)
    s_np, ld_np = np.linalg.slogdet(A)
    assert rc == 0 and sg == int(s_np)
    assert abs(ld - ld_np) < 1e-12 * max(1.0, abs(ld_np))
    np.testing.assert_allclose(inv, np.linalg.inv(A), rtol=1e-10, atol=1e-12 * np.abs(inv).max())


def test_lu_singular():
    A = np.ones((3, 3))
    sg, ld, inv, rc = oracle.lu_slogdet_inv(A)
    assert rc == 1 and sg == 0 and ld == -math.inf


# ------------------------------------------------------------------ basis --
def _fd_grad_lap(f, r, h=1e-4):
    g = np.zeros((3,) + np.shape(f(r)))
    lap = 0.0
    f0 = f(r)
    for x in range(3):
        e = np.zeros(3)
        e[x] = h
        fp, fm = f(r + e), f(r - e)
        g[x] = (fp - fm) / (2 * h)
        lap = lap + (fp - 2 * f0 + fm) / (h * h)
    return g, lap


def test_basis_single_s_closed_form():
    s = _one_electron_system(0, 0, 0.7)
    r = np.array([0.3, -0.4, 0.5])
    v = oracle.basis_vgl(s, r)[0]
    r2 = r @ r
    e = math.exp(-0.7 * r2)
    np.testing.assert_allclose(v[0], e, rtol=1e-15)
    np.testing.assert_allclose(v[1:4], -2 * 0.7 * r * e, rtol=1e-14)
    np.testing.assert_allclose(v[4], (4 * 0.49 * r2 - 6 * 0.7) * e, rtol=1e-14)


def test_basis_fd_all_shell_types():
    s = synth.small_random_system(11, n_atom=2, shells=(0, 1, 2, 2), nprim=3)
    rng = np.random.default_rng(0)
    for _ in range(4):
        r = s.ion_xyz[0] + 0.7 * rng.standard_normal(3)
        v = oracle.basis_vgl(s, r)
        g, lap = _fd_grad_lap(lambda q: oracle.basis_vgl(s, q)[:, 0], r, h=1e-4)
        scale = np.abs(v[:, 0]).max() + np.abs(v[:, 1:4]).max()
        np.testing.assert_allclose(v[:, 1:4].T, g, atol=1e-7 * scale)
        np.testing.assert_allclose(v[:, 4], lap, atol=2e-4 * np.abs(v[:, 4]).max())


def test_basis_cartesian_order_and_count():
    s = synth.small_random_system(12, n_atom=1, shells=(2,), nprim=1)
    r = s.ion_xyz[0] + np.array([0.2, 0.3, 0.5])
    v = oracle.basis_vgl(s, r)[:, 0]
    d = r - s.ion_xyz[0]
    R = s.prim_coef[0] * math.exp(-s.prim_alpha[0] * d @ d)
    x, y, z = d
    np.testing.assert_allclose(v, R * np.array([x * x, x * y, x * z, y * y, y * z, z * z]),
                               rtol=1e-14)


def test_orbitals_are_lcao_of_basis():
    s = synth.small_random_system(13, n_atom=3, shells=(0, 0, 1, 2), nprim=2, n_up=3, n_dn=2)
    r = np.array([0.4, 1.1, -0.3])
    b = oracle.basis_vgl(s, r)
    o = oracle.orbitals_vgl(s, r, 3)
    np.testing.assert_allclose(o, (s.mo_coef[:, :3].T @ b).T, rtol=1e-12, atol=1e-14)
    g, lap = _fd_grad_lap(lambda q: oracle.orbitals_vgl(s, q, 3)[0], r)
    np.testing.assert_allclose(o[1:4], g, atol=1e-7 * np.abs(o).max())
    np.testing.assert_allclose(o[4], lap, atol=2e-4 * np.abs(o).max())


# ----------------------------------------------------------------- Jastrow --
def test_jastrow_two_electrons_closed_form():
    s = synth.small_random_system(14, n_atom=1, n_up=1, n_dn=1)
    s.jen_a = np.zeros(1)
    R = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.3]])
    J, g, lap = oracle.jastrow(s, R)
    a, b, r = 0.5, s.jee_b, 1.3
    assert abs(J - a * r / (1 + b * r)) < 1e-15
    up = a / (1 + b * r) ** 2
    np.testing.assert_allclose(g[0], [0, 0, -up], atol=1e-15)
    np.testing.assert_allclose(g[1], [0, 0, up], atol=1e-15)
    # parallel spins use a = 1/4
    s2 = synth.small_random_system(14, n_atom=1, n_up=2, n_dn=0)
    s2.jen_a = np.zeros(1)
    J2, _, _ = oracle.jastrow(s2, R)
    assert abs(J2 - 0.25 * r / (1 + b * r)) < 1e-15


def test_jastrow_fd():
    s = synth.small_random_system(15, n_atom=2, n_up=3, n_dn=2)
    R = synth.make_walkers(s, 1, 5)[0]
    J, g, lap = oracle.jastrow(s, R)
    for i in range(s.n_elec):
        def f(q, i=i):
            R2 = R.copy()
            R2[i] = q
            return np.array(oracle.jastrow(s, R2)[0])
        gf, lf = _fd_grad_lap(f, R[i])
        np.testing.assert_allclose(g[i], gf, atol=1e-7)
        np.testing.assert_allclose(lap[i], lf, atol=1e-4)


def test_potential_closed_form():
    s = synth.System("pot", np.array([[0, 0, 0], [0, 0, 2.0]]), np.array([2.0, 1.0]), [0, 1],
                     [0, 0], [1, 1], [1.0, 1.0], [1.0, 1.0], np.eye(2)[:, :1], 1, 1)
    R = np.array([[1.0, 0, 0], [0, 0, 3.0]])
    v = oracle.potential(s, R)
    r12 = math.sqrt(1 + 9)
    expect = (1 / r12 - 2 / 1.0 - 1 / math.sqrt(1 + 4) - 2 / 3.0 - 1 / 1.0 + 2 * 1 / 2.0)
    assert abs(v - expect) < 1e-14


# ------------------------------------------------------------ local energy --
@pytest.mark.parametrize("Z", [1.0, 2.0, 3.0])
def test_zero_variance_hydrogenic(Z):
    """Psi = exp(-Z r) through a constant orbital and a Pade e-n term with
    a = -Z, b = 0: E_L = -Z^2/2 at every point and drift = -Z r_hat."""
    s = _one_electron_system(0, 0, 0.0, Z=Z, jen_a=-Z, jen_b=0.0)
    rng = np.random.default_rng(int(Z))
    for _ in range(20):
        r = rng.standard_normal(3) * rng.uniform(0.05, 3.0)
        lp, sg, el, dr, rc = oracle.evaluate(s, r[None, :])
        assert rc == 0 and sg == 1
        assert abs(el + Z * Z / 2) < 1e-12
        np.testing.assert_allclose(dr[0], -Z * r / np.linalg.norm(r), atol=1e-13)
        assert abs(lp + Z * np.linalg.norm(r)) < 1e-13


@pytest.mark.parametrize("l,comp,coef", [(0, 0, 3.0), (1, 0, 5.0), (2, 1, 7.0)])
def test_single_gaussian_closed_form(l, comp, coef):
    """No Jastrow, one Cartesian Gaussian: E_L = c*alpha - 2 alpha^2 r^2 - Z/r
    with c = 3 (s), 5 (p_x), 7 (d_xy)."""
    alpha, Z = 0.8, 1.0
    s = _one_electron_system(l, comp, alpha, Z=Z)
    rng = np.random.default_rng(l)
    for _ in range(10):
        r = rng.standard_normal(3)
        el = oracle.evaluate(s, r[None, :])[2]
        r2 = r @ r
        assert abs(el - (coef * alpha - 2 * alpha ** 2 * r2 - Z / math.sqrt(r2))) < 1e-11


def _logpsi(s, R):
    return oracle.evaluate(s, R)[0]


def test_local_energy_and_drift_vs_fd():
    """E_L = -1/2 sum_i (lap_i ln|Psi| + |grad_i ln|Psi||^2) + V, by FD of
    ln|Psi| (independent of the tr(A^-1 B) assembly)."""
    s = synth.small_random_system(16, n_atom=2, n_up=3, n_dn=2, shells=(0, 0, 1, 2), nprim=2)
    R = synth.make_walkers(s, 1, 9)[0]
    lp, sg, el, dr, rc = oracle.evaluate(s, R)
    h = 1e-4
    kin = 0.0
    for i in range(s.n_elec):
        for x in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[i, x] += h
            Rm[i, x] -= h
            fp, fm = _logpsi(s, Rp), _logpsi(s, Rm)
            g = (fp - fm) / (2 * h)
            l2 = (fp - 2 * lp + fm) / (h * h)
            assert abs(g - dr[i, x]) < 1e-6 * max(1, abs(g))
            kin += l2 + g * g
    el_fd = -0.5 * kin + oracle.potential(s, R)
    assert abs(el - el_fd) < 2e-4 * max(1.0, abs(el))


def test_invariances():
    s = synth.small_random_system(17, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2)
    R = synth.make_walkers(s, 1, 3)[0]
    lp, sg, el, dr, _ = oracle.evaluate(s, R)
    # occupied-space mixing C -> C U
    U = np.random.default_rng(1).standard_normal((3, 3))
    s2 = synth.System(**{**s.__dict__, "mo_coef": s.mo_coef[:, :3] @ U})
    lp2, sg2, el2, dr2, _ = oracle.evaluate(s2, R)
    su, ldu = np.linalg.slogdet(U)
    assert abs(lp2 - (lp + 2 * ldu)) < 1e-10
    assert abs(el2 - el) < 1e-9 * max(1, abs(el))
    np.testing.assert_allclose(dr2, dr, atol=1e-9)
    # global translation of ions and electrons
    t = np.array([0.3, -1.2, 2.2])
    s3 = synth.System(**{**s.__dict__, "ion_xyz": s.ion_xyz + t})
    lp3, sg3, el3, _, _ = oracle.evaluate(s3, R + t)
    assert abs(lp3 - lp) < 1e-10 and sg3 == sg and abs(el3 - el) < 1e-9 * max(1, abs(el))
    # exchange of two same-spin electrons
    R4 = R.copy()
    R4[[0, 1]] = R4[[1, 0]]
    lp4, sg4, el4, _, _ = oracle.evaluate(s, R4)
    assert sg4 == -sg and abs(lp4 - lp) < 1e-10 and abs(el4 - el) < 1e-9 * max(1, abs(el))


# --------------------------------------------------------------- ion grads --
def test_ion_grads_vs_fd_and_sum_rules():
    s = synth.small_random_system(18, n_atom=3, n_up=3, n_dn=2, shells=(0, 0, 1, 2), nprim=2)
    R = synth.make_walkers(s, 1, 4)[0]
    dl, dv, rc = oracle.ion_grads(s, R)
    assert rc == 0
    h = 1e-4
    for a in range(s.n_atom):
        for x in range(3):
            sp = synth.System(**{**s.__dict__, "ion_xyz": s.ion_xyz.copy()})
            sm = synth.System(**{**s.__dict__, "ion_xyz": s.ion_xyz.copy()})
            sp.ion_xyz[a, x] += h
            sm.ion_xyz[a, x] -= h
            fd = (_logpsi(sp, R) - _logpsi(sm, R)) / (2 * h)
            fv = (oracle.potential(sp, R) - oracle.potential(sm, R)) / (2 * h)
            assert abs(fd - dl[a, x]) < 1e-6 * max(1, abs(fd))
            assert abs(fv - dv[a, x]) < 1e-6 * max(1, abs(fv))
    # translation sum rules: sum_A d/dR_A = - sum_i d/dr_i
    dr = oracle.evaluate(s, R)[3]
    np.testing.assert_allclose(dl.sum(0), -dr.sum(0), atol=1e-9)
    h = 1e-5
    gv = np.zeros(3)
    for x in range(3):
        Rp, Rm = R.copy(), R.copy()
        Rp[:, x] += h
        Rm[:, x] -= h
        gv[x] = (oracle.potential(s, Rp) - oracle.potential(s, Rm)) / (2 * h)
    np.testing.assert_allclose(dv.sum(0), -gv, atol=1e-6)


# ------------------------------------------------------------------- sweep --
def _brute_force_sweep(s, R, step, mode, tau, seed, walker):
    """One sweep with a complete re-evaluation of Psi at every proposal."""
    R = R.copy()
    acc = np.zeros(s.n_elec, dtype=np.uint8)
    for i in range(s.n_elec):
        lp, sg, _, dr, _ = oracle.evaluate(s, R)
        chi, u = oracle.move_draws(seed, step, walker, i)
        rn = R[i] + tau * dr[i] + math.sqrt(tau) * chi
        R2 = R.copy()
        R2[i] = rn
        lp2, sg2, _, dr2, _ = oracle.evaluate(s, R2)
        if mode == 1 and sg2 * sg <= 0:
            continue
        fwd = np.sum((rn - R[i] - tau * dr[i]) ** 2)
        bwd = np.sum((R[i] - rn - tau * dr2[i]) ** 2)
        lnq = 2 * (lp2 - lp) + (fwd - bwd) / (2 * tau)
        p = 1.0 if lnq >= 0 else math.exp(lnq)
        if u < p:
            R = R2
            acc[i] = 1
    return R, acc


@pytest.mark.parametrize("mode", [0, 1])
def test_sweep_matches_brute_force(mode):
    s = synth.small_random_system(19, n_atom=2, n_up=3, n_dn=2, shells=(0, 0, 1, 2), nprim=2)
    W, tau, seed = 4, 0.05, 99
    R0 = synth.make_walkers(s, W, 8)
    out = oracle.run(s, R0, n_steps=2, mode=mode, tau=tau, seed=seed, e_trial=-1.0,
                     walker_offset=10)
    for w in range(W):
        R = R0[w]
        for st in range(2):
            R, acc = _brute_force_sweep(s, R, st, mode, tau, seed, 10 + w)
            np.testing.assert_array_equal(out["accept_log"][st, w], acc)
        np.testing.assert_allclose(out["R"][w], R, atol=1e-12)
    assert out["accept_log"].mean() > 0.5


def test_dmc_weights_exact_for_zero_variance():
    """With E_L = -Z^2/2 everywhere, log w = -tau * n * (E - E_T) exactly."""
    Z, tau, n = 2.0, 0.01, 5
    s = _one_electron_system(0, 0, 0.0, Z=Z, jen_a=-Z, jen_b=0.0)
    R = np.random.default_rng(2).standard_normal((8, 1, 3))
    out = oracle.run(s, R, n_steps=n, mode=1, tau=tau, seed=5, e_trial=-1.5)
    np.testing.assert_allclose(out["log_w"], -tau * n * (-Z * Z / 2 + 1.5), atol=1e-13)
    np.testing.assert_allclose(out["e_log"], -Z * Z / 2, atol=1e-12)


def _msd_small_system():
    """3+3 electrons, 10 MOs, a reference plus singles and doubles of both spins."""
    import dataclasses
    s = synth.small_random_system(31, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2,
                                  n_mo=10)
    exc = np.array([[0, 0] + [-1] * 8,
                    [1, 0, 1, -1, 5, -1, -1, -1, -1, -1],
                    [0, 1, -1, -1, -1, -1, 2, -1, 4, -1],
                    [2, 0, 0, 2, 4, 6, -1, -1, -1, -1],
                    [1, 1, 0, -1, 7, -1, 1, -1, 3, -1]], dtype=np.int32)
    return dataclasses.replace(s, n_det=len(exc), det_exc=exc,
                               ci_coef=np.array([1.0, 0.4, -0.3, 0.2, -0.25]))


@pytest.mark.parametrize("msd", [False, True])
def test_dmc_log_weights_rebuilt_from_step_end_energies(msd):
    """Eq. 1 weight update, log w += -tau((E_L,old + E_L,new)/2 - E_T), rebuilt
    from E_L evaluated afresh (oracle.evaluate, pinned by the E_L tests above)
    at the configuration before step 0 and at every step end, for walkers whose
    E_L varies from step to step.  An update that used only E_new or only E_old
    differs from the rebuilt weights by tau/2 |E_first - E_last|, which the test
    asserts is far above its tolerance."""
    s = _msd_small_system() if msd else synth.small_random_system(
        19, n_atom=2, n_up=3, n_dn=2, shells=(0, 0, 1, 2), nprim=2)
    W, n, tau, seed, e_t = 3, 5, 0.05, 41, -1.25
    R0 = synth.make_walkers(s, W, 8)
    lw0 = np.array([0.3, -0.7, 1.1])
    out = oracle.run(s, R0, log_w=lw0, n_steps=n, mode=1, tau=tau, seed=seed, e_trial=e_t)
    R = R0.copy()
    e_prev = np.array([oracle.evaluate(s, R[w])[2] for w in range(W)])
    e_first = e_prev.copy()
    expect = lw0.copy()
    for st in range(n):
        R = oracle.run(s, R, n_steps=1, step0=st, mode=1, tau=tau, seed=seed, e_trial=e_t)["R"]
        e_new = np.array([oracle.evaluate(s, R[w])[2] for w in range(W)])
        np.testing.assert_allclose(out["e_log"][st], e_new, rtol=1e-12, atol=1e-12)
        expect += -tau * (0.5 * (e_prev + e_new) - e_t)
        e_prev = e_new
    np.testing.assert_allclose(out["R"], R, rtol=0, atol=1e-13)
    tol = 1e-13 * np.maximum(1.0, np.abs(expect))
    assert np.all(np.abs(out["log_w"] - expect) <= tol)
    # the trapezoid is distinguishable from the one-sided updates on these walkers
    one_sided = 0.5 * tau * np.abs(e_first - e_prev)
    assert np.all(one_sided > 1e3 * tol), one_sided
    assert out["accept_log"].mean() > 0.3


def test_vmc_variational_bound_hydrogen():
    """VMC of H with a non-exact Jastrow exponent (b > 0): <E> >= -1/2."""
    s = _one_electron_system(0, 0, 0.0, Z=1.0, jen_a=-1.0, jen_b=0.3)
    R = np.random.default_rng(3).standard_normal((256, 1, 3))
    out = oracle.run(s, R, n_steps=60, mode=0, tau=0.1, seed=11)
    e = out["e_log"][20:].mean()
    err = out["e_log"][20:].std() / math.sqrt(out["e_log"][20:].size / 10)
    assert e > -0.5 - 3 * err


# --------------------------------------------------------------------- MSD --
def test_msd_direct_reference_and_single_excitation():
    s = synth.small_random_system(20, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2,
                                  n_mo=8)
    R = synth.make_walkers(s, 1, 1)[0]
    s1 = synth.System(**{**s.__dict__, "n_det": 1, "det_exc": np.array([[0, 0] + [-1] * 8]),
                         "ci_coef": np.array([1.0])})
    assert abs(oracle.msd_ratio_direct(s1, R) - 1.0) < 1e-14
    # one single excitation up: hole 1 -> particle 5, c = 0.3
    exc = np.array([[0, 0] + [-1] * 8, [1, 0, 1, -1, 5, -1, -1, -1, -1, -1]])
    s2 = synth.System(**{**s.__dict__, "n_det": 2, "det_exc": exc, "ci_coef": np.array([1.0, 0.3])})
    A = np.array([oracle.orbitals_vgl(s, R[i], 8)[0] for i in range(3)])
    cols = [0, 5, 2]
    ratio = np.linalg.det(A[:, cols]) / np.linalg.det(A[:, :3])
    assert abs(oracle.msd_ratio_direct(s2, R) - (1.0 + 0.3 * ratio)) < 1e-11


@pytest.mark.parametrize("gain,target", [(0.3, 0), (1.0, 0), (0.3, 12), (0.6, 4)])
def test_et_feedback_zero_variance_closed_form(gain, target):
    """E_T feedback on the exact hydrogen-like wavefunction, where E_L = -Z^2/2
    at every point: every walker's log-weight changes by -tau (E - E_T) per
    step, W_tot = W exp(log w), so the feedback E_T = E - (gain / tau)
    (log w + c), c = ln(W / W_T) for the target population W_T (c = 0 for the
    default W_T = W), gives, from log w = 0 and E_T = E + delta, log w after
    step s (s >= 1) equal to -c + (tau delta + c) (1 - gain)^(s - 1) for
    every walker."""
    Z = 1.6
    s = _one_electron_system(0, 0, 0.0, Z=Z, jen_a=-Z, jen_b=0.0)
    W, n, tau, delta = 6, 7, 0.02, 0.4
    R = np.random.default_rng(3).standard_normal((W, 1, 3))
    E = -Z * Z / 2.0
    lw = np.zeros(W)
    for k in range(1, n + 1):
        out = oracle.run_feedback(s, R, log_w=np.zeros(W), n_steps=k, tau=tau, seed=5,
                                  e_trial=E + delta, gain=gain, target=target)
        assert out["rc"] == 0
        np.testing.assert_allclose(out["e_local"], E, rtol=0, atol=1e-12)
        c = math.log(W / target) if target else 0.0
        np.testing.assert_allclose(out["log_w"], -c + (tau * delta + c) * (1 - gain) ** (k - 1),
                                   rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(out["et_log"][0], E + delta, rtol=0, atol=0)


def test_et_feedback_first_step_is_plain_dmc():
    """The first step uses the E_T it is given: one step with feedback equals
    one plain DMC step at that E_T bit for bit."""
    s = synth.small_molecule()
    R = synth.make_walkers(s, 5, 81)
    a = oracle.run(s, R, n_steps=1, mode=1, tau=0.01, seed=9, e_trial=-7.0)
    b = oracle.run_feedback(s, R, n_steps=1, tau=0.01, seed=9, e_trial=-7.0, gain=0.7)
    np.testing.assert_array_equal(a["accept_log"], b["accept_log"])
    np.testing.assert_array_equal(a["log_w"], b["log_w"])
    np.testing.assert_array_equal(a["R"], b["R"])
    assert b["et_log"][0] == -7.0
