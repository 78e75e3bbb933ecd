"""Pins of the oracle's multideterminant trial function (Eq. 2 with M > 1)
against facts that do not come from the multideterminant code itself.

* Multilinearity: a determinant is linear in each column, so an expansion
  over the excitations h -> p of a column (and of two columns) sums to ONE
  determinant whose column h holds phi_h + c phi_p.  The oracle's
  single-determinant path (pinned elsewhere) evaluates that determinant;
  log|Psi|, sign, E_L, drift and whole runs must agree.
* A zero coefficient on every excitation reduces to the single determinant.
* E_L against a finite-difference kinetic energy of ln|Psi|, and the drift
  against finite differences of ln|Psi|.
* |Psi_MSD / Psi_0| against the direct-LU ratio routine.
* Exchanging two electrons of one spin flips the sign only.
"""
import dataclasses

import numpy as np

import oracle
from paper_2504_07948_amd import synth


def _base(seed=31, n_mo=10):
    return synth.small_random_system(seed, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2,
                                     n_mo=n_mo)


def _with_exc(s, rows, coef):
    exc = np.array([[0, 0] + [-1] * 8] + rows, dtype=np.int32)
    return dataclasses.replace(s, n_det=len(exc), det_exc=exc,
                               ci_coef=np.array([1.0] + list(coef), dtype=np.float64))


def _single(spin, h, p):
    return [1, 0, h, -1, p, -1, -1, -1, -1, -1] if spin == 0 else [0, 1, -1, -1, -1, -1, h, -1, p, -1]


def _double_same(spin, h1, h2, p1, p2):
    return ([2, 0, h1, h2, p1, p2, -1, -1, -1, -1] if spin == 0 else
            [0, 2, -1, -1, -1, -1, h1, h2, p1, p2])


def _combine(up, dn):
    """Excitation row with the up part of `up` and the down part of `dn`."""
    return [up[0], dn[1]] + up[2:6] + dn[6:10]


def _check_same(a, b, R, tol=1e-11):
    for Rw in R:
        la, sa, ea, da = oracle.evaluate(a, Rw)[:4]
        lb, sb, eb, db = oracle.evaluate(b, Rw)[:4]
        assert sa == sb
        assert abs(la - lb) <= tol * max(1.0, abs(lb))
        assert abs(ea - eb) <= tol * max(1.0, abs(eb))
        np.testing.assert_allclose(da, db, rtol=tol, atol=tol)


def test_zero_coefficients_reduce_to_single_determinant():
    s = _base()
    m = _with_exc(s, [_single(0, 1, 5), _double_same(1, 0, 2, 4, 6)], [0.0, 0.0])
    R = synth.make_walkers(s, 4, 3)
    _check_same(m, s, R)


def test_single_excitations_sum_to_one_determinant():
    s = _base()
    c, h, p = 0.37, 1, 6
    rows = [_single(0, h, p), _single(1, h, p), _combine(_single(0, h, p), _single(1, h, p))]
    m = _with_exc(s, rows, [c, c, c * c])
    mo = s.mo_coef.copy()
    mo[:, h] += c * mo[:, p]
    eq = dataclasses.replace(s, mo_coef=mo)
    R = synth.make_walkers(s, 5, 4)
    _check_same(m, eq, R)
    # whole runs: same accept sequence, energies and weights
    ra = oracle.run(m, R, n_steps=3, mode=1, tau=0.02, seed=5, e_trial=-3.0)
    rb = oracle.run(eq, R, n_steps=3, mode=1, tau=0.02, seed=5, e_trial=-3.0)
    np.testing.assert_array_equal(ra["accept_log"], rb["accept_log"])
    np.testing.assert_allclose(ra["e_log"], rb["e_log"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(ra["R"], rb["R"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ra["log_w"], rb["log_w"], rtol=1e-10, atol=1e-12)


def test_double_excitations_sum_to_one_determinant():
    """(D + a D_{h1->p1} + b D_{h2->p2} + ab D_{h1h2->p1p2}) per spin, product
    over spins: 16 determinants with up to two excitations per spin."""
    s = _base()
    (h1, p1, a), (h2, p2, b) = (0, 5, -0.41), (2, 7, 0.23)
    per_spin = [(None, 1.0), ("s1", a), ("s2", b), ("d", a * b)]

    def part(kind, spin):
        if kind is None:
            return [0, 0] + [-1] * 8
        if kind == "s1":
            return _single(spin, h1, p1)
        if kind == "s2":
            return _single(spin, h2, p2)
        return _double_same(spin, h1, h2, p1, p2)

    rows, coef = [], []
    for ku, cu in per_spin:
        for kd, cd in per_spin:
            if ku is None and kd is None:
                continue
            rows.append(_combine(part(ku, 0), part(kd, 1)))
            coef.append(cu * cd)
    m = _with_exc(s, rows, coef)
    mo = s.mo_coef.copy()
    mo[:, h1] += a * s.mo_coef[:, p1]
    mo[:, h2] += b * s.mo_coef[:, p2]
    eq = dataclasses.replace(s, mo_coef=mo)
    R = synth.make_walkers(s, 5, 6)
    _check_same(m, eq, R)
    ra = oracle.run(m, R, n_steps=2, mode=0, tau=0.02, seed=8)
    rb = oracle.run(eq, R, n_steps=2, mode=0, tau=0.02, seed=8)
    np.testing.assert_array_equal(ra["accept_log"], rb["accept_log"])
    np.testing.assert_allclose(ra["e_log"], rb["e_log"], rtol=1e-10, atol=1e-10)


def _random_msd(seed=41):
    s = _base(seed, n_mo=8)
    return synth.make_msd(s, n_det=15, n_active=6, seed=seed + 1)


def test_local_energy_and_drift_vs_finite_differences():
    m = _random_msd()
    R = synth.make_walkers(m, 3, 9)

    def lp(Rx):
        return oracle.evaluate(m, Rx)[0]

    for Rw in R:
        l0, _, e0, d0 = oracle.evaluate(m, Rw)[:4]
        kin_fd = 0.0
        for i in range(m.n_elec):
            for x in range(3):
                vals = {}
                for h in (1e-3, 5e-4):
                    Rp = Rw.copy(); Rp[i, x] += h
                    Rm = Rw.copy(); Rm[i, x] -= h
                    fp, fm = lp(Rp), lp(Rm)
                    vals[h] = ((fp - fm) / (2 * h), (fp - 2 * l0 + fm) / h ** 2)
                g = (4 * vals[5e-4][0] - vals[1e-3][0]) / 3  # Richardson
                d2 = (4 * vals[5e-4][1] - vals[1e-3][1]) / 3
                assert abs(g - d0[i, x]) <= 1e-6 * max(1.0, abs(g))
                kin_fd += d2 + g * g
        e_fd = -0.5 * kin_fd + oracle.potential(m, Rw)
        assert abs(e_fd - e0) <= 1e-5 * max(1.0, abs(e0)), (e_fd, e0)


def test_ratio_matches_direct_lu_routine():
    m = _random_msd()
    ref = dataclasses.replace(m, n_det=0, det_exc=None, ci_coef=None)
    for Rw in synth.make_walkers(m, 4, 10):
        lm, sm, _, _ = oracle.evaluate(m, Rw)[:4]
        l0, s0, _, _ = oracle.evaluate(ref, Rw)[:4]
        r = oracle.msd_ratio_direct(m, Rw)
        assert abs(np.exp(lm - l0) - abs(r)) <= 1e-11 * max(1.0, abs(r))
        assert sm * s0 == (1 if r > 0 else -1)


def test_exchange_of_two_same_spin_electrons():
    m = _random_msd()
    for Rw in synth.make_walkers(m, 3, 11):
        l0, s0, e0, d0 = oracle.evaluate(m, Rw)[:4]
        Rx = Rw.copy()
        Rx[[0, 2]] = Rx[[2, 0]]
        l1, s1, e1, d1 = oracle.evaluate(m, Rx)[:4]
        assert s1 == -s0
        assert abs(l1 - l0) <= 1e-12 * max(1.0, abs(l0))
        assert abs(e1 - e0) <= 1e-10 * max(1.0, abs(e0))
        np.testing.assert_allclose(d1[[2, 0]], d0[[0, 2]], rtol=1e-10, atol=1e-10)


def test_ion_gradients_sum_to_one_determinant():
    """Forward-mode ion gradients of the 16-determinant expansion equal those
    of the single determinant with the mixed columns (multilinearity)."""
    s = _base()
    (h1, p1, a), (h2, p2, b) = (1, 6, 0.35), (2, 8, -0.27)
    per_spin = [([0, 0] + [-1] * 8, 1.0)]

    def rows_for(spin):
        return [(_single(spin, h1, p1), a), (_single(spin, h2, p2), b),
                (_double_same(spin, h1, h2, p1, p2), a * b)]

    rows, coef = [], []
    for ru, cu in per_spin + rows_for(0):
        for rd, cd in per_spin + rows_for(1):
            if cu == 1.0 and cd == 1.0 and ru[0] == 0 and rd[1] == 0:
                continue
            rows.append(_combine(ru, rd))
            coef.append(cu * cd)
    m = _with_exc(s, rows, coef)
    mo = s.mo_coef.copy()
    mo[:, h1] += a * s.mo_coef[:, p1]
    mo[:, h2] += b * s.mo_coef[:, p2]
    eq = dataclasses.replace(s, mo_coef=mo)
    for Rw in synth.make_walkers(s, 3, 12):
        dl_m, dv_m = oracle.ion_grads(m, Rw)[:2]
        dl_e, dv_e = oracle.ion_grads(eq, Rw)[:2]
        np.testing.assert_allclose(dl_m, dl_e, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(dv_m, dv_e, rtol=1e-12, atol=1e-12)


def test_ion_gradients_vs_finite_differences():
    m = _random_msd()
    Rw = synth.make_walkers(m, 1, 13)[0]
    dl = oracle.ion_grads(m, Rw)[0]

    def lp_at(xyz):
        return oracle.evaluate(dataclasses.replace(m, ion_xyz=xyz), Rw)[0]

    for a in range(m.n_atom):
        for x in range(3):
            est = {}
            for h in (2e-4, 1e-4):
                xp = m.ion_xyz.copy(); xp[a, x] += h
                xm = m.ion_xyz.copy(); xm[a, x] -= h
                est[h] = (lp_at(xp) - lp_at(xm)) / (2 * h)
            fd = (4 * est[1e-4] - est[2e-4]) / 3
            assert abs(fd - dl[a, x]) <= 1e-6 * max(1.0, abs(fd)), (a, x, fd, dl[a, x])
