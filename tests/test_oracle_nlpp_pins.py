"""Pins of the oracle's semilocal pseudopotential (the ccECP form of the
paper's QMC runs; the tables themselves are synthetic stand-ins) against
facts that do not come from that code:

* the 12-point icosahedral rule integrates every polynomial of degree <= 5 on
  the sphere exactly, so for one electron in an orbital of pure angular
  momentum L about the pseudopotential's atom (the Jastrow factor there is
  spherical) the non-local energy is v_L(r) exactly, whatever the rotation:
  s, p and d orbitals against channels 0, 1 and 2 at once;
* the quadrature rotations are proper rotations (orthogonal, det +1) and
  average to zero over many draws (uniform over the rotation group);
* the local terms add beta r^(n-2) exp(-alpha r^2) to the potential;
* for many electrons, the sum rebuilt point by point from the definition
  (directions written out here from the icosahedron, ratios from full
  re-evaluations of ln|Psi| at the moved configurations);
* electrons outside the cutoff contribute nothing;
* DMC runs: log w rebuilt from independent step-end energies that include
  each step's non-local energy with that step's rotations;
* the Hellmann-Feynman force term d(V_loc + V_NL)/dR_A (Psi fixed) against
  Richardson differences in the position of a ghost centre that carries the
  pseudopotential alone (no charge, no basis functions, no Jastrow term).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import synth

PHI = (1 + math.sqrt(5)) / 2


def _one_electron_pp(l, comp, terms, Z=1.0, alpha=0.6):
    nc = synth.NCART[l]
    mo = np.zeros((nc, 1))
    mo[comp, 0] = 1.0
    s = synth.System("one", np.zeros((1, 3)), np.array([Z]), [0], [l], [1], [alpha], [1.0], mo,
                     1, 0, jen_a=np.array([-0.3]), jen_b=0.5)
    return synth.with_pseudopotential(s, [terms])


def _v(terms, l, r):
    return sum(b * r ** (n - 2) * math.exp(-a * r * r) for (ll, n, b, a) in terms if ll == l)


TERMS = [(0, 2, 2.0, 1.3), (1, 2, -1.5, 0.9), (1, 3, 0.7, 1.1), (2, 2, 0.8, 1.6), (-1, 2, -1.0, 0.7)]


@pytest.mark.parametrize("l,comp", [(0, 0), (1, 0), (1, 2), (2, 1), (2, 4)])
def test_pure_angular_momentum_closed_form(l, comp):
    s = _one_electron_pp(l, comp, TERMS)
    rng = np.random.default_rng(l * 10 + comp)
    for k in range(5):
        r = rng.standard_normal(3) * rng.uniform(0.3, 1.5)
        rr = np.linalg.norm(r)
        v, rc = oracle.nlpp(s, r[None, :], seed=11 + k, step=k, walker=3)
        assert rc == 0
        ref = _v(TERMS, l, rr)
        print(f"[nlpp] L={l} r={rr:.3f} V_NL={v:.15f} v_L={ref:.15f}")
        assert abs(v - ref) < 1e-13 * max(1.0, abs(ref))


def test_rotations_are_uniform_proper_rotations():
    mats = np.array([oracle.nlpp_rotation(7, st, w, e) for st in range(40) for w in range(25)
                     for e in range(20)])
    eye = np.einsum("nij,nkj->nik", mats, mats)
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(mats) - 1.0).max() < 1e-14
    # Haar measure: E[R] = 0, E[R_ij^2] = 1/3 (20000 draws: standard error 0.004)
    assert np.abs(mats.mean(axis=0)).max() < 0.02
    assert np.abs((mats ** 2).mean(axis=0) - 1.0 / 3.0).max() < 0.02
    # different counters, different rotations
    assert not np.allclose(oracle.nlpp_rotation(7, 0, 0, 0), oracle.nlpp_rotation(7, 0, 0, 1))


def test_local_terms_in_the_potential():
    s = _one_electron_pp(0, 0, TERMS, Z=1.5)
    bare = dataclasses.replace(s, pp_atom=None, pp_l=None, pp_n=None, pp_beta=None,
                               pp_alpha=None, pp_rcut=None)
    r = np.array([[0.4, -0.7, 0.2]])
    rr = np.linalg.norm(r)
    assert abs(oracle.potential(bare, r) + 1.5 / rr) < 1e-15
    assert abs(oracle.potential(s, r) - (-1.5 / rr + _v(TERMS, -1, rr))) < 1e-14


def _ico():
    v = []
    for q in range(12):
        a = -PHI if q & 1 else PHI
        b = -1.0 if q & 2 else 1.0
        v.append([(0.0, b, a), (b, a, 0.0), (a, 0.0, b)][q >> 2])
    return np.array(v) / math.sqrt(1 + PHI * PHI)


def _legendre(l, x):
    return [1.0, x, 0.5 * (3 * x * x - 1), 0.5 * (5 * x ** 3 - 3 * x)][l]


def test_many_electrons_against_point_by_point_definition():
    s = synth.small_molecule_pp()
    R = synth.make_walkers(s, 2, 44)
    seed, step = 5, 3
    ico = _ico()
    # the icosahedron: 12 unit vectors, each with 5 nearest neighbours at one angle
    dots = ico @ ico.T
    assert np.allclose(np.sort(dots, axis=1)[:, -2], 1 / math.sqrt(5))
    for w in range(2):
        lp0, sg0, _, _, _ = oracle.evaluate(s, R[w])
        ref = 0.0
        for i in range(s.n_elec):
            rot = oracle.nlpp_rotation(seed, step, w, i)
            for A in range(s.n_atom):
                d = R[w, i] - s.ion_xyz[A]
                r = np.linalg.norm(d)
                if not r < s.pp_rcut[A]:
                    continue
                terms = [(l, n, b, a) for (at, l, n, b, a) in zip(s.pp_atom, s.pp_l, s.pp_n,
                                                                  s.pp_beta, s.pp_alpha) if at == A]
                for q in range(12):
                    od = rot @ ico[q]
                    Rq = R[w].copy()
                    Rq[i] = s.ion_xyz[A] + r * od
                    lp, sg, _, _, _ = oracle.evaluate(s, Rq)
                    ratio = sg * sg0 * math.exp(lp - lp0)
                    cth = od @ d / r
                    f = sum(_v(terms, l, r) * (2 * l + 1) * _legendre(l, cth) for l in range(3))
                    ref += f * ratio / 12
        v, rc = oracle.nlpp(s, R[w], seed, step, w)
        assert rc == 0
        print(f"[nlpp] walker {w}: {v:.12f} point by point {ref:.12f}")
        assert abs(v - ref) < 1e-11 * max(1.0, abs(ref))


def test_cutoff_excludes_far_electrons():
    s = synth.small_molecule_pp()
    R = synth.make_walkers(s, 1, 45)[0]
    tiny = dataclasses.replace(s, pp_rcut=np.full(s.n_atom, 1e-3))
    assert oracle.nlpp(tiny, R, 1, 0, 0)[0] == 0.0
    assert oracle.nlpp(s, R, 1, 0, 0)[0] != 0.0


def test_dmc_weights_rebuilt_with_nonlocal_energies():
    """log w after DMC steps rebuilt from step-end energies evaluated apart
    (E_L of the configuration + the non-local energy with that step's
    rotations; before step 0 the step-0 rotations)."""
    s = synth.small_molecule_pp()
    W, tau, seed, et = 3, 0.02, 9, -6.0
    R0 = synth.make_walkers(s, W, 46)
    Rs = [R0]
    R = R0
    for st in range(3):
        out = oracle.run(s, R, step0=st, n_steps=1, mode=1, tau=tau, seed=seed, e_trial=et)
        assert out["rc"] == 0
        R = out["R"]
        Rs.append(R)
    full = oracle.run(s, R0, step0=0, n_steps=3, mode=1, tau=tau, seed=seed, e_trial=et)
    np.testing.assert_array_equal(full["R"], Rs[-1])

    def energy(Rc, st):
        e = np.array([oracle.evaluate(s, Rc[w])[2] for w in range(W)])
        v = np.array([oracle.nlpp(s, Rc[w], seed, st, w)[0] for w in range(W)])
        return e + v

    es = [energy(Rs[0], 0)] + [energy(Rs[k + 1], k) for k in range(3)]
    lw = np.zeros(W)
    for k in range(3):
        lw += -tau * (0.5 * (es[k] + es[k + 1]) - et)
    np.testing.assert_allclose(full["e_log"][-1], es[-1], rtol=1e-13)
    np.testing.assert_allclose(full["log_w"], lw, rtol=1e-12, atol=1e-13)


def _ghost_pp_system(pos):
    """The small molecule with a pseudopotential on a ghost centre (no
    charge, no basis functions, no Jastrow term): moving the ghost moves the
    pseudopotential operator alone, Psi stays fixed."""
    s = synth.small_molecule()
    ion = np.vstack([s.ion_xyz, np.asarray(pos, dtype=np.float64)[None, :]])
    g = dataclasses.replace(s, ion_xyz=ion, ion_charge=np.append(s.ion_charge, 0.0),
                            jen_a=np.append(s.jen_a, 0.0))
    return synth.with_pseudopotential(g, [[]] * s.n_atom + [PP_GHOST])


PP_GHOST = [(-1, 2, -1.2, 0.9), (-1, 3, 0.6, 1.3), (0, 2, 2.5, 0.8), (1, 2, -1.1, 0.7),
            (2, 3, 0.9, 1.2)]


def test_pp_ion_grads_against_ghost_centre_differences():
    """d(V_loc + V_NL)/dR_A with Psi fixed: Richardson differences of the
    local potential plus the non-local energy (same rotations) in the
    position of a ghost centre that carries only the pseudopotential."""
    pos0 = np.array([0.9, 1.7, 2.2])
    s = _ghost_pp_system(pos0)
    R = synth.make_walkers(synth.small_molecule(), 2, 47)
    seed, step = 13, 2
    for w in range(2):
        g, rc = oracle.pp_ion_grads(s, R[w], seed, step, w)
        assert rc == 0
        assert np.all(g[:-1] == 0.0)
        for x in range(3):
            def energy(t):
                p = pos0.copy()
                p[x] += t
                sg = _ghost_pp_system(p)
                return oracle.potential(sg, R[w]) + oracle.nlpp(sg, R[w], seed, step, w)[0]
            h = 1e-3
            d1 = (energy(h) - energy(-h)) / (2 * h)
            d2 = (energy(2 * h) - energy(-2 * h)) / (4 * h)
            fd = (4 * d1 - d2) / 3
            print(f"[nlpp] walker {w} x{x}: analytic {g[-1, x]:.10f} fd {fd:.10f}")
            assert abs(g[-1, x] - fd) < 1e-7 * max(1.0, abs(fd))


def test_nlpp_param_grads_pade_against_differences():
    """d V_NL / d b for the two Pade b (rotations fixed): Richardson
    differences of the oracle's non-local energy in jee_b and jen_b."""
    s = synth.small_molecule_pp()
    R = synth.make_walkers(s, 2, 51)
    for w in range(2):
        dv, rc = oracle.nlpp_param_grads(s, R[w], 3, 1, w)
        assert rc == 0
        for name, p in (("jee_b", 0), ("jen_b", 1)):
            b0 = getattr(s, name)

            def V(t):
                return oracle.nlpp(dataclasses.replace(s, **{name: b0 + t}), R[w], 3, 1, w)[0]
            h = 1e-4
            d1 = (V(h) - V(-h)) / (2 * h)
            d2 = (V(2 * h) - V(-2 * h)) / (4 * h)
            fd = (4 * d1 - d2) / 3
            print(f"[nlpp] walker {w} {name}: {dv[p]:.12f} fd {fd:.12f}")
            assert abs(dv[p] - fd) < 1e-8 * max(1.0, abs(fd))


def test_nlpp_param_grads_three_body_point_by_point():
    """The three-body directions: sum over the quadrature points, rebuilt
    here from the icosahedron, the Legendre polynomials, ratios from full
    evaluations of ln|Psi| and the three-body sums F_k of each moved
    configuration (the exponent of a trial function J + c F_k moves each
    ratio by c (F_k(R_q) - F_k(R)))."""
    s = synth.small_molecule_pp()
    R = synth.make_walkers(s, 1, 52)[0]
    seed, step, w = 7, 2, 0
    ico = _ico()
    lp0, sg0, _, _, _ = oracle.evaluate(s, R)
    F0 = oracle.j3_values(s, R)
    ref = np.zeros(6)
    for i in range(s.n_elec):
        rot = oracle.nlpp_rotation(seed, step, w, i)
        for A in range(s.n_atom):
            d = R[i] - s.ion_xyz[A]
            r = np.linalg.norm(d)
            if not r < s.pp_rcut[A]:
                continue
            terms = [(l, n, b, a) for (at, l, n, b, a) in zip(s.pp_atom, s.pp_l, s.pp_n,
                                                              s.pp_beta, s.pp_alpha) if at == A]
            for q in range(12):
                od = rot @ ico[q]
                Rq = R.copy()
                Rq[i] = s.ion_xyz[A] + r * od
                lp, sg, _, _, _ = oracle.evaluate(s, Rq)
                ratio = sg * sg0 * math.exp(lp - lp0)
                f = sum(_v(terms, l, r) * (2 * l + 1) * _legendre(l, od @ d / r) for l in range(3))
                ref += f * ratio * (oracle.j3_values(s, Rq) - F0) / 12
    dv, rc = oracle.nlpp_param_grads(s, R, seed, step, w)
    assert rc == 0
    print(f"[nlpp] three-body directions {dv[2:]} point by point {ref}")
    np.testing.assert_allclose(dv[2:], ref, rtol=1e-11, atol=1e-13)
