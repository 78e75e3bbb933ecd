"""Multideterminant trial function (Eq. 2 with M > 1) by the table method on
the GPU, against the oracle's one-LU-per-determinant evaluation.

Bars (FP64): signs and accept sequences exact; positions within 1e-10;
log|Psi| and E_L within 1e-10 x max(|x|, 1) x max(1, cond(A_0) kappa_S / 100)
per walker, where cond(A_0) is the reference determinant's condition number
and kappa_S = sum_d |c_d R_d| / |S| the cancellation in the determinant sum
(the table method expresses every ratio relative to the reference, so its
rounding grows with both; the synthetic expansions give every determinant a
coefficient of order one, which makes weak references common).  Graph
replays are bit-identical to eager runs.  The mixed form is compared with
the FP64 path at identical configurations.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import dmcx, synth

pytestmark = pytest.mark.gpu


def _close(a, b, rel=1e-10, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = rel * np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)
    bad = np.abs(a - b) > tol
    if bad.any():
        i = np.argmax(np.abs(a - b) / tol)
        raise AssertionError(f"{bad.sum()} of {bad.size} outside; worst {a.ravel()[i]!r} vs "
                             f"{b.ravel()[i]!r}")


def _conditioning(s, Rw):
    """cond(A_0) of the worse spin and the cancellation kappa_S =
    sum_d |c_d R_d| / |S| at one configuration, from plain numpy
    determinants of the oracle's orbital values.  The table method writes
    every ratio relative to the reference determinant, so its rounding
    grows with both."""
    nmo = s.mo_coef.shape[1]
    orb = np.array([oracle.orbitals_vgl(s, r, nmo)[0] for r in Rw])
    blocks = ((0, s.n_up), (s.n_up, s.n_dn))
    terms = []
    for d in range(s.n_det):
        e, t = s.det_exc[d], s.ci_coef[d]
        for sp, (lo, n) in enumerate(blocks):
            cols = list(range(n))
            h, p = (e[2:4], e[4:6]) if sp == 0 else (e[6:8], e[8:10])
            for k in range(e[sp]):
                cols[h[k]] = p[k]
            t *= np.linalg.det(orb[lo:lo + n][:, cols]) / np.linalg.det(orb[lo:lo + n, :n])
        terms.append(t)
    terms = np.array(terms)
    cond = max(np.linalg.cond(orb[lo:lo + n, :n]) for lo, n in blocks)
    return cond, np.abs(terms).sum() / abs(terms.sum())


def _close_conditioned(a, b, s, R, label, rel=1e-10):
    """|a - b| <= rel * max(|b|, 1) * max(1, cond(A_0) kappa_S / 100) per walker."""
    amp = np.array([max(1.0, np.prod(_conditioning(s, Rw)) / 100.0) for Rw in R])
    err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    w = int(np.argmax(err / amp))
    print(f"[msd] {label}: max rel err {err.max():.2e}; worst vs bar: walker {w} err {err[w]:.2e} "
          f"amplification {amp[w]:.3g}", flush=True)
    assert np.all(err <= rel * amp)


def _msd_small(n_det=30, n_active=12):
    return synth.make_msd(synth.small_molecule(), n_det, n_active, 901)


def _msd_large(n_det=120, n_active=40):
    return synth.make_msd(synth.large_molecule(), n_det, n_active, 902)


@pytest.mark.parametrize("which,W", [("small", 13), ("large", 5)])
def test_msd_measure_matches_oracle(which, W):
    s = _msd_small() if which == "small" else _msd_large()
    R = synth.make_walkers(s, W, 910)
    print(f"[msd] measure {which}: {s.n_elec} e, {s.n_det} dets, W={W}", flush=True)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    e, lp, sg = ctx.measure()
    lp_o, sg_o, e_o, rc = oracle.evaluate_batch(s, R)
    assert rc == 0
    np.testing.assert_array_equal(sg, sg_o)
    _close_conditioned(lp, lp_o, s, R, f"{which} log|Psi|")
    _close_conditioned(e, e_o, s, R, f"{which} E_L")


@pytest.mark.parametrize("mode,k,P", [(dmcx.DMCX_DMC, 2, 2), (dmcx.DMCX_VMC, 4, 64),
                                      (dmcx.DMCX_DMC, 1, 1)])
def test_msd_run_small_matches_oracle(mode, k, P):
    """Three steps, compared step by step (the E_L bar of each walker is
    scaled by the conditioning at that step's configuration)."""
    s = _msd_small()
    W = 16
    R = synth.make_walkers(s, W, 911)
    e_t = -8.0
    ctx = dmcx.Context(s, W, delay_rank=k, recompute_period=P, seed=21)
    ctx.set_walkers(R)
    Ro, lwo = R, np.zeros(W)
    for step in range(3):
        acc, el = ctx.run(1, mode=mode, e_trial=e_t, logs=True)
        ref = oracle.run(s, Ro, log_w=lwo, step0=step, n_steps=1, mode=mode, tau=0.01, seed=21,
                         e_trial=e_t)
        Ro, lwo = ref["R"], ref["log_w"]
        np.testing.assert_array_equal(acc, ref["accept_log"])
        _close_conditioned(el[0], ref["e_log"][0], s, Ro, f"step {step} E_L")
        Rg, lw = ctx.get_walkers()
        _close(Rg, Ro)
    e, lp, sg = ctx.measure()
    lp_o, sg_o, e_o, _ = oracle.evaluate_batch(s, Ro)
    _close_conditioned(lp, lp_o, s, Ro, "log|Psi|")
    np.testing.assert_array_equal(sg, sg_o)


def test_msd_run_large_matches_oracle():
    """112 electrons, 120 determinants over 40 active orbitals, 8 walkers,
    one DMC step with delayed rank-16 updates."""
    s = _msd_large()
    W = 8
    R = synth.make_walkers(s, W, 912)
    ctx = dmcx.Context(s, W, delay_rank=16, recompute_period=64, seed=22)
    ctx.set_walkers(R)
    print(f"[msd] large run: {s.n_det} dets", flush=True)
    acc, el = ctx.run(1, mode=dmcx.DMCX_DMC, e_trial=-100.0, logs=True)
    Rg, _ = ctx.get_walkers()
    ref = oracle.run(s, R, n_steps=1, mode=dmcx.DMCX_DMC, tau=0.01, seed=22, e_trial=-100.0)
    np.testing.assert_array_equal(acc, ref["accept_log"])
    _close_conditioned(el[0], ref["e_log"][0], s, ref["R"], "large step E_L")
    _close(Rg, ref["R"])


def test_msd_equals_single_determinant_with_mixed_column():
    """D + c D_{h->p} per spin is one determinant with column h = phi_h + c phi_p
    (multilinearity): the table path and the plain single-determinant path
    agree on whole runs."""
    base = synth.small_molecule()
    s0 = synth.make_msd(base, 2, 12, 913)  # extends the MO set
    h, p, c = 2, 6, 0.31
    single = lambda sp: ([1, 0, h, -1, p, -1, -1, -1, -1, -1] if sp == 0 else
                         [0, 1, -1, -1, -1, -1, h, -1, p, -1])
    exc = np.array([[0, 0] + [-1] * 8, single(0), single(1),
                    [1, 1, h, -1, p, -1, h, -1, p, -1]], dtype=np.int32)
    m = dataclasses.replace(s0, n_det=4, det_exc=exc, ci_coef=np.array([1.0, c, c, c * c]))
    mo = s0.mo_coef.copy()
    mo[:, h] += c * mo[:, p]
    eq = dataclasses.replace(s0, mo_coef=mo, n_det=0, det_exc=None, ci_coef=None)
    W = 16
    R = synth.make_walkers(base, W, 914)
    out = []
    for sys_ in (m, eq):
        ctx = dmcx.Context(sys_, W, delay_rank=3, recompute_period=2, seed=23)
        ctx.set_walkers(R)
        out.append(ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=-8.0, logs=True) + (ctx.measure(),))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    _close(out[0][1], out[1][1])
    _close(out[0][2][1], out[1][2][1])


def test_msd_graph_matches_eager():
    s = _msd_small()
    W = 16
    R = synth.make_walkers(s, W, 915)
    res = []
    for graph in (False, True):
        ctx = dmcx.Context(s, W, delay_rank=4, recompute_period=2, seed=24, graph=graph)
        ctx.set_walkers(R)
        a, e = ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=-8.0, logs=True)
        res.append((a, e, ctx.get_walkers()[0]))
    for x, y in zip(res[0], res[1]):
        np.testing.assert_array_equal(x, y)


def test_msd_group_of_alkanes_matches_individual_and_oracle():
    """Two alkane stand-ins (20 and 44 electrons) with 200-determinant
    expansions in one group, graph-captured."""
    systems = [synth.make_msd(synth.alkane(n, 77 + n), 200, 40, 78 + n) for n in (3, 7)]
    walkers = [9, 8]
    ne_max = max(s.n_elec for s in systems)
    Rs = [synth.make_walkers(s, w, 916 + i) for i, (s, w) in enumerate(zip(systems, walkers))]
    pad = lambda R: np.concatenate([R, np.zeros((R.shape[0], ne_max - R.shape[1], 3))], axis=1)
    grp = dmcx.Context(systems, walkers, delay_rank=8, recompute_period=2, seed=25, graph=True)
    grp.set_walkers(np.concatenate([pad(R) for R in Rs]))
    acc, el = grp.run(2, mode=dmcx.DMCX_DMC, e_trial=-30.0, logs=True)
    for i, (s, w, R) in enumerate(zip(systems, walkers, Rs)):
        sl = slice(grp.offsets[i], grp.offsets[i] + w)
        one = dmcx.Context(s, w, delay_rank=8, recompute_period=2, seed=25)
        one.set_walkers(R)
        a1, e1 = one.run(2, mode=dmcx.DMCX_DMC, e_trial=-30.0, logs=True)
        np.testing.assert_array_equal(acc[:, sl, :s.n_elec], a1)
        np.testing.assert_array_equal(el[:, sl], e1)
        if i == 0:
            ref = oracle.run(s, R, n_steps=2, mode=dmcx.DMCX_DMC, tau=0.01, seed=25, e_trial=-30.0)
            np.testing.assert_array_equal(a1, ref["accept_log"])
            _close_conditioned(e1[-1], ref["e_log"][-1], s, ref["R"], "alkane E_L")


def test_msd_mixed_precision_error():
    s = _msd_large()
    W = 16
    R = synth.make_walkers(s, W, 917)
    mx = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED)
    mx.set_walkers(R)
    e_m, lp_m, sg_m = mx.measure()
    f64 = dmcx.Context(s, W)
    f64.set_walkers(R)
    e_f, lp_f, sg_f = f64.measure()
    de = (e_m - e_f) / s.n_elec
    print(f"[msd] mixed vs FP64: median |dE_L|/N_e {np.median(np.abs(de)):.3e}, "
          f"max {np.abs(de).max():.3e}; max |dlog Psi| {np.abs(lp_m - lp_f).max():.3e}")
    np.testing.assert_array_equal(sg_m, sg_f)
    assert np.median(np.abs(de)) <= 1e-4
    assert np.abs(lp_m - lp_f).max() <= 1e-2


@pytest.mark.parametrize("which,W", [("small", 8), ("large", 3)])
def test_msd_ion_grads_match_oracle(which, W):
    """Reverse mode through the table (adjoint weights X, Y of the minors)
    against the oracle's forward mode per determinant."""
    s = _msd_small() if which == "small" else _msd_large()
    R = synth.make_walkers(s, W, 919)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    dl, dv = ctx.ion_grads()
    dl_o, dv_o, rc = oracle.ion_grads_batch(s, R)
    assert rc == 0
    _close(dv, dv_o, rel=1e-12)
    amp = np.array([max(1.0, np.prod(_conditioning(s, Rw)) / 100.0) for Rw in R])
    err = np.abs(dl - dl_o).max(axis=(1, 2)) / max(1.0, np.abs(dl_o).max())
    print(f"[msd] {which} ion grads: max rel err {err.max():.2e}", flush=True)
    assert np.all(err <= 1e-10 * amp)


def test_msd_ion_grads_after_moves_and_fd():
    s = _msd_small()
    W = 8
    R = synth.make_walkers(s, W, 920)
    ctx = dmcx.Context(s, W, delay_rank=2, recompute_period=100, seed=26)
    ctx.set_walkers(R)
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-8.0)
    Rg, _ = ctx.get_walkers()
    dl, _ = ctx.ion_grads()
    dl_o, _, _ = oracle.ion_grads_batch(s, Rg)
    amp = np.array([max(1.0, np.prod(_conditioning(s, Rw)) / 100.0) for Rw in Rg])
    err = np.abs(dl - dl_o).max(axis=(1, 2)) / max(1.0, np.abs(dl_o).max())
    assert np.all(err <= 1e-9 * amp), err
    # central differences of the library's own log|Psi| (Richardson, h = 2e-4, 1e-4)
    ctx.set_walkers(Rg)
    dl0, _ = ctx.ion_grads()
    base = s.ion_xyz.copy()
    for a, x in [(0, 0), (2, 1), (3, 2)]:
        est = {}
        for h in (2e-4, 1e-4):
            vals = []
            for sgn in (1, -1):
                xyz = base.copy()
                xyz[a, x] += sgn * h
                ctx.set_ions(xyz)
                vals.append(ctx.measure()[1])
            est[h] = (vals[0] - vals[1]) / (2 * h)
        fd = (4 * est[1e-4] - est[2e-4]) / 3
        np.testing.assert_allclose(dl0[:, a, x], fd, rtol=1e-6, atol=1e-6)
    ctx.set_ions(base)


def test_msd_forces_estimator_runs_in_a_group():
    systems = [synth.make_msd(synth.alkane(3, 80), 100, 30, 81), _msd_small()]
    walkers = [8, 8]
    ne_max = max(x.n_elec for x in systems)
    R = np.zeros((16, ne_max, 3))
    for i, x in enumerate(systems):
        R[i * 8:(i + 1) * 8, :x.n_elec] = synth.make_walkers(x, 8, 921 + i)
    grp = dmcx.Context(systems, walkers)
    grp.set_walkers(R)
    F = grp.forces()
    for i, x in enumerate(systems):
        one = dmcx.Context(x, 8)
        one.set_walkers(R[i * 8:(i + 1) * 8, :x.n_elec])
        _close(F[i, :x.n_atom], one.forces(), rel=1e-10)
