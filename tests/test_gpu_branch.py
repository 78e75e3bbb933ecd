"""Birth/death branching on the GPU (the DMC weights of Eq. 1 as walker
counts; the population size varies within the context's capacity) against
the oracle.

* Selection: the copies of every walker and the new count W' are bit-exact
  against the oracle's on the same log-weights, seed and step (integer work
  decided in FP64 on both sides).
* Layout: the new positions equal the oracle's slot rule applied to the old
  ones, log w is 0, and every copy's E_L, log|Psi| and sign equal its
  source's bit for bit (the state moved with it).
* Continuation: DMC steps from the new population agree with the oracle run
  from the laid-out positions (accept sequences bit-exact, E_L, positions
  and log w to the FP64 bar): a wrong copied inverse, orbital row or padding
  slot would show there.  Growing and shrinking populations, across tile
  boundaries; mixed and multideterminant forms; the E_T feedback's target
  population after a branch; the refusal cases (nothing survives, over the
  capacity) leave the population unchanged.
"""
import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import dmcx, synth

pytestmark = pytest.mark.gpu


def _close(a, b, rel=1e-10, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)
    print(f"[branch] max rel err {err.max():.2e}", flush=True)
    assert np.all(err <= rel)


def _layout(W, copies, pairs, wn, X):
    """The oracle's new population of X (per-walker rows) from its pairs."""
    Y = np.zeros((max(W, wn),) + X.shape[1:], dtype=X.dtype)
    Y[:W] = X
    src = np.arange(max(W, wn))
    for d, s in pairs:
        Y[d] = X[s]
        src[d] = s
    return Y[:wn], src[:wn]


def _branch_and_check(ctx, s, R1, lw1, step, seed, cap):
    W = R1.shape[0]
    ctx.set_walkers(R1, lw1)
    ctx.set_step(step)
    e_b, lp_b, sg_b = ctx.measure()
    ref_c, ref_p, ref_w, rc = oracle.branch(lw1, seed, step, cap)
    assert rc == 0
    copies, wn = ctx.branch(step)
    print(f"[branch] W {W} -> {wn} (oracle {ref_w}), {ref_p.shape[0]} pairs", flush=True)
    np.testing.assert_array_equal(copies, ref_c)
    assert wn == ref_w == ctx.walker_count()[0]
    R2, lw2 = ctx.get_walkers()
    Rx, src = _layout(W, ref_c, ref_p, wn, R1)
    np.testing.assert_array_equal(R2, Rx)
    np.testing.assert_array_equal(lw2, np.zeros(wn))
    e_a, lp_a, sg_a = ctx.measure()
    np.testing.assert_array_equal(e_a, e_b[src])
    np.testing.assert_array_equal(lp_a, lp_b[src])
    np.testing.assert_array_equal(sg_a, sg_b[src])
    return R2


@pytest.mark.parametrize("shift,k,graph", [(0.45, 1, False), (-0.5, 4, False), (0.0, 2, False),
                                           (0.45, 2, True)])
def test_branch_then_run_matches_oracle(shift, k, graph):
    s = synth.small_molecule()
    cap, W0, tau, seed, et = 96, 37, 0.02, 43, -8.0
    ctx = dmcx.Context(s, cap, delay_rank=k, recompute_period=3, tau=tau, seed=seed, graph=graph)
    assert ctx.walker_count() == (cap, cap)
    ctx.set_walker_count(W0)
    assert ctx.walker_count() == (W0, cap)
    ctx.set_walkers(synth.make_walkers(s, W0, 511))
    ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=et)
    R1, lw1 = ctx.get_walkers()
    assert R1.shape[0] == W0
    step = ctx.get_step()
    # log-weights of a chosen spread (the run's own are far wider at this E_T)
    lw1 = shift + np.random.default_rng(17).normal(0.0, 0.6, W0)
    R2 = _branch_and_check(ctx, s, R1, lw1, step, seed, cap)
    wn = R2.shape[0]
    if shift > 0:
        assert wn > W0
    elif shift < 0:
        assert wn < W0
    acc, el = ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=et, logs=True)
    ref = oracle.run(s, R2, log_w=np.zeros(wn), step0=step, n_steps=3, mode=1, tau=tau, seed=seed,
                     e_trial=et)
    np.testing.assert_array_equal(acc, ref["accept_log"])
    _close(el, ref["e_log"])
    R3, lw3 = ctx.get_walkers()
    _close(R3, ref["R"])
    _close(lw3, ref["log_w"])


@pytest.mark.parametrize("form,prec", [("mixed", dmcx.DMCX_MIXED), ("msd", dmcx.DMCX_FP64),
                                       ("msd", dmcx.DMCX_MIXED)])
def test_branch_carries_state_mixed_and_multideterminant(form, prec):
    base = synth.small_random_system(77, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2,
                                     n_mo=10)
    s = synth.make_msd(base, n_det=15, n_active=6, seed=78) if form == "msd" else base
    cap, W0, seed = 64, 29, 3
    ctx = dmcx.Context(s, cap, precision=prec, delay_rank=2, recompute_period=4, seed=seed)
    ctx.set_walker_count(W0)
    ctx.set_walkers(synth.make_walkers(s, W0, 79))
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-4.0)
    R1, lw1 = ctx.get_walkers()
    lw1 = 0.2 + np.random.default_rng(6).normal(0.0, 0.6, W0)
    _branch_and_check(ctx, s, R1, lw1, ctx.get_step(), seed, cap)
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-4.0)
    assert not ctx.walker_flags().any()


def test_feedback_target_after_branch():
    """E_T feedback keeps the population it was switched on with as its
    target: after a branch to W' walkers, the run agrees with the oracle's
    feedback run with target W."""
    s = synth.small_molecule()
    cap, W0, tau, seed, gain = 80, 40, 0.01, 31, 0.5
    ctx = dmcx.Context(s, cap, delay_rank=1, recompute_period=4, tau=tau, seed=seed)
    ctx.set_walker_count(W0)
    R = synth.make_walkers(s, W0, 701)
    ctx.set_walkers(R)
    ctx.set_et_feedback(gain)
    step = ctx.get_step()
    lw = np.random.default_rng(8).normal(0.25, 0.5, W0)
    R2 = _branch_and_check(ctx, s, R, lw, step, seed, cap)
    wn = R2.shape[0]
    assert wn != W0
    _, _, e0, _ = oracle.evaluate_batch(s, R2)
    e_t = float(np.mean(e0)) + 0.2
    acc, el = ctx.run(4, mode=dmcx.DMCX_DMC, e_trial=e_t, logs=True)
    ref = oracle.run_feedback(s, R2, n_steps=4, step0=step, tau=tau, seed=seed, e_trial=e_t,
                              gain=gain, target=W0)
    np.testing.assert_array_equal(acc, ref["accept_log"])
    _close(el, ref["e_log"])
    _close(ctx.trial_energy()[0], ref["e_trial"])


def test_refusals_leave_the_population():
    s = synth.small_molecule()
    cap, W0, seed = 24, 16, 5
    ctx = dmcx.Context(s, cap, seed=seed)
    ctx.set_walker_count(W0)
    R = synth.make_walkers(s, W0, 521)
    # every walker would get 2 copies: 32 > 24
    ctx.set_walkers(R, np.full(W0, np.log(2.0) + 1e-9))
    with pytest.raises(dmcx.DmcxError):
        ctx.branch(0)
    assert ctx.walker_count() == (W0, cap)
    R2, lw2 = ctx.get_walkers()
    np.testing.assert_array_equal(R2, R)
    # nothing survives
    ctx.set_walkers(R, np.full(W0, -np.inf))
    with pytest.raises(dmcx.DmcxError):
        ctx.branch(0)
    assert ctx.walker_count() == (W0, cap)
    np.testing.assert_array_equal(ctx.get_walkers()[0], R)
    # unit weights: everyone keeps one copy, nothing moves
    ctx.set_walkers(R, np.zeros(W0))
    copies, wn = ctx.branch(3)
    np.testing.assert_array_equal(copies, np.ones(W0))
    assert wn == W0
    np.testing.assert_array_equal(ctx.get_walkers()[0], R)
    with pytest.raises(dmcx.DmcxError):
        ctx.set_walker_count(cap + 1)
    with pytest.raises(dmcx.DmcxError):
        ctx.set_walker_count(0)


def test_group_context_refuses_branching():
    a = synth.small_molecule()
    b = synth.small_random_system(91, n_atom=2, n_up=2, n_dn=1, shells=(0, 1), nprim=1,
                                  charge=1.5)
    g = dmcx.Context([a, b], [8, 8], seed=1)
    with pytest.raises(dmcx.DmcxError):
        g.set_walker_count(4)


def test_calls_after_growth_match_a_fresh_context():
    """After a branch that grows the population, the per-walker calls whose
    buffers are sized by the capacity (estimators, ion derivatives, Jastrow
    parameter derivatives, linear-method matrices) agree with a context made
    for the new count on the same positions."""
    s = synth.small_molecule()
    cap, W0, seed = 64, 20, 9
    ctx = dmcx.Context(s, cap, delay_rank=2, seed=seed)
    ctx.set_walker_count(W0)
    R = synth.make_walkers(s, W0, 531)
    ctx.set_walkers(R, 0.5 + np.random.default_rng(10).normal(0.0, 0.4, W0))
    _, wn = ctx.branch(0)
    assert wn > W0
    Rb, lw = ctx.get_walkers()
    fresh = dmcx.Context(s, wn, delay_rank=2, seed=seed)
    fresh.set_walkers(Rb, lw)
    est, est_f = ctx.estimators(), fresh.estimators()
    assert est[0][0] == wn
    np.testing.assert_allclose(est[0][:9], est_f[0][:9], rtol=1e-13, atol=0)
    dl, dv = ctx.ion_grads()
    dl_f, dv_f = fresh.ion_grads()
    _close(dl, dl_f, rel=1e-12)
    _close(dv, dv_f, rel=1e-12)
    O, D = ctx.jastrow_param_grads()
    O_f, D_f = fresh.jastrow_param_grads()
    _close(O, O_f, rel=1e-12)
    _close(D, D_f, rel=1e-12)
    S, H = ctx.linear_method()
    S_f, H_f = fresh.linear_method()
    _close(S, S_f, rel=1e-11)
    _close(H, H_f, rel=1e-11)


@pytest.mark.parametrize("case", ["one", "full"])
def test_branch_to_one_walker_and_to_capacity(case):
    """The extremes: one walker left (every other weight zero), and the
    population filling the capacity exactly (every walker doubled, W' a
    multiple of the 8-walker tile so no padding copy runs); the next DMC step
    against the oracle run from the laid-out positions."""
    s = synth.small_molecule()
    cap, W0, tau, seed, et = 24, 12, 0.02, 17, -8.0
    ctx = dmcx.Context(s, cap, delay_rank=2, recompute_period=4, tau=tau, seed=seed)
    ctx.set_walker_count(W0)
    R = synth.make_walkers(s, W0, 541)
    if case == "one":
        lw = np.full(W0, -np.inf)
        lw[7] = 0.0
    else:
        lw = np.full(W0, np.log(2.0))
    R2 = _branch_and_check(ctx, s, R, lw, 5, seed, cap)
    assert R2.shape[0] == (1 if case == "one" else cap)
    acc, el = ctx.run(1, mode=dmcx.DMCX_DMC, e_trial=et, logs=True)
    ref = oracle.run(s, R2, log_w=np.zeros(R2.shape[0]), step0=5, n_steps=1, mode=1, tau=tau,
                     seed=seed, e_trial=et)
    np.testing.assert_array_equal(acc, ref["accept_log"])
    _close(el, ref["e_log"])
