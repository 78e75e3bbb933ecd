"""E_T feedback on the GPU (QMC section, Eq. 1: the trial energy of the
projection, fed back from the population after every DMC step) against the
oracle's step-by-step run with the same rule: accept sequences bit-exact,
E_L, positions and log-weights within 1e-10, and the E_T of the next step
within 1e-10 (relative, floor 1 Ha)."""
import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import dmcx, synth

pytestmark = pytest.mark.gpu


def _close(a, b, rel=1e-10, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = rel * np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)
    assert np.all(np.abs(a - b) <= tol), f"max diff {np.abs(a - b).max():.3e}"


@pytest.mark.parametrize("graph", [False, True])
def test_feedback_run_matches_oracle(graph):
    s = synth.small_molecule()
    W, n, gain, tau = 40, 6, 0.5, 0.01
    R = synth.make_walkers(s, W, 701)
    _, _, e0, _ = oracle.evaluate_batch(s, R)
    e_t = float(np.mean(e0)) + 0.3
    ctx = dmcx.Context(s, W, delay_rank=1, recompute_period=4, tau=tau, seed=31, graph=graph)
    ctx.set_walkers(R)
    ctx.set_et_feedback(gain)
    acc, el = ctx.run(n, mode=dmcx.DMCX_DMC, e_trial=e_t, logs=True)
    Rg, lw = ctx.get_walkers()
    et_next = ctx.trial_energy()[0]
    ref = oracle.run_feedback(s, R, n_steps=n, tau=tau, seed=31, e_trial=e_t, gain=gain)
    np.testing.assert_array_equal(acc, ref["accept_log"])
    _close(el, ref["e_log"])
    _close(Rg, ref["R"])
    _close(lw, ref["log_w"])
    _close(et_next, ref["e_trial"])
    print(f"[feedback] E_T per step {np.round(ref['et_log'], 4)} next {et_next:.6f}", flush=True)
    # switched off: E_T stays at the value a run starts with
    ctx.set_et_feedback(-1.0)
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-9.0)
    assert ctx.trial_energy()[0] == -9.0


def test_feedback_group_one_e_trial_per_system():
    a = synth.small_molecule()
    b = synth.small_random_system(91, n_atom=2, n_up=2, n_dn=1, shells=(0, 1), nprim=1,
                                  charge=1.5)
    Ws = [24, 17]
    ne = max(a.n_elec, b.n_elec)
    Ra = synth.make_walkers(a, Ws[0], 702)
    Rb = synth.make_walkers(b, Ws[1], 703)
    R = np.zeros((sum(Ws), ne, 3))
    R[:Ws[0], :a.n_elec] = Ra
    R[Ws[0]:, :b.n_elec] = Rb
    g = dmcx.Context([a, b], Ws, delay_rank=1, seed=32)
    g.set_walkers(R)
    g.set_et_feedback(0.8)
    g.run(4, mode=dmcx.DMCX_DMC, e_trial=-5.0)
    et = g.trial_energy()
    for i, (x, Rx) in enumerate(((a, Ra), (b, Rb))):
        ref = oracle.run_feedback(x, Rx, n_steps=4, tau=0.01, seed=32, e_trial=-5.0, gain=0.8)
        _close(et[i], ref["e_trial"])
