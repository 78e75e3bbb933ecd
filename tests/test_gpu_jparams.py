"""Jastrow parameter derivatives and linear-method matrices on the GPU
against the oracle (the optimisation of the Jastrow factor of Eq. 2).

Bars: FP64 contexts give O_p = d ln Psi/dp and dE_L/dp per walker within
1e-10 x max(|x|, 1) of the oracle at the same configurations (FP64 sums in a
different order; the three-body sums of the 112-electron molecule hold some
10^5 terms per walker, so that case is held to 1e-9).  The mixed form takes
grad ln|Psi| from FP32 inverse and orbital rows: O_p (positions only) stays
at the FP64 bar, dE_L/dp is held to 1e-4 x max(|x|, 1).  The linear-method
matrices are compared with the oracle's matrices built from the oracle's own
per-walker values, E_L and the test's log-weights, within 1e-9 x max(|x|, 1).
Electron counts 1, 2, odd and even cover the pair enumeration; groups,
moved walkers, excluded walkers and the unsupported multideterminant form
are covered too.
"""
import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import dmcx, synth

pytestmark = pytest.mark.gpu


def _close(a, b, rel=1e-10, floor=1.0, label=""):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)
    print(f"[jparams] {label}: max rel err {err.max():.2e}", flush=True)
    assert np.all(err <= rel), f"{(err > rel).sum()} of {err.size} outside"


def _systems():
    return {
        "small": synth.small_molecule(),
        "odd": synth.small_random_system(81, n_atom=3, n_up=4, n_dn=3, shells=(0, 0, 1, 2),
                                         nprim=2),
        "two": synth.small_random_system(82, n_atom=2, n_up=1, n_dn=1, shells=(0, 1), nprim=1),
        "one": synth.small_random_system(83, n_atom=2, n_up=1, n_dn=0, shells=(0, 1), nprim=1,
                                         charge=1.0),
    }


@pytest.mark.parametrize("name", ["small", "odd", "two", "one"])
def test_param_grads_match_oracle(name):
    s = _systems()[name]
    W = 37
    R = synth.make_walkers(s, W, 9100)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    O, D = ctx.jastrow_param_grads()
    Oo, Do, rc = oracle.jastrow_param_grads_batch(s, R)
    assert rc == 0
    _close(O, Oo, label=f"{name} O")
    _close(D, Do, label=f"{name} dE_L")


def test_after_moves_and_linear_method():
    """After VMC steps with delayed updates the derivatives follow the moved
    walkers; the linear-method matrices match the oracle's."""
    s = _systems()["odd"]
    W = 300
    ctx = dmcx.Context(s, W, delay_rank=3, recompute_period=5, seed=17)
    ctx.set_walkers(synth.make_walkers(s, W, 9101))
    ctx.run(4, mode=dmcx.DMCX_VMC)
    R, _ = ctx.get_walkers()
    lw = np.random.default_rng(3).normal(0.0, 0.7, W)
    lw[5] = -np.inf
    ctx.set_walkers(R, lw)
    O, D = ctx.jastrow_param_grads()
    Oo, Do, rc = oracle.jastrow_param_grads_batch(s, R)
    assert rc == 0
    _close(O, Oo, label="moved O")
    _close(D, Do, label="moved dE_L")
    S, H = ctx.linear_method()
    _, _, Eo, _ = oracle.evaluate_batch(s, R)
    So, Ho = oracle.linear_method(lw, Eo, Oo, Do)
    _close(S[0], So, rel=1e-9, label="S")
    _close(H[0], Ho, rel=1e-9, label="H")


def test_mixed_precision():
    s = _systems()["odd"]
    W = 64
    R = synth.make_walkers(s, W, 9102)
    ctx = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED)
    ctx.set_walkers(R)
    O, D = ctx.jastrow_param_grads()
    Oo, Do, _ = oracle.jastrow_param_grads_batch(s, R)
    _close(O, Oo, label="mixed O")
    _close(D, Do, rel=1e-4, label="mixed dE_L")


def test_group_of_systems():
    a = _systems()["small"]
    b = _systems()["odd"]
    Ws = [20, 13]
    ctx = dmcx.Context([a, b], Ws, seed=4)
    Ra = synth.make_walkers(a, Ws[0], 9103)
    Rb = synth.make_walkers(b, Ws[1], 9104)
    ne = max(a.n_elec, b.n_elec)
    R = np.zeros((sum(Ws), ne, 3))
    R[: Ws[0], : a.n_elec] = Ra
    R[Ws[0]:, : b.n_elec] = Rb
    lw = np.random.default_rng(8).normal(0.0, 0.5, sum(Ws))
    ctx.set_walkers(R, lw)
    O, D = ctx.jastrow_param_grads()
    S, H = ctx.linear_method()
    for i, (sysi, Ri, sl) in enumerate(((a, Ra, slice(0, Ws[0])), (b, Rb, slice(Ws[0], None)))):
        Oo, Do, _ = oracle.jastrow_param_grads_batch(sysi, Ri)
        _close(O[sl], Oo, label=f"group {i} O")
        _close(D[sl], Do, label=f"group {i} dE_L")
        _, _, Eo, _ = oracle.evaluate_batch(sysi, Ri)
        So, Ho = oracle.linear_method(lw[sl], Eo, Oo, Do)
        _close(S[i], So, rel=1e-9, label=f"group {i} S")
        _close(H[i], Ho, rel=1e-9, label=f"group {i} H")


def test_large_molecule_sampled():
    """The 112-electron, 64-ion molecule at 2048 walkers (the launch the
    benchmark times): every walker's O and dE_L finite, sampled walkers
    against the oracle."""
    s = synth.large_molecule()
    W = 2048
    R = synth.make_walkers(s, W, 9105)
    ctx = dmcx.Context(s, W, delay_rank=32, recompute_period=64)
    ctx.set_walkers(R)
    O, D = ctx.jastrow_param_grads()
    assert np.all(np.isfinite(O)) and np.all(np.isfinite(D))
    idx = np.array([0, 1, 777, 1500, W - 1])
    Oo, Do, rc = oracle.jastrow_param_grads_batch(s, R[idx])
    assert rc == 0
    _close(O[idx], Oo, rel=1e-9, label="large O")
    _close(D[idx], Do, rel=1e-9, label="large dE_L")


def test_multideterminant_unsupported():
    base = synth.small_random_system(77, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2,
                                     n_mo=10)
    s = synth.make_msd(base, n_det=5, n_active=6, seed=78)
    ctx = dmcx.Context(s, 8)
    ctx.set_walkers(synth.make_walkers(s, 8, 1))
    with pytest.raises(dmcx.DmcxError):
        ctx.jastrow_param_grads()
    with pytest.raises(dmcx.DmcxError):
        ctx.linear_method()


def test_optimisation_on_the_gpu_reaches_the_exact_jastrow():
    """The linear method end to end on the GPU path: VMC runs, the
    walkers' derivatives and the matrices S, H from the library, the step
    from optimize.linear_method_update; the hydrogen-like 1s with the Pade
    e-n term goes from b = 0.4 to the exact b = 0 (E_L = -Z^2/2)."""
    from paper_2504_07948_amd import optimize
    b, W = 0.4, 512
    R = np.random.default_rng(5).normal(0.0, 1.0, (W, 1, 3))
    for it in range(6):
        s = synth.System("h1s", np.zeros((1, 3)), np.array([1.0]), [0], [0], [1], [0.0], [1.0],
                         np.ones((1, 1)), 1, 0, jen_a=np.array([-1.0]), jen_b=b)
        ctx = dmcx.Context(s, W, tau=0.1, seed=11 + it, delay_rank=1)
        ctx.set_walkers(R)
        ctx.run(30, mode=dmcx.DMCX_VMC)
        R, _ = ctx.get_walkers()
        S, H = ctx.linear_method()
        dp, _ = optimize.linear_method_update(S[0], H[0], params=[1], shift=1e-4)
        print(f"[jparams] optimisation step {it}: b {b:.5f} -> {b + dp[0]:.5f}, "
              f"<E> {H[0][0, 0]:.6f}", flush=True)
        b += dp[0]
    assert abs(b) < 0.02
