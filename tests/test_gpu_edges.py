"""Edge cases of the HIP path: the exactly solvable one-electron case, the
largest supported shapes, unequal spin counts and a spin with no electrons.

* Zero variance: Psi = exp(-Z r) (constant orbital, Pade e-n term with
  a = -Z, b = 0) gives E_L = -Z^2/2 at every configuration, so every E_L the
  GPU reports -- initial, after VMC and DMC sweeps -- equals it, and the DMC
  log-weights are exactly -tau n (E - E_T).
* Largest shapes: 128 electrons per spin (eight 16-orbital blocks) with the
  largest delay rank (64), two walker tiles with a ragged end, against the
  oracle.
* Unequal spins (3 up, 1 down) and one spin empty (2 up, 0 down) against
  the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2504_07948_amd import dmcx, synth

pytestmark = pytest.mark.gpu


def _close(a, b, rel=1e-10, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = rel * np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)
    err = np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), floor)
    print(f"[edges] max rel err {err.max():.2e}", flush=True)
    assert np.all(np.abs(a - b) <= tol)


def _hydrogenic(Z):
    mo = np.ones((1, 1))
    return synth.System("one", np.zeros((1, 3)), np.array([Z]), [0], [0], [1], [0.0], [1.0], mo, 1,
                        0, jen_a=np.array([-Z]), jen_b=0.0)


@pytest.mark.parametrize("Z", [1.0, 2.0])
def test_zero_variance_exact_on_gpu(Z):
    s = _hydrogenic(Z)
    W = 24
    R = np.random.default_rng(int(Z)).standard_normal((W, 1, 3)) * 0.8
    ctx = dmcx.Context(s, W, delay_rank=1, recompute_period=3, tau=0.01, seed=31)
    ctx.set_walkers(R)
    e, lp, sg = ctx.measure()
    np.testing.assert_allclose(e, -Z * Z / 2, rtol=0, atol=1e-12)
    np.testing.assert_allclose(lp, -Z * np.linalg.norm(R[:, 0], axis=1), rtol=0, atol=1e-12)
    assert np.all(sg == 1)
    _, el = ctx.run(3, mode=dmcx.DMCX_VMC, logs=True)
    np.testing.assert_allclose(el, -Z * Z / 2, rtol=0, atol=1e-12)
    ctx.set_walkers(R)
    e_t, n, tau = -0.3, 4, 0.01
    acc, el = ctx.run(n, mode=dmcx.DMCX_DMC, e_trial=e_t, logs=True)
    np.testing.assert_allclose(el, -Z * Z / 2, rtol=0, atol=1e-12)
    _, lw = ctx.get_walkers()
    np.testing.assert_allclose(lw, -tau * n * (-Z * Z / 2 - e_t), rtol=0, atol=1e-13)
    ref = oracle.run(s, R, n_steps=n, mode=1, tau=tau, seed=31, e_trial=e_t)
    np.testing.assert_array_equal(acc, ref["accept_log"])


def test_largest_shapes_match_oracle():
    """128 + 128 electrons, 512 basis functions, 128 orbitals per spin (NOB 8),
    delay rank 64 (two blocks per spin), 9 walkers (one full and one ragged
    tile), one DMC step."""
    s = synth.small_random_system(611, n_atom=64, n_up=128, n_dn=128, shells=(0, 0, 1, 1), nprim=2,
                                  box=14.0, alpha=(0.3, 3.0), charge=4.0)
    W = 9
    R = synth.make_walkers(s, W, 612)
    print(f"[edges] {s.n_elec} electrons, {s.n_basis} functions", flush=True)
    ctx = dmcx.Context(s, W, delay_rank=64, recompute_period=100, seed=33)
    ctx.set_walkers(R)
    e0, lp0, sg0 = ctx.measure()
    lp_o, sg_o, e_o, rc = oracle.evaluate_batch(s, R)
    np.testing.assert_array_equal(sg0, sg_o)
    _close(lp0, lp_o)
    print(f"[edges] initial E_L max rel err "
          f"{(np.abs(e0 - e_o) / np.maximum(np.abs(e_o), 1.0)).max():.2e}", flush=True)
    _close(e0, e_o)
    acc, el = ctx.run(1, mode=dmcx.DMCX_DMC, e_trial=-200.0, logs=True)
    ref = oracle.run(s, R, n_steps=1, mode=1, tau=0.01, seed=33, e_trial=-200.0)
    np.testing.assert_array_equal(acc, ref["accept_log"])
    print(f"[edges] step E_L max rel err "
          f"{(np.abs(el - ref['e_log']) / np.maximum(np.abs(ref['e_log']), 1.0)).max():.2e}",
          flush=True)
    _close(el, ref["e_log"])
    _close(ctx.get_walkers()[0], ref["R"])


@pytest.mark.parametrize("n_up,n_dn", [(3, 1), (2, 0)])
def test_unequal_and_empty_spin_match_oracle(n_up, n_dn):
    s = synth.small_random_system(620 + n_dn, n_atom=2, n_up=n_up, n_dn=n_dn, shells=(0, 0, 1, 2),
                                  nprim=2, charge=(n_up + n_dn) / 2)
    W = 11
    R = synth.make_walkers(s, W, 621)
    for k in (1, 2):
        ctx = dmcx.Context(s, W, delay_rank=k, recompute_period=2, seed=34)
        ctx.set_walkers(R)
        acc, el = ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=-3.0, logs=True)
        ref = oracle.run(s, R, n_steps=3, mode=1, tau=0.01, seed=34, e_trial=-3.0)
        np.testing.assert_array_equal(acc, ref["accept_log"])
        _close(el, ref["e_log"])
        _close(ctx.get_walkers()[0], ref["R"])
