"""GPU parity of the ion-force path (reverse-mode adjoint) against the CPU
oracle's forward-mode Eq. 3 gradients, central finite differences of the
library's own log|Psi| and V, the VJP definitions and the force estimator."""
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
    assert not bad.any(), (f"{bad.sum()}/{bad.size} outside; max rel "
                           f"{(np.abs(a - b) / np.maximum(np.abs(b), floor)).max():.3e}")


@pytest.mark.parametrize("mol,W", [("small", 16), ("large", 9)])
def test_ion_grads_match_oracle_forward_mode(mol, W):
    s = synth.molecule(mol)
    R = synth.make_walkers(s, W, 500 + synth.SEED_OFFSET[mol])
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    dl, dv = ctx.ion_grads()
    dl_o, dv_o, rc = oracle.ion_grads_batch(s, R)
    assert rc == 0
    _close(dv, dv_o)
    _close(dl, dl_o)


def test_ion_grads_after_moves_match_oracle():
    """Gradients use the delayed-updated inverse after a DMC step."""
    s = synth.large_molecule()
    W = 8
    R = synth.make_walkers(s, W, 510)
    ctx = dmcx.Context(s, W, delay_rank=32, recompute_period=100)
    ctx.set_walkers(R)
    ctx.run(1, mode=dmcx.DMCX_DMC, e_trial=-100.0)
    Rg, _ = ctx.get_walkers()
    dl, dv = ctx.ion_grads()
    dl_o, dv_o, _ = oracle.ion_grads_batch(s, Rg)
    print(f"[forces] after a DMC step: d ln|Psi|/dR max rel err "
          f"{(np.abs(dl - dl_o) / np.maximum(np.abs(dl_o), 1.0)).max():.2e}", flush=True)
    _close(dl, dl_o)
    _close(dv, dv_o)


def test_ion_grads_vs_finite_differences():
    s = synth.small_molecule()
    W = 8
    R = synth.make_walkers(s, W, 520)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    dl, dv = ctx.ion_grads()
    base = s.ion_xyz.copy()

    def central(a, x, h):
        vals = []
        for sgn in (+1, -1):
            xyz = base.copy()
            xyz[a, x] += sgn * h
            ctx.set_ions(xyz)
            _, lp, _ = ctx.measure()
            vals.append((lp, ctx.potential()))
        return ((vals[0][0] - vals[1][0]) / (2 * h), (vals[0][1] - vals[1][1]) / (2 * h))

    for a, x in [(0, 0), (1, 2), (3, 1)]:
        # central differences at h = 1e-4 and 2e-4, Richardson-extrapolated (O(h^4))
        l1, v1 = central(a, x, 2e-4)
        l2, v2 = central(a, x, 1e-4)
        fd_l = (4 * l2 - l1) / 3
        fd_v = (4 * v2 - v1) / 3
        np.testing.assert_allclose(dl[:, a, x], fd_l, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(dv[:, a, x], fd_v, rtol=1e-6, atol=1e-6)
    ctx.set_ions(base)


def test_translation_sum_rule():
    """sum_A dlnPsi/dR_A = -sum_i grad_i lnPsi (the oracle's drift)."""
    s = synth.small_molecule()
    W = 4
    R = synth.make_walkers(s, W, 530)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    dl, _ = ctx.ion_grads()
    for w in range(W):
        drift = oracle.evaluate(s, R[w])[3]
        np.testing.assert_allclose(dl[w].sum(0), -drift.sum(0), rtol=1e-9, atol=1e-9)


def test_vjps_and_force_estimator():
    s = synth.small_molecule()
    W = 24
    R = synth.make_walkers(s, W, 540)
    lw = np.random.default_rng(0).normal(0, 0.3, W)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R, lw)
    dl, dv = ctx.ion_grads()
    g = np.random.default_rng(1).standard_normal(W)
    _close(ctx.logpsi_vjp(g), np.einsum("w,wak->ak", g, dl), rel=1e-12)
    _close(ctx.potential_vjp(g), np.einsum("w,wak->ak", g, dv), rel=1e-12)
    e, _, _ = ctx.measure()
    om = np.exp(lw - lw.max())
    om /= om.sum()
    mean = lambda x: np.einsum("w,w...->...", om, x)
    F_ref = -mean(dv) - 2 * (mean(e[:, None, None] * dl) - mean(e) * mean(dl))
    _close(ctx.forces(), F_ref, rel=1e-11)


def _force_objective(log_psi, v_pot, e_local, omega):
    """<V> + 2 (<E_L lnPsi> - <E_L><lnPsi>) with E_L and omega held constant;
    minus its ion gradient is the Hellmann-Feynman + Pulay force estimate."""
    wsum = omega.sum()
    e = e_local.detach()
    e_mean = (omega * e).sum() / wsum
    return (omega * v_pot).sum() / wsum + 2.0 * ((omega * (e - e_mean) * log_psi).sum() / wsum)


@pytest.mark.parametrize("where", ["cuda", "cpu"])
def test_autograd_function_matches_vjp(where):
    torch = pytest.importorskip("torch")
    from paper_2504_07948_amd.autograd import IonGradFn
    s = synth.small_molecule()
    W = 16
    R = synth.make_walkers(s, W, 550)
    ctx = dmcx.Context(s, W, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_walkers(R)
    ion = torch.tensor(s.ion_xyz, dtype=torch.float64, device=where, requires_grad=True)
    lp, v, e = IonGradFn.apply(ion, ctx)
    assert lp.device == ion.device and v.device == ion.device and e.device == ion.device
    e_ref, lp_ref, _ = ctx.measure()
    _close(lp.detach().cpu().numpy(), lp_ref, rel=0.0)
    _close(e.cpu().numpy(), e_ref, rel=0.0)
    om = torch.ones(W, dtype=torch.float64, device=where)
    obj = _force_objective(lp, v, e, om)
    obj.backward()
    assert ion.grad.device == ion.device
    _close(-ion.grad.cpu().numpy(), ctx.forces(), rel=1e-11)


def test_large_system_ion_grads_vs_richardson_fd():
    """The 64-atom, 192-component force workload: per-walker d ln|Psi|/dR and
    dV/dR of a handful of components (carbons and hydrogens, every axis)
    against Richardson-extrapolated central differences (h = 2e-4, 1e-4 bohr)
    of the library's own log|Psi| and V, electrons fixed."""
    s = synth.large_molecule()
    W = 3
    R = synth.make_walkers(s, W, 530)
    ctx = dmcx.Context(s, W)
    ctx.set_walkers(R)
    dl, dv = ctx.ion_grads()
    base = s.ion_xyz.copy()
    comps = [(0, 0), (5, 2), (15, 1), (16, 0), (33, 1), (63, 2)]
    worst = 0.0
    for a, x in comps:
        est_l, est_v = {}, {}
        for h in (2e-4, 1e-4):
            lp, vv = [], []
            for sgn in (1, -1):
                xyz = base.copy()
                xyz[a, x] += sgn * h
                ctx.set_ions(xyz)
                lp.append(ctx.measure()[1])
                vv.append(ctx.potential())
            est_l[h] = (lp[0] - lp[1]) / (2 * h)
            est_v[h] = (vv[0] - vv[1]) / (2 * h)
        fd_l = (4 * est_l[1e-4] - est_l[2e-4]) / 3
        fd_v = (4 * est_v[1e-4] - est_v[2e-4]) / 3
        worst = max(worst, np.max(np.abs(dl[:, a, x] - fd_l) / np.maximum(np.abs(fd_l), 1.0)))
        np.testing.assert_allclose(dl[:, a, x], fd_l, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(dv[:, a, x], fd_v, rtol=1e-6, atol=1e-6)
    ctx.set_ions(base)
    print(f"[forces] 64-atom FD: worst rel deviation of d ln|Psi|/dR {worst:.2e}", flush=True)


def test_mixed_force_estimator_against_oracle_runs():
    """F_mixed = 2 F_DMC - F_VMC (the paper's mixed estimator in its force
    comparison): F_DMC from a DMC-weighted population, F_VMC from a VMC
    population of the same start (equal weights), each the Hellmann-Feynman +
    Pulay estimate of dmcx_forces.  The oracle runs the same chains (accept
    sequences bit-exact); its per-walker ion derivatives (forward mode, Eq. 3)
    and energies at the final configurations, combined by the estimator's
    definition with its log-weights, give the reference at 1e-10."""
    s = synth.small_molecule()
    W, steps = 32, 4
    R = synth.make_walkers(s, W, 560)
    _, _, e0, _ = oracle.evaluate_batch(s, R)
    e_t = float(np.mean(e0))
    F = {}
    for mode in (dmcx.DMCX_DMC, dmcx.DMCX_VMC):
        ctx = dmcx.Context(s, W, delay_rank=1, recompute_period=4, seed=23)
        ctx.set_walkers(R)
        acc, _ = ctx.run(steps, mode=mode, e_trial=e_t, logs=True)
        ref = oracle.run(s, R, n_steps=steps, mode=mode, tau=0.01, seed=23, e_trial=e_t)
        np.testing.assert_array_equal(acc, ref["accept_log"])
        dl_o, dv_o, _ = oracle.ion_grads_batch(s, ref["R"])
        _, _, e_o, _ = oracle.evaluate_batch(s, ref["R"])
        lw = ref["log_w"] if mode == dmcx.DMCX_DMC else np.zeros(W)
        om = np.exp(lw - lw.max())
        om /= om.sum()
        mean = lambda x: np.einsum("w,w...->...", om, x)
        F_ref = -mean(dv_o) - 2 * (mean(e_o[:, None, None] * dl_o) - mean(e_o) * mean(dl_o))
        # the estimator subtracts terms of size <|E_L| |dlnPsi|>: the bar scales with them
        terms = np.abs(mean(np.abs(dv_o))) + 2 * mean(np.abs(e_o)[:, None, None] * np.abs(dl_o))
        F[mode] = (ctx.forces(), F_ref, terms)
        ctx.close()
    mixed = 2 * F[dmcx.DMCX_DMC][0] - F[dmcx.DMCX_VMC][0]
    mixed_ref = 2 * F[dmcx.DMCX_DMC][1] - F[dmcx.DMCX_VMC][1]
    bar = 1e-10 * np.maximum(2 * F[dmcx.DMCX_DMC][2] + F[dmcx.DMCX_VMC][2], 1.0)
    print(f"[forces] mixed estimator max |dF| {np.abs(mixed - mixed_ref).max():.3e}", flush=True)
    assert np.all(np.abs(mixed - mixed_ref) <= bar)
