"""Semilocal pseudopotential on the GPU (local terms in V, the non-local
energy by the rotated 12-point rule, ratios through y_e = C (A^-1)_{:,e})
against the oracle, with synthetic stand-ins for the ccECP tables.

Bars: E_L (which now carries the pseudopotential energy with the rotations of
(electron, walker, step)) within 1e-10 x max(|E_L|, 1) of the oracle's
E_L + V_NL at the same configurations; DMC runs with the accept sequence
bit-exact and E_L, positions and log-weights within 1e-10; in the mixed form
the pseudopotential part (from the FP64 inverse) within 1e-10 and E_L at the
mixed form's bars; graph replays bit-identical to eager steps;
a group equal to its systems' own contexts; Eq. 3 ion derivatives with the
pseudopotential's Hellmann-Feynman term and the force estimate at 1e-10;
zero-variance forces, Jastrow derivatives and multideterminant expansions
with a pseudopotential rejected.
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
    print(f"[pp] {label}: max rel err {err.max():.2e}", flush=True)
    assert np.all(err <= rel), f"{(err > rel).sum()} of {err.size} outside"


def _oracle_energy(s, R, seed, step, offset=0):
    _, _, e, rc = oracle.evaluate_batch(s, R)
    assert rc == 0
    v, rc = oracle.nlpp_batch(s, R, seed, step, offset)
    assert rc == 0
    return e + v


def test_measure_small_against_oracle():
    s = synth.small_molecule_pp()
    W, seed = 40, 21
    R = synth.make_walkers(s, W, 3300)
    ctx = dmcx.Context(s, W, seed=seed)
    ctx.set_walkers(R)
    e, _, _ = ctx.measure()
    ref = _oracle_energy(s, R, seed, 0)
    _close(e, ref, label="small E_L with pseudopotential")
    # the pseudopotential moves E_L by O(1) Ha: the comparison would fail without it
    bare = dmcx.Context(synth.small_molecule(), W, seed=seed)
    bare.set_walkers(R)
    assert np.abs(bare.measure()[0] - e).max() > 0.1


@pytest.mark.parametrize("k", [1, 4])
def test_dmc_run_small_against_oracle(k):
    s = synth.small_molecule_pp()
    W, seed, tau, et = 24, 22, 0.02, -10.0
    R = synth.make_walkers(s, W, 3301)
    ctx = dmcx.Context(s, W, seed=seed, tau=tau, delay_rank=k, recompute_period=3)
    ctx.set_walkers(R)
    acc, el = ctx.run(4, mode=dmcx.DMCX_DMC, e_trial=et, logs=True)
    ref = oracle.run(s, R, n_steps=4, mode=1, tau=tau, seed=seed, e_trial=et)
    assert ref["rc"] == 0
    np.testing.assert_array_equal(acc, ref["accept_log"])
    _close(el, ref["e_log"], label="E_L log")
    Rg, lw = ctx.get_walkers()
    _close(Rg, ref["R"], label="positions")
    _close(lw, ref["log_w"], label="log w")


def test_large_molecule_sampled_and_run():
    s = synth.large_molecule_pp()
    W, seed = 64, 23
    R = synth.make_walkers(s, W, 3302)
    ctx = dmcx.Context(s, W, seed=seed, delay_rank=32, recompute_period=64)
    ctx.set_walkers(R)
    e, _, _ = ctx.measure()
    assert np.all(np.isfinite(e))
    idx = np.array([0, 17, W - 1])
    ref = np.array([_oracle_energy(s, R[i:i + 1], seed, 0, offset=int(i))[0] for i in idx])
    _close(e[idx], ref, label="large E_L with pseudopotential")
    # one DMC step of the first 3 walkers, against the oracle
    ctx3 = dmcx.Context(s, 3, seed=seed, delay_rank=32, recompute_period=64, tau=0.01)
    ctx3.set_walkers(R[:3])
    acc, el = ctx3.run(1, mode=dmcx.DMCX_DMC, e_trial=-150.0, logs=True)
    out = oracle.run(s, R[:3], n_steps=1, mode=1, tau=0.01, seed=seed, e_trial=-150.0)
    np.testing.assert_array_equal(acc, out["accept_log"])
    _close(el, out["e_log"], label="large E_L after a step")
    _close(ctx3.get_walkers()[1], out["log_w"], label="large log w")


def test_mixed_form_against_oracle():
    """The mixed form takes the kinetic energy from FP32 derivative rows
    (per-walker errors near 1e-6 relative), so E_L is held to the mixed
    form's bars; the pseudopotential part itself, computed from the FP64
    inverse, is isolated as the difference to the same context without it
    (the moves do not depend on the pseudopotential, so both contexts move
    the walkers identically) and held to 1e-10 x max(|E_L|, 1)."""
    s = synth.small_molecule_pp()
    bare_s = synth.small_molecule()
    W, seed = 32, 24
    R = synth.make_walkers(s, W, 3303)
    ctx = dmcx.Context(s, W, seed=seed, precision=dmcx.DMCX_MIXED)
    bare = dmcx.Context(bare_s, W, seed=seed, precision=dmcx.DMCX_MIXED)
    ne = s.n_elec
    for st, nsteps in ((0, 0), (1, 2)):
        if nsteps == 0:
            ctx.set_walkers(R)
            bare.set_walkers(R)
        else:
            ctx.run(nsteps, mode=dmcx.DMCX_VMC)
            bare.run(nsteps, mode=dmcx.DMCX_VMC)
        Rg, _ = ctx.get_walkers()
        np.testing.assert_array_equal(Rg, bare.get_walkers()[0])
        e, _, _ = ctx.measure()
        eb, _, _ = bare.measure()
        ref = _oracle_energy(s, Rg, seed, st)
        dv = np.array([oracle.potential(s, Rg[w]) - oracle.potential(bare_s, Rg[w])
                       for w in range(W)])
        vnl, _ = oracle.nlpp_batch(s, Rg, seed, st)
        scale = np.maximum(np.abs(e), 1.0)
        err = np.abs((e - eb) - (dv + vnl)) / scale
        print(f"[pp] mixed step {st}: pseudopotential part max rel err {err.max():.2e}", flush=True)
        assert np.all(err <= 1e-10)
        assert abs(np.mean(e - ref)) / ne <= 1e-6
        assert np.all(np.abs(e - ref) <= 1e-5 * np.maximum(np.abs(ref), ne))


def test_graph_replay_matches_eager():
    s = synth.small_molecule_pp()
    W, seed = 16, 25
    R = synth.make_walkers(s, W, 3304)
    out = []
    for graph in (False, True):
        ctx = dmcx.Context(s, W, seed=seed, graph=graph, delay_rank=2, recompute_period=2)
        ctx.set_walkers(R)
        acc, el = ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=-10.0, logs=True)
        out.append((acc, el, ctx.get_walkers()))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2][0], out[1][2][0])
    np.testing.assert_array_equal(out[0][2][1], out[1][2][1])


def test_group_with_and_without_pseudopotential():
    a = synth.small_molecule_pp()
    b = synth.small_random_system(91, n_atom=2, n_up=2, n_dn=1, shells=(0, 1), nprim=1,
                                  charge=1.5)
    Ws = [12, 9]
    Ra = synth.make_walkers(a, Ws[0], 3305)
    Rb = synth.make_walkers(b, Ws[1], 3306)
    ne = max(a.n_elec, b.n_elec)
    R = np.zeros((sum(Ws), ne, 3))
    R[: Ws[0], : a.n_elec] = Ra
    R[Ws[0]:, : b.n_elec] = Rb
    grp = dmcx.Context([a, b], Ws, seed=26)
    grp.set_walkers(R)
    acc, el = grp.run(2, mode=dmcx.DMCX_DMC, e_trial=-8.0, logs=True)
    for i, (sysi, Ri, sl) in enumerate(((a, Ra, slice(0, Ws[0])), (b, Rb, slice(Ws[0], None)))):
        one = dmcx.Context(sysi, Ws[i], seed=26)
        one.set_walkers(Ri)
        acc1, el1 = one.run(2, mode=dmcx.DMCX_DMC, e_trial=-8.0, logs=True)
        np.testing.assert_array_equal(acc[:, sl, : sysi.n_elec], acc1)
        np.testing.assert_array_equal(el[:, sl], el1)


def _oracle_dv(s, R, seed, step):
    _, dv, rc = oracle.ion_grads_batch(s, R)
    assert rc == 0
    for w in range(R.shape[0]):
        g, rc = oracle.pp_ion_grads(s, R[w], seed, step, w)
        assert rc == 0
        dv[w] += g
    return dv


def test_ion_grads_and_forces_with_pseudopotential():
    """Eq. 3 ion derivatives with the pseudopotential's Hellmann-Feynman term
    (its centre moved at fixed electrons and Psi, rotations of the current
    step counter) against the oracle, at set-up and after DMC steps; the
    force estimate F = -<dV> - 2(<E_L dlnPsi> - <E_L><dlnPsi>) against the
    oracle's per-walker values (E_L with the rotations of its own step)."""
    s = synth.small_molecule_pp()
    W, seed = 16, 27
    R = synth.make_walkers(s, W, 3307)
    lw = np.random.default_rng(2).normal(0.0, 0.3, W)
    ctx = dmcx.Context(s, W, seed=seed, delay_rank=2, recompute_period=3)
    ctx.set_walkers(R, lw)
    dl, dv = ctx.ion_grads()
    dl_o, _, _ = oracle.ion_grads_batch(s, R)
    _close(dl, dl_o, label="dln|Psi|/dR (set-up)")
    _close(dv, _oracle_dv(s, R, seed, 0), label="dV/dR with pseudopotential (set-up)")
    e, _, _ = ctx.measure()
    om = np.exp(lw - lw.max())
    om /= om.sum()
    mean = lambda x: np.einsum("w,w...->...", om, x)
    e_o = _oracle_energy(s, R, seed, 0)
    dv_o = _oracle_dv(s, R, seed, 0)
    F_ref = -mean(dv_o) - 2 * (mean(e_o[:, None, None] * dl_o) - mean(e_o) * mean(dl_o))
    _close(ctx.forces(), F_ref, rel=1e-10, label="force estimate")
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-10.0)
    Rg, _ = ctx.get_walkers()
    dl, dv = ctx.ion_grads()
    _close(dv, _oracle_dv(s, Rg, seed, 2), label="dV/dR with pseudopotential (after steps)")


def test_ion_grads_after_population_control():
    """The pseudopotential's force term after walkers were copied: comb
    reconfiguration and branching replace slots' inverses after the last
    energy evaluation, and dV/dR of every slot must follow its new walker
    (rotations of the slot's own index and the current step)."""
    s = synth.small_molecule_pp()
    cap, W, seed = 40, 16, 29
    ctx = dmcx.Context(s, cap, seed=seed, delay_rank=2, recompute_period=3)
    ctx.set_walker_count(W)
    ctx.set_walkers(synth.make_walkers(s, W, 3309))
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-10.0)
    R1, lw1 = ctx.get_walkers()
    ctx.set_walkers(R1, np.random.default_rng(4).normal(0.0, 1.0, W))
    ctx.set_step(2)
    copies, _ = ctx.reconfigure(0.37)
    assert (copies != 1).any()
    Rg, _ = ctx.get_walkers()
    _, dv = ctx.ion_grads()
    _close(dv, _oracle_dv(s, Rg, seed, 2), label="dV/dR after reconfiguration")
    ctx.set_walkers(Rg, 0.4 + np.random.default_rng(5).normal(0.0, 0.5, W))
    ctx.set_step(2)
    _, wn = ctx.branch(2)
    assert wn > W
    Rb, _ = ctx.get_walkers()
    _, dv = ctx.ion_grads()
    _close(dv, _oracle_dv(s, Rb, seed, 2), label="dV/dR after branching")


def test_ion_grads_large_molecule_sampled():
    s = synth.large_molecule_pp()
    W, seed = 32, 28
    R = synth.make_walkers(s, W, 3308)
    ctx = dmcx.Context(s, W, seed=seed, delay_rank=32, recompute_period=64)
    ctx.set_walkers(R)
    _, dv = ctx.ion_grads()
    idx = [0, W - 1]
    ref = np.array([_oracle_dv(s, R[i:i + 1], seed, 0)[0] if i == 0 else
                    _oracle_dv_one(s, R[i], seed, 0, i) for i in idx])
    _close(dv[idx], ref, label="large dV/dR with pseudopotential")


def _oracle_dv_one(s, Rw, seed, step, w):
    _, dv, _ = oracle.ion_grads_batch(s, Rw[None])
    g, rc = oracle.pp_ion_grads(s, Rw, seed, step, w)
    assert rc == 0
    return dv[0] + g


def _oracle_jparams(s, R, seed, step):
    O, D, rc = oracle.jastrow_param_grads_batch(s, R)
    assert rc == 0
    for w in range(R.shape[0]):
        dv, rc = oracle.nlpp_param_grads(s, R[w], seed, step, w)
        assert rc == 0
        D[w] += dv
    return O, D


def _medium_pp():
    base = synth.small_random_system(431, n_atom=10, n_up=14, n_dn=13, shells=(0, 0, 1, 2),
                                     nprim=2, box=7.0, charge=2.7)
    return synth.with_pseudopotential(base, [synth.PP_SMALL if a % 2 == 0 else []
                                             for a in range(10)])


@pytest.mark.parametrize("mol", ["small", "medium"])
def test_jastrow_param_grads_with_pseudopotential(mol):
    """dE_L/dp with the non-local energy's part (each quadrature ratio
    carries the Jastrow factor's change) against the oracle's kinetic part
    plus its pseudopotential part, at set-up (rotations of the step set by
    dmcx_set_step) and after DMC steps; the linear-method matrices built on
    them are finite."""
    s = synth.small_molecule_pp() if mol == "small" else _medium_pp()
    W, seed = 6, 61
    R = synth.make_walkers(s, W, 3410)
    ctx = dmcx.Context(s, W, seed=seed, delay_rank=2, recompute_period=3)
    ctx.set_walkers(R)
    ctx.set_step(3)
    O, D = ctx.jastrow_param_grads()
    O_o, D_o = _oracle_jparams(s, R, seed, 3)
    _close(O, O_o, rel=1e-12, label="O_p with pseudopotential")
    _close(D, D_o, rel=1e-10, label="dE_L/dp with pseudopotential")
    ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-10.0)
    Rg, _ = ctx.get_walkers()
    step = ctx.get_step()
    O, D = ctx.jastrow_param_grads()
    O_o, D_o = _oracle_jparams(s, Rg, seed, step)
    _close(D, D_o, rel=1e-10, label="dE_L/dp with pseudopotential after steps")
    S, H = ctx.linear_method()
    assert np.all(np.isfinite(S)) and np.all(np.isfinite(H))


def test_jastrow_param_grads_with_pseudopotential_mixed():
    s = synth.small_molecule_pp()
    W, seed = 6, 62
    R = synth.make_walkers(s, W, 3411)
    ctx = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED, seed=seed)
    ctx.set_walkers(R)
    ctx.set_step(4)
    _, D = ctx.jastrow_param_grads()
    _, D_o = _oracle_jparams(s, R, seed, 4)
    _close(D, D_o, rel=1e-4, label="dE_L/dp with pseudopotential, mixed")


def test_unsupported_with_pseudopotential():
    s = synth.small_molecule_pp()
    ctx = dmcx.Context(s, 8)
    ctx.set_walkers(synth.make_walkers(s, 8, 1))
    with pytest.raises(dmcx.DmcxError) as e:
        ctx.zv_grads(warp=True)
    assert e.value.status == dmcx.DMCX_E_UNSUPPORTED
    base = synth.small_random_system(77, n_atom=2, n_up=3, n_dn=3, shells=(0, 0, 1, 2), nprim=2,
                                     n_mo=10)
    msd = synth.with_pseudopotential(synth.make_msd(base, n_det=5, n_active=6, seed=78),
                                     [synth.PP_SMALL] * 2)
    with pytest.raises(dmcx.DmcxError) as e:
        dmcx.Context(msd, 8)
    assert e.value.status == dmcx.DMCX_E_UNSUPPORTED


def test_mixed_fp32_energy_form():
    """The mixed form with its FP32 energy (E_L from the FP32 rows and the
    FP32 inverse, which also feeds y_e): E_L and the pseudopotential part at
    that form's bar, |dE| <= 1e-6 cond(A) max(|E|, N_e) per walker at set-up
    (no FP32 update has accumulated yet)."""
    s = synth.small_molecule_pp()
    bare_s = synth.small_molecule()
    W, seed = 24, 29
    R = synth.make_walkers(s, W, 3309)
    ctx = dmcx.Context(s, W, seed=seed, precision=dmcx.DMCX_MIXED, fp32_energy=True)
    bare = dmcx.Context(bare_s, W, seed=seed, precision=dmcx.DMCX_MIXED, fp32_energy=True)
    ctx.set_walkers(R)
    bare.set_walkers(R)
    e, _, _ = ctx.measure()
    eb, _, _ = bare.measure()
    ref = _oracle_energy(s, R, seed, 0)
    dv = np.array([oracle.potential(s, R[w]) - oracle.potential(bare_s, R[w]) for w in range(W)])
    vnl, _ = oracle.nlpp_batch(s, R, seed, 0)
    cond = []
    for w in range(W):
        for sp, (a, b) in enumerate(((0, s.n_up), (s.n_up, s.n_elec))):
            A = np.array([oracle.orbitals_vgl(s, R[w, i], b - a)[0] for i in range(a, b)])
            cond.append(np.linalg.cond(A))
    cmax = max(cond)
    ne = s.n_elec
    err_pp = np.abs((e - eb) - (dv + vnl)) / np.maximum(np.abs(e), 1.0)
    err = np.abs(e - ref) / np.maximum(np.abs(ref), ne)
    print(f"[pp] fp32-energy: max cond {cmax:.1e}, pseudopotential part {err_pp.max():.2e}, "
          f"E_L {err.max():.2e}", flush=True)
    assert np.all(err_pp <= 1e-6 * cmax)
    assert np.all(err <= 1e-6 * cmax)
