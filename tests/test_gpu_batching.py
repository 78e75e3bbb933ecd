"""Batching form: captured step graphs, groups of systems with uneven
electron counts in one context, and the delay-rank autotuner.

Bars: a graph run and an eager run of the same context options produce the
same bits (accept logs, E_L logs, positions, weights); every system of a
group moves exactly as it does in a context of its own (same bits), and
both agree with the CPU oracle (accept sequence bit-exact, E_L and
positions within 1e-10); the autotuner picks one of its candidates and the
run it precedes matches a run at that rank from the same walkers.
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
    bad = np.abs(a - b) > tol
    assert not bad.any(), f"{bad.sum()} of {bad.size} outside tolerance"


def _group_systems():
    """Three systems with 8, 6 and 112 electrons (uneven shapes, ragged walkers)."""
    return [synth.small_molecule(),
            synth.small_random_system(71, n_atom=3, n_up=3, n_dn=3, shells=(0, 0, 1, 2),
                                      nprim=3, charge=2.0),
            synth.large_molecule()], [13, 21, 9]


def _pad(R, ne_max):
    out = np.zeros((R.shape[0], ne_max, 3))
    out[:, :R.shape[1]] = R
    return out


@pytest.mark.parametrize("mol,W,P", [("small", 24, 3), ("large", 11, 2)])
def test_graph_matches_eager(mol, W, P):
    """Replays of the captured step graph reproduce eager steps bit for bit,
    with eager work (a measure) between replays and a recompute period that
    the graph's kernels decide from the device step counter."""
    s = synth.molecule(mol)
    R = synth.make_walkers(s, W, 700 + synth.SEED_OFFSET[mol])
    out = {}
    for graph in (False, True):
        print(f"[batching] {mol} W={W} P={P} graph={graph}", flush=True)
        ctx = dmcx.Context(s, W, delay_rank=8, recompute_period=P, seed=5, graph=graph)
        ctx.set_walkers(R)
        a1, e1 = ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-10.0, logs=True)
        m1 = ctx.measure()
        a2, e2 = ctx.run(3, mode=dmcx.DMCX_DMC, e_trial=-10.0, logs=True)
        a3, _ = ctx.run(1, mode=dmcx.DMCX_VMC, e_trial=0.0, logs=True)  # new mode, same graph
        Rg, lw = ctx.get_walkers()
        out[graph] = (a1, e1, m1, a2, e2, a3, Rg, lw, ctx.measure())
    for x, y in zip(out[False], out[True]):
        if isinstance(x, tuple):
            for u, v in zip(x, y):
                np.testing.assert_array_equal(u, v)
        else:
            np.testing.assert_array_equal(x, y)


def test_graph_device_logs():
    torch = pytest.importorskip("torch")
    s = synth.small_molecule()
    W = 16
    R = synth.make_walkers(s, W, 710)
    res = []
    for graph in (False, True):
        ctx = dmcx.Context(s, W, delay_rank=1, seed=9, graph=graph)
        ctx.set_walkers(torch.from_numpy(R).cuda())
        acc = torch.zeros((4, W, s.n_elec), dtype=torch.uint8, device="cuda")
        el = torch.zeros((4, W), dtype=torch.float64, device="cuda")
        ctx.run_device(4, mode=dmcx.DMCX_DMC, e_trial=-8.0, accept_log=acc, e_log=el)
        ctx.sync()
        res.append((acc.cpu().numpy(), el.cpu().numpy()))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("graph", [False, True])
def test_group_matches_individual_and_oracle(graph):
    systems, walkers = _group_systems()
    ne_max = max(s.n_elec for s in systems)
    Rs = [synth.make_walkers(s, w, 720 + i) for i, (s, w) in enumerate(zip(systems, walkers))]
    n_steps, e_t = 2, -20.0
    print(f"[batching] group of {[s.n_elec for s in systems]} electrons, graph={graph}", flush=True)
    grp = dmcx.Context(systems, walkers, delay_rank=16, recompute_period=2, seed=11, graph=graph)
    grp.set_walkers(np.concatenate([_pad(R, ne_max) for R in Rs]))
    acc, el = grp.run(n_steps, mode=dmcx.DMCX_DMC, e_trial=e_t, logs=True)
    Rg, lwg = grp.get_walkers()
    eg, lpg, sgg = grp.measure()
    assert acc.shape == (n_steps, sum(walkers), ne_max)
    for i, (s, w, R) in enumerate(zip(systems, walkers, Rs)):
        o = grp.offsets[i]
        sl = slice(o, o + w)
        one = dmcx.Context(s, w, delay_rank=16, recompute_period=2, seed=11)
        one.set_walkers(R)
        a1, e1 = one.run(n_steps, mode=dmcx.DMCX_DMC, e_trial=e_t, logs=True)
        R1, lw1 = one.get_walkers()
        np.testing.assert_array_equal(acc[:, sl, :s.n_elec], a1)
        assert not acc[:, sl, s.n_elec:].any()
        np.testing.assert_array_equal(el[:, sl], e1)
        np.testing.assert_array_equal(Rg[sl, :s.n_elec], R1)
        np.testing.assert_array_equal(lwg[sl], lw1)
        np.testing.assert_array_equal(eg[sl], one.measure()[0])
        if s.n_elec <= 8:  # the oracle run is cheap for the small systems
            ref = oracle.run(s, R, n_steps=n_steps, mode=dmcx.DMCX_DMC, tau=0.01, seed=11,
                             e_trial=e_t)
            np.testing.assert_array_equal(a1, ref["accept_log"])
            _close(e1, ref["e_log"])
            _close(R1, ref["R"])


def test_group_forces_and_grads_match_individual():
    systems, walkers = _group_systems()
    ne_max = max(s.n_elec for s in systems)
    na_max = max(s.n_atom for s in systems)
    Rs = [synth.make_walkers(s, w, 740 + i) for i, (s, w) in enumerate(zip(systems, walkers))]
    grp = dmcx.Context(systems, walkers, delay_rank=16)
    grp.set_walkers(np.concatenate([_pad(R, ne_max) for R in Rs]))
    dl, dv = grp.ion_grads()
    assert dl.shape == (sum(walkers), na_max, 3)
    F = grp.forces()
    assert F.shape == (len(systems), na_max, 3)
    g = np.random.default_rng(3).standard_normal(sum(walkers))
    vj = grp.logpsi_vjp(g)
    for i, (s, w, R) in enumerate(zip(systems, walkers, Rs)):
        sl = slice(grp.offsets[i], grp.offsets[i] + w)
        one = dmcx.Context(s, w, delay_rank=16)
        one.set_walkers(R)
        dl1, dv1 = one.ion_grads()
        # per-atom sums are accumulated with atomics: equal up to summation order
        _close(dl[sl, :s.n_atom], dl1, rel=1e-12)
        _close(dv[sl, :s.n_atom], dv1, rel=1e-12)
        _close(F[i, :s.n_atom], one.forces(), rel=1e-12)
        _close(vj[i, :s.n_atom], one.logpsi_vjp(g[sl]), rel=1e-12)


def test_group_rejects_move_by_move_calls():
    systems, walkers = _group_systems()
    grp = dmcx.Context(systems, walkers)
    ne_max = max(s.n_elec for s in systems)
    grp.set_walkers(np.concatenate([_pad(synth.make_walkers(s, w, 750), ne_max)
                                    for s, w in zip(systems, walkers)]))
    with pytest.raises(dmcx.DmcxError) as e:
        grp.ratio_grad(0, np.zeros((sum(walkers), 3)))
    assert e.value.status == dmcx.DMCX_E_UNSUPPORTED


def test_autotuner_picks_a_candidate_and_preserves_the_run():
    s = synth.large_molecule()
    W = 16
    R = synth.make_walkers(s, W, 760)
    ctx = dmcx.Context(s, W, delay_rank=0, recompute_period=64, seed=13)
    ctx.set_walkers(R)
    acc, el = ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-50.0, logs=True)  # tunes first
    ranks, shapes, ms = ctx.autotune_report()
    k = ctx.delay_rank()
    print(f"[batching] autotune ranks {ranks.tolist()} ms {np.round(ms, 3).tolist()} -> k={k}")
    assert ranks.tolist() == [8, 16, 24, 32, 48, 56]
    assert np.all(shapes == dmcx.DMCX_TILE_DEEP) and ctx.tile_shape() == dmcx.DMCX_TILE_DEEP
    assert np.all(ms > 0) and k in ranks.tolist()
    assert ms[ranks.tolist().index(k)] == ms.min()
    ref = dmcx.Context(s, W, delay_rank=k, recompute_period=64, seed=13)
    ref.set_walkers(R)
    acc_r, el_r = ref.run(2, mode=dmcx.DMCX_DMC, e_trial=-50.0, logs=True)
    np.testing.assert_array_equal(acc, acc_r)
    np.testing.assert_array_equal(el, el_r)
    # an explicit call keeps configurations and weights
    Rb, lwb = ctx.get_walkers()
    eb = ctx.measure()[0]
    kk = ctx.autotune(steps=1)
    Ra, lwa = ctx.get_walkers()
    np.testing.assert_array_equal(Ra, Rb)
    np.testing.assert_array_equal(lwa, lwb)
    _close(ctx.measure()[0], eb, rel=1e-9)
    assert kk[0] == ctx.delay_rank()


def test_autotuner_chooses_tile_shape_and_rank_mixed():
    """The FP32 sweep offers two tile shapes: the tuner times every (shape,
    rank) pair and keeps the fastest; a run after it is bit-identical to a
    run of a fresh context given that shape and rank."""
    s = synth.large_molecule()
    W = 64
    R = synth.make_walkers(s, W, 761)
    ctx = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED, delay_rank=0, recompute_period=32,
                       seed=14)
    ctx.set_walkers(R)
    acc, el = ctx.run(2, mode=dmcx.DMCX_DMC, e_trial=-50.0, logs=True)
    ranks, shapes, ms = ctx.autotune_report()
    k, shape = ctx.delay_rank(), ctx.tile_shape()
    print(f"[batching] mixed autotune {list(zip(shapes.tolist(), ranks.tolist()))} "
          f"ms {np.round(ms, 3).tolist()} -> shape {shape}, k={k}", flush=True)
    assert sorted(set(shapes.tolist())) == [dmcx.DMCX_TILE_DEEP, dmcx.DMCX_TILE_SHALLOW]
    assert ranks.tolist() == [8, 16, 24, 32, 48, 56] * 2
    best = int(np.argmin(ms))
    assert (shapes[best], ranks[best]) == (shape, k)
    ref = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED, delay_rank=k, recompute_period=32,
                       seed=14)
    ref.set_tile_shape(shape)
    ref.set_walkers(R)
    acc_r, el_r = ref.run(2, mode=dmcx.DMCX_DMC, e_trial=-50.0, logs=True)
    np.testing.assert_array_equal(acc, acc_r)
    np.testing.assert_array_equal(el, el_r)


@pytest.mark.parametrize("shape", [0, 1])
def test_tile_shapes_mixed_against_oracle(shape):
    """Both tile shapes of the FP32 sweep: VMC steps against the oracle run
    on the same stream (every walker's accept sequence equal to the oracle's
    but for at most two walkers, where a near-threshold FP32 ratio may fall
    the other way; energies of the final configurations within the mixed
    form's bar)."""
    s = synth.small_molecule()
    W = 48
    R = synth.make_walkers(s, W, 762)
    ctx = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED, delay_rank=2, recompute_period=4,
                       seed=15, tau=0.02)
    ctx.set_tile_shape(shape)
    assert ctx.tile_shape() == shape
    ctx.set_walkers(R)
    acc, _ = ctx.run(3, mode=dmcx.DMCX_VMC, logs=True)
    ref = oracle.run(s, R, n_steps=3, mode=0, tau=0.02, seed=15)
    same = np.all(acc == ref["accept_log"], axis=(0, 2))
    print(f"[batching] shape {shape}: {same.sum()} of {W} walkers with the oracle's accept "
          f"sequence", flush=True)
    assert same.sum() >= W - 2
    Rg, _ = ctx.get_walkers()
    e = ctx.measure()[0]
    _, _, eo, _ = oracle.evaluate_batch(s, Rg)
    ne = s.n_up + s.n_dn
    assert abs(np.mean(e - eo)) / ne <= 1e-6
    assert np.all(np.abs(e - eo) <= 1e-5 * np.maximum(np.abs(eo), ne))


def test_tile_shape_errors():
    s = synth.small_molecule()
    ctx = dmcx.Context(s, 8)  # FP64: deep only
    with pytest.raises(dmcx.DmcxError) as e:
        ctx.set_tile_shape(dmcx.DMCX_TILE_SHALLOW)
    assert e.value.status == dmcx.DMCX_E_UNSUPPORTED
    for bad in (2, -1):
        with pytest.raises(dmcx.DmcxError):
            ctx.set_tile_shape(bad)
    with pytest.raises(dmcx.DmcxError):
        ctx.set_tile_shape(0, sys_index=1)
    ctx.set_tile_shape(dmcx.DMCX_TILE_DEEP)
