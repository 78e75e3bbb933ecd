"""Diagnostics on the GPU: the inverse residual max|A A^{-1} - I| (Eq. 3's
inverse as the delayed updates keep it) and the JSON-lines metrics log.

* Residual: at round-off right after the FP64 set-up; small but larger
  after DMC steps without a recompute; back at round-off after
  dmcx_recompute; a pending electron block of the move-by-move calls is
  flushed first (the moved electron's row is then part of A); the mixed
  form's stored FP32 inverse shows FP32-size residuals; a group reports each
  system's walkers in its own rows.
* Metrics: a logged run writes one line per chunk; the last line's weighted
  estimators agree with numpy sums over the walkers' log w and E_L read
  back after the run, its move count is steps x walkers x electrons.
"""
import json

import numpy as np
import pytest

from paper_2504_07948_amd import dmcx, metrics, synth

pytestmark = pytest.mark.gpu


def test_inverse_residual_fp64_and_mixed():
    s = synth.small_molecule()
    W = 16
    R = synth.make_walkers(s, W, 801)
    ctx = dmcx.Context(s, W, delay_rank=4, recompute_period=100, seed=5)
    ctx.set_walkers(R)
    r0 = ctx.inverse_residual()
    print(f"[metrics] residual after set-up {r0.max():.2e}", flush=True)
    assert r0.shape == (W, 2) and np.all(r0 < 1e-12)
    ctx.run(5, mode=dmcx.DMCX_DMC, e_trial=-8.0)
    r1 = ctx.inverse_residual()
    print(f"[metrics] residual after 5 steps {r1.max():.2e}", flush=True)
    assert np.all(r1 < 1e-9) and r1.max() > 0.0
    ctx.recompute()
    assert np.all(ctx.inverse_residual() < 1e-12)
    # a pending block: one accepted move of electron 0, not flushed
    Rg, _ = ctx.get_walkers()
    r_new = Rg[:, 0, :] + 0.05
    ratio, _ = ctx.ratio_grad(0, r_new)
    ctx.accept(0, np.ones(W, dtype=np.uint8))
    r2 = ctx.inverse_residual()
    print(f"[metrics] residual after a pending move {r2.max():.2e}", flush=True)
    assert np.all(r2 < 1e-9)
    m = dmcx.Context(s, W, precision=dmcx.DMCX_MIXED, delay_rank=4, recompute_period=100, seed=5)
    m.set_walkers(R)
    m.run(3, mode=dmcx.DMCX_DMC, e_trial=-8.0)
    rm = m.inverse_residual()
    print(f"[metrics] mixed residual {rm.max():.2e}", flush=True)
    assert 1e-9 < rm.max() < 1e-2


def test_inverse_residual_group_rows():
    a = synth.small_molecule()
    b = synth.small_random_system(91, n_atom=2, n_up=2, n_dn=1, shells=(0, 1), nprim=1,
                                  charge=1.5)
    Ws = [8, 5]
    ne = max(a.n_elec, b.n_elec)
    R = np.zeros((sum(Ws), ne, 3))
    R[:Ws[0], :a.n_elec] = synth.make_walkers(a, Ws[0], 802)
    R[Ws[0]:, :b.n_elec] = synth.make_walkers(b, Ws[1], 803)
    g = dmcx.Context([a, b], Ws, delay_rank=2, seed=6)
    g.set_walkers(R)
    g.run(2, mode=dmcx.DMCX_DMC, e_trial=-5.0)
    r = g.inverse_residual()
    assert r.shape == (13, 2) and np.all(r < 1e-9)
    solo = dmcx.Context(b, Ws[1], delay_rank=2, seed=6)
    solo.set_walkers(R[Ws[0]:, :b.n_elec])
    solo.run(2, mode=dmcx.DMCX_DMC, e_trial=-5.0)
    np.testing.assert_array_equal(r[Ws[0]:], solo.inverse_residual())


def test_metrics_log_matches_walker_sums(tmp_path):
    s = synth.small_molecule()
    W = 24
    ctx = dmcx.Context(s, W, delay_rank=4, recompute_period=8, tau=0.01, seed=7)
    ctx.set_walkers(synth.make_walkers(s, W, 804))
    path = tmp_path / "metrics.jsonl"
    with metrics.MetricsLog(str(path)) as log:
        recs = metrics.run_logged(ctx, 4, log, mode=dmcx.DMCX_DMC, e_trial=-8.0, every=2)
    lines = [json.loads(x) for x in open(path).read().strip().split("\n")]
    assert len(lines) == 2 and [x["step"] for x in lines] == [2, 4]
    last = lines[-1]["systems"][0]
    _, lw = ctx.get_walkers()
    e, _, _ = ctx.measure()
    om = np.exp(lw - lw.max())
    mean = float((om * e).sum() / om.sum())
    var = float((om * (e - mean) ** 2).sum() / om.sum())
    print(f"[metrics] last line {last}", flush=True)
    assert last["counted"] == W and last["flagged"] == 0
    assert abs(last["e_mean"] - mean) <= 1e-12 * max(1.0, abs(mean))
    assert abs(last["e_var"] - var) <= 1e-10 * max(1.0, var)
    assert abs(last["log_w_max"] - lw.max()) <= 1e-14 and abs(last["log_w_min"] - lw.min()) <= 1e-14
    n_eff = om.sum() ** 2 / (om ** 2).sum()
    assert abs(last["n_eff"] - n_eff) <= 1e-10 * n_eff
    assert last["moves"] == 2 * W * s.n_elec
    assert 0.0 < last["acceptance"] <= 1.0
    assert last["residual_max"] is not None and last["residual_max"] < 1e-9
    assert recs[-1]["systems"][0] == last


def test_metrics_log_for_a_group(tmp_path):
    """A context of two systems: one record per system, each over its own
    walkers (counts, estimators equal to the systems' own contexts)."""
    a = synth.small_molecule()
    b = synth.small_random_system(91, n_atom=2, n_up=2, n_dn=1, shells=(0, 1), nprim=1,
                                  charge=1.5)
    Ws = [16, 9]
    ne = max(a.n_elec, b.n_elec)
    Ra = synth.make_walkers(a, Ws[0], 805)
    Rb = synth.make_walkers(b, Ws[1], 806)
    R = np.zeros((sum(Ws), ne, 3))
    R[:Ws[0], :a.n_elec] = Ra
    R[Ws[0]:, :b.n_elec] = Rb
    g = dmcx.Context([a, b], Ws, delay_rank=2, seed=8)
    g.set_walkers(R)
    with metrics.MetricsLog(str(tmp_path / "g.jsonl")) as log:
        recs = metrics.run_logged(g, 2, log, mode=dmcx.DMCX_DMC, e_trial=-5.0, every=2)
    sysrec = recs[-1]["systems"]
    assert [r["walkers"] for r in sysrec] == Ws and [r["system"] for r in sysrec] == [0, 1]
    for i, (s, Rs) in enumerate(((a, Ra), (b, Rb))):
        solo = dmcx.Context(s, Ws[i], delay_rank=2, seed=8)
        solo.set_walkers(Rs)
        solo.run(2, mode=dmcx.DMCX_DMC, e_trial=-5.0)
        est = solo.estimators()[0]
        assert sysrec[i]["counted"] == Ws[i] and sysrec[i]["flagged"] == 0
        assert sysrec[i]["e_mean"] == est[6]
        assert sysrec[i]["moves"] == int(est[10])
