"""The JSON-lines metrics log (host logic) on a stand-in context: the
estimator fields map to their records, non-finite values become null, the
flagged count and the largest residual are taken per system, and a run in
chunks writes one line per chunk."""
import json
import math

import numpy as np

from paper_2504_07948_amd import metrics


class _Stub:
    def __init__(self):
        self.n_sys = 2
        self.offsets = [0, 3]
        self.walkers = [3, 2]
        self.step = 0
        self.runs = []

    def estimators(self):
        # [counted, m, S0, S1, S2, Q, <E>, var, min log w, acceptance, moves]
        return np.array([[3, 0.5, 2.0, -4.0, 8.5, 1.5, -2.0, 0.25, -0.2, 0.75, 120],
                         [0, np.nan, np.nan, np.nan, np.nan, np.nan, np.nan, np.nan, np.nan,
                          np.nan, 0]])

    def walker_flags(self):
        return np.array([0, 1, 0, 2, 2], dtype=np.uint8)

    def inverse_residual(self):
        return np.array([[1e-14, 3e-13], [2e-14, 0.0], [5e-15, 1e-15], [np.nan, 0.0], [1e-9, 0.0]])

    def get_step(self):
        return self.step

    def run(self, k, mode, e_trial):
        self.runs.append(k)
        self.step += k


def test_records_and_nulls(tmp_path):
    ctx = _Stub()
    with metrics.MetricsLog(str(tmp_path / "m.jsonl")) as log:
        rec = log.write(ctx)
    a, b = rec["systems"]
    assert a["counted"] == 3 and a["e_mean"] == -2.0 and a["e_var"] == 0.25
    assert a["acceptance"] == 0.75 and a["moves"] == 120
    assert abs(a["log_w_total"] - (0.5 + math.log(2.0))) < 1e-15
    assert a["log_w_min"] == -0.2 and a["log_w_max"] == 0.5
    assert abs(a["n_eff"] - 4.0 / 1.5) < 1e-15
    assert a["flagged"] == 1 and a["residual_max"] == 3e-13
    assert b["counted"] == 0 and b["e_mean"] is None and b["log_w_total"] is None
    assert b["n_eff"] is None and b["flagged"] == 2 and b["residual_max"] is None
    line = json.loads(open(tmp_path / "m.jsonl").read().strip())
    assert line["systems"] == rec["systems"] and line["step"] == 0


def test_run_in_chunks(tmp_path):
    ctx = _Stub()
    with metrics.MetricsLog(str(tmp_path / "r.jsonl"), residual=False) as log:
        recs = metrics.run_logged(ctx, 7, log, mode=1, e_trial=-1.0, every=3)
    assert ctx.runs == [3, 3, 1]
    assert [r["step"] for r in recs] == [3, 6, 7]
    lines = open(tmp_path / "r.jsonl").read().strip().split("\n")
    assert len(lines) == 3 and "residual_max" not in json.loads(lines[0])["systems"][0]
