"""Per-step metrics of a DMC run as JSON lines, written on the host after a
run call returns (never from inside the eager or captured step).

One line per logging point holds the step counter, the wall time since the
log was opened and, for every system of the context:

* the weighted estimators of ``dmcx_estimators`` (the weights of Eq. 1):
  walkers counted, <E_L>, its weighted variance, the acceptance ratio and
  the moves proposed since the previous logging point, the log of the total
  weight, the smallest and largest log w, the effective walker count;
* the number of walkers with a status flag (non-finite or singular);
* the largest inverse residual max |A A^{-1} - I| over its walkers
  (``dmcx_inverse_residual``).

Non-finite numbers are written as null (JSON has no NaN).  Reading the
estimators clears the context's move counters, so each line's acceptance
covers the steps since the line before.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np


def _num(x):
    x = float(x)
    return x if math.isfinite(x) else None


def step_metrics(ctx, residual=True):
    """The per-system records of one logging point (a list of dicts)."""
    est = np.asarray(ctx.estimators(), dtype=np.float64)
    flags = np.asarray(ctx.walker_flags())
    res = np.asarray(ctx.inverse_residual(), dtype=np.float64) if residual else None
    out = []
    for s in range(ctx.n_sys):
        o, n = ctx.offsets[s], ctx.walkers[s]
        e = est[s]
        counted = int(e[0])
        m, s0, q = e[1], e[2], e[5]
        rec = {
            "system": s,
            "walkers": int(n),
            "counted": counted,
            "e_mean": _num(e[6]),
            "e_var": _num(e[7]),
            "acceptance": _num(e[9]),
            "moves": int(e[10]) if math.isfinite(e[10]) else 0,
            "log_w_total": _num(m + math.log(s0)) if counted and s0 > 0 else None,
            "log_w_min": _num(e[8]),
            "log_w_max": _num(m),
            "n_eff": _num(s0 * s0 / q) if counted and q > 0 else None,
            "flagged": int(np.count_nonzero(flags[o:o + n])),
        }
        if res is not None:
            r = res[o:o + n]
            rec["residual_max"] = None if np.isnan(r).any() else _num(r.max() if r.size else 0.0)
        out.append(rec)
    return out


class MetricsLog:
    """A JSON-lines metrics file (opened for appending)."""

    def __init__(self, path, residual=True):
        self.path = path
        self.residual = residual
        self.t0 = time.perf_counter()
        self.f = open(path, "a", encoding="utf-8")

    def write(self, ctx, step=None, **extra):
        rec = {"step": int(ctx.get_step() if step is None else step),
               "time_s": round(time.perf_counter() - self.t0, 6),
               "systems": step_metrics(ctx, self.residual)}
        rec.update(extra)
        self.f.write(json.dumps(rec) + "\n")
        self.f.flush()
        return rec

    def close(self):
        if self.f:
            self.f.close()
            self.f = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run_logged(ctx, n_steps, log, mode, e_trial=0.0, every=1):
    """n_steps steps of ``ctx.run`` in chunks of ``every``, one log line after
    each chunk.  Returns the records written."""
    if every < 1:
        raise ValueError("every must be >= 1")
    recs = []
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        ctx.run(k, mode=mode, e_trial=e_trial)
        done += k
        recs.append(log.write(ctx))
    return recs
