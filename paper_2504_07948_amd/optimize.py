"""One step of the linear method for the Jastrow parameters, from the
matrices of ``dmcx_linear_method`` (host logic: a (1+P) x (1+P) generalised
eigenproblem; the walkers' derivatives and the matrices come from the GPU).

The paper optimises the Jastrow factor of Eq. 2 in VMC with a variant of
Umrigar's linear method (QMC section).  In the basis {Psi, (O_k - <O_k>) Psi}
the matrices S and H of the sample give the lowest eigenpair of
H c = E S c; the parameter change is c_k / c_0.  The variant here is the
published stabilisation: a shift added to the diagonal of H outside the
(0, 0) entry, which damps the step (Toulouse and Umrigar), raised until the
step's change of the wavefunction stays small.
"""
from __future__ import annotations

import math

import numpy as np


def _solve(Ss, Hs, shift):
    import scipy.linalg

    Hh = Hs.copy()
    Hh[1:, 1:] += shift * np.eye(Hs.shape[0] - 1)
    w, v = scipy.linalg.eig(Hh, Ss)
    for j in np.argsort(w.real):
        c = v[:, j].real
        if np.isfinite(w[j].real) and abs(c[0]) > 1e-12 * np.abs(c).max():
            return c[1:] / c[0], float(w[j].real)
    raise ValueError("linear method: no eigenvector with a usable c_0")


def linear_method_update(S, H, params=None, shift=1e-3, max_change=0.3):
    """Parameter change of one linear-method step.

    S, H: [1 + P][1 + P] (one system of ``Context.linear_method()``).
    params: indices (0-based, into the P parameters) to optimise; the
    others are held (their rows and columns are dropped).  The diagonal
    shift starts at ``shift`` and is raised fourfold until the linearised
    wavefunction changes by at most ``max_change`` in norm,
    sqrt(dp^T S dp) <= max_change (the linear expansion holds only for small
    changes of nonlinear parameters; a step beyond it can overshoot into
    an unphysical region).  Returns (dp [len(params)], E): the change of
    those parameters and the lowest eigenvalue of the shifted problem.
    Raises ValueError when no eigenvector has a usable c_0 (|c_0| below
    1e-12 of the vector's largest entry).
    """
    S = np.asarray(S, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    P = S.shape[0] - 1
    idx = np.arange(P) if params is None else np.asarray(params, dtype=int)
    keep = np.concatenate(([0], 1 + idx))
    Ss = S[np.ix_(keep, keep)]
    Hs = H[np.ix_(keep, keep)]
    a = shift
    for _ in range(40):
        dp, E = _solve(Ss, Hs, a)
        if max_change is None or math.sqrt(max(dp @ Ss[1:, 1:] @ dp, 0.0)) <= max_change:
            return dp, E
        a = 4.0 * a if a > 0.0 else 1e-4
    return dp, E
