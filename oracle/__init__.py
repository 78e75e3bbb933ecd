"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports or links
this package, and this package imports nothing from the product.  Systems are
passed as any object with the attributes of a seeded synthetic system
(ion_xyz, shell tables, mo_coef, n_up, n_dn, Jastrow parameters).

Every function here follows a passage of the paper (arXiv 2504.07948, QMC
section); see oracle.c for the mapping (Eq. 1-3).  Parity is pinned by the
CPU tests against direct determinants, finite differences, closed forms and
the zero-variance hydrogen-like case.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [
        ("n_atom", C.c_int32), ("ion_xyz", C.c_void_p), ("ion_charge", C.c_void_p),
        ("n_shell", C.c_int32), ("shell_atom", C.c_void_p), ("shell_l", C.c_void_p),
        ("shell_nprim", C.c_void_p), ("prim_alpha", C.c_void_p), ("prim_coef", C.c_void_p),
        ("n_basis", C.c_int32), ("n_mo", C.c_int32), ("mo_coef", C.c_void_p),
        ("n_up", C.c_int32), ("n_dn", C.c_int32),
        ("jee_a_anti", C.c_double), ("jee_a_para", C.c_double), ("jee_b", C.c_double),
        ("jen_a", C.c_void_p), ("jen_b", C.c_double),
        ("n_det", C.c_int32), ("det_exc", C.c_void_p), ("ci_coef", C.c_void_p),
        ("pp_n_term", C.c_int32), ("pp_atom", C.c_void_p), ("pp_l", C.c_void_p),
        ("pp_n", C.c_void_p), ("pp_beta", C.c_void_p), ("pp_alpha", C.c_void_p),
        ("pp_rcut", C.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_basis_vgl.argtypes = [P, P, P]
        lib.orc_orbitals_vgl.argtypes = [P, P, C.c_int32, P]
        lib.orc_lu_slogdet_inv.argtypes = [C.c_int32, P, P, P, P]
        lib.orc_jastrow.argtypes = [P, P, P, P, P]
        lib.orc_potential.argtypes = [P, P]
        lib.orc_potential.restype = C.c_double
        lib.orc_evaluate.argtypes = [P, P, P, P, P, P]
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox4x32_10.restype = None
        lib.orc_move_draws.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, P, P]
        lib.orc_move_draws.restype = None
        lib.orc_run.argtypes = [P, C.c_int32, P, P, P, C.c_int64, C.c_int32, C.c_int32,
                                C.c_double, C.c_uint64, C.c_double, C.c_int32, P, P, C.c_int32]
        lib.orc_run_feedback.argtypes = [P, C.c_int32, P, P, P, C.c_int64, C.c_int32, C.c_double,
                                         C.c_uint64, C.c_double, C.c_double, C.c_int32,
                                         C.c_int32, P, P, P, P, C.c_int32]
        lib.orc_ion_grads.argtypes = [P, P, P, P]
        lib.orc_ion_grads_batch.argtypes = [P, C.c_int32, P, P, P, C.c_int32]
        lib.orc_evaluate_batch.argtypes = [P, C.c_int32, P, P, P, P, C.c_int32]
        lib.orc_msd_ratio_direct.argtypes = [P, P, P]
        lib.orc_reconfigure.argtypes = [C.c_int32, P, C.c_double, P, P, P, P]
        lib.orc_branch.argtypes = [C.c_int32, P, P, C.c_uint64, C.c_int64, C.c_int32, P, P, P, P]
        lib.orc_local_energy_dir.argtypes = [P, P, P, P, P, P]
        lib.orc_zv_grads.argtypes = [P, P, C.c_int32, P, P, P]
        lib.orc_zv_grads_batch.argtypes = [P, C.c_int32, P, C.c_int32, P, P, P, C.c_int32]
        lib.orc_basis_d3.argtypes = [P, P, P]
        lib.orc_warp_weights.argtypes = [P, P, P, P]
        lib.orc_jastrow_param_grads.argtypes = [P, P, P, P]
        lib.orc_jastrow_param_grads_batch.argtypes = [P, C.c_int32, P, P, P, C.c_int32]
        lib.orc_j3_values.argtypes = [P, P, P]
        lib.orc_nlpp.argtypes = [P, P, C.c_uint64, C.c_int64, C.c_int32, P]
        lib.orc_nlpp_param_grads.argtypes = [P, P, C.c_uint64, C.c_int64, C.c_int32, P]
        lib.orc_nlpp_batch.argtypes = [P, C.c_int32, P, C.c_uint64, C.c_int64, C.c_int32, P,
                                       C.c_int32]
        lib.orc_nlpp_rotation.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, P]
        lib.orc_pp_ion_grads.argtypes = [P, P, C.c_uint64, C.c_int64, C.c_int32, P]
        lib.orc_nlpp_rotation.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class OracleSystem:
    """Holds contiguous copies of a system's arrays and the C struct."""

    def __init__(self, sys):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self.sys = sys
        self.keep = dict(
            ion_xyz=f64(sys.ion_xyz), ion_charge=f64(sys.ion_charge), shell_atom=i32(sys.shell_atom),
            shell_l=i32(sys.shell_l), shell_nprim=i32(sys.shell_nprim), prim_alpha=f64(sys.prim_alpha),
            prim_coef=f64(sys.prim_coef), mo_coef=f64(sys.mo_coef), jen_a=f64(sys.jen_a))
        n_det = int(getattr(sys, "n_det", 0) or 0)
        if n_det:
            self.keep["det_exc"] = i32(sys.det_exc)
            self.keep["ci_coef"] = f64(sys.ci_coef)
        k = self.keep
        n_pp = 0 if getattr(sys, "pp_atom", None) is None else len(sys.pp_atom)
        if n_pp:
            for name in ("pp_atom", "pp_l", "pp_n"):
                k[name] = i32(getattr(sys, name))
            for name in ("pp_beta", "pp_alpha", "pp_rcut"):
                k[name] = f64(getattr(sys, name))
        self.c = _Sys(
            n_atom=k["ion_xyz"].shape[0], ion_xyz=_ptr(k["ion_xyz"]), ion_charge=_ptr(k["ion_charge"]),
            n_shell=k["shell_l"].shape[0], shell_atom=_ptr(k["shell_atom"]), shell_l=_ptr(k["shell_l"]),
            shell_nprim=_ptr(k["shell_nprim"]), prim_alpha=_ptr(k["prim_alpha"]),
            prim_coef=_ptr(k["prim_coef"]), n_basis=k["mo_coef"].shape[0], n_mo=k["mo_coef"].shape[1],
            mo_coef=_ptr(k["mo_coef"]), n_up=sys.n_up, n_dn=sys.n_dn, jee_a_anti=sys.jee_a_anti,
            jee_a_para=sys.jee_a_para, jee_b=sys.jee_b, jen_a=_ptr(k["jen_a"]), jen_b=sys.jen_b,
            n_det=n_det, det_exc=_ptr(k.get("det_exc")), ci_coef=_ptr(k.get("ci_coef")),
            pp_n_term=n_pp, pp_atom=_ptr(k.get("pp_atom")), pp_l=_ptr(k.get("pp_l")),
            pp_n=_ptr(k.get("pp_n")), pp_beta=_ptr(k.get("pp_beta")),
            pp_alpha=_ptr(k.get("pp_alpha")), pp_rcut=_ptr(k.get("pp_rcut")))
        self.n_elec = sys.n_up + sys.n_dn
        self.n_atom = k["ion_xyz"].shape[0]
        self.n_basis = k["mo_coef"].shape[0]

    @property
    def ref(self):
        return C.byref(self.c)


def _osys(sys):
    return sys if isinstance(sys, OracleSystem) else OracleSystem(sys)


def basis_vgl(sys, r):
    o = _osys(sys)
    out = np.zeros((o.n_basis, 5))
    rc = _load().orc_basis_vgl(o.ref, _ptr(np.ascontiguousarray(r, dtype=np.float64)), _ptr(out))
    assert rc == 0
    return out


def orbitals_vgl(sys, r, n_orb):
    o = _osys(sys)
    out = np.zeros((5, n_orb))
    rc = _load().orc_orbitals_vgl(o.ref, _ptr(np.ascontiguousarray(r, dtype=np.float64)), n_orb,
                                  _ptr(out))
    assert rc == 0
    return out


def lu_slogdet_inv(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    ld = C.c_double()
    sg = C.c_int32()
    inv = np.zeros_like(A)
    rc = _load().orc_lu_slogdet_inv(n, _ptr(A), C.byref(ld), C.byref(sg), _ptr(inv))
    return int(sg.value), float(ld.value), inv, rc


def jastrow(sys, R):
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    J = C.c_double()
    g = np.zeros((o.n_elec, 3))
    l = np.zeros(o.n_elec)
    _load().orc_jastrow(o.ref, _ptr(R), C.byref(J), _ptr(g), _ptr(l))
    return float(J.value), g, l


def potential(sys, R):
    o = _osys(sys)
    return float(_load().orc_potential(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64))))


def evaluate(sys, R):
    """-> (log|Psi|, sign, E_L, drift[n_elec,3]) at one configuration."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    lp = C.c_double()
    sg = C.c_int32()
    el = C.c_double()
    dr = np.zeros((o.n_elec, 3))
    rc = _load().orc_evaluate(o.ref, _ptr(R), C.byref(lp), C.byref(sg), C.byref(el), _ptr(dr))
    return float(lp.value), int(sg.value), float(el.value), dr, rc


def evaluate_batch(sys, R, n_threads=0):
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    W = R.shape[0]
    lp = np.zeros(W)
    sg = np.zeros(W, dtype=np.int32)
    el = np.zeros(W)
    rc = _load().orc_evaluate_batch(o.ref, W, _ptr(R), _ptr(lp), _ptr(sg), _ptr(el), n_threads)
    return lp, sg, el, rc


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def move_draws(seed, step, walker, elec):
    chi = np.zeros(3)
    u = C.c_double()
    _load().orc_move_draws(seed, step, walker, elec, _ptr(chi), C.byref(u))
    return chi, float(u.value)


def run(sys, R, log_w=None, step0=0, n_steps=1, mode=1, tau=0.01, seed=1, e_trial=0.0,
        walker_offset=0, want_logs=True, n_threads=0):
    """Run n_steps sweeps on a copy of R. mode 0 = VMC, 1 = DMC.
    Returns dict(R, log_w, e_local, accept_log[n_steps,W,ne], e_log[n_steps,W])."""
    o = _osys(sys)
    R = np.array(R, dtype=np.float64, copy=True, order="C")
    W = R.shape[0]
    lw = np.zeros(W) if log_w is None else np.array(log_w, dtype=np.float64, copy=True)
    el = np.zeros(W)
    acc = np.zeros((n_steps, W, o.n_elec), dtype=np.uint8) if want_logs else None
    elog = np.zeros((n_steps, W)) if want_logs else None
    rc = _load().orc_run(o.ref, W, _ptr(R), _ptr(lw), _ptr(el), step0, n_steps, mode, tau, seed,
                         e_trial, walker_offset, _ptr(acc), _ptr(elog), n_threads)
    return dict(R=R, log_w=lw, e_local=el, accept_log=acc, e_log=elog, rc=rc)


def run_feedback(sys, R, log_w=None, step0=0, n_steps=1, tau=0.01, seed=1, e_trial=0.0, gain=0.5,
                 walker_offset=0, n_threads=0, target=0):
    """DMC steps with E_T fed back from the population after every step (see
    orc_run_feedback; target: the target population, 0 for the walker
    count).  Returns dict(R, log_w, e_local, accept_log, e_log,
    et_log[n_steps] (the E_T each step used), e_trial (the next one))."""
    o = _osys(sys)
    R = np.array(R, dtype=np.float64, copy=True, order="C")
    W = R.shape[0]
    lw = np.zeros(W) if log_w is None else np.array(log_w, dtype=np.float64, copy=True)
    el = np.zeros(W)
    acc = np.zeros((n_steps, W, o.n_elec), dtype=np.uint8)
    elog = np.zeros((n_steps, W))
    etlog = np.zeros(n_steps)
    et = C.c_double()
    rc = _load().orc_run_feedback(o.ref, W, _ptr(R), _ptr(lw), _ptr(el), step0, n_steps, tau,
                                  seed, e_trial, gain, target, walker_offset, _ptr(acc),
                                  _ptr(elog),
                                  _ptr(etlog), C.byref(et), n_threads)
    return dict(R=R, log_w=lw, e_local=el, accept_log=acc, e_log=elog, et_log=etlog,
                e_trial=float(et.value), rc=rc)


def ion_grads(sys, R):
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    dl = np.zeros((o.n_atom, 3))
    dv = np.zeros((o.n_atom, 3))
    rc = _load().orc_ion_grads(o.ref, _ptr(R), _ptr(dl), _ptr(dv))
    return dl, dv, rc


def ion_grads_batch(sys, R, n_threads=0):
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    W = R.shape[0]
    dl = np.zeros((W, o.n_atom, 3))
    dv = np.zeros((W, o.n_atom, 3))
    rc = _load().orc_ion_grads_batch(o.ref, W, _ptr(R), _ptr(dl), _ptr(dv), n_threads)
    return dl, dv, rc


def msd_ratio_direct(sys, R):
    o = _osys(sys)
    out = C.c_double()
    _load().orc_msd_ratio_direct(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)),
                                 C.byref(out))
    return float(out.value)


def reconfigure(log_w, u):
    """Comb reconfiguration at fixed population (see oracle.h).
    Returns (copies[W] int32, pairs[n, 2] (destination, source), log_wbar, rc)."""
    lw = np.ascontiguousarray(log_w, dtype=np.float64)
    W = lw.shape[0]
    copies = np.zeros(W, dtype=np.int32)
    pairs = np.zeros((max(W, 1), 2), dtype=np.int32)
    n = C.c_int32(0)
    lwbar = C.c_double(0.0)
    rc = _load().orc_reconfigure(W, _ptr(lw), float(u), _ptr(copies), _ptr(pairs), C.byref(n),
                                 C.byref(lwbar))
    return copies, pairs[: n.value].copy(), float(lwbar.value), rc


def estimators(log_w, e_local, flags=None, n_accepted=0, n_proposed=0):
    """Weighted walker estimators of the fixed-node DMC population (QMC section,
    Eq. 1: each walker carries the weight w = exp(log w)), written out from their
    definitions with numpy.  A walker counts when log w and E_L are finite and its
    status flag (if given) is zero.  m is the largest counted log w and
    omega = exp(log w - m).  Returns the 11 numbers
      [n, m, sum omega, sum omega E, sum omega E^2, sum omega^2,
       <E> = sum omega E / sum omega,
       var = sum omega (E - <E>)^2 / sum omega,
       min log w, accepted / proposed, proposed]
    (NaN where undefined).  The move counts are passed in: they are counts of the
    accept decisions of the run, not arithmetic of the method."""
    lw = np.asarray(log_w, dtype=np.float64)
    e = np.asarray(e_local, dtype=np.float64)
    ok = np.isfinite(lw) & np.isfinite(e)
    if flags is not None:
        ok &= np.asarray(flags) == 0
    nan = float("nan")
    acc = float(n_accepted) / float(n_proposed) if n_proposed else nan
    if not ok.any():
        return np.array([0.0, nan, nan, nan, nan, nan, nan, nan, nan, acc, float(n_proposed)])
    lw, e = lw[ok], e[ok]
    m = lw.max()
    om = np.exp(lw - m)
    s0 = om.sum()
    mean = (om * e).sum() / s0
    var = (om * (e - mean) ** 2).sum() / s0
    return np.array([float(ok.sum()), m, s0, (om * e).sum(), (om * e * e).sum(), (om * om).sum(),
                     mean, var, lw.min(), acc, float(n_proposed)])


def basis_d3(sys, r):
    """Basis value, gradient, Hessian (xx, xy, xz, yy, yz, zz), Laplacian and
    gradient of the Laplacian at r: [n_basis][14]."""
    o = _osys(sys)
    out = np.zeros((o.n_basis, 14))
    _load().orc_basis_d3(o.ref, _ptr(np.ascontiguousarray(r, dtype=np.float64)), _ptr(out))
    return out


def warp_weights(sys, r):
    """Space-warp weights omega_a(r) [n_atom] and their gradients [n_atom][3]."""
    o = _osys(sys)
    om = np.zeros(o.n_atom)
    dom = np.zeros((o.n_atom, 3))
    _load().orc_warp_weights(o.ref, _ptr(np.ascontiguousarray(r, dtype=np.float64)), _ptr(om),
                             _ptr(dom))
    return om, dom


def local_energy_dir(sys, R, dion, del_):
    """Eq. 4 derivative of E_L and Eq. 3 derivative of ln|Psi| along the
    direction (ion displacements dion [n_atom][3], electron displacements
    del_ [n_elec][3]).  Returns (dE_L, dln|Psi|, rc)."""
    o = _osys(sys)
    de = C.c_double()
    dl = C.c_double()
    rc = _load().orc_local_energy_dir(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)),
                                      _ptr(np.ascontiguousarray(dion, dtype=np.float64)),
                                      _ptr(np.ascontiguousarray(del_, dtype=np.float64)),
                                      C.byref(de), C.byref(dl))
    return float(de.value), float(dl.value), rc


def zv_grads_batch(sys, R, warp, n_threads=0):
    """Per walker and ion coordinate: dE_L, d ln|Psi| and d ln(Jacobian)
    [W][n_atom][3] each, along the ion displacement alone (warp=False) or with
    the space warp (warp=True)."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    W = R.shape[0]
    de = np.zeros((W, o.n_atom, 3))
    dl = np.zeros((W, o.n_atom, 3))
    dj = np.zeros((W, o.n_atom, 3))
    rc = _load().orc_zv_grads_batch(o.ref, W, _ptr(R), int(bool(warp)), _ptr(de), _ptr(dl),
                                    _ptr(dj), n_threads)
    return de, dl, dj, rc


def zv_force_estimator(log_w, e_local, dEL, dlogpsi, dlogjac):
    """F = -<dE_L> - <(E_L - <E_L>)(2 dln|Psi| + dln J)> over the walkers,
    weights exp(log w - max) (zero-variance force with the Pulay covariance;
    dln J = 0 without the space warp).  Walkers with a non-finite log w or E_L
    are left out."""
    lw = np.asarray(log_w, dtype=np.float64)
    e = np.asarray(e_local, dtype=np.float64)
    ok = np.isfinite(lw) & np.isfinite(e)
    om = np.exp(lw[ok] - lw[ok].max())
    om /= om.sum()
    mean = lambda x: np.einsum("w,w...->...", om, np.asarray(x)[ok])
    em = mean(e)
    de = e - em
    return -mean(dEL) - mean(de[:, None, None] * (2.0 * np.asarray(dlogpsi) + np.asarray(dlogjac)))


# the Jastrow parameters whose derivatives jastrow_param_grads returns
JASTROW_PARAMS = ("b_ee", "b_en", "c3_110", "c3_101", "c3_111", "c3_210", "c3_201", "c3_102")


def jastrow_param_grads(sys, R):
    """O_p = d ln Psi / dp and dE_L / dp for the eight Jastrow parameters
    (JASTROW_PARAMS: the two Pade b, then six three-body e-e-n coefficients at
    zero) at one configuration R [n_elec][3].  Returns (O[8], dEL[8], rc)."""
    o = _osys(sys)
    O = np.zeros(8)
    D = np.zeros(8)
    rc = _load().orc_jastrow_param_grads(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)),
                                         _ptr(O), _ptr(D))
    return O, D, rc


def jastrow_param_grads_batch(sys, R, n_threads=0):
    """The same for a crowd R [W][n_elec][3]: O [W][8], dEL [W][8], rc."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    W = R.shape[0]
    O = np.zeros((W, 8))
    D = np.zeros((W, 8))
    rc = _load().orc_jastrow_param_grads_batch(o.ref, W, _ptr(R), _ptr(O), _ptr(D), n_threads)
    return O, D, rc


def j3_values(sys, R):
    """The six three-body sums F_k(R) = sum_A sum_{i<j} (s_iA^l s_jA^m +
    s_iA^m s_jA^l) s_ij^n, s(r) = r / (1 + r)."""
    o = _osys(sys)
    F = np.zeros(6)
    _load().orc_j3_values(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)), _ptr(F))
    return F


def linear_method(log_w, e_local, O, dEL, flags=None):
    """Linear-method matrices of the parameter derivatives (the first step of
    the Jastrow optimisation), over the walkers with weights
    omega = exp(log w - max), normalised; walkers with a non-finite log w or
    E_L, or a non-zero flag, are left out.  With <.> the weighted mean,
    dO_k = O_k - <O_k> and the basis {Psi, dO_k Psi}:
      S[0][0] = 1, S[0][k] = S[k][0] = 0, S[k][l] = <dO_k dO_l>,
      H[0][0] = <E_L>, H[k][0] = <dO_k E_L>,
      H[0][l] = <E_L dO_l> + <dE_L/dp_l>,
      H[k][l] = <dO_k (dO_l E_L + dE_L/dp_l)>.
    Returns (S, H), each [1 + P][1 + P]."""
    lw = np.asarray(log_w, dtype=np.float64)
    e = np.asarray(e_local, dtype=np.float64)
    O = np.asarray(O, dtype=np.float64)
    D = np.asarray(dEL, dtype=np.float64)
    ok = np.isfinite(lw) & np.isfinite(e)
    if flags is not None:
        ok &= np.asarray(flags) == 0
    P = O.shape[1]
    S = np.zeros((1 + P, 1 + P))
    H = np.zeros((1 + P, 1 + P))
    om = np.exp(lw[ok] - lw[ok].max())
    om /= om.sum()
    e, O, D = e[ok], O[ok], D[ok]
    mean = lambda x: np.einsum("w,w...->...", om, x)
    dO = O - mean(O)
    S[0, 0] = 1.0
    S[1:, 1:] = mean(dO[:, :, None] * dO[:, None, :])
    H[0, 0] = mean(e)
    H[1:, 0] = mean(dO * e[:, None])
    H[0, 1:] = mean(e[:, None] * dO) + mean(D)
    H[1:, 1:] = mean(dO[:, :, None] * (dO[:, None, :] * e[:, None, None] + D[:, None, :]))
    return S, H


def nlpp(sys, R, seed, step, walker):
    """Non-local pseudopotential energy of one walker at R [n_elec][3], with
    the quadrature rotations of (electron, walker, step) under key seed.
    Returns (v_nl, rc)."""
    o = _osys(sys)
    v = C.c_double()
    rc = _load().orc_nlpp(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)), seed, step,
                          walker, C.byref(v))
    return float(v.value), rc


def nlpp_param_grads(sys, R, seed, step, walker):
    """d V_NL / dp [8] for the Jastrow parameter directions (the non-local
    part of dE_L/dp) at fixed rotations.  Returns (dv, rc)."""
    o = _osys(sys)
    dv = np.zeros(8)
    rc = _load().orc_nlpp_param_grads(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)),
                                      seed, step, walker, _ptr(dv))
    return dv, rc


def nlpp_batch(sys, R, seed, step, walker_offset=0, n_threads=0):
    """The same for a crowd R [W][n_elec][3], walker w with index offset + w."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, dtype=np.float64)
    v = np.zeros(R.shape[0])
    rc = _load().orc_nlpp_batch(o.ref, R.shape[0], _ptr(R), seed, step, walker_offset, _ptr(v),
                                n_threads)
    return v, rc


def nlpp_rotation(seed, step, walker, elec):
    """The random rotation [3][3] of one electron's quadrature."""
    rot = np.zeros(9)
    _load().orc_nlpp_rotation(seed, step, walker, elec, _ptr(rot))
    return rot.reshape(3, 3)


def pp_ion_grads(sys, R, seed, step, walker):
    """d(V_loc + V_NL)/dR_A [n_atom][3] at fixed electrons, rotations and
    Psi: the pseudopotential's Hellmann-Feynman force term.  Returns (g, rc)."""
    o = _osys(sys)
    g = np.zeros((o.n_atom, 3))
    rc = _load().orc_pp_ion_grads(o.ref, _ptr(np.ascontiguousarray(R, dtype=np.float64)), seed,
                                  step, walker, _ptr(g))
    return g, rc


def branch(log_w, seed, step, cap, flags=None):
    """Birth/death branching: (copies [W], pairs [n][2] (destination,
    source), W', rc)."""
    lw = np.ascontiguousarray(log_w, dtype=np.float64)
    W = lw.shape[0]
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    copies = np.zeros(W, dtype=np.int32)
    pairs = np.zeros((W + cap + 1, 2), dtype=np.int32)
    n = C.c_int32()
    wn = C.c_int32()
    rc = _load().orc_branch(W, _ptr(lw), _ptr(fl), seed, step, cap, _ptr(copies), _ptr(pairs),
                            C.byref(n), C.byref(wn))
    return copies, pairs[: n.value].copy(), int(wn.value), rc
