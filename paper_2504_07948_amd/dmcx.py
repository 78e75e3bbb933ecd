"""ctypes binding of libdmcx.so (include/dmcx.h), argument marshalling only.

Every ``dmcx_*`` function below forwards to the C function of the same name.
Arrays are numpy (host, DMCX_HOST) or torch CUDA/HIP tensors (device,
DMCX_DEVICE; the pointer is ``tensor.data_ptr()``).  ``Context`` wraps a
handle for the common calls.  The library must have been built
(``paper_2504_07948_amd.build_ext.build()``); loading fails loudly otherwise:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmcx.so")

DMCX_OK, DMCX_E_INVALID, DMCX_E_NOMEM, DMCX_E_HIP, DMCX_E_SINGULAR, DMCX_E_NONFINITE, \
    DMCX_E_STATE, DMCX_E_UNSUPPORTED = range(8)
DMCX_FP64, DMCX_MIXED = 0, 1
DMCX_VMC, DMCX_DMC = 0, 1
DMCX_HOST, DMCX_DEVICE = 0, 1
DMCX_FLAG_GRAPH = 1
DMCX_FLAG_FP32_ENERGY = 2
DMCX_N_ESTIMATORS = 11
DMCX_NOALLOC_MAX_WALKERS = 1048576
DMCX_N_JASTROW_PARAMS = 8
DMCX_TILE_DEEP, DMCX_TILE_SHALLOW = 0, 1

EXPORTED = [
    "dmcx_create", "dmcx_destroy", "dmcx_set_walkers", "dmcx_get_walkers", "dmcx_set_step",
    "dmcx_get_step", "dmcx_set_ions", "dmcx_recompute", "dmcx_eval_orbitals", "dmcx_ratio_grad",
    "dmcx_accept", "dmcx_flush", "dmcx_run", "dmcx_measure", "dmcx_ion_grads", "dmcx_logpsi_vjp",
    "dmcx_potential_vjp", "dmcx_forces", "dmcx_potential", "dmcx_walker_flags", "dmcx_sync", "dmcx_last_run_timing",
    "dmcx_selftest", "dmcx_philox", "dmcx_strerror", "dmcx_last_error", "dmcx_autotune",
    "dmcx_autotune_report", "dmcx_get_delay_rank", "dmcx_reconfigure", "dmcx_estimators",
    "dmcx_zv_grads", "dmcx_forces_zv", "dmcx_estimators_noalloc",
    "dmcx_energy_escalations", "dmcx_set_et_feedback", "dmcx_get_trial_energy",
    "dmcx_jastrow_param_grads", "dmcx_linear_method", "dmcx_set_tile_shape",
    "dmcx_get_tile_shape", "dmcx_branch", "dmcx_set_walker_count", "dmcx_walker_count",
    "dmcx_inverse_residual", "dmcx_set_energy_escalation_cap",
]


class dmcx_system(C.Structure):
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


class dmcx_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("delay_rank", C.c_int32),
                ("recompute_period", C.c_int32), ("tau", C.c_double), ("seed", C.c_uint64),
                ("flags", C.c_uint32)]


_lib = None


def load():
    """Load libdmcx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2504_07948_amd.build_ext.build()")
    # PyTorch ships its own HIP runtime; when both live in one process, torch's
    # must initialise the device before this library's does, or torch later
    # finds no device.  Start it first when torch and a GPU are present.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "dmcx_create": [P, I32, P, P, P, P],
        "dmcx_destroy": [P],
        "dmcx_set_walkers": [P, P, P, I32],
        "dmcx_get_walkers": [P, P, P, I32],
        "dmcx_set_step": [P, I64],
        "dmcx_get_step": [P, P],
        "dmcx_set_ions": [P, I32, P, I32],
        "dmcx_recompute": [P],
        "dmcx_eval_orbitals": [P, I32, P, P, I32],
        "dmcx_ratio_grad": [P, I32, P, P, P, I32],
        "dmcx_accept": [P, I32, P, I32],
        "dmcx_flush": [P],
        "dmcx_run": [P, I32, I32, D, P, P, I32],
        "dmcx_measure": [P, P, P, P, I32],
        "dmcx_ion_grads": [P, P, P, I32],
        "dmcx_logpsi_vjp": [P, P, P, I32],
        "dmcx_potential_vjp": [P, P, P, I32],
        "dmcx_forces": [P, P, I32],
        "dmcx_potential": [P, P, I32],
        "dmcx_walker_flags": [P, P, I32],
        "dmcx_reconfigure": [P, P, P, P, I32],
        "dmcx_branch": [P, I64, P, P, I32],
        "dmcx_set_walker_count": [P, I32],
        "dmcx_walker_count": [P, P, P],
        "dmcx_inverse_residual": [P, P, I32],
        "dmcx_set_energy_escalation_cap": [P, D],
        "dmcx_sync": [P],
        "dmcx_last_run_timing": [P, P, P, P],
        "dmcx_selftest": [P],
        "dmcx_philox": [P, P, I32, P],
        "dmcx_strerror": [I32],
        "dmcx_last_error": [P],
        "dmcx_autotune": [P, I32, P],
        "dmcx_autotune_report": [P, I32, I32, P, P, P, P],
        "dmcx_set_tile_shape": [P, I32, I32],
        "dmcx_get_tile_shape": [P, I32, P],
        "dmcx_get_delay_rank": [P, I32, P],
        "dmcx_estimators": [P, P, I32],
        "dmcx_zv_grads": [P, I32, P, P, P, I32],
        "dmcx_forces_zv": [P, I32, P, I32],
        "dmcx_estimators_noalloc": [I32, P, P, P, P, P, P, P],
        "dmcx_energy_escalations": [P, P],
        "dmcx_set_et_feedback": [P, D],
        "dmcx_get_trial_energy": [P, P],
        "dmcx_jastrow_param_grads": [P, P, P, I32],
        "dmcx_linear_method": [P, P, P, I32],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I32
    lib.dmcx_destroy.restype = None
    lib.dmcx_strerror.restype = C.c_char_p
    lib.dmcx_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class DmcxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dmcx status {status}: {msg}")
        self.status = status


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def _mem(a):
    if a is None or isinstance(a, np.ndarray):
        return DMCX_HOST
    return DMCX_DEVICE if a.is_cuda else DMCX_HOST


# ---------------------------------------------------------- same names ----
def dmcx_create(sys_struct, n_sys, walkers_per_sys, opt, stream, out):
    return load().dmcx_create(sys_struct, n_sys, walkers_per_sys, opt, stream, out)


def dmcx_destroy(ctx):
    load().dmcx_destroy(ctx)


def dmcx_set_walkers(ctx, R, log_w, mem):
    return load().dmcx_set_walkers(ctx, R, log_w, mem)


def dmcx_get_walkers(ctx, R, log_w, mem):
    return load().dmcx_get_walkers(ctx, R, log_w, mem)


def dmcx_set_step(ctx, step):
    return load().dmcx_set_step(ctx, step)


def dmcx_get_step(ctx, step_ptr):
    return load().dmcx_get_step(ctx, step_ptr)


def dmcx_set_ions(ctx, sys_index, ion_xyz, mem):
    return load().dmcx_set_ions(ctx, sys_index, ion_xyz, mem)


def dmcx_recompute(ctx):
    return load().dmcx_recompute(ctx)


def dmcx_eval_orbitals(ctx, spin, r, vgl, mem):
    return load().dmcx_eval_orbitals(ctx, spin, r, vgl, mem)


def dmcx_ratio_grad(ctx, iel, r_new, ratio, grad, mem):
    return load().dmcx_ratio_grad(ctx, iel, r_new, ratio, grad, mem)


def dmcx_accept(ctx, iel, accept, mem):
    return load().dmcx_accept(ctx, iel, accept, mem)


def dmcx_flush(ctx):
    return load().dmcx_flush(ctx)


def dmcx_run(ctx, mode, n_steps, e_trial, accept_log, e_log, mem):
    return load().dmcx_run(ctx, mode, n_steps, e_trial, accept_log, e_log, mem)


def dmcx_measure(ctx, e_local, log_psi, sign, mem):
    return load().dmcx_measure(ctx, e_local, log_psi, sign, mem)


def dmcx_ion_grads(ctx, dlogpsi, dv, mem):
    return load().dmcx_ion_grads(ctx, dlogpsi, dv, mem)


def dmcx_logpsi_vjp(ctx, gbar, grad_R, mem):
    return load().dmcx_logpsi_vjp(ctx, gbar, grad_R, mem)


def dmcx_potential_vjp(ctx, gbar, grad_R, mem):
    return load().dmcx_potential_vjp(ctx, gbar, grad_R, mem)


def dmcx_forces(ctx, F, mem):
    return load().dmcx_forces(ctx, F, mem)


def dmcx_zv_grads(ctx, warp, dEL, dlogpsi, dlogjac, mem):
    return load().dmcx_zv_grads(ctx, warp, dEL, dlogpsi, dlogjac, mem)


def dmcx_forces_zv(ctx, warp, F, mem):
    return load().dmcx_forces_zv(ctx, warp, F, mem)


def dmcx_estimators(ctx, out, mem):
    return load().dmcx_estimators(ctx, out, mem)


def dmcx_estimators_noalloc(n_walkers, log_w, e_local, flags, n_accepted, n_proposed, out,
                            hip_stream):
    return load().dmcx_estimators_noalloc(n_walkers, log_w, e_local, flags, n_accepted,
                                          n_proposed, out, hip_stream)


def dmcx_energy_escalations(ctx, n):
    return load().dmcx_energy_escalations(ctx, n)


def dmcx_set_et_feedback(ctx, gain):
    return load().dmcx_set_et_feedback(ctx, gain)


def dmcx_get_trial_energy(ctx, e_trial):
    return load().dmcx_get_trial_energy(ctx, e_trial)


def dmcx_jastrow_param_grads(ctx, dlogpsi, dEL, mem):
    return load().dmcx_jastrow_param_grads(ctx, dlogpsi, dEL, mem)


def dmcx_linear_method(ctx, S, H, mem):
    return load().dmcx_linear_method(ctx, S, H, mem)


def dmcx_potential(ctx, v, mem):
    return load().dmcx_potential(ctx, v, mem)


def dmcx_walker_flags(ctx, flags, mem):
    return load().dmcx_walker_flags(ctx, flags, mem)


def dmcx_reconfigure(ctx, u, copies, log_wbar, mem):
    return load().dmcx_reconfigure(ctx, u, copies, log_wbar, mem)


def dmcx_branch(ctx, step, copies, n_walkers, mem):
    return load().dmcx_branch(ctx, step, copies, n_walkers, mem)


def dmcx_set_walker_count(ctx, n):
    return load().dmcx_set_walker_count(ctx, n)


def dmcx_walker_count(ctx, n, cap):
    return load().dmcx_walker_count(ctx, n, cap)


def dmcx_inverse_residual(ctx, res, mem):
    return load().dmcx_inverse_residual(ctx, res, mem)


def dmcx_set_energy_escalation_cap(ctx, cap):
    return load().dmcx_set_energy_escalation_cap(ctx, cap)


def dmcx_sync(ctx):
    return load().dmcx_sync(ctx)


def dmcx_last_run_timing(ctx, ms_avg, n, total):
    return load().dmcx_last_run_timing(ctx, ms_avg, n, total)


def dmcx_selftest(stream):
    return load().dmcx_selftest(stream)


def dmcx_philox(ctr, key, n, out):
    return load().dmcx_philox(ctr, key, n, out)


def dmcx_autotune(ctx, steps, chosen_k):
    return load().dmcx_autotune(ctx, steps, chosen_k)


def dmcx_autotune_report(ctx, sys_index, max_n, ranks, shapes, ms, n_cand):
    return load().dmcx_autotune_report(ctx, sys_index, max_n, ranks, shapes, ms, n_cand)


def dmcx_set_tile_shape(ctx, sys_index, shape):
    return load().dmcx_set_tile_shape(ctx, sys_index, shape)


def dmcx_get_tile_shape(ctx, sys_index, shape):
    return load().dmcx_get_tile_shape(ctx, sys_index, shape)


def dmcx_get_delay_rank(ctx, sys_index, k):
    return load().dmcx_get_delay_rank(ctx, sys_index, k)


def dmcx_strerror(status):
    return load().dmcx_strerror(status).decode()


def dmcx_last_error(ctx):
    return load().dmcx_last_error(ctx).decode()


# ------------------------------------------------------------- wrapper ----
class SystemStruct:
    """dmcx_system built from a synthetic system (keeps its arrays alive)."""

    def __init__(self, sys):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        k = dict(ion_xyz=f64(sys.ion_xyz), ion_charge=f64(sys.ion_charge),
                 shell_atom=i32(sys.shell_atom), shell_l=i32(sys.shell_l),
                 shell_nprim=i32(sys.shell_nprim), prim_alpha=f64(sys.prim_alpha),
                 prim_coef=f64(sys.prim_coef), mo_coef=f64(sys.mo_coef), jen_a=f64(sys.jen_a))
        n_det = int(getattr(sys, "n_det", 0) or 0)
        if n_det:
            k["det_exc"] = i32(sys.det_exc)
            k["ci_coef"] = f64(sys.ci_coef)
        n_pp = 0 if getattr(sys, "pp_atom", None) is None else len(sys.pp_atom)
        if n_pp:
            for name in ("pp_atom", "pp_l", "pp_n"):
                k[name] = i32(getattr(sys, name))
            for name in ("pp_beta", "pp_alpha", "pp_rcut"):
                k[name] = f64(getattr(sys, name))
        self.keep = k
        self.c = dmcx_system(
            n_atom=k["ion_xyz"].shape[0], ion_xyz=_ptr(k["ion_xyz"]),
            ion_charge=_ptr(k["ion_charge"]), n_shell=k["shell_l"].shape[0],
            shell_atom=_ptr(k["shell_atom"]), shell_l=_ptr(k["shell_l"]),
            shell_nprim=_ptr(k["shell_nprim"]), prim_alpha=_ptr(k["prim_alpha"]),
            prim_coef=_ptr(k["prim_coef"]), n_basis=k["mo_coef"].shape[0],
            n_mo=k["mo_coef"].shape[1], mo_coef=_ptr(k["mo_coef"]), n_up=sys.n_up,
            n_dn=sys.n_dn, jee_a_anti=sys.jee_a_anti, jee_a_para=sys.jee_a_para,
            jee_b=sys.jee_b, jen_a=_ptr(k["jen_a"]), jen_b=sys.jen_b, n_det=n_det,
            det_exc=_ptr(k.get("det_exc")), ci_coef=_ptr(k.get("ci_coef")),
            pp_n_term=n_pp, pp_atom=_ptr(k.get("pp_atom")), pp_l=_ptr(k.get("pp_l")),
            pp_n=_ptr(k.get("pp_n")), pp_beta=_ptr(k.get("pp_beta")),
            pp_alpha=_ptr(k.get("pp_alpha")), pp_rcut=_ptr(k.get("pp_rcut")))


class Context:
    """Owns one dmcx context for one or more systems."""

    def __init__(self, systems, walkers, precision=DMCX_FP64, delay_rank=32, recompute_period=64,
                 tau=0.01, seed=1, stream=None, graph=False, fp32_energy=False):
        if not isinstance(systems, (list, tuple)):
            systems = [systems]
            walkers = [walkers]
        self.systems = list(systems)
        self.structs = [SystemStruct(s) for s in systems]
        arr = (dmcx_system * len(systems))(*[s.c for s in self.structs])
        wps = np.ascontiguousarray(walkers, dtype=np.int32)
        self.W = int(wps.sum())
        self.ne = max(s.n_up + s.n_dn for s in systems)
        self.n_atom = max(s.n_atom for s in systems)
        self.n_sys = len(systems)
        self.walkers = [int(x) for x in wps]
        self.offsets = np.concatenate([[0], np.cumsum(wps)[:-1]]).astype(int).tolist()
        opt = dmcx_options(precision=precision, delay_rank=delay_rank,
                           recompute_period=recompute_period, tau=tau, seed=seed,
                           flags=(DMCX_FLAG_GRAPH if graph else 0)
                           | (DMCX_FLAG_FP32_ENERGY if fp32_energy else 0))
        h = C.c_void_p()
        st = load().dmcx_create(arr, len(systems), _ptr(wps), C.byref(opt), stream, C.byref(h))
        if st != DMCX_OK:
            raise DmcxError(st, "dmcx_create failed: " + dmcx_strerror(st))
        self.h = h
        self._keep = (arr, wps, opt)

    def close(self):
        if getattr(self, "h", None):
            load().dmcx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != DMCX_OK:
            raise DmcxError(st, dmcx_last_error(self.h) or dmcx_strerror(st))

    def set_walkers(self, R, log_w=None):
        if isinstance(R, np.ndarray):
            R = np.ascontiguousarray(R, dtype=np.float64)
            log_w = None if log_w is None else np.ascontiguousarray(log_w, dtype=np.float64)
        self.check(dmcx_set_walkers(self.h, _ptr(R), _ptr(log_w), _mem(R)))

    def get_walkers(self):
        R = np.zeros((self.W, self.ne, 3))
        lw = np.zeros(self.W)
        self.check(dmcx_get_walkers(self.h, _ptr(R), _ptr(lw), DMCX_HOST))
        return R, lw

    def set_step(self, step):
        """Set the step counter (the Philox step field of later draws, and
        the pseudopotential rotations of evaluations outside a run)."""
        self.check(dmcx_set_step(self.h, step))

    def run(self, n_steps, mode=DMCX_DMC, e_trial=0.0, logs=False):
        acc = np.zeros((n_steps, self.W, self.ne), dtype=np.uint8) if logs else None
        el = np.zeros((n_steps, self.W)) if logs else None
        self.check(dmcx_run(self.h, mode, n_steps, e_trial, _ptr(acc), _ptr(el), DMCX_HOST))
        return acc, el

    def run_device(self, n_steps, mode=DMCX_DMC, e_trial=0.0, accept_log=None, e_log=None):
        self.check(dmcx_run(self.h, mode, n_steps, e_trial, _ptr(accept_log), _ptr(e_log),
                            DMCX_DEVICE))

    def measure(self):
        e = np.zeros(self.W)
        lp = np.zeros(self.W)
        sg = np.zeros(self.W, dtype=np.int8)
        self.check(dmcx_measure(self.h, _ptr(e), _ptr(lp), _ptr(sg), DMCX_HOST))
        return e, lp, sg

    def recompute(self):
        self.check(dmcx_recompute(self.h))

    def eval_orbitals(self, spin, r):
        n = self.systems[0].n_up if spin == 0 else self.systems[0].n_dn
        out = np.zeros((self.W, 5, n))
        self.check(dmcx_eval_orbitals(self.h, spin, _ptr(np.ascontiguousarray(r, dtype=np.float64)),
                                      _ptr(out), DMCX_HOST))
        return out

    def ratio_grad(self, iel, r_new):
        r_new = np.ascontiguousarray(r_new, dtype=np.float64)
        ratio = np.zeros(self.W)
        grad = np.zeros((self.W, 3))
        self.check(dmcx_ratio_grad(self.h, iel, _ptr(r_new), _ptr(ratio), _ptr(grad), DMCX_HOST))
        return ratio, grad

    def accept(self, iel, mask):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.check(dmcx_accept(self.h, iel, _ptr(mask), DMCX_HOST))

    def flush(self):
        self.check(dmcx_flush(self.h))

    def potential(self):
        v = np.zeros(self.W)
        self.check(dmcx_potential(self.h, _ptr(v), DMCX_HOST))
        return v

    def set_ions(self, ion_xyz, sys_index=0):
        if isinstance(ion_xyz, np.ndarray):
            ion_xyz = np.ascontiguousarray(ion_xyz, dtype=np.float64)
        self.check(dmcx_set_ions(self.h, sys_index, _ptr(ion_xyz), _mem(ion_xyz)))

    def ion_grads(self):
        dl = np.zeros((self.W, self.n_atom, 3))
        dv = np.zeros((self.W, self.n_atom, 3))
        self.check(dmcx_ion_grads(self.h, _ptr(dl), _ptr(dv), DMCX_HOST))
        return dl, dv

    def _per_system(self):
        # [n_atom][3] for one system, [n_sys][n_atom_max][3] for a group
        return np.zeros((self.n_atom, 3) if self.n_sys == 1 else (self.n_sys, self.n_atom, 3))

    def logpsi_vjp(self, gbar):
        out = self._per_system()
        self.check(dmcx_logpsi_vjp(self.h, _ptr(np.ascontiguousarray(gbar, dtype=np.float64)),
                                   _ptr(out), DMCX_HOST))
        return out

    def potential_vjp(self, gbar):
        out = self._per_system()
        self.check(dmcx_potential_vjp(self.h, _ptr(np.ascontiguousarray(gbar, dtype=np.float64)),
                                      _ptr(out), DMCX_HOST))
        return out

    def forces(self):
        F = self._per_system()
        self.check(dmcx_forces(self.h, _ptr(F), DMCX_HOST))
        return F

    def zv_grads(self, warp=True):
        """Per-walker (dE_L/dR, d ln|Psi|/dR, d ln J/dR), [W][n_atom][3] each."""
        out = [np.zeros((self.W, self.n_atom, 3)) for _ in range(3)]
        self.check(dmcx_zv_grads(self.h, int(bool(warp)), *[_ptr(a) for a in out], DMCX_HOST))
        return tuple(out)

    def forces_zv(self, warp=True):
        F = self._per_system()
        self.check(dmcx_forces_zv(self.h, int(bool(warp)), _ptr(F), DMCX_HOST))
        return F

    def estimators(self):
        """[n_sys][DMCX_N_ESTIMATORS] weighted estimators (see include/dmcx.h)."""
        out = np.zeros((self.n_sys, DMCX_N_ESTIMATORS))
        self.check(dmcx_estimators(self.h, _ptr(out), DMCX_HOST))
        return out

    def set_et_feedback(self, gain):
        """E_T <- <E_L>_w - (gain/tau) ln(W_tot/W) after every DMC step (gain < 0: off)."""
        self.check(load().dmcx_set_et_feedback(self.h, float(gain)))

    def trial_energy(self):
        """E_T the next step would use, one per system."""
        out = np.zeros(self.n_sys)
        self.check(load().dmcx_get_trial_energy(self.h, _ptr(out)))
        return out

    def jastrow_param_grads(self):
        """Per walker (d ln Psi/dp, dE_L/dp) [W][8] each for the Jastrow
        parameters (e-e Pade b, e-n Pade b, six three-body coefficients);
        with a pseudopotential dE_L/dp includes the non-local energy's part
        (rotations of the current step counter)."""
        O = np.zeros((self.W, DMCX_N_JASTROW_PARAMS))
        D = np.zeros((self.W, DMCX_N_JASTROW_PARAMS))
        self.check(load().dmcx_jastrow_param_grads(self.h, _ptr(O), _ptr(D), DMCX_HOST))
        return O, D

    def linear_method(self):
        """Linear-method matrices (S, H), [n_sys][9][9] each."""
        n = DMCX_N_JASTROW_PARAMS + 1
        S = np.zeros((self.n_sys, n, n))
        H = np.zeros((self.n_sys, n, n))
        self.check(load().dmcx_linear_method(self.h, _ptr(S), _ptr(H), DMCX_HOST))
        return S, H

    def energy_escalations(self):
        """Walkers whose E_L the last energy evaluation took from FP64 rows."""
        n = C.c_int32(0)
        self.check(load().dmcx_energy_escalations(self.h, C.byref(n)))
        return int(n.value)

    def walker_flags(self):
        f = np.zeros(self.W, dtype=np.uint8)
        self.check(dmcx_walker_flags(self.h, _ptr(f), DMCX_HOST))
        return f

    def get_step(self):
        s = C.c_int64(0)
        self.check(dmcx_get_step(self.h, C.byref(s)))
        return int(s.value)

    def reconfigure(self, u):
        """Comb reconfiguration of each system's walkers (fixed population).
        u: comb offset(s) in [0, 1), one per system.  Returns (copies[W],
        log_wbar[n_sys])."""
        uu = np.ascontiguousarray(np.broadcast_to(np.asarray(u, dtype=np.float64), (self.n_sys,)))
        copies = np.zeros(self.W, dtype=np.int32)
        lwbar = np.zeros(self.n_sys)
        self.check(dmcx_reconfigure(self.h, _ptr(uu), _ptr(copies), _ptr(lwbar), DMCX_HOST))
        return copies, lwbar

    def branch(self, step):
        """Birth/death branching (one system): M_j = floor(w_j + u_j) copies
        of walker j.  Returns (copies[W before], W after).  Raises DmcxError
        when nothing would survive or the capacity would be exceeded (the
        population is then unchanged)."""
        copies = np.zeros(self.W, dtype=np.int32)
        n = C.c_int32(0)
        st = dmcx_branch(self.h, int(step), _ptr(copies), C.byref(n), DMCX_HOST)
        self.check(st)
        self._set_w(int(n.value))
        return copies, self.W

    def set_walker_count(self, n):
        """Set the walker count (1 .. capacity) of a one-system context;
        set_walkers must follow."""
        self.check(dmcx_set_walker_count(self.h, int(n)))
        self._set_w(int(n))

    def walker_count(self):
        n, cap = C.c_int32(0), C.c_int32(0)
        self.check(dmcx_walker_count(self.h, C.byref(n), C.byref(cap)))
        return int(n.value), int(cap.value)

    def set_energy_escalation_cap(self, cap):
        """Bound (Ha per electron) above which the mixed form's FP64 energy
        recomputes a walker's E_L from FP64 rows (0: every walker)."""
        self.check(dmcx_set_energy_escalation_cap(self.h, float(cap)))

    def inverse_residual(self):
        """[W][2] max_ij |A A^{-1} - I| of each walker's spin matrices (the
        stored inverse of the working precision)."""
        out = np.zeros((self.W, 2))
        self.check(dmcx_inverse_residual(self.h, _ptr(out), DMCX_HOST))
        return out

    def _set_w(self, n):
        self.W = n
        self.walkers = [n]

    def sync(self):
        self.check(dmcx_sync(self.h))

    def autotune(self, steps=2):
        k = np.zeros(self.n_sys, dtype=np.int32)
        self.check(dmcx_autotune(self.h, steps, _ptr(k)))
        return k

    def autotune_report(self, sys_index=0):
        """The tuner's candidates: (ranks, shapes, ms per sweep)."""
        r = np.zeros(32, dtype=np.int32)
        sh = np.zeros(32, dtype=np.int32)
        t = np.zeros(32, dtype=np.float32)
        n = C.c_int32()
        self.check(dmcx_autotune_report(self.h, sys_index, 32, _ptr(r), _ptr(sh), _ptr(t),
                                        C.byref(n)))
        return r[:n.value].copy(), sh[:n.value].copy(), t[:n.value].copy()

    def set_tile_shape(self, shape, sys_index=0):
        self.check(dmcx_set_tile_shape(self.h, sys_index, int(shape)))

    def tile_shape(self, sys_index=0):
        v = C.c_int32()
        self.check(dmcx_get_tile_shape(self.h, sys_index, C.byref(v)))
        return int(v.value)

    def delay_rank(self, sys_index=0):
        k = C.c_int32()
        self.check(dmcx_get_delay_rank(self.h, sys_index, C.byref(k)))
        return k.value

    def last_run_timing(self):
        a = C.c_double()
        n = C.c_int32()
        t = C.c_double()
        self.check(dmcx_last_run_timing(self.h, C.byref(a), C.byref(n), C.byref(t)))
        return a.value, n.value, t.value


def selftest(stream=None):
    return load().dmcx_selftest(stream)


def philox(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(ctr)
    st = load().dmcx_philox(_ptr(ctr), _ptr(key), ctr.shape[0], _ptr(out))
    if st != DMCX_OK:
        raise DmcxError(st, "dmcx_philox")
    return out
