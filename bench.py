"""Benchmark: electron-moves/s of the DMC step on one MI355X.

Workload (default): the 112-electron, 64-atom, 1024-function synthetic
system, 2048 walkers, FP64, delayed rank k = 32, FP64 inverse recompute
every 64 steps, tau = 0.01.  One step = one full sweep (every electron of
every walker proposes one drift-diffusion move, fixed-node Metropolis test,
delayed inverse update with rank-k flushes), then local energies and DMC
weights, plus the periodic recompute.  Inputs are resident in HBM before the
timed region; the timed region is exactly --steps steps bracketed by
torch.cuda.synchronize().

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (the sweep kernel, timed with HIP events on the stream it runs on)
and the CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3

# HBM traffic of one sweep launch, from two counter passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) over the default FP64 workload, each scaled by
# what the same counter reads for a 512 MiB device copy (fetch x 2.0, write x
# 1.0).  Reported only while the kernel sources and their compiler flags hash
# to the value they had when the counters were taken, and only for that workload.
SWEEP_TRAFFIC = {
    "sources_sha256": "54412998c6fb32f0cdbbc37d7c756552b1d8cab23aec0cc346cf73776b24ab7b",
    "workload": {"walkers": 2048, "delay": 32, "precision": "fp64"},
    "fetch_bytes": 3.2659e+09,
    "write_bytes": 2.7239e+09,
}


# the sources the FP64 sweep kernel is compiled from (the host runtime is not);
# its flags are hashed with them
SWEEP_SOURCES = ("device_common.h", "kernels.h", "launch.h", "sweep_impl.h", "sweep_f64.hip")


def kernel_sources_sha256():
    """Hash of the FP64 sweep's sources and of the compiler flags they are
    built with (a scheduler flag changes the code as much as an edit)."""
    import hashlib
    from paper_2504_07948_amd import build_ext
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2504_07948_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(build_ext.HIPCC_FLAGS + build_ext.SOURCE_FLAGS.get("sweep_f64.hip", [])).encode())
    return h.hexdigest()


def host_cpu_info():
    """Sockets, physical cores and logical CPUs of the host, and the CPUs this
    process may run on."""
    info = {"logical_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}
    try:
        phys, cores = set(), set()
        pid = cid = None
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("physical id"):
                    pid = line.split(":")[1].strip()
                    phys.add(pid)
                elif line.startswith("core id"):
                    cid = line.split(":")[1].strip()
                    cores.add((pid, cid))
                elif line.startswith("model name") and "model" not in info:
                    info["model"] = line.split(":", 1)[1].strip()
        info["sockets"] = len(phys) or None
        info["physical_cores"] = len(cores) or None
    except OSError:
        pass
    return info


def flops_per_move(n_basis, n_prim, n_sigma, n_elec, n_atom, k):
    """Algorithmic FLOP per proposed single-electron move:
    MO VGL contraction 2*5*N_b*N_s, basis assembly ~20*N_b plus one per
    primitive exponential, ratio/drift dots 14*N_s, block Sherman-Morrison
    updates 2*N_s*(k-1) (per accepted move, counted per move), amortised
    rank-k flush 4*N_s^2 + 2*k*N_s, Jastrow sums 40*(N_e + N_atom)."""
    return (2 * 5 * n_basis * n_sigma + 20 * n_basis + n_prim + 14 * n_sigma
            + 2 * n_sigma * max(k - 1, 0) + 4 * n_sigma ** 2 + 2 * k * n_sigma
            + 40 * (n_elec + n_atom))


def _timed_ctx(s, torch, dmcx, stream, W, steps, seed, **kw):
    """Context on W walkers of s, one warm-up step, then `steps` timed steps;
    returns (ctx, ms per step, sweep kernel ms)."""
    from paper_2504_07948_amd import synth
    R0 = synth.make_walkers(s, W, 2026)
    ctx = dmcx.Context(s, W, tau=0.01, seed=seed, stream=stream, **kw)
    ctx.set_walkers(torch.from_numpy(R0).cuda())
    e0, _, _ = ctx.measure()
    e_t = float(np.mean(e0[np.isfinite(e0)]))
    ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_device(steps, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_sweep, _, _ = ctx.last_run_timing()
    return ctx, dt * 1e3 / steps, ms_sweep


def _energy_errors(s, torch, dmcx, stream, ctx, W):
    """E_L and log|Psi| of ctx against the FP64 GPU path (held to the oracle
    within 1e-10 by the tests) at ctx's own configurations."""
    Rm, _ = ctx.get_walkers()
    em, lpm, _ = ctx.measure()
    ref = dmcx.Context(s, W, precision=dmcx.DMCX_FP64, stream=stream)
    ref.set_walkers(torch.from_numpy(Rm).cuda())
    ef, lpf, _ = ref.measure()
    ref.close()
    ok = np.isfinite(em) & np.isfinite(ef)
    de = (em - ef)[ok]
    dl = (lpm - lpf)[ok]
    return {"e_err_per_electron_mean": float(abs(de.mean()) / s.n_elec),
            "e_err_per_electron_median_walker": float(np.median(np.abs(de)) / s.n_elec),
            "e_err_per_electron_rms_walker": float(np.sqrt(np.mean(de ** 2)) / s.n_elec),
            "e_err_per_electron_max_walker": float(np.abs(de).max() / s.n_elec),
            "logpsi_err_median": float(np.median(np.abs(dl))),
            "logpsi_err_max": float(np.abs(dl).max())}


def mixed_leg(s, torch, dmcx, stream, args, W=4096, steps=10, P=32):
    """Mixed precision on the same system at 4096 walkers against FP64 at the
    same 4096 walkers, each with the sweep's tile shape and delay rank chosen
    by the autotuner in its warm-up step (ranks 8..56 of the 56 orbitals per
    spin; the FP32 sweep offers two tile shapes, the FP64 sweep one).  Two
    mixed forms: the default (FP32 sweep, FP64 value rows, inverse and E_L at
    the end of every step) and the FP32-energy variant (E_L from the FP32
    rows and inverse, FP64 recompute every 32 steps).  Reports moves/s and ms
    per step of each, the speedup over FP64 at equal walker count, the FP32
    sweep kernel's fraction of the FP32 peak, and the energy error per
    electron at identical configurations."""
    ne, ns = s.n_elec, max(s.n_up, s.n_dn)
    c64, ms64, sw64 = _timed_ctx(s, torch, dmcx, stream, W, steps, 19, precision=dmcx.DMCX_FP64,
                                 delay_rank=0, recompute_period=64)
    k64 = c64.delay_rank()
    c64.close()
    out = {"walkers": W, "steps": steps, "unit": "electron-moves/s",
           "fp64_same_walkers": {"ms_per_step": ms64, "value": W * ne / (ms64 * 1e-3),
                                 "sweep_ms_avg": sw64, "recompute_period": 64,
                                 "delay_rank": k64, "tile_shape": "deep"}}
    shape_name = {dmcx.DMCX_TILE_DEEP: "deep", dmcx.DMCX_TILE_SHALLOW: "shallow"}
    for name, fp32e in (("fp64_energy", False), ("fp32_energy", True)):
        ctx, ms, sw = _timed_ctx(s, torch, dmcx, stream, W, steps, 19, precision=dmcx.DMCX_MIXED,
                                 delay_rank=0, recompute_period=P, fp32_energy=fp32e)
        k = ctx.delay_rank()
        ranks, shapes, tms = ctx.autotune_report()
        fpm = flops_per_move(s.n_basis, len(s.prim_alpha), ns, ne, s.n_atom, k)
        n_esc = ctx.energy_escalations()
        ach = fpm * W * ne / (sw * 1e-3) / 1e12
        rec = {"ms_per_step": ms, "value": W * ne / (ms * 1e-3), "speedup_vs_fp64_same_walkers":
               ms64 / ms, "sweep_ms_avg": sw, "delay_rank": k,
               "tile_shape": shape_name[ctx.tile_shape()],
               "autotune_ms_per_sweep": {f"{shape_name[int(a)]}/k={int(b)}": round(float(t), 3)
                                         for a, b, t in zip(shapes, ranks, tms)},
               "sweep_roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                                  "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS},
               "recompute_period": 1 if not fp32e else P,
               "walkers_with_fp64_derivative_rows_last_step": n_esc}
        rec.update(_energy_errors(s, torch, dmcx, stream, ctx, W))
        ctx.close()
        out[name] = rec
    out["value"] = out["fp64_energy"]["value"]
    out["reference"] = "FP64 GPU path at each mixed run's final configurations"
    return out


def flush_leg(s, torch, dmcx, stream, W=2048, k=32, reps=5):
    """The delayed-update GEMMs alone: the rank-kb flush G <- G0 - (M Z)^T U
    (Z = Delta G0, M = (I + L)^-1) of kb = k - 1 pending moves of every walker,
    run through the move-by-move calls (dmcx_ratio_grad / dmcx_accept, then
    dmcx_flush launches k_flush, the same code the sweep runs at each block
    end) and timed with events on the context's stream.  Algorithmic FLOP per
    walker: 2 kb n^2 (Z) + kb^2 n (M Z, M lower triangular) + 2 kb n^2
    (the update), n = electrons per spin."""
    from paper_2504_07948_amd import synth
    ctx = dmcx.Context(s, W, precision=dmcx.DMCX_FP64, delay_rank=k, recompute_period=64,
                       stream=stream)
    R0 = synth.make_walkers(s, W, 2040)
    ctx.set_walkers(torch.from_numpy(R0).cuda())
    rng = np.random.default_rng(2041)
    acc = torch.ones(W, dtype=torch.uint8, device="cuda")
    ratio = torch.empty(W, dtype=torch.float64, device="cuda")
    grad = torch.empty((W, 3), dtype=torch.float64, device="cuda")
    kb = k - 1
    times = []
    for rep in range(reps + 1):
        for i in range(kb):
            rn = torch.from_numpy(R0[:, i, :] + 0.05 * rng.standard_normal((W, 3))).cuda()
            ctx.check(dmcx.dmcx_ratio_grad(ctx.h, i, rn.data_ptr(), ratio.data_ptr(),
                                           grad.data_ptr(), dmcx.DMCX_DEVICE))
            ctx.check(dmcx.dmcx_accept(ctx.h, i, acc.data_ptr(), dmcx.DMCX_DEVICE))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.check(dmcx.dmcx_flush(ctx.h))
        e1.record()
        torch.cuda.synchronize()
        if rep:  # the first flush is a warm-up
            times.append(e0.elapsed_time(e1))
    n = s.n_up
    flop = W * (4 * kb * n * n + kb * kb * n)
    ms = float(np.mean(times))
    ach = flop / (ms * 1e-3) / 1e12
    ctx.close()
    return {"walkers": W, "pending_moves": kb, "electrons_per_spin": n, "kernel": "k_flush",
            "ms_avg": ms, "flop_per_launch": flop,
            "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS}}


# FP64 additions and multiplications per electron pair and atom in the
# three-body part of k_jparam as written (R_A . d, the two cosine terms, the
# six terms and their sums; a fused multiply-add counts two)
JPARAM_FLOP_PER_UNIT = 87


def jparams_leg(s, torch, dmcx, stream, W=2048, reps=5, cpu_walkers=4):
    """Jastrow parameter derivatives (two Pade b, six three-body e-e-n
    coefficients) of the 2048 walkers, FP64: k_jparam timed with events on
    the context's stream (a new configuration before each call, so nothing is
    cached), then the linear-method matrices (four short launches).  Work unit:
    one electron pair and one atom, W n(n-1)/2 n_atom per launch; the oracle
    timed on a few walkers beside it."""
    from paper_2504_07948_amd import synth
    ctx = dmcx.Context(s, W, precision=dmcx.DMCX_FP64, delay_rank=32, recompute_period=64,
                       stream=stream)
    O = torch.empty((W, dmcx.DMCX_N_JASTROW_PARAMS), dtype=torch.float64, device="cuda")
    D = torch.empty_like(O)
    n9 = dmcx.DMCX_N_JASTROW_PARAMS + 1
    S = torch.empty((n9, n9), dtype=torch.float64, device="cuda")
    H = torch.empty_like(S)
    t_jp, t_lm = [], []
    for rep in range(reps + 1):
        R = torch.from_numpy(synth.make_walkers(s, W, 2050 + rep)).cuda()
        ctx.set_walkers(R)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        ctx.check(dmcx.dmcx_jastrow_param_grads(ctx.h, O.data_ptr(), D.data_ptr(),
                                                dmcx.DMCX_DEVICE))
        ev[1].record()
        ctx.check(dmcx.dmcx_linear_method(ctx.h, S.data_ptr(), H.data_ptr(), dmcx.DMCX_DEVICE))
        ev[2].record()
        torch.cuda.synchronize()
        if rep:  # the first call is a warm-up
            t_jp.append(ev[0].elapsed_time(ev[1]))
            t_lm.append(ev[1].elapsed_time(ev[2]))
    ne = s.n_elec
    units = W * ne * (ne - 1) // 2 * s.n_atom
    ms = float(np.mean(t_jp))
    ach = JPARAM_FLOP_PER_UNIT * units / (ms * 1e-3) / 1e12
    import oracle
    R = synth.make_walkers(s, cpu_walkers, 2050)
    tc = time.perf_counter()
    oracle.jastrow_param_grads_batch(s, R, n_threads=1)
    tcpu = (time.perf_counter() - tc) / cpu_walkers
    ctx.close()
    return {"walkers": W, "params": dmcx.DMCX_N_JASTROW_PARAMS, "kernel": "k_jparam",
            "ms_avg": ms, "pair_atom_units": units, "ns_per_unit_chip": 1e6 * ms / units,
            "linear_method_ms_avg": float(np.mean(t_lm)),
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                         "flop_per_unit": JPARAM_FLOP_PER_UNIT},
            "oracle_ms_per_walker_one_thread": 1e3 * tcpu,
            "gpu_ms_per_walker": ms / W}


def pp_leg(torch, dmcx, stream, W=2048, steps=5, cpu_walkers=2):
    """DMC steps of the large molecule with a semilocal pseudopotential on its
    16 "C" atoms (synthetic stand-in tables in the ccECP form: a local term
    and a non-local s channel, cutoff 2.15 bohr), FP64, k = 32, P = 64,
    against the same steps without it, each also with the Eq. 3 force
    estimate after every step (with the pseudopotential its Hellmann-Feynman
    term comes in).  Every step's E_L then carries the
    non-local energy: 12 quadrature points per (electron, atom) pair within
    the cutoff, each a basis evaluation dotted with y_e = C (A^-1)_{:,e} and
    a Jastrow ratio.  Points are counted on the host from the final walkers;
    the oracle's non-local energy is timed on a few walkers beside it."""
    from paper_2504_07948_amd import synth
    out = {"walkers": W, "steps": steps}
    for name, s in (("without", synth.large_molecule()), ("with", synth.large_molecule_pp())):
        ctx, ms, sw = _timed_ctx(s, torch, dmcx, stream, W, steps, 31, precision=dmcx.DMCX_FP64,
                                 delay_rank=32, recompute_period=64)
        out[f"ms_per_step_{name}_pp"] = ms
        # the same steps with the Eq. 3 force estimate after each
        F = torch.empty((s.n_atom, 3), dtype=torch.float64, device="cuda")
        e_t = float(np.mean(ctx.measure()[0]))
        ctx.check(dmcx.dmcx_forces(ctx.h, F.data_ptr(), dmcx.DMCX_DEVICE))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
            ctx.check(dmcx.dmcx_forces(ctx.h, F.data_ptr(), dmcx.DMCX_DEVICE))
        torch.cuda.synchronize()
        out[f"ms_per_step_with_forces_{name}_pp"] = 1e3 * (time.perf_counter() - t0) / steps
        # the Jastrow parameter derivatives (with the pseudopotential, its
        # non-local part too); dmcx_set_step forces a fresh evaluation
        O = torch.empty((W, 8), dtype=torch.float64, device="cuda")
        Dd = torch.empty((W, 8), dtype=torch.float64, device="cuda")
        jt = []
        for i in range(3):
            ctx.set_step(ctx.get_step())
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.check(dmcx.dmcx_jastrow_param_grads(ctx.h, O.data_ptr(), Dd.data_ptr(),
                                                    dmcx.DMCX_DEVICE))
            torch.cuda.synchronize()
            if i > 0:
                jt.append(1e3 * (time.perf_counter() - t1))
        out[f"jastrow_param_grads_ms_{name}_pp"] = float(np.mean(jt))
        if name == "with":
            R, _ = ctx.get_walkers()
            nl = [a for a in range(s.n_atom) if np.any((s.pp_atom == a) & (s.pp_l >= 0))]
            d = np.linalg.norm(R[:, :, None, :] - s.ion_xyz[None, None, nl, :], axis=-1)
            pairs = int((d < s.pp_rcut[nl][None, None, :]).sum())
            out["quadrature_points_per_step"] = 12 * pairs
            out["points_per_walker"] = 12 * pairs / W
            import oracle
            tc = time.perf_counter()
            oracle.nlpp_batch(s, R[:cpu_walkers], 31, 0, 0, n_threads=1)
            out["oracle_nlpp_ms_per_walker_one_thread"] = 1e3 * (time.perf_counter() - tc) / cpu_walkers
        ctx.close()
    out["pp_cost_ratio"] = out["ms_per_step_with_pp"] / out["ms_per_step_without_pp"]
    out["force_energy_cost_ratio_with_pp"] = (out["ms_per_step_with_forces_with_pp"] /
                                              out["ms_per_step_with_pp"])
    extra = out["ms_per_step_with_pp"] - out["ms_per_step_without_pp"]
    out["pp_ms_per_step"] = extra
    out["points_per_s"] = out["quadrature_points_per_step"] / (extra * 1e-3) if extra > 0 else None
    return out


def batch5_leg(torch, dmcx, stream, steps=5, W=512, n_det=1000, n_active=100, P=32):
    """Eight alkane stand-ins (20..200 electrons), 512 walkers each, 1000-
    determinant expansions over 100 active orbitals (table method), mixed
    precision, one group whose steps replay a captured graph; the delay rank
    of every molecule is chosen by the autotuner during the warm-up step."""
    from paper_2504_07948_amd import synth
    systems = synth.make_batch5(n_det=n_det, n_active=n_active)
    walkers = [W] * len(systems)
    ne_max = max(x.n_elec for x in systems)
    R = np.zeros((W * len(systems), ne_max, 3))
    for i, x in enumerate(systems):
        R[i * W:(i + 1) * W, :x.n_elec] = synth.make_walkers(x, W, 2030 + i)
    ctx = dmcx.Context(systems, walkers, precision=dmcx.DMCX_MIXED, delay_rank=0,
                       recompute_period=P, tau=0.01, seed=29, stream=stream, graph=True)
    ctx.set_walkers(torch.from_numpy(R).cuda())
    e0, _, _ = ctx.measure()
    e_t = float(np.mean(e0[np.isfinite(e0)]))
    t0 = time.perf_counter()
    ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)  # autotune + capture + one step
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.run_device(steps, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    moves = W * sum(x.n_elec for x in systems) * steps
    # the same steps with the force estimate of every molecule after each step
    F = torch.zeros((len(systems), ctx.n_atom, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
        ctx.check(dmcx.dmcx_forces(ctx.h, F.data_ptr(), dmcx.DMCX_DEVICE))
    torch.cuda.synchronize()
    dt_f = time.perf_counter() - t0
    return {"molecules": [x.name for x in systems], "electrons": [x.n_elec for x in systems],
            "walkers_each": W, "determinants": n_det, "active_orbitals": n_active,
            "steps": steps, "recompute_period": P, "precision": "mixed", "graph": True,
            "delay_rank": [ctx.delay_rank(i) for i in range(len(systems))],
            "warmup_s_incl_autotune": t_warm,
            "value": moves / dt, "unit": "electron-moves/s", "ms_per_step": 1e3 * dt / steps,
            "walker_flags_nonzero": int((ctx.walker_flags() != 0).sum()),
            "ms_per_step_with_forces": 1e3 * dt_f / steps,
            "force_energy_cost_ratio": dt_f / dt}


def forces_leg(s, torch, dmcx, stream, args, W=1024, steps=5):
    """Forces every step (192 components) vs energy-only steps, 1024 walkers,
    FP64 and mixed: Hellmann-Feynman + Pulay via the Eq. 3 adjoint, and the
    zero-variance estimator (Eq. 4 derivative of E_L) with the space warp."""
    from paper_2504_07948_amd import synth
    R0 = synth.make_walkers(s, W, 2027)
    out = {"walkers": W, "steps": steps, "components": 3 * s.n_atom}
    for prec, name in ((dmcx.DMCX_FP64, "fp64"), (dmcx.DMCX_MIXED, "mixed")):
        ctx = dmcx.Context(s, W, precision=prec, delay_rank=32, recompute_period=64, tau=0.01,
                           seed=23, stream=stream)
        ctx.set_walkers(torch.from_numpy(R0).cuda())
        e0, _, _ = ctx.measure()
        e_t = float(np.mean(e0[np.isfinite(e0)]))
        F = torch.empty((s.n_atom, 3), dtype=torch.float64, device="cuda")
        ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
        ctx.check(dmcx.dmcx_forces(ctx.h, F.data_ptr(), dmcx.DMCX_DEVICE))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
        torch.cuda.synchronize()
        t_e = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
            ctx.check(dmcx.dmcx_forces(ctx.h, F.data_ptr(), dmcx.DMCX_DEVICE))
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        # zero-variance force (Eq. 4 derivative of E_L) with the space warp, every step
        ctx.check(dmcx.dmcx_forces_zv(ctx.h, 1, F.data_ptr(), dmcx.DMCX_DEVICE))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
            ctx.check(dmcx.dmcx_forces_zv(ctx.h, 1, F.data_ptr(), dmcx.DMCX_DEVICE))
        torch.cuda.synchronize()
        t_z = time.perf_counter() - t0
        out[name] = {"ms_step_energy": 1e3 * t_e / steps, "ms_step_with_forces": 1e3 * t_f / steps,
                     "force_energy_cost_ratio": t_f / t_e,
                     "ms_step_with_zv_warp_forces": 1e3 * t_z / steps,
                     "zv_warp_force_energy_cost_ratio": t_z / t_e}
    return out


def population_leg(s, torch, dmcx, stream, W=2048, steps=10, sigma=0.5):
    """Comb reconfiguration (fixed population) of the 2048 walkers, FP64,
    after one DMC step.  Before each timed call the log-weights are set to a
    seeded normal spread (sigma 0.5; with this synthetic trial function and
    no local-energy cutoff, weights accumulated by the steps themselves
    collapse onto a few walkers within a few steps).  The copy of a replaced
    walker moves its whole carried state; bytes = 2 x that x walkers
    replaced."""
    from paper_2504_07948_amd import synth
    ctx = dmcx.Context(s, W, delay_rank=32, recompute_period=64, tau=0.01, seed=29, stream=stream)
    ctx.set_walkers(torch.from_numpy(synth.make_walkers(s, W, 2029)).cuda())
    e0, _, _ = ctx.measure()
    e_t = float(np.mean(e0[np.isfinite(e0)]))
    ctx.run_device(1, mode=dmcx.DMCX_DMC, e_trial=e_t)
    R1 = torch.from_numpy(ctx.get_walkers()[0]).cuda()
    rng = np.random.default_rng(31)
    u_host = rng.uniform(0.0, 1.0, steps + 1)
    copies = torch.zeros((steps + 1, W), dtype=torch.int32, device="cuda")
    lwbar = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    cur = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps + 1)]
    for i in range(steps + 1):  # call 0 is a warm-up
        ctx.set_walkers(R1, torch.from_numpy(rng.normal(0.0, sigma, W)).cuda())
        u = np.ascontiguousarray(u_host[i:i + 1])
        ev[i][0].record(cur)
        ctx.check(dmcx.dmcx_reconfigure(ctx.h, u.ctypes.data, copies[i].data_ptr(),
                                        lwbar[i:i + 1].data_ptr(), dmcx.DMCX_DEVICE))
        ev[i][1].record(cur)
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev[1:]])
    replaced = (copies[1:] == 0).sum(dim=1).cpu().numpy()
    NP = (max(s.n_up, s.n_dn) + 15) // 16 * 16
    ne = s.n_elec
    state = ne * 3 * 8 + ne * 5 * NP * 8 + 2 * NP * NP * 8 + 8 * 8
    gbs = 2.0 * state * replaced / (ms * 1e-3) / 1e9
    ctx.close()
    # birth/death branching of the same walkers in a context of twice the
    # capacity: the call includes the host read of the new count (the
    # launches after it are sized by it), so it is timed on the host clock
    bctx = dmcx.Context(s, 2 * W, delay_rank=32, recompute_period=64, tau=0.01, seed=29,
                        stream=stream)
    bms, wnew = [], []
    for i in range(steps + 1):
        bctx.set_walker_count(W)
        bctx.set_walkers(R1, torch.from_numpy(rng.normal(0.0, sigma, W)).cuda())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, wn = bctx.branch(100 + i)
        bctx.sync()
        t1 = time.perf_counter()
        if i > 0:
            bms.append((t1 - t0) * 1e3)
            wnew.append(wn)
    bctx.close()
    return {"walkers": W, "calls": steps, "log_w_sigma": sigma,
            "reconfigure_ms_avg": float(ms.mean()),
            "walkers_replaced_avg": float(replaced.mean()),
            "state_bytes_per_walker": state,
            "copy_GB_per_s_avg": float(gbs.mean()),
            "hbm_fraction": float(gbs.mean() / 8000.0),
            "branch_capacity": 2 * W,
            "branch_ms_avg": float(np.mean(bms)),
            "branch_walkers_after_avg": float(np.mean(wnew))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--walkers", type=int, default=2048)
    ap.add_argument("--delay", type=int, default=32)
    ap.add_argument("--recompute", type=int, default=64)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-extras", action="store_true",
                    help="only the FP64 leg (same as --extras none)")
    ap.add_argument("--extras", default="mixed,forces,batch,population,flush,jparams,pp",
                    help="comma list of the extra legs to run after the FP64 leg: mixed, forces, "
                         "batch (eight multideterminant alkanes), population, flush (the "
                         "delayed-update GEMMs alone), jparams (Jastrow parameter derivatives "
                         "and linear-method matrices), pp (pseudopotential), or none")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, run one device copy of this many MiB "
                         "(a known-size kernel for scaling FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for {args.gpus}); "
              "walkers are independent, so N GPUs would each run this workload on their own "
              "walker shard with one small all-reduce of estimators per step.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_07948_amd import dmcx, synth

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    s = synth.large_molecule()
    W = args.walkers
    R0 = synth.make_walkers(s, W, 2025)
    prec = dmcx.DMCX_FP64 if args.precision == "fp64" else dmcx.DMCX_MIXED
    ctx = dmcx.Context(s, W, precision=prec, delay_rank=args.delay,
                       recompute_period=args.recompute, tau=0.01, seed=17, stream=stream)
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    Rd = torch.from_numpy(R0).cuda()
    ctx.set_walkers(Rd)
    e0, _, _ = ctx.measure()
    e_t = float(np.mean(e0[np.isfinite(e0)]))
    if args.warmup:
        ctx.run_device(args.warmup, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_device(args.steps, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweep_ms, n_launch, sweep_total = ctx.last_run_timing()
    flags = ctx.walker_flags()
    # A window shorter than the recompute period holds no FP64 recompute; time
    # one whole period as well (aligned so that it starts with the recompute).
    step_now = ctx.get_step()
    align = (-step_now) % args.recompute
    if align:
        ctx.run_device(align, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    ctx.run_device(args.recompute, mode=dmcx.DMCX_DMC, e_trial=e_t)
    torch.cuda.synchronize()
    dt_period = time.perf_counter() - tp0

    mixed = forces = batch5 = population = flush = jparams = pp = None
    extras = set() if args.skip_extras else set(args.extras.split(",")) - {"none", ""}
    unknown = extras - {"mixed", "forces", "batch", "population", "flush", "jparams", "pp"}
    if unknown:
        sys.exit(f"bench.py: unknown extra legs {sorted(unknown)}")
    if "mixed" in extras:
        mixed = mixed_leg(s, torch, dmcx, stream, args)
    if "forces" in extras:
        forces = forces_leg(s, torch, dmcx, stream, args)
    if "batch" in extras:
        batch5 = batch5_leg(torch, dmcx, stream)
    if "population" in extras:
        population = population_leg(s, torch, dmcx, stream)
    if "flush" in extras:
        flush = flush_leg(s, torch, dmcx, stream)
    if "jparams" in extras:
        jparams = jparams_leg(s, torch, dmcx, stream)
    if "pp" in extras:
        pp = pp_leg(torch, dmcx, stream)

    ne, ns = s.n_elec, max(s.n_up, s.n_dn)
    moves = W * ne * args.steps
    value = moves / dt
    fpm = flops_per_move(s.n_basis, len(s.prim_alpha), ns, ne, s.n_atom, args.delay)
    sweep_flops = fpm * W * ne
    achieved = sweep_flops / (sweep_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if prec == dmcx.DMCX_FP64 else PEAK_FP32_TFLOPS
    traffic = None
    if (kernel_sources_sha256() == SWEEP_TRAFFIC["sources_sha256"]
            and SWEEP_TRAFFIC["workload"] == {"walkers": W, "delay": args.delay,
                                              "precision": args.precision}):
        tb = SWEEP_TRAFFIC["fetch_bytes"] + SWEEP_TRAFFIC["write_bytes"]
        traffic = {"bytes_per_launch": tb, "fetch_bytes": SWEEP_TRAFFIC["fetch_bytes"],
                   "write_bytes": SWEEP_TRAFFIC["write_bytes"],
                   "bytes_per_move": tb / (W * s.n_elec),
                   "GB_per_s": tb / (sweep_ms * 1e-3) / 1e9}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        host = host_cpu_info()
        n_threads = min(16, host["affinity_cpus"])
        # pilot: one step of n_threads walkers, then size the sample to ~cpu-seconds
        pilot = R0[:n_threads]
        tp = time.perf_counter()
        oracle.run(s, pilot, n_steps=1, mode=1, tau=0.01, seed=17, e_trial=e_t,
                   want_logs=False, n_threads=n_threads)
        rate_pilot = n_threads * ne / (time.perf_counter() - tp)
        w_sample = int(min(W, max(n_threads, rate_pilot * args.cpu_seconds / ne)))
        w_sample = max(n_threads, (w_sample // n_threads) * n_threads)
        tc = time.perf_counter()
        oracle.run(s, R0[:w_sample], n_steps=1, mode=1, tau=0.01, seed=17, e_trial=e_t,
                   want_logs=False, n_threads=n_threads)
        tcpu = time.perf_counter() - tc
        # one thread: one DMC step of two walkers
        t1 = time.perf_counter()
        oracle.run(s, R0[:2], n_steps=1, mode=1, tau=0.01, seed=17, e_trial=e_t,
                   want_logs=False, n_threads=1)
        t1 = time.perf_counter() - t1
        cpu = {"value": w_sample * ne / tcpu, "unit": "electron-moves/s", "cores": n_threads,
               "kind": "oracle",
               "sample": f"1 DMC step of the first {w_sample} of {W} walkers "
                         f"({w_sample * ne} moves, {tcpu:.1f} s, FP64, k=1 with fresh LU)",
               "one_thread_value": 2 * ne / t1,
               "one_thread_sample": f"1 DMC step of 2 walkers ({2 * ne} moves, {t1:.1f} s)",
               "host": host}

    out = {
        "metric": "electron-moves/s, FP64 vs mixed at stated error; forces-vs-energy cost ratio",
        "value": value,
        "unit": "electron-moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "full_recompute_period": {"steps": args.recompute, "ms_per_step":
                                  dt_period * 1e3 / args.recompute,
                                  "value": W * ne * args.recompute / dt_period,
                                  "note": "one FP64 recompute (every P steps) inside the window"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == dmcx.DMCX_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "DMC step, 64-atom 112-electron synthetic molecule "
                               "(1024 Cartesian GTOs, 400 shells x 3 primitives), "
                               f"{W} walkers, delayed rank k={args.delay}, FP64 LU recompute "
                               f"every {args.recompute} steps, tau=0.01",
                   "walkers": W, "electrons": ne, "basis": s.n_basis, "precision": args.precision},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_sweep", "kernel_ms_avg": sweep_ms, "launches": n_launch,
                     "flop_per_launch": sweep_flops, "flop_per_move": fpm},
        "cpu_baseline": cpu,
        "mixed": mixed,
        "forces": forces,
        "batch_multideterminant": batch5,
        "population_control": population,
        "delayed_update_flush": flush,
        "jastrow_param_derivatives": jparams,
        "pseudopotential": pp,
        "walker_flags_nonzero": int((flags != 0).sum()),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
