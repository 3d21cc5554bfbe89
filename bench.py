"""Benchmark: forward + reverse-time adjoint particle-mesh simulation on one
MI355X.

One benchmark step = one full pass of the hot path on a synthetic LambdaCDM
box: 2LPT initial conditions, 63 KDK steps (a = 1/64 -> 1), the final-density
MSE objective, 63 adjoint steps with reverse-time integration and the 2LPT
VJP, giving J, dJ/domega and dJ/d(Omega_m, sigma8).  Default workload:
512^3 particles on a 512^3 mesh in a 512 Mpc/h box, FP32 mesh/FFT with FP64
particle state.  The metric is particle-steps/s = N_p * 63 / (time per pass).

Prints one JSON line (see README/DESIGN for the fields).
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (particles per side, mesh per side, box Mpc/h, steps, a_start)
    "512": (512, 512, 512.0, 63, 1.0 / 64),
    "128": (128, 128, 256.0, 63, 1.0 / 64),
    "32": (32, 64, 128.0, 10, 1.0 / 16),
    "1024": (1024, 1024, 1024.0, 63, 1.0 / 64),
}
HBM_PEAK_GBS = 8000.0

# sources of each kernel family: a committed traffic summary under profiles/
# applies only while these files are unchanged
FAMILY_SOURCES = {
    "gather": ["paper_2211_09815_amd/csrc/particles.hip", "paper_2211_09815_amd/csrc/tiles.h"],
    "paint_tiles": ["paper_2211_09815_amd/csrc/paint.hip", "paper_2211_09815_amd/csrc/tiles.h"],
    "bin": ["paper_2211_09815_amd/csrc/paint.hip", "paper_2211_09815_amd/csrc/tiles.h"],
    "scatter": ["paper_2211_09815_amd/csrc/paint.hip", "paper_2211_09815_amd/csrc/tiles.h"],
    "halo_add": ["paper_2211_09815_amd/csrc/paint.hip", "paper_2211_09815_amd/csrc/tiles.h"],
    "fft_lines": ["paper_2211_09815_amd/csrc/fft_lines.hip", "paper_2211_09815_amd/csrc/fft_core.h"],
    "fft_poisson": ["paper_2211_09815_amd/csrc/fft_fused.hip", "paper_2211_09815_amd/csrc/fft_core.h"],
    "fft_r2c_z": ["paper_2211_09815_amd/csrc/fft_z.hip", "paper_2211_09815_amd/csrc/fft_core.h"],
    "fft_c2r_z": ["paper_2211_09815_amd/csrc/fft_z.hip", "paper_2211_09815_amd/csrc/fft_core.h"],
}


def measured_traffic(family, workload):
    """HBM bytes per launch of `family` at `workload` from the rocprofv3
    counter summary in profiles/, or None if there is none for that workload
    or the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    import re
    if family not in FAMILY_SOURCES:
        return None
    h = hashlib.sha256()
    for f in FAMILY_SOURCES[family]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    digest = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            m = re.search(r"traffic_per_launch_bytes=([0-9.e+]+) family=(\w+) workload=(\w+) source_sha256=(\w+)",
                          line)
            if m and m.group(2) == family and m.group(3) == workload and m.group(4) == digest:
                return float(m.group(1))
    return None



def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(seconds_hint=20.0):
    """Time the FP64 oracle (numpy, as it stands) on a bounded sample: 2LPT,
    2 forward KDK steps, the objective and 2 reverse-time adjoint steps at
    128^3 particles on a 128^3 mesh (256 Mpc/h)."""
    import numpy as np

    from oracle import cosmology, integrate, lpt, objective, simulate
    from paper_2211_09815_amd import inputs
    n, nm, box, steps = 128, 128, 256.0, 2
    cfg = simulate.SimConfig(n, nm, box, 1.0 / 64, 1.0 / 64 + 2.0 / 64, steps)
    omega = inputs.white_noise(n, inputs.SEED_RUN)
    target = np.zeros(cfg.mesh_shape)
    t0 = time.perf_counter()
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    coefs, dcoefs = cosmology.step_coefficients_with_derivative(cfg.a_grid(), 0.3)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, 0.3)
    s, p, a, _ = integrate.forward(q, s0, p0, coefs, F, store=False)
    J, xbar = objective.density_mse(q + s, target, cfg.n_particles)
    _, _, xi0, pi0, _ = integrate.adjoint_reverse(q, s, p, a, xbar, np.zeros_like(xbar), coefs, dcoefs, F)
    lpt.lpt_vjp(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r, xi0, pi0)
    dt = time.perf_counter() - t0
    return {
        "value": n ** 3 * steps / dt,
        "unit": "particle-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "FP64 numpy oracle, 128^3 particles on a 128^3 mesh, 2LPT + 2 KDK steps + objective + "
                  "2 reverse-time adjoint steps + 2LPT VJP, %.1f s wall (numpy FFT and bincount run on one core)"
                  % dt,
    }


def _setup_run(n, nm, box, nsteps, a0, mdt, sdt, seed=None, checkpoint_steps=(), deterministic=True):
    import torch
    from paper_2211_09815_amd import api, inputs
    from paper_2211_09815_amd.simulate import SimConfig, Simulation
    sim = Simulation(SimConfig(n, nm, box, a0, 1.0, nsteps, mdt, sdt, checkpoint_steps=tuple(checkpoint_steps),
                               deterministic=deterministic))
    cosmo = api.Cosmology()
    tabs = sim.tables(cosmo)
    npdt = "float32" if mdt == torch.float32 else "float64"
    omega = torch.as_tensor(inputs.white_noise(n, inputs.SEED_RUN if seed is None else seed, dtype=npdt),
                            device="cuda")
    return sim, cosmo, tabs, omega


def hbm_warmup(gib):
    """Allocate device memory in 1 GiB pieces, up to `gib` GiB or all but
    8 GiB of what is free, and release it, before the plan and the state are
    allocated.  On MI355X the large buffers allocated after such a cycle run
    the whole pass several percent faster than buffers allocated first in a
    fresh process (measured; the kernels are the same).  Returns (GiB cycled,
    seconds)."""
    import torch
    if gib <= 0:
        return 0, 0.0
    t0 = time.perf_counter()
    free, _ = torch.cuda.mem_get_info()
    want = min(int(gib), int(free >> 30) - 8)
    chunks = []
    try:
        for _ in range(max(want, 0)):
            chunks.append(torch.empty(1 << 30, dtype=torch.uint8, device="cuda"))
    except RuntimeError:
        pass
    got = len(chunks)
    del chunks
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    return got, time.perf_counter() - t0


def _timed_pass(sim, omega, cosmo, target, tabs):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g, th = sim.value_and_grad(omega, cosmo, target, tabs)
    torch.cuda.synchronize()
    return J, g, th, time.perf_counter() - t0


def _rel_l2(a, b):
    import torch
    return float(torch.linalg.vector_norm((a.double() - b.double()).reshape(-1))
                 / torch.linalg.vector_norm(b.double().reshape(-1)))


def stream_bandwidth(plan, gib=2, reps=5):
    """Best rate of the library's STREAM-like kernels (pm_stream) over a
    `gib` GiB buffer: pure read, copy (read + write bytes) and pure write."""
    import torch
    from paper_2211_09815_amd import _lib
    x = torch.zeros((gib << 30) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, mode, src, dst in (("read", _lib.PM_STREAM_READ, x, None), ("copy", _lib.PM_STREAM_COPY, x, y),
                                 ("write", _lib.PM_STREAM_WRITE, None, y)):
        plan.stream(mode, src, dst)
        best = 0.0
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nbytes = plan.stream(mode, src, dst)
            e1.record()
            e1.synchronize()
            best = max(best, nbytes / 1e9 / (e0.elapsed_time(e1) / 1e3))
        out[name] = best
    del x, y
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(gib=2, reps=5):
    """Best device-to-device copy rate (read + write bytes / time) of a
    `gib` GiB buffer: the practical HBM ceiling next to the published peak."""
    import torch
    x = torch.empty((gib << 30) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * x.numel() * 4 / 1e9 / (e0.elapsed_time(e1) / 1e3))
    del x, y
    torch.cuda.empty_cache()
    return best


def final_state_outputs(sim, omega, cosmo, tabs):
    """Forward pass only: the final displacement s_n (FP64 copy) and the
    power spectrum (k, P) of the final density contrast (pm_power_spectrum)."""
    sim.forward(omega, cosmo, tabs)
    s_fin = sim.s.double().clone()
    k, P, _ = sim.plan.power_spectrum(sim.plan.density(sim.s))
    return s_fin, k.clone(), P.clone()


def fp64_reference(args, target64, g_mixed, th_mixed, s_mixed, pk_mixed):
    """One all-FP64 pass on the same workload (same white noise and target):
    its throughput, and the error of each benchmarked output against it:
    final positions, the density power spectrum and the gradients."""
    import torch
    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    log("all-FP64 reference pass")
    sim, cosmo, tabs, omega = _setup_run(n, nm, box, nsteps, a0, torch.float64, torch.float64)
    _timed_pass(sim, omega, cosmo, target64, tabs)  # warm-up
    J, g, th, dt = _timed_pass(sim, omega, cosmo, target64, tabs)
    s64, k64, P64 = final_state_outputs(sim, omega, cosmo, tabs)
    ds = s_mixed - s64
    relP = (pk_mixed[1].double() / P64 - 1.0).abs().cpu()
    nq = max(1, (nm // 2) // 2)           # shells b = 1 .. N/4
    return {
        "fp64_reference": {"value": n ** 3 * nsteps / dt, "unit": "particle-steps/s", "ms_per_step": 1000 * dt,
                           "J": float(J.cpu()[0]), "dJ_dtheta": th.cpu().tolist()},
        "grad_omega_rel_l2_vs_fp64": _rel_l2(g_mixed, g),
        "dJ_dtheta_rel_err_vs_fp64": [abs(float(a) - float(b)) / abs(float(b)) for a, b in zip(th_mixed.cpu(), th.cpu())],
        "final_positions_vs_fp64": {"rel_l2_of_displacement": _rel_l2(s_mixed, s64),
                                    "rms_err_cells": float(ds.pow(2).mean().sqrt()),
                                    "max_err_cells": float(ds.abs().max())},
        "power_spectrum_vs_fp64": {"max_rel_err_first_quarter": float(relP[:nq].max()),
                                   "max_rel_err_all": float(relP.max()),
                                   "rel_err_per_shell": [float(x) for x in relP],
                                   "k_h_per_mpc": [float(x) for x in k64.cpu()],
                                   "P_fp64": [float(x) for x in P64.cpu()],
                                   "note": "final density contrast of the forward pass at a = 1, shells "
                                           "round(|m|) = 1 .. N/2 (pm_power_spectrum); first quarter: "
                                           "shells 1 .. N/4"},
    }


def study_precision(args):
    """FP32 throughout vs FP32 mesh + FP64 state vs all-FP64 at one workload:
    reversibility of the recovered initial state, gradient error against the
    FP64 run, throughput, and peak memory against the number of steps."""
    import torch
    from paper_2211_09815_amd import inputs
    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    modes = [("f64", "f64"), ("f32", "f64"), ("f32", "f32")]
    dt_of = {"f32": torch.float32, "f64": torch.float64}
    # target: the all-FP64 run of the target seed
    sim, cosmo, tabs, omega_t = _setup_run(n, nm, box, nsteps, a0, torch.float64, torch.float64,
                                           seed=inputs.SEED_TARGET)
    sim.forward(omega_t, cosmo, tabs)
    target64 = sim.plan.density(sim.s).clone()
    del sim, omega_t
    torch.cuda.empty_cache()
    res = {}
    grads = {}
    finals = {}
    for mdt, sdt in modes:
        key = "%s-mesh/%s-state" % (mdt, sdt)
        log("precision: " + key)
        sim, cosmo, tabs, omega = _setup_run(n, nm, box, nsteps, a0, dt_of[mdt], dt_of[sdt])
        target = target64.to(dt_of[mdt])
        coefs, ic = tabs
        st0 = {"s": torch.zeros_like(sim.s), "p": torch.zeros_like(sim.p), "acc": None}
        sim.plan.lpt(omega, cosmo, ic, st0)
        _timed_pass(sim, omega, cosmo, target, tabs)  # warm-up
        J, g, th, dt = _timed_pass(sim, omega, cosmo, target, tabs)
        s0, p0 = st0["s"].double(), st0["p"].double()
        ds = (sim.s.double() - s0)
        dp = (sim.p.double() - p0)
        res[key] = {
            "particle_steps_per_s": n ** 3 * nsteps / dt,
            "ms_per_pass": 1000 * dt,
            "J": float(J.cpu()[0]),
            "dJ_dtheta": th.cpu().tolist(),
            "reversibility": {
                "s0_rms_err_cells": float(ds.pow(2).mean().sqrt()),
                "s0_rms_err_over_std": float(ds.pow(2).mean().sqrt() / s0.std()),
                "s0_max_err_cells": float(ds.abs().max()),
                "p0_rms_err_over_std": float(dp.pow(2).mean().sqrt() / p0.std()),
            },
        }
        grads[key] = (g.double().clone(), th.clone())
        finals[key] = final_state_outputs(sim, omega, cosmo, tabs)
        del sim, omega, target, st0, s0, p0, ds, dp, g
        torch.cuda.empty_cache()
    g64, th64 = grads["f64-mesh/f64-state"]
    s64, _, P64 = finals["f64-mesh/f64-state"]
    nq = max(1, nm // 4)
    for key, (g, th) in grads.items():
        res[key]["grad_omega_rel_l2_vs_fp64"] = _rel_l2(g, g64)
        res[key]["dJ_dtheta_rel_err_vs_fp64"] = [abs(float(a) - float(b)) / abs(float(b))
                                                 for a, b in zip(th.cpu(), th64.cpu())]
        s_fin, _, P = finals[key]
        relP = (P / P64 - 1.0).abs()
        res[key]["final_positions_vs_fp64"] = {"rel_l2_of_displacement": _rel_l2(s_fin, s64),
                                               "max_err_cells": float((s_fin - s64).abs().max())}
        res[key]["power_spectrum_vs_fp64"] = {"max_rel_err_first_quarter": float(relP[:nq].max()),
                                              "max_rel_err_all": float(relP.max())}
    del grads, g64, finals, s64
    torch.cuda.empty_cache()
    # adjoint memory against the number of steps (mixed precision)
    mem = {}
    for steps in (10, 31, 63):
        log("memory: %d steps" % steps)
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        sim, cosmo, tabs, omega = _setup_run(n, nm, box, steps, a0, torch.float32, torch.float64)
        sim.value_and_grad(omega, cosmo, target64.float(), tabs)
        torch.cuda.synchronize()
        ws = sim.plan.workspace_bytes((nm,) * 3, (n,) * 3, torch.float32, torch.float64)
        mem[str(steps)] = {"torch_peak_gb": (torch.cuda.max_memory_allocated() - base) / 1e9,
                           "plan_workspace_gb": ws / 1e9,
                           "total_gb": (torch.cuda.max_memory_allocated() - base + ws) / 1e9}
        del sim, omega
        torch.cuda.empty_cache()
    return {"study": "precision", "workload": "%d^3 particles, %d^3 mesh, %.0f Mpc/h, %d steps a=%.5f..1"
            % (n, nm, box, nsteps, a0), "modes": res, "peak_memory_vs_steps": mem,
            "reversibility_metric": "recovered minus true 2LPT initial state after the reverse-time pass; "
                                    "rms over all particles and axes, in cells and relative to the std of s0 / p0"}


def study_checkpoints(args):
    """Piecewise reverse from forward checkpoints (Sec. 3.5): for FP32 state
    and for FP32 mesh + FP64 state, the pass time, the checkpoint memory, the
    reversibility of the recovered initial state and the gradient error
    against the all-FP64 pass, with 0, 7, 21 and 63 evenly spaced
    checkpoints."""
    import torch
    from paper_2211_09815_amd import inputs
    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    sim, cosmo, tabs, omega_t = _setup_run(n, nm, box, nsteps, a0, torch.float64, torch.float64,
                                           seed=inputs.SEED_TARGET)
    sim.forward(omega_t, cosmo, tabs)
    target64 = sim.plan.density(sim.s).clone()
    del sim, omega_t
    torch.cuda.empty_cache()
    log("checkpoints: all-FP64 reference")
    sim, cosmo, tabs, omega = _setup_run(n, nm, box, nsteps, a0, torch.float64, torch.float64)
    _, g64, th64, _ = _timed_pass(sim, omega, cosmo, target64, tabs)
    g64 = g64.float()
    del sim, omega
    torch.cuda.empty_cache()
    res = {}
    for sdt_name, sdt, counts in (("f32", torch.float32, (0, 7, 21, nsteps)), ("f64", torch.float64, (0, 7))):
        for k in counts:
            steps = [round((i + 1) * nsteps / k) for i in range(k)] if k else []
            key = "f32-mesh/%s-state/%d-checkpoints" % (sdt_name, k)
            log("checkpoints: " + key)
            sim, cosmo, tabs, omega = _setup_run(n, nm, box, nsteps, a0, torch.float32, sdt, checkpoint_steps=steps)
            coefs, ic = tabs
            st0 = {"s": torch.zeros_like(sim.s), "p": torch.zeros_like(sim.p), "acc": None}
            sim.plan.lpt(omega, cosmo, ic, st0)
            target = target64.float()
            _timed_pass(sim, omega, cosmo, target, tabs)  # warm-up
            J, g, th, dt = _timed_pass(sim, omega, cosmo, target, tabs)
            s0 = st0["s"].double()
            ds = sim.s.double() - s0
            res[key] = {
                "checkpoint_steps": steps,
                "checkpoint_memory_gb": 2 * k * sim.s.numel() * sim.s.element_size() / 1e9,
                "ms_per_pass": 1000 * dt,
                "particle_steps_per_s": n ** 3 * nsteps / dt,
                "s0_rms_err_over_std": float(ds.pow(2).mean().sqrt() / s0.std()),
                "grad_omega_rel_l2_vs_fp64": _rel_l2(g, g64),
                "dJ_dtheta_rel_err_vs_fp64": [abs(float(a) - float(b)) / abs(float(b))
                                              for a, b in zip(th.cpu(), th64.cpu())],
            }
            del sim, omega, st0, s0, ds, g, target
            torch.cuda.empty_cache()
    return {"study": "checkpoints", "workload": "%d^3 particles, %d^3 mesh, %.0f Mpc/h, %d steps a=%.5f..1"
            % (n, nm, box, nsteps, a0), "runs": res,
            "note": "checkpoint j holds (s_j, p_{j-1/2}); the reverse pass lands its drift on s_j and takes "
                    "p_{j-1/2} after its kick; the forward pass is bitwise the same with or without them"}


def study_force(args, reps=10):
    """Single force and force VJP, stage by stage: 256^3 particles displaced by
    2LPT at a = 0.5, painted to a 512^3 FP32 mesh in a 512 Mpc/h box; the VJP
    uses a seeded Gaussian cotangent.  Algorithmic bytes per stage: particles
    and meshes read or written once (FP32 displacements and fields)."""
    import torch
    from paper_2211_09815_amd import _lib, api, inputs
    n, nm, box = 256, 512, 512.0
    plan = api.Plan(nm, n, box=box, mesh_dtype=torch.float32, state_dtype=torch.float32)
    cosmo = api.Cosmology()
    _, ic = api.tables(cosmo, [0.5, 1.0])
    omega = torch.as_tensor(inputs.white_noise(n, inputs.SEED_RUN, dtype="float32"), device="cuda")
    st = {"s": torch.zeros((3, n ** 3), dtype=torch.float32, device="cuda"),
          "p": torch.zeros((3, n ** 3), dtype=torch.float32, device="cuda"), "acc": None}
    plan.lpt(omega, cosmo, ic, st)
    s = st["s"]
    cot = torch.as_tensor(inputs.normal((3, n ** 3), inputs.SEED_COTANGENT, dtype=np.float32), device="cuda")
    om = cosmo.omega_m
    N, Nc = n ** 3, nm ** 3
    Ns = nm * nm * (nm // 2 + 1)
    f4, c8 = 4.0, 8.0
    rho = plan.paint(s)
    dk = plan.fft_r2c(rho)
    gk = plan.poisson_grad(dk[0], om)
    g = plan.fft_c2r(gk)
    stages = [
        ("paint", lambda: plan.paint(s, out=rho), N * 12 + Nc * f4),
        ("r2c", lambda: plan.fft_r2c(rho, out=dk), Nc * f4 + Ns * c8),
        ("poisson_grad (unfused)", lambda: plan.poisson_grad(dk[0], om, out=gk), 4 * Ns * c8),
        # the inverse transform works in place on its input; the timing of a
        # transform does not depend on the values it is given
        ("3x c2r", lambda: plan.fft_c2r(gk, out=g, destroy_input=True), 3 * (Ns * c8 + Nc * f4)),
        ("readout (3 fields)", lambda: plan.readout(s, g), N * 12 + 3 * Nc * f4 + 3 * N * f4),
        ("force (fused: paint, r2c, gradient in the x pass, 3x c2r, readout)", lambda: plan.force(s, om),
         N * 12 + Nc * f4 + (Nc * f4 + Ns * c8) + 3 * (Ns * c8 + Nc * f4) + 3 * Nc * f4 + 3 * N * f4),
        ("force VJP (4-channel paint, 4x r2c, combine in the x pass, 4x c2r, 4-field gather)",
         lambda: plan.force_vjp(s, cot, om, want_acc=False),
         N * 12 + 3 * N * f4 + 4 * Nc * f4 + 4 * (Nc * f4 + Ns * c8) + 4 * (Ns * c8 + Nc * f4) + 4 * Nc * f4
         + N * 12 + 3 * N * f4 + 3 * N * f4),
    ]
    rows = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, fn, by in stages:
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        rows.append({"stage": name, "ms": ms, "algorithmic_GB": by / 1e9, "GBps": by / 1e9 / (ms / 1e3),
                     "frac_of_peak": by / 1e9 / (ms / 1e3) / HBM_PEAK_GBS})
    # kernel families inside the fused force and the VJP
    fams = {}
    for label, fn in (("force", lambda: plan.force(s, om)),
                      ("force_vjp", lambda: plan.force_vjp(s, cot, om, want_acc=False))):
        plan.timing_enable(_lib.KERNEL_FAMILIES.values())
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        fams[label] = {}
        for fam, kid in _lib.KERNEL_FAMILIES.items():
            ms, nl, b = plan.timing_read(kid)
            if nl:
                fams[label][fam] = {"ms": ms / reps, "GBps": (b / 1e9) / (ms / 1e3)}
        plan.timing_enable(())
    return {"study": "force", "workload": "256^3 particles (2LPT at a=0.5), 512^3 FP32 mesh, 512 Mpc/h, "
            "FP32 displacements; cotangent seed %d" % inputs.SEED_COTANGENT, "reps": reps, "stages": rows,
            "kernel_families": fams, "peak_GBps": HBM_PEAK_GBS}


def study_cpu_oracle(args, reps=3, n=256, nm=512):
    """The FP64 oracle (numpy, as it stands) on the host, stage by stage, at
    the single-force shape: 256^3 particles displaced by the oracle's 2LPT at
    a = 0.5 on a 512^3 mesh in a 512 Mpc/h box, Gaussian cotangent.  Each
    stage is timed `reps` times after a warm-up (median).  Beside it, the FFT
    stages with scipy.fft on every host core (a library FFT, not the oracle).
    The whole 512^3 pass per particle-step is then extrapolated: the mesh
    stages of one force and one force VJP as measured, their particle stages
    scaled by 8 (512^3 particles), over 512^3 particle-steps.  Needs no GPU."""
    import numpy as np
    import scipy.fft

    from oracle import cosmology, lpt, pm, simulate
    from paper_2211_09815_amd import inputs
    box = float(nm)
    shape = (nm, nm, nm)
    cfg = simulate.SimConfig(n, nm, box, 0.5, 1.0, 1)
    omega = inputs.white_noise(n, inputs.SEED_RUN)
    t0 = time.perf_counter()
    s0, _ = lpt.lpt(omega, cfg.box, cfg.cosmo, 0.5, cfg.r)
    t_lpt = time.perf_counter() - t0
    x = simulate.lattice(cfg) + s0
    N = n ** 3
    coef = 1.5 * cfg.cosmo.omega_m
    abar = inputs.normal((N, 3), inputs.SEED_COTANGENT)
    workers = os.cpu_count() or 1

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    delta = pm.density_contrast(x, shape, N)
    dk = np.fft.rfftn(delta)
    gk = pm.poisson_gradient(dk, shape, coef)
    g = [np.fft.irfftn(gj, s=shape, axes=(0, 1, 2)) for gj in gk]
    rows = {
        "paint (density contrast)": timed(lambda: pm.density_contrast(x, shape, N)),
        "r2c (numpy, 1 core)": timed(lambda: np.fft.rfftn(delta)),
        "poisson gradient": timed(lambda: pm.poisson_gradient(dk, shape, coef)),
        "3x c2r (numpy, 1 core)": timed(lambda: [np.fft.irfftn(gj, s=shape, axes=(0, 1, 2)) for gj in gk]),
        "readout (3 fields)": timed(lambda: [pm.readout(x, gj) for gj in g]),
        "force": timed(lambda: pm.force(x, shape, N, coef)),
        "force VJP": timed(lambda: pm.force_vjp(x, abar, shape, N, coef)),
    }
    lib = {
        "r2c (scipy.fft, %d workers)" % workers: timed(lambda: scipy.fft.rfftn(delta, workers=workers)),
        "3x c2r (scipy.fft, %d workers)" % workers:
            timed(lambda: [scipy.fft.irfftn(gj, s=shape, axes=(0, 1, 2), workers=workers) for gj in gk]),
    }
    # mesh and particle parts of the force and of the VJP (the VJP runs one
    # r2c and three c2r for the force, three r2c and one c2r for the
    # cotangent fields, and the multipliers twice)
    t_fft1 = rows["r2c (numpy, 1 core)"]
    t_c2r = rows["3x c2r (numpy, 1 core)"] / 3
    t_mul = rows["poisson gradient"]
    mesh_force = t_fft1 + t_mul + 3 * t_c2r
    mesh_vjp = 4 * t_fft1 + 2 * t_mul + 4 * t_c2r
    part_force = max(rows["force"] - mesh_force, 0.0)
    part_vjp = max(rows["force VJP"] - mesh_vjp, 0.0)
    n4 = 512
    scale = (n4 / n) ** 3
    t_step = mesh_force + scale * part_force + mesh_vjp + scale * part_vjp
    return {"study": "cpu-oracle", "workload": "%d^3 particles (oracle 2LPT at a=0.5), %d^3 FP64 mesh, "
            "%g Mpc/h; cotangent seed %d" % (n, nm, box, inputs.SEED_COTANGENT), "reps": reps, "lpt_s": t_lpt,
            "oracle_stage_s": rows, "library_fft_s": lib, "host_cpus": workers,
            "oracle_cores": 1,
            "extrapolated_512": {
                "s_per_step": t_step, "particle_steps_per_s": n4 ** 3 / t_step,
                "note": "extrapolated, not measured: one force (forward) and one force VJP (adjoint) per "
                        "step at 512^3 particles on a 512^3 mesh; mesh stages as measured at 512^3, "
                        "particle stages x8 from 256^3"}}


def study_paint_modes(args):
    """The fixed-point paint against the floating-point-atomic one, and the
    precision modes against each other (Sec. 4.1, Tables rep and rev): per
    mode the pass time, run-to-run reproducibility (two identical passes
    compared element by element), the reversibility of the recovered initial
    state, and the gradient error against the all-FP64 fixed-point pass;
    then, for each gradient-error target, the fastest mode that meets it."""
    import torch
    from paper_2211_09815_amd import inputs
    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    f32, f64 = torch.float32, torch.float64
    modes = [  # (name, mesh, state, deterministic, checkpoints)
        ("f64-mesh/f64-state/fixed", f64, f64, True, 0),
        ("f64-mesh/f64-state/float-atomic", f64, f64, False, 0),
        ("f32-mesh/f64-state/fixed", f32, f64, True, 0),
        ("f32-mesh/f64-state/float-atomic", f32, f64, False, 0),
        ("f32-mesh/f64-state/fixed/7-checkpoints", f32, f64, True, 7),
        ("f32-mesh/f32-state/fixed", f32, f32, True, 0),
        ("f32-mesh/f32-state/float-atomic", f32, f32, False, 0),
    ]
    sim, cosmo, tabs, omega_t = _setup_run(n, nm, box, nsteps, a0, f64, f64, seed=inputs.SEED_TARGET)
    sim.forward(omega_t, cosmo, tabs)
    target64 = sim.plan.density(sim.s).clone()
    del sim, omega_t
    torch.cuda.empty_cache()
    res, ref = {}, None
    for name, mdt, sdt, det, nck in modes:
        log("paint-modes: " + name)
        steps = [round((i + 1) * nsteps / nck) for i in range(nck)] if nck else []
        sim, cosmo, tabs, omega = _setup_run(n, nm, box, nsteps, a0, mdt, sdt, checkpoint_steps=steps,
                                             deterministic=det)
        coefs, ic = tabs
        st0 = {"s": torch.zeros_like(sim.s), "p": torch.zeros_like(sim.p), "acc": None}
        sim.plan.lpt(omega, cosmo, ic, st0)
        target = target64.to(mdt)
        _timed_pass(sim, omega, cosmo, target, tabs)  # warm-up
        J1, g1, th1, dt = _timed_pass(sim, omega, cosmo, target, tabs)
        g1, th1, s1 = g1.double().clone(), th1.clone(), sim.s.double().clone()
        J2, g2, th2, _ = _timed_pass(sim, omega, cosmo, target, tabs)
        s0 = st0["s"].double()
        ds = s1 - s0
        r = {"particle_steps_per_s": n ** 3 * nsteps / dt, "ms_per_pass": 1000 * dt, "checkpoints": nck,
             "reproducibility": {"grad_omega_max_abs_diff_over_max": float((g2.double() - g1).abs().max() /
                                                                           g1.abs().max()),
                                 "grad_omega_bitwise_equal": bool(torch.equal(g2.double(), g1)),
                                 "recovered_s0_bitwise_equal": bool(torch.equal(sim.s.double(), s1)),
                                 "J_rel_diff": abs(float(J2.cpu()[0]) - float(J1.cpu()[0])) / abs(float(J1.cpu()[0])),
                                 "dJ_dtheta_rel_diff": [abs(float(a) - float(b)) / abs(float(b))
                                                        for a, b in zip(th2.cpu(), th1.cpu())]},
             "reversibility_s0_rms_err_over_std": float(ds.pow(2).mean().sqrt() / s0.std())}
        if ref is None:
            ref = (g1, th1)
        r["grad_omega_rel_l2_vs_fp64"] = _rel_l2(g1, ref[0])
        r["dJ_dtheta_rel_err_vs_fp64"] = [abs(float(a) - float(b)) / abs(float(b))
                                          for a, b in zip(th1.cpu(), ref[1].cpu())]
        res[name] = r
        del sim, omega, st0, s0, ds, g1, g2, s1, target
        torch.cuda.empty_cache()
    frontier = {}
    for tgt in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        ok = [(v["particle_steps_per_s"], k) for k, v in res.items()
              if k != modes[0][0] and v["grad_omega_rel_l2_vs_fp64"] <= tgt]
        ok.append((res[modes[0][0]]["particle_steps_per_s"], modes[0][0]))   # the reference meets any target
        best = max(ok)
        frontier["%g" % tgt] = {"fastest_mode": best[1], "particle_steps_per_s": best[0]}
    return {"study": "paint-modes", "workload": "%d^3 particles, %d^3 mesh, %.0f Mpc/h, %d steps a=%.5f..1"
            % (n, nm, box, nsteps, a0), "modes": res, "fastest_mode_per_gradient_error_target": frontier,
            "reference": modes[0][0] + " (errors are against it; its own error against the oracle is at the "
                                       "1e-8 level at 32^3, GPU tests)"}


def study_lightcone(args):
    """Light-cone observation (Sec. 2.4) and the exact gradient of an
    objective on the observables (Sec. 3.4): an observer at the centre of
    the box of the workload, FP32 mesh and FP64 state, a linear objective
    with seeded weights on the 7 observed values of every particle.  Reports
    the forward and gradient times next to the plain final-density pass, the
    light-cone kernels' share and rate, a check that every particle is
    observed exactly once, and the FP64 oracle on a small run beside it."""
    import numpy as np
    import torch

    from paper_2211_09815_amd import inputs
    from paper_2211_09815_amd._lib import PM_K_LIGHTCONE
    from paper_2211_09815_amd.lightcone import LightCone
    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    sim, cosmo, tabs, omega = _setup_run(n, nm, box, nsteps, a0, torch.float32, torch.float64)
    N = n ** 3
    lc = LightCone(sim, (nm / 2.0,) * 3)
    ltabs = lc.tables(cosmo)
    w = torch.empty((7, N), dtype=torch.float32, device="cuda")
    for k in range(7):   # seeded weights, one row at a time to bound host memory
        w[k].copy_(torch.as_tensor(inputs.normal(N, inputs.SEED_COTANGENT + k, dtype=np.float32)))
    res = {}
    for rep in range(2):     # the first repetition is the warm-up
        sim.plan.timing_enable([PM_K_LIGHTCONE])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        counts = lc.forward(omega, cosmo, ltabs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_f, nl_f, by_f = sim.plan.timing_read(PM_K_LIGHTCONE)
        sim.plan.timing_enable([PM_K_LIGHTCONE])
        g, th = lc.gradient(omega, cosmo, w, ltabs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ms_g, nl_g, by_g = sim.plan.timing_read(PM_K_LIGHTCONE)
        sim.plan.timing_enable(())
        log("lightcone rep %d: forward %.3f s, gradient %.3f s" % (rep, t1 - t0, t2 - t1))
    steps_seen = [int(i) for i in np.nonzero(counts)[0]]
    ostep = lc.obs_step.cpu().numpy()
    grid = sim.cfg.a_grid()
    ah = lc.obs[6].cpu().numpy()
    in_step = bool(np.all((ah > grid[ostep - 1]) & (ah <= grid[ostep]))) if np.all(ostep > 0) else False
    res["forward_ms"] = 1000 * (t1 - t0)
    res["gradient_ms"] = 1000 * (t2 - t1)
    res["particle_steps_per_s"] = N * nsteps / (t2 - t0)
    res["observed_per_step"] = {str(i): int(counts[i]) for i in steps_seen}
    res["every_particle_observed_once"] = bool(int(counts.sum()) == N and np.all(ostep > 0) and in_step)
    gbs = (by_f / 1e9) / (ms_f / 1e3) if ms_f > 0 else None
    res["k_lightcone"] = {"launches": nl_f, "ms_total": ms_f, "avg_launch_ms": ms_f / max(nl_f, 1),
                          "algorithmic_bytes_per_launch": by_f / max(nl_f, 1), "algorithmic_GBps": gbs,
                          "frac_of_peak": gbs / HBM_PEAK_GBS if gbs else None,
                          "bytes_note": "two FP64 displacement arrays read per step; the momenta and the "
                                        "outputs of the observed particles are extra"}
    res["gradient_lightcone_kernels"] = {"launches": nl_g, "ms_total": ms_g}
    res["dJ_dtheta"] = th.cpu().tolist()
    res["grad_omega_norm"] = float(torch.linalg.vector_norm(g.double()))
    # the truncated adjoint of Sec. 3.4 (the observed particles' sourcing
    # frozen from the end of their crossing step) on the same run: its time
    # and how far its gradient is from the exact one
    g_ex, th_ex = g.double().clone(), th.clone()
    lc.forward(omega, cosmo, ltabs)        # the reverse pass consumed the final state
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_tr, th_tr = lc.gradient(omega, cosmo, w, ltabs, truncate=True)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t0
    res["truncated_gradient"] = {
        "gradient_ms": 1000 * t_tr,
        "grad_omega_rel_l2_vs_exact": float(torch.linalg.vector_norm(g_tr.double() - g_ex)
                                            / torch.linalg.vector_norm(g_ex)),
        "dJ_dtheta": th_tr.cpu().tolist(),
        "dJ_dtheta_rel_diff_vs_exact": [abs(a - b) / abs(b) for a, b in zip(th_tr.cpu().tolist(),
                                                                          th_ex.cpu().tolist())]}
    # the plain pass of the same run for comparison
    target = torch.zeros((nm,) * 3, dtype=torch.float32, device="cuda")
    _timed_pass(sim, omega, cosmo, target, tabs)
    _, _, _, dt = _timed_pass(sim, omega, cosmo, target, tabs)
    res["plain_pass_ms"] = 1000 * dt
    # the oracle beside it: forward with observation and the stored-trajectory
    # gradient, 32^3 particles on a 64^3 mesh (128 Mpc/h), 10 steps a=1/16..1
    from oracle import lightcone as olc
    from oracle import simulate as osim
    ocfg = osim.SimConfig(32, 64, 128.0, 1.0 / 16, 1.0, 10)
    om_o = inputs.white_noise(32, inputs.SEED_RUN)
    wo = inputs.normal((32 ** 3, 7), inputs.SEED_COTANGENT)
    t0 = time.perf_counter()
    olc.value_and_grad(om_o, ocfg, np.array([32.0, 32.0, 32.0]), wo)
    dt_o = time.perf_counter() - t0
    res["oracle"] = {"value": 32 ** 3 * 10 / dt_o, "unit": "particle-steps/s", "seconds": dt_o,
                     "sample": "32^3 particles, 64^3 mesh, 10 steps, forward with observation and the "
                               "stored-trajectory gradient (FP64 numpy oracle)"}
    return {"study": "lightcone", "workload": "%d^3 particles, %d^3 mesh, %.0f Mpc/h, %d steps a=%.5f..1, "
            "observer at the box centre, FP32 mesh / FP64 state" % (n, nm, box, nsteps, a0), "result": res}


def study_fd_theta(args, hs=(1e-3, 3e-4)):
    """dJ/d(Omega_m, sigma8) from the adjoint pass against central finite
    differences of the forward model (two step sizes, relative to theta)."""
    import torch
    from paper_2211_09815_amd import inputs
    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    mdt = torch.float32 if args.mesh_dtype == "f32" else torch.float64
    sdt = torch.float32 if args.state_dtype == "f32" else torch.float64
    sim, cosmo, tabs, omega_t = _setup_run(n, nm, box, nsteps, a0, mdt, sdt, seed=inputs.SEED_TARGET)
    log("fd-theta: target run")
    sim.forward(omega_t, cosmo, tabs)
    target = sim.plan.density(sim.s).clone()
    del omega_t
    npdt = "float32" if mdt == torch.float32 else "float64"
    omega = torch.as_tensor(inputs.white_noise(n, inputs.SEED_RUN, dtype=npdt), device="cuda")
    log("fd-theta: adjoint pass")
    J, g, th, dt = _timed_pass(sim, omega, cosmo, target, tabs)
    del g
    fd = {}
    for name, idx in (("omega_m", 0), ("sigma8", 1)):
        base = getattr(cosmo, name)
        fd[name] = []
        for h in hs:
            vals = []
            for sg in (1, -1):
                c = cosmo.replace(**{name: base * (1 + sg * h)})
                sim.forward(omega, c)
                Jp, _ = sim.plan.density_mse(sim.s, target, want_grad=False)
                vals.append(float(Jp.cpu()[0]))
                log("fd-theta: %s h=%g sign=%d J=%.12e" % (name, h, sg, vals[-1]))
            d = (vals[0] - vals[1]) / (2 * h * base)
            fd[name].append({"h_rel": h, "fd": d, "adjoint": float(th[idx]),
                             "rel_diff": abs(d - float(th[idx])) / abs(d)})
    return {"study": "fd-theta", "workload": "%d^3 particles, %d^3 mesh, %.0f Mpc/h, %d steps a=%.5f..1, %s-mesh/%s-state"
            % (n, nm, box, nsteps, a0, args.mesh_dtype, args.state_dtype), "J": float(J.cpu()[0]),
            "adjoint_pass_s": dt, "particle_steps_per_s": n ** 3 * nsteps / dt, "fd": fd}


# kernel families of each stage of the hot path (the paint includes the drift
# and kick fused into its binning)
STAGES = {
    "paint": ("bin", "scatter", "paint_tiles", "halo_add"),
    "fft": ("fft_r2c_z", "fft_lines", "fft_poisson", "fft_c2r_z"),
    "gather": ("gather",),
}


def family_table(plan, families, passes=1):
    """Per-family time, launches, algorithmic and method bytes since the last
    timing_enable, per pass, with the rates against the HBM peak."""
    out = {}
    for name, kid in families.items():
        ms, nl, by, mby = plan.timing_read(kid, method=True)
        if not nl:
            continue
        gbs = (by / 1e9) / (ms / 1e3)
        mgbs = (mby / 1e9) / (ms / 1e3)
        out[name] = {"ms_per_step": ms / passes, "launches_per_step": nl / passes, "avg_launch_ms": ms / nl,
                     "algorithmic_bytes_per_step": by / passes, "method_bytes_per_step": mby / passes,
                     "algorithmic_GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
                     "method_GBps": mgbs, "frac_method": mgbs / HBM_PEAK_GBS}
    return out


def stage_table(kernels):
    """The paint, FFT and gather stages (sums of their families)."""
    out = {}
    for st, fams in STAGES.items():
        ms = sum(kernels[f]["ms_per_step"] for f in fams if f in kernels)
        by = sum(kernels[f]["algorithmic_bytes_per_step"] for f in fams if f in kernels)
        mby = sum(kernels[f]["method_bytes_per_step"] for f in fams if f in kernels)
        if ms <= 0:
            continue
        out[st] = {"families": [f for f in fams if f in kernels], "ms_per_step": ms,
                   "algorithmic_GBps": by / 1e9 / (ms / 1e3), "frac": by / 1e9 / (ms / 1e3) / HBM_PEAK_GBS,
                   "method_GBps": mby / 1e9 / (ms / 1e3), "frac_method": mby / 1e9 / (ms / 1e3) / HBM_PEAK_GBS}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-warmup-child", dest="warmup_child", action="store_false",
                    help="with --hbm-warmup: skip its child process (for a run whose previous process already "
                         "cycled the memory)")
    ap.add_argument("--hbm-warmup", type=int, default=0, metavar="GIB",
                    help="untimed setup, off by default: allocate and release up to GIB GiB (at most all but "
                         "8 GiB of the free device memory), first in a child process and then in this one, "
                         "before the plan and the state are allocated")
    ap.add_argument("--workload", default="512", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto",
                    help="kernel family for the roofline object (default: the one with the most time)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference for profiler byte counters)")
    ap.add_argument("--mesh-dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--state-dtype", default="f64", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="skip the all-FP64 reference pass used for the errors against FP64")
    ap.add_argument("--study", choices=["precision", "force", "fd-theta", "checkpoints", "lightcone",
                                        "paint-modes", "cpu-oracle"],
                    help="print a study instead of the benchmark line: precision = FP32 / mixed / FP64 "
                         "reversibility, gradient error and memory vs steps; force = single force and VJP "
                         "per stage at 256^3 particles on a 512^3 mesh; fd-theta = dJ/dtheta against central "
                         "differences; checkpoints = piecewise reverse from forward checkpoints; "
                         "lightcone = light-cone observation and its gradient; paint-modes = fixed-point vs "
                         "float-atomic paint and precision modes: speed, reproducibility, reversibility, "
                         "gradient error, fastest mode per error target; cpu-oracle = the FP64 oracle on the "
                         "host per stage at the single-force shape, and the 512^3 rate extrapolated from it "
                         "(no GPU)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the mesh would shard as slabs with all-to-all transposes; not built)", file=sys.stderr)
        sys.exit(2)

    if args.study == "cpu-oracle":
        print(json.dumps(study_cpu_oracle(args)), flush=True)
        return

    if args.hbm_warmup > 0 and args.warmup_child and not args.study:
        # the same cycle first in a short child process, before this process
        # touches the GPU
        t0 = time.perf_counter()
        rc = subprocess.run([sys.executable, "-c", "import bench; bench.hbm_warmup(%d)" % args.hbm_warmup],
                            cwd=os.path.dirname(os.path.abspath(__file__))).returncode
        log("HBM warm-up in a child process: exit %d, %.1f s" % (rc, time.perf_counter() - t0))

    import torch

    from paper_2211_09815_amd import _lib, api, inputs
    from paper_2211_09815_amd.simulate import SimConfig, Simulation
    families = _lib.KERNEL_FAMILIES
    if args.study:
        out = {"precision": study_precision, "force": study_force, "fd-theta": study_fd_theta,
               "checkpoints": study_checkpoints, "lightcone": study_lightcone,
               "paint-modes": study_paint_modes}[args.study](args)
        print(json.dumps(out), flush=True)
        return

    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    mdt = torch.float32 if args.mesh_dtype == "f32" else torch.float64
    sdt = torch.float32 if args.state_dtype == "f32" else torch.float64
    torch.cuda.set_device(0)
    warm_gib, warm_s = hbm_warmup(args.hbm_warmup)
    if warm_gib:
        log("HBM warm-up: %d GiB allocated and released in %.1f s" % (warm_gib, warm_s))
    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB done")
        del x, y
    cfg = SimConfig(n, nm, box, a0, 1.0, nsteps, mdt, sdt)
    log("workload %s: %d^3 particles, %d^3 mesh, box %.0f, %d steps, mesh %s state %s"
        % (args.workload, n, nm, box, nsteps, args.mesh_dtype, args.state_dtype))
    sim = Simulation(cfg)
    cosmo = api.Cosmology()
    tabs = sim.tables(cosmo)
    log("generating white noise")
    omega = torch.as_tensor(inputs.white_noise(n, inputs.SEED_RUN, dtype="float32" if mdt == torch.float32 else "float64"),
                            device="cuda")
    omega_t = torch.as_tensor(inputs.white_noise(n, inputs.SEED_TARGET, dtype="float32" if mdt == torch.float32 else "float64"),
                              device="cuda")
    log("target run")
    sim.forward(omega_t, cosmo, tabs)
    target = sim.plan.density(sim.s).clone()
    del omega_t
    torch.cuda.synchronize()

    # The last warmup pass times every kernel family (the per-family table);
    # the timed passes then time only the roofline family, because an event
    # around every launch slows the whole pass down by several percent.
    kernels = {}
    for w in range(args.warmup):
        last = w == args.warmup - 1
        if last:
            sim.plan.timing_enable(families.values())
        t0 = time.perf_counter()
        J, g, th = sim.value_and_grad(omega, cosmo, target, tabs)
        torch.cuda.synchronize()
        log("warmup %d: %.3f s" % (w, time.perf_counter() - t0))
        if last:
            kernels = family_table(sim.plan, families)
            sim.plan.timing_enable(())
    if args.kernel != "auto":
        top = args.kernel
    elif kernels:
        top = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    else:
        top = None   # no warmup: time every family in the timed passes and pick afterwards
    timed = [families[top]] if top else list(families.values())

    sim.plan.timing_enable(timed)
    torch.cuda.reset_peak_memory_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fam = {}
    for k in range(args.steps):
        J, g, th = sim.value_and_grad(omega, cosmo, target, tabs)
        for name, kid in families.items():   # waits for this pass's timed kernels
            if kid in timed:
                fam[name] = sim.plan.timing_read(kid, method=True)
        log("step %d done (%.3f s elapsed)" % (k, time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.plan.timing_enable(())
    peak_mem = torch.cuda.max_memory_allocated()
    plan_ws = sim.plan.workspace_bytes((nm,) * 3, (n,) * 3, mdt, sdt)
    if not kernels:
        for name, (ms, nl, by, mby) in fam.items():
            if nl:
                gbs, mgbs = (by / 1e9) / (ms / 1e3), (mby / 1e9) / (ms / 1e3)
                kernels[name] = {"ms_per_step": ms / args.steps, "launches_per_step": nl / args.steps,
                                 "avg_launch_ms": ms / nl, "algorithmic_bytes_per_step": by / args.steps,
                                 "method_bytes_per_step": mby / args.steps, "algorithmic_GBps": gbs,
                                 "frac_of_peak": gbs / HBM_PEAK_GBS, "method_GBps": mgbs,
                                 "frac_method": mgbs / HBM_PEAK_GBS}
        top = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kms, klaunch, kbytes, kmbytes = fam[top]
    ms_per_step = 1000.0 * elapsed / args.steps
    value = n ** 3 * nsteps / (elapsed / args.steps)
    achieved = (kbytes / 1e9) / (kms / 1e3) if kms > 0 else None
    achieved_m = (kmbytes / 1e9) / (kms / 1e3) if kms > 0 else None
    Jv = float(J.cpu()[0])
    thv = th.cpu().tolist()
    gn = float(torch.linalg.vector_norm(g.double()).cpu())
    ok = math.isfinite(Jv) and all(math.isfinite(x) for x in thv) and math.isfinite(gn)
    log("J %.6e  |dJ/domega| %.6e  dJ/dtheta %s  finite %s" % (Jv, gn, thv, ok))
    copy_gbs = copy_bandwidth()
    log("device copy: %.0f GB/s" % copy_gbs)
    stream_gbs = stream_bandwidth(sim.plan)
    log("stream kernels: read %.0f, copy %.0f, write %.0f GB/s" % (stream_gbs["read"], stream_gbs["copy"],
                                                                   stream_gbs["write"]))
    # the whole pass's method bytes (last warmup pass) over the timed pass time
    pass_method = sum(v["method_bytes_per_step"] for v in kernels.values())
    pass_alg = sum(v["algorithmic_bytes_per_step"] for v in kernels.values())
    ref = None
    if not args.no_fp64_ref and (args.mesh_dtype, args.state_dtype) != ("f64", "f64"):
        g_keep, th_keep = g.double().clone(), th.clone()
        s_fin, k_fin, P_fin = final_state_outputs(sim, omega, cosmo, tabs)
        del sim, g
        torch.cuda.empty_cache()
        ref = fp64_reference(args, target.double(), g_keep, th_keep, s_fin, (k_fin, P_fin))

    out = {
        "metric": "particle-steps/s for forward+adjoint at %d^3" % n,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "%s-mesh/%s-state" % (args.mesh_dtype, args.state_dtype),
        "data": "synthetic",
        "config": {
            "workload": "%d^3 particles, %d^3 mesh, %.0f Mpc/h box, %d KDK steps a=%.5f..1, 2LPT + forward + "
                        "objective + reverse-time adjoint + 2LPT VJP" % (n, nm, box, nsteps, a0),
            "particles": n ** 3,
            "mesh": nm ** 3,
            "box_mpc_h": box,
            "kdk_steps": nsteps,
            "mesh_dtype": args.mesh_dtype,
            "state_dtype": args.state_dtype,
            "peak_mem_gb": (peak_mem + plan_ws) / 1e9,
            "peak_mem_note": "torch allocator peak plus the plan's own workspace",
            "hbm_warmup_gib": warm_gib,
            "process": "cold: the plan and the state are the first device memory this process and the GPU's "
                       "last process allocated" if not warm_gib else
                       "after an untimed HBM warm-up (%d GiB allocated and released%s)"
                       % (warm_gib, ", first in a child process" if args.warmup_child else ""),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": top,
            "symbol": _lib.KERNEL_SYMBOLS[top],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(top, args.workload),
            "launches": klaunch,
            "avg_launch_ms": kms / klaunch if klaunch else None,
            "algorithmic_bytes_per_launch": kbytes / klaunch if klaunch else None,
            "method_bytes_per_launch": kmbytes / klaunch if klaunch else None,
            "achieved_method": achieved_m,
            "frac_method": (achieved_m / HBM_PEAK_GBS) if achieved_m else None,
            "bytes_note": "achieved/frac: algorithmic bytes (the implementation's intermediates included: sort "
                          "keys, CIC records, lists, halos, FFT inter-pass spectra); achieved_method/frac_method: "
                          "the method's own state and field traffic only (pm_timing_read)",
            "stages": stage_table(kernels),
            "pass": {"ms": ms_per_step, "algorithmic_bytes": pass_alg, "method_bytes": pass_method,
                     "frac": pass_alg / 1e9 / (ms_per_step / 1e3) / HBM_PEAK_GBS,
                     "frac_method": pass_method / 1e9 / (ms_per_step / 1e3) / HBM_PEAK_GBS,
                     "method_bytes_per_particle_step": pass_method / (n ** 3 * nsteps)},
            "device_copy_GBps": copy_gbs,
            "frac_of_copy": (achieved / copy_gbs) if achieved else None,
            "stream_GBps": stream_gbs,
            "stream_note": "the library's own STREAM-like kernels (pm_stream), best of 5 over 2 GiB: pure "
                           "read, copy (read + write bytes), pure write",
        },
        "kernels": kernels,
        "kernels_note": ("per-family times of the last warmup pass, which times every family; the timed "
                         "passes time only the roofline family") if args.warmup else
                        "per-family times averaged over the timed passes, which time every family",
        "result": {"J": Jv, "dJ_dtheta": thv, "grad_omega_norm": gn, "finite": ok},
    }
    if ref is not None:
        out["result"].update(ref)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
