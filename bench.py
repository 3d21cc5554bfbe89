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
import sys
import time

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
    "fft_lines": ["paper_2211_09815_amd/csrc/fft.hip"],
    "fft_poisson": ["paper_2211_09815_amd/csrc/fft.hip"],
    "fft_c2r_z": ["paper_2211_09815_amd/csrc/fft.hip"],
}


def measured_traffic(family):
    """HBM bytes per launch of `family` from the rocprofv3 counter summary in
    profiles/, or None if there is none or the kernel source changed since."""
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
            m = re.search(r"traffic_per_launch_bytes=([0-9.e+]+) family=(\w+) source_sha256=(\w+)", line)
            if m and m.group(2) == family and m.group(3) == digest:
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="512", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto",
                    help="kernel family for the roofline object (default: the one with the most time)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference for profiler byte counters)")
    ap.add_argument("--mesh-dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--state-dtype", default="f64", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the mesh would shard as slabs with all-to-all transposes; not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2211_09815_amd import _lib, api, inputs
    from paper_2211_09815_amd.simulate import SimConfig, Simulation
    families = _lib.KERNEL_FAMILIES

    n, nm, box, nsteps, a0 = WORKLOADS[args.workload]
    mdt = torch.float32 if args.mesh_dtype == "f32" else torch.float64
    sdt = torch.float32 if args.state_dtype == "f32" else torch.float64
    torch.cuda.set_device(0)
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

    for w in range(args.warmup):
        t0 = time.perf_counter()
        J, g, th = sim.value_and_grad(omega, cosmo, target, tabs)
        torch.cuda.synchronize()
        log("warmup %d: %.3f s" % (w, time.perf_counter() - t0))

    sim.plan.timing_enable(families.values())
    torch.cuda.reset_peak_memory_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fam = {k: [0.0, 0, 0.0] for k in families}
    for k in range(args.steps):
        J, g, th = sim.value_and_grad(omega, cosmo, target, tabs)
        for name, kid in families.items():   # waits for this pass's timed kernels
            fam[name] = list(sim.plan.timing_read(kid))
        log("step %d done (%.3f s elapsed)" % (k, time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.plan.timing_enable(())
    peak_mem = torch.cuda.max_memory_allocated()
    kernels = {}
    for name, (ms, nl, by) in fam.items():
        if nl:
            gbs = (by / 1e9) / (ms / 1e3)
            kernels[name] = {"ms_per_step": ms / args.steps, "launches_per_step": nl / args.steps,
                             "avg_launch_ms": ms / nl, "algorithmic_GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    top = max(kernels, key=lambda k: kernels[k]["ms_per_step"]) if args.kernel == "auto" else args.kernel
    kms, klaunch, kbytes = fam[top]
    ms_per_step = 1000.0 * elapsed / args.steps
    value = n ** 3 * nsteps / (elapsed / args.steps)
    achieved = (kbytes / 1e9) / (kms / 1e3) if kms > 0 else None
    Jv = float(J.cpu()[0])
    thv = th.cpu().tolist()
    gn = float(torch.linalg.vector_norm(g.double()).cpu())
    ok = math.isfinite(Jv) and all(math.isfinite(x) for x in thv) and math.isfinite(gn)
    log("J %.6e  |dJ/domega| %.6e  dJ/dtheta %s  finite %s" % (Jv, gn, thv, ok))

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
            "peak_mem_gb": peak_mem / 1e9,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": top,
            "symbol": _lib.KERNEL_SYMBOLS[top],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(top),
            "launches": klaunch,
            "avg_launch_ms": kms / klaunch if klaunch else None,
            "algorithmic_bytes_per_launch": kbytes / klaunch if klaunch else None,
        },
        "kernels": kernels,
        "result": {"J": Jv, "dJ_dtheta": thv, "grad_omega_norm": gn, "finite": ok},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
