"""Write tests/golden/c2_oracle.json: the FP64 oracle's results for the
63-step configuration (128^3 particles on a 128^3 mesh, 256 Mpc/h, a from
1/64 to 1, Eisenstein-Hu no-wiggle LambdaCDM with Omega_m 0.3, Omega_b 0.05,
h 0.7, n_s 0.96, sigma8 0.8; white noise from seed 0, target density from a
seed-1 run with the same parameters).

Everything here calls the oracle only.  Stored:
  * J, dJ/d(Omega_m, sigma8) and |dJ/domega| (stored-trajectory adjoint);
  * dJ/domega and the final displacement s_n at 4096 sampled particles, and
    the target density contrast at 4096 sampled cells;
  * central finite differences of J on 16 white-noise entries at
    h = 1e-2 and 3e-3, and on Omega_m, sigma8 at h = 1e-3 and 3e-4 of the
    value, next to the adjoint's values.

Runs for about an hour on 6 cores:
    python tests/golden/make_c2_golden.py [--workers 6]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import simulate  # noqa: E402
from paper_2211_09815_amd import inputs  # noqa: E402

N, NM, BOX, STEPS, A0 = 128, 128, 256.0, 63, 1.0 / 64
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle.json")
H_OMEGA = (1e-2, 3e-3)
H_THETA = (1e-3, 3e-4)   # relative to the parameter value
N_FD, N_SAMPLE = 16, 4096
SAMPLE_SEED, CELL_SEED = inputs.SEED_PROBES + 100, inputs.SEED_PROBES + 101

_G = {}


def cfg(cosmo=None):
    return simulate.SimConfig(N, NM, BOX, A0, 1.0, STEPS, cosmo=cosmo)


def _init(target):
    _G["target"] = target
    _G["omega"] = inputs.white_noise(N, inputs.SEED_RUN)
    _G["obj"] = simulate.FixedThetaObjective(cfg(), target)


def _task(t):
    kind = t[0]
    omega = _G["omega"]
    t0 = time.time()
    if kind == "main":
        st = {}
        J, g, th = simulate.value_and_grad(omega, cfg(), _G["target"], mode="stored", final_state_out=st)
        res = (t, (J, g, th, st["s"]))
    elif kind == "omega":
        _, idx, h, sign = t
        w = omega.copy().reshape(-1)
        w[idx] += sign * h
        res = (t, _G["obj"](w.reshape(omega.shape)))
    else:
        _, name, h, sign = t
        base = cfg().cosmo
        val = getattr(base, name)
        c = cfg(base.replace(**{name: val * (1 + sign * h)}))
        res = (t, simulate.objective_value(omega, c, _G["target"]))
    print("done %s in %.0f s" % (str(t), time.time() - t0), flush=True)
    return res


def target_sample(target):
    cells = inputs.probe_indices(target.size, N_SAMPLE, seed=CELL_SEED)
    flat = target.reshape(-1)
    return {"idx": [int(i) for i in cells], "value": [float(flat[i]) for i in cells]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    args = ap.parse_args()
    t0 = time.time()
    target = simulate.final_density(inputs.white_noise(N, inputs.SEED_TARGET), cfg())
    print("target done in %.0f s" % (time.time() - t0), flush=True)
    npart = N ** 3
    fd_idx = inputs.probe_indices(npart, N_FD, seed=inputs.SEED_PROBES)
    sample = inputs.probe_indices(npart, N_SAMPLE, seed=SAMPLE_SEED)
    tasks = [("main",)]
    tasks += [("omega", int(i), h, sg) for h in H_OMEGA for i in fd_idx for sg in (1, -1)]
    tasks += [("theta", nm, h, sg) for nm in ("omega_m", "sigma8") for h in H_THETA for sg in (1, -1)]
    with Pool(args.workers, initializer=_init, initargs=(target,)) as pool:
        results = dict(pool.map(_task, tasks, chunksize=1))
    J, g, th, s_n = results[("main",)]
    g = g.reshape(-1)
    fd = [[(results[("omega", int(i), h, 1)] - results[("omega", int(i), h, -1)]) / (2 * h) for i in fd_idx]
          for h in H_OMEGA]
    base = cfg().cosmo
    fd_th = [[(results[("theta", nm, h, 1)] - results[("theta", nm, h, -1)]) / (2 * h * getattr(base, nm))
              for nm in ("omega_m", "sigma8")] for h in H_THETA]
    out = {
        "config": {"particles_per_side": N, "mesh_per_side": NM, "box": BOX, "steps": STEPS, "a_start": A0,
                   "a_end": 1.0, "seed_run": inputs.SEED_RUN, "seed_target": inputs.SEED_TARGET},
        "J": J,
        "dJ_dtheta": [float(th[0]), float(th[1])],
        "grad_norm": float(np.linalg.norm(g)),
        "sample_idx": [int(i) for i in sample],
        "grad_sample": [float(g[i]) for i in sample],
        "s_final_sample": [[float(v) for v in s_n[i]] for i in sample],
        "target_sample": target_sample(target),
        "fd_omega": {"idx": [int(i) for i in fd_idx], "adjoint": [float(g[i]) for i in fd_idx],
                     "h": list(H_OMEGA), "fd": fd},
        "fd_theta": {"h_rel": list(H_THETA), "adjoint": [float(th[0]), float(th[1])], "fd": fd_th},
        "wall_seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
