"""Write tests/golden/c3_oracle.json: the FP64 oracle's single force and
force VJP for the single-force configuration (256^3 particles displaced by
2LPT at a = 0.5, painted to a 512^3 mesh in a 512 Mpc/h box; Eisenstein-Hu
no-wiggle LambdaCDM with Omega_m 0.3, Omega_b 0.05, h 0.7, n_s 0.96,
sigma8 0.8; white noise from seed 0, cotangent of the accelerations from
seed 3).  The displacements are rounded to float32 first, the form in which
the GPU path holds them, so both sides see identical positions.

Everything here calls the oracle only.  Stored: accelerations and the VJP's
displacement cotangent at 4096 sampled particles, the full coefficient
cotangent, and sum(a) (momentum conservation).

    python tests/golden/make_c3_golden.py          # about 5 minutes
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cosmology, lpt, pm  # noqa: E402
from paper_2211_09815_amd import inputs  # noqa: E402

N, NM, BOX, A = 256, 512, 512.0, 0.5
COEF = 1.5 * 0.3
N_SAMPLE = 4096
SAMPLE_SEED = inputs.SEED_PROBES + 200
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle.json")


def displacements():
    """The float32-rounded 2LPT displacement (N^3, 3) in mesh cells."""
    s, _ = lpt.lpt(inputs.white_noise(N, inputs.SEED_RUN), BOX, cosmology.Cosmo(), A, NM / N)
    return s.astype(np.float32).astype(np.float64)


def cotangent():
    """Seeded cotangent of the accelerations, (N^3, 3), float32 values."""
    return inputs.normal((3, N ** 3), inputs.SEED_COTANGENT, dtype=np.float32).astype(np.float64).T


def main():
    t0 = time.time()
    s = displacements()
    x = pm.lattice_positions((N,) * 3, NM / N) + s
    print("lpt done in %.0f s" % (time.time() - t0), flush=True)
    shape = (NM,) * 3
    xbar, coef_bar, a = pm.force_vjp(x, cotangent(), shape, N ** 3, COEF)
    print("force and vjp done in %.0f s" % (time.time() - t0), flush=True)
    idx = inputs.probe_indices(N ** 3, N_SAMPLE, seed=SAMPLE_SEED)
    out = {
        "config": {"particles_per_side": N, "mesh_per_side": NM, "box": BOX, "a": A, "coef": COEF,
                   "seed_run": inputs.SEED_RUN, "seed_cotangent": inputs.SEED_COTANGENT},
        "sample_idx": [int(i) for i in idx],
        "acc_sample": [[float(v) for v in a[i]] for i in idx],
        "acc_rms": float(np.sqrt(np.mean(a * a))),
        "acc_sum": [float(v) for v in a.sum(0)],
        "xbar_sample": [[float(v) for v in xbar[i]] for i in idx],
        "coef_bar": float(coef_bar),
        "wall_seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
