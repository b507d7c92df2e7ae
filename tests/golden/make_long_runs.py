"""Writes the FP64 oracle's state after long runs, sampled, for the GPU
parity tests at full iteration counts. Calls only oracle/ and synth/.

  long_256x256x128_5000.json: the 256 x 256 x 128 benchmark cube after 5000
  iterations of Alg. 1 from its initial point (the iteration count the
  workload is quoted for): the last trace entry (relative change, r, tau_s,
  tau_t), the MPSNR of u against the clean cube (eq. (29)), per-band means
  of u, and u, s, t at 4096 seeded sample voxels.

Run from the repository root: python tests/golden/make_long_runs.py
(about 40 minutes on 8 cores)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth.cubes import CUBE_256x256x128, make_cube  # noqa: E402

SAMPLES, SAMPLE_SEED, ITERS = 4096, 12345, 5000


def sample_index(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=SAMPLES, replace=False))


def main():
    c = make_cube(CUBE_256x256x128)
    v = np.asarray(c["v"], dtype=np.float32).astype(np.float64)  # what the GPU sees
    S = oracle.Solver(v, c["eps"], c["alpha"], c["beta"], omega=c["omega"])
    t0 = time.time()
    for done in range(0, ITERS, 500):
        S.step(500)
        print(f"{done + 500} iterations, {time.time() - t0:.0f} s, rel {S.trace[-1][0]:.3e}",
              flush=True)
    idx = sample_index(v.size)
    out = {
        "cube": "256x256x128", "iterations": ITERS, "omega": c["omega"],
        "eps": c["eps"], "alpha": c["alpha"], "beta": c["beta"],
        "last_trace": {"rel": S.trace[-1][0], "r": S.trace[-1][1], "tau_s": S.trace[-1][2],
                       "tau_t": S.trace[-1][3]},
        "mpsnr": oracle.mpsnr(S.u, c["u_clean"]),
        "band_mean_u": S.u.reshape(S.u.shape[0], -1).mean(axis=1).tolist(),
        "sample_seed": SAMPLE_SEED,
        "sample_index": idx.tolist(),
        "u": S.u.ravel()[idx].tolist(),
        "s": S.s.ravel()[idx].tolist(),
        "t": S.t.ravel()[idx].tolist(),
    }
    path = os.path.join(ROOT, "tests", "golden", "long_256x256x128_5000.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
