"""Writes the FP64 oracle's state after long runs, sampled, for the GPU
parity tests at full iteration counts. Calls only oracle/ and synth/.

Runs (pick any with their names on the command line; default: all):

  256    long_256x256x128_5000.json: the 256 x 256 x 128 benchmark cube after
         5000 iterations from the initial point: the last trace entry
         (relative change, r, tau_s, tau_t), the MPSNR of u against the clean
         cube (eq. (29)), per-band means of u, and u, s, t at 4096 seeded
         sample voxels. About 40 minutes on 8 cores.
  batch  batch32_3000.json: three cubes of the 32-cube uneven batch (the
         smallest, the largest and the one whose width fills the 64- and
         128-column tiles worst) after 3000 iterations, the same fields for
         each. About 40 minutes on 8 cores.
  512    long_512x512x224_5000.json: the 512 x 512 x 224 cube after 5000
         iterations, the same fields at checkpoints after 1, 10, 100, 1000
         and 5000 iterations. About 5 hours on 8 cores and 31 GB of memory.
  quality quality_cases_300.json: the paper's noise cases 1 and 5 (Sec.
         IV-A) on a 120 x 120 x 99 synthetic cube with the radii of eqs.
         (25)-(27), for omega 0.01, 0.03 and 0.05: 300 iterations each, the
         same fields plus MSSIM (eq. (30)). A few minutes.

Run from the repository root: python tests/golden/make_long_runs.py [runs]"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth.cubes import CUBE_256x256x128, CUBE_512x512x224, batch_specs, make_cube  # noqa: E402

SAMPLES, SAMPLE_SEED = 4096, 12345
# cubes of the uneven batch checked against the oracle: the smallest
# (123 x 107 x 44), the largest (246 x 248 x 154) and the one of 137 columns
# (9 columns past a whole number of 64- and of 128-column tiles)
BATCH_CUBES = (20, 28, 4)
BATCH_ITERS = 3000


def sample_index(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=SAMPLES, replace=False))


def snapshot(S, u_clean, idx, iters):
    return {
        "iterations": iters,
        "last_trace": {"rel": S.trace[-1][0], "r": S.trace[-1][1], "tau_s": S.trace[-1][2],
                       "tau_t": S.trace[-1][3]},
        "mpsnr": oracle.mpsnr(S.u, u_clean),
        "band_mean_u": S.u.reshape(S.u.shape[0], -1).mean(axis=1).tolist(),
        "u": S.u.ravel()[idx].tolist(),
        "s": S.s.ravel()[idx].tolist(),
        "t": S.t.ravel()[idx].tolist(),
    }


def solver_for(c):
    v = np.asarray(c["v"], dtype=np.float32).astype(np.float64)  # what the GPU sees
    return oracle.Solver(v, c["eps"], c["alpha"], c["beta"], omega=c["omega"])


def run_to(S, label, target, t0, every=100):
    while len(S.trace) < target:
        S.step(min(every, target - len(S.trace)))
        print(f"{label}: {len(S.trace)} iterations, {time.time() - t0:.0f} s, "
              f"rel {S.trace[-1][0]:.3e}", flush=True)


def write(name, out):
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


def run_256():
    c = make_cube(CUBE_256x256x128)
    S = solver_for(c)
    t0 = time.time()
    run_to(S, "256x256x128", 5000, t0, every=500)
    idx = sample_index(S.u.size)
    out = {"cube": "256x256x128", "omega": c["omega"], "eps": c["eps"], "alpha": c["alpha"],
           "beta": c["beta"], "sample_seed": SAMPLE_SEED, "sample_index": idx.tolist()}
    out.update(snapshot(S, c["u_clean"], idx, 5000))
    write("long_256x256x128_5000.json", out)


def run_batch():
    specs = batch_specs()
    cubes = []
    for q in BATCH_CUBES:
        sp = specs[q]
        c = make_cube(sp)
        S = solver_for(c)
        t0 = time.time()
        run_to(S, f"batch cube {q} ({sp.n1}x{sp.n2}x{sp.n3})", BATCH_ITERS, t0, every=250)
        idx = sample_index(S.u.size)
        e = {"index": q, "n1": sp.n1, "n2": sp.n2, "n3": sp.n3, "eps": c["eps"],
             "alpha": c["alpha"], "beta": c["beta"], "omega": c["omega"],
             "sample_index": idx.tolist()}
        e.update(snapshot(S, c["u_clean"], idx, BATCH_ITERS))
        cubes.append(e)
        del S, c
    write("batch32_3000.json", {"iterations": BATCH_ITERS, "sample_seed": SAMPLE_SEED,
                                "cubes": cubes})


def run_512():
    c = make_cube(CUBE_512x512x224)
    u_clean = c["u_clean"]
    S = solver_for(c)
    head = {"cube": "512x512x224", "omega": c["omega"], "eps": c["eps"], "alpha": c["alpha"],
            "beta": c["beta"], "sample_seed": SAMPLE_SEED}
    del c
    idx = sample_index(S.u.size)
    head["sample_index"] = idx.tolist()
    t0 = time.time()
    checkpoints = []
    for target in (1, 10, 100, 1000, 5000):
        run_to(S, "512x512x224", target, t0)
        checkpoints.append(snapshot(S, u_clean, idx, target))
        # partial file after every checkpoint, so a long run leaves something
        write("long_512x512x224_5000.json", dict(head, checkpoints=checkpoints,
                                                  complete=target == 5000))


QUALITY_CASES, QUALITY_OMEGAS, QUALITY_ITERS = (1, 5), (0.01, 0.03, 0.05), 300


def run_quality():
    from synth.cubes import PAVIA_SHAPE, paper_case
    from synth.quality import mssim
    n1, n2, n3 = PAVIA_SHAPE
    solves = []
    for case in QUALITY_CASES:
        for omega in QUALITY_OMEGAS:
            c = paper_case(case, n1, n2, n3, seed=0, omega=omega)
            S = solver_for(c)
            t0 = time.time()
            run_to(S, f"case {case} omega {omega}", QUALITY_ITERS, t0, every=QUALITY_ITERS)
            idx = sample_index(S.u.size)
            e = {"case": case, "omega": omega, "eps": c["eps"], "alpha": c["alpha"],
                 "beta": c["beta"], "sample_index": idx.tolist(),
                 "mssim": mssim(S.u, c["u_clean"])}
            e.update(snapshot(S, c["u_clean"], idx, QUALITY_ITERS))
            solves.append(e)
    write("quality_cases_300.json", {"shape": [n3, n1, n2], "iterations": QUALITY_ITERS,
                                     "sample_seed": SAMPLE_SEED, "solves": solves})


RUNS = {"256": run_256, "batch": run_batch, "512": run_512, "quality": run_quality}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(RUNS)):
        RUNS[name]()
