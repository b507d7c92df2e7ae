"""Benchmark of the GeoSSTV P-PDS hot path on one MI355X.

One "step" is one iteration of Alg. 1 (all of its steps) over a synthetic
256 x 256 x 128 cube with the paper's mixed noise (Gaussian sigma 0.05, sparse
rate 0.05, stripes on 10% of columns, dead columns on 2% of columns in 10% of
bands). Inputs are resident in HBM before the timed region. Prints one JSON
line: voxel-iterations/s, the roofline of the dominant kernel (HIP events over
the timed region) and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E bytes/s
ALGO_BYTES_ITER = 172  # bytes per voxel-iteration, every state word read and written once + v

# Compulsory bytes per voxel of each phase: every array it reads or writes,
# once (FP32 state and intermediates).
PHASE_BYTES = {
    # reads u, w1 (6), w2 (6), y1 (2), y2 (2), y4, v (steps 1, 4, 5, 11, 12 and
    # the u' part of 14) and s, t, y3 (inputs of the l1 projections of steps 2
    # and 3); writes u, w1, w2, y1, y2 and y4 + u'/5
    "sweep_a": 4 * (22 + 18),
    # reads s, t, y3, y4 and 5 y4 + u' - v; writes s, t, y3, y4 (steps 2, 3,
    # 13-15; y4 is kept as the residual 5 y4' - v, so v is not needed)
    "sweep_b": 4 * (5 + 4),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cube", default="256x256x128", help="N1xN2xN3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles",
                                                       "sweep_a_traffic_256x256x128.txt"))
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB five times (calibration of the HBM byte counters)")
    return ap.parse_args()


def copy_probe():
    """A plain device copy of known size: 256 MiB read and 256 MiB written per
    launch. The FETCH_SIZE / WRITE_SIZE counters of this launch give the
    factors that turn the counters of the solver's kernels into bytes."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy probe: 5 copies of 256 MiB", flush=True)


def read_traffic(path, cube):
    """HBM bytes per launch of sweep A from the stored counter summary, or None
    when it is missing, for another cube, or taken from other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v_ = line.split(":", 1)
                kv[k.strip()] = v_.strip()
    try:
        if kv["cube"] != cube or kv["source_hash"] != geo_source_hash():
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_bytes_per_kib"])
        write = float(kv["write_kib_per_dispatch"]) * float(kv["write_bytes_per_kib"])
    except (KeyError, ValueError):
        return None
    return fetch + write


def cpu_baseline(c, seconds):
    """The FP64 oracle on the same cube: as many full iterations as fit in
    about `seconds` (at least 2), on all host threads."""
    import numpy as np

    import oracle
    v = np.asarray(c["v"], dtype=np.float64)
    S = oracle.Solver(v, c["eps"], c["alpha"], c["beta"], omega=c["omega"])
    S.step(1)  # first-touch of the oracle's buffers
    done, t0 = 0, time.perf_counter()
    while True:
        S.step(1)
        done += 1
        el = time.perf_counter() - t0
        if done >= 2 and el >= seconds:
            break
    n = v.size
    return {"value": n * done / el, "unit": "voxel-iterations/s",
            "cores": int(oracle.threads_for(n)), "kind": "oracle",
            "sample": f"{done} full iterations of the FP64 oracle on the same "
                      f"{c['shape'][1]}x{c['shape'][2]}x{c['shape'][0]} cube "
                      f"({el:.1f} s)"}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from synth.cubes import CUBE_256x256x128, like, make_cube

    n1, n2, n3 = (int(x) for x in args.cube.lower().split("x"))
    spec = CUBE_256x256x128 if (n1, n2, n3) == (256, 256, 128) else like(CUBE_256x256x128, n1=n1,
                                                                          n2=n2, n3=n3)
    c = make_cube(spec)
    v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
    N = v.numel()
    dims = geo.dims_of(v.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"], tol=0.0)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, v, ws)
    geo.geo_step(dims, p, v, ws, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, phase_ms = geo.geo_step_profiled(dims, p, v, ws, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    K = args.steps
    value = N * K / el
    dom = max(PHASE_BYTES, key=lambda k: phase_ms[k])
    avg_s = phase_ms[dom] / K / 1e3
    achieved = PHASE_BYTES[dom] * N / avg_s
    traffic = read_traffic(args.traffic, f"{n1}x{n2}x{n3}") if dom == "sweep_a" else None
    out = {
        "metric": "P-PDS voxel-iterations/s",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"P-PDS (Alg. 1) on one {n1}x{n2}x{n3} cube, synthetic mixed "
                               "noise, FP32 iterates, FP64 reductions",
                   "n1": n1, "n2": n2, "n3": n3, "voxels": N, "omega": c["omega"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": traffic, "bytes_per_voxel": PHASE_BYTES[dom],
                     "traffic_bytes_per_voxel": None if traffic is None else traffic / N,
                     "avg_launch_ms": 1e3 * avg_s},
        "iteration_hbm_frac": ALGO_BYTES_ITER * value / HBM_PEAK,
        "phase_ms_per_step": {k: v_ / K for k, v_ in phase_ms.items()},
        "last": {"rel_change": res.rel_change, "r": res.r, "tau_s": res.tau_s,
                 "tau_t": res.tau_t, "iters": res.total_iters},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def geo_source_hash():
    """Hash of the kernel sources (traffic counters go stale when they change)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2510_00562_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
