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


def algo_bytes_iter(db):
    """Algorithmic bytes per voxel-iteration: the 21 state words read and
    written once (15 FP32 words of u, s, t, w1, w2; 6 dual words of y1..y4 in
    db bytes each) plus v: 172 B with FP32 duals, 148 B with BF16."""
    return 2 * (15 * 4 + 6 * db) + 4


def phase_bytes(db):
    """Compulsory bytes per voxel of each phase (every array it reads or
    writes, once), duals and the y4 intermediate in db bytes."""
    return {
        # reads u, w1 (6), w2 (6), v, s, t (FP32) and y1 (2), y2 (2), y4, y3
        # (steps 1, 4, 5, 11, 12, the u' part of 14 and the inputs of the l1
        # projections of steps 2 and 3); writes u, w1, w2 and y1, y2 and
        # 5 y4 + u' - v
        "sweep_a": 4 * 16 + db * 6 + 4 * 13 + db * 5,
        # reads s, t and y3, y4, 5 y4 + u' - v; writes s, t and y3, y4 (steps
        # 2, 3, 13-15; y4 is kept as the residual 5 y4' - v, so v is not read)
        "sweep_b": 4 * 2 + db * 3 + 4 * 2 + db * 2,
    }


PHASE_BYTES = phase_bytes(4)
ALGO_BYTES_ITER = algo_bytes_iter(4)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cube", default="256x256x128", help="N1xN2xN3")
    ap.add_argument("--workload", choices=("cube", "batch", "serve", "quality", "realshape",
                                           "regularizer"),
                    default="cube",
                    help="cube: one cube (default); batch: 32 uneven cubes, batched launches "
                         "vs the per-cube loop; serve: a request stream through the "
                         "request loop (p50/p99 latency); quality: the paper's five noise cases "
                         "on cubes of its two image shapes, omega sweep, MPSNR/MSSIM; realshape: "
                         "the shapes and fixed radii of its real-image experiment, solved to "
                         "tol 1e-5; regularizer: the cube solved with a comparison "
                         "regularizer of Sec. IV-A (--regularizer) in place of GeoSSTV")
    ap.add_argument("--regularizer", choices=("sstv", "hsstv1", "hsstv2"), default="hsstv2",
                    help="regularizer workload: which comparison regularizer")
    ap.add_argument("--requests", type=int, default=0,
                    help="serve: requests in the stream (0: those arriving within --seconds)")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: Poisson arrivals per second")
    ap.add_argument("--seconds", type=float, default=120.0,
                    help="serve: arrivals stop after this many seconds; the queue then drains")
    ap.add_argument("--pool", type=int, default=4, help="serve: distinct cubes per size")
    ap.add_argument("--hbm-budget-gb", type=float, default=96.0, help="serve: admission budget")
    ap.add_argument("--active-mvoxels", type=float, default=16.0,
                    help="serve: admit while fewer voxels than this (millions) are in flight; "
                         "0 = by HBM footprint alone")
    ap.add_argument("--dual", choices=("f32", "bf16"), default="f32",
                    help="storage of the dual variables y1..y4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare", action="store_true",
                    help="quality: also solve the cases with SSTV, HSSTV1 and HSSTV2 (Sec. IV-A)")
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


def copy_ceiling():
    """Bytes/s of a plain device copy (torch's copy kernel, 512 MiB read and
    512 MiB written per launch, well beyond the 256 MB memory-side cache):
    the streaming rate this chip reaches in practice, beside its 8 TB/s
    peak. Mean of 10 launches after 2 untimed ones."""
    import torch
    a = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / 10
    del a, b
    return 2 * 512 * 1024 * 1024 / sec


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


def cpu_baseline(c, seconds, reg=0, what="the FP64 oracle"):
    """The FP64 oracle on the same cube, on all host threads, timed over one
    call of k full iterations: k grows from 2 until a call takes at least
    half of `seconds`. One call per iteration would time the oracle's
    per-call set-up too (its scratch, 42 doubles per voxel, is allocated and
    first touched by every call: 0.25 instead of 0.16 s per iteration at
    256x256x128 on 16 threads)."""
    import numpy as np

    import oracle
    v = np.asarray(c["v"], dtype=np.float64)
    if reg:
        S = oracle.VariantSolver(v, c["eps"], c["alpha"], c["beta"], reg, omega=c["omega"])
    else:
        S = oracle.Solver(v, c["eps"], c["alpha"], c["beta"], omega=c["omega"])
    k = 2
    while True:
        t0 = time.perf_counter()
        S.step(k)
        el = time.perf_counter() - t0
        if el >= 0.5 * seconds or k >= 1 << 20:
            break
        k = max(2 * k, int(k * 0.75 * seconds / max(el, 1e-6)))
    n = v.size
    n3, n1, n2 = c["shape"]
    return {"value": n * k / el, "unit": "voxel-iterations/s",
            "cores": int(oracle.threads_for(n)), "kind": "oracle",
            "sample": f"{k} full iterations of {what} in one call on the same "
                      f"{n1}x{n2}x{n3} cube ({el:.1f} s)"}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "quality":
        return bench_quality(args)
    if args.workload == "realshape":
        return bench_realshape(args)
    if args.workload == "regularizer":
        return bench_regularizer(args)
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from synth.cubes import CUBE_256x256x128, CUBE_512x512x224, like, make_cube

    n1, n2, n3 = (int(x) for x in args.cube.lower().split("x"))
    named = {(256, 256, 128): CUBE_256x256x128, (512, 512, 224): CUBE_512x512x224}
    spec = named.get((n1, n2, n3)) or like(CUBE_256x256x128, n1=n1, n2=n2, n3=n3)
    c = make_cube(spec)
    v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
    N = v.numel()
    dims = geo.dims_of(v.shape)
    db = 2 if args.dual == "bf16" else 4
    PB = phase_bytes(db)
    p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"], tol=0.0,
                   dual_storage=geo.GEO_STORE_BF16 if db == 2 else geo.GEO_STORE_F32)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, v, ws)
    geo.geo_step(dims, p, v, ws, args.warmup)
    torch.cuda.synchronize()
    # timed region: HIP events around the dominant kernel (the fused sweep)
    # only, on the stream it runs on
    t0 = time.perf_counter()
    res, sweep_a_ms = geo.geo_step_timed(dims, p, v, ws, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    K = args.steps
    value = N * K / el
    # per-phase breakdown from a separate, untimed run with events at every
    # phase boundary (they add about 4% to the iteration)
    _, phase_ms = geo.geo_step_profiled(dims, p, v, ws, min(K, 100))
    phase_ms = {k: x * K / min(K, 100) for k, x in phase_ms.items()}
    dom = "sweep_a"
    avg_s = sweep_a_ms / K / 1e3
    achieved = PB[dom] * N / avg_s
    # one sweep A launch per iteration: its time cannot exceed the step's
    consistent = avg_s * 1e3 <= 1e3 * el / K
    traffic = (read_traffic(args.traffic, f"{n1}x{n2}x{n3}")
               if dom == "sweep_a" and db == 4 else None)
    copy_bps = copy_ceiling()
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
                               "noise, FP32 iterates" + (", BF16-stored duals" if db == 2 else "")
                               + ", FP64 reductions",
                   "n1": n1, "n2": n2, "n3": n3, "voxels": N, "omega": c["omega"],
                   "dual_storage": args.dual},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK if consistent else None,
                     "traffic": traffic, "bytes_per_voxel": PB[dom],
                     "traffic_bytes_per_voxel": None if traffic is None else traffic / N,
                     "avg_launch_ms": 1e3 * avg_s,
                     # the same figures against what a plain copy reaches
                     "copy_ceiling": copy_bps / 1e9, "frac_of_copy": achieved / copy_bps,
                     "traffic_rate": None if traffic is None else traffic / avg_s / 1e9},
        "iteration_hbm_frac": algo_bytes_iter(db) * value / HBM_PEAK,
        "phase_ms_per_step": {k: v_ / K for k, v_ in phase_ms.items()},
        "last": {"rel_change": res.rel_change, "r": res.r, "tau_s": res.tau_s,
                 "tau_t": res.tau_t, "iters": res.total_iters},
        # the timed call: launch slots issued (one per iteration: a missed
        # l1 window is resolved inside its slot) and missed windows in it
        "timed_call": {"slots": res.slots, "missed_windows": res.fallback_passes,
                       "sweep_a_samples": len(range(7, K, 8)) if K >= 8 else K},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """32 uneven cubes: the batched launches (persistent sweep over every
    cube's tiles, one graph-replayed launch sequence per iteration, band
    chunk from the autotuner) against the per-cube loop (geo_step on each
    cube in turn) on the same GPU, same iterations, same results (the
    batched iterates are bit-identical to the per-cube ones)."""
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from paper_2510_00562_amd.tune import tune_band_chunk
    from synth.cubes import batch_specs, make_cube

    specs = batch_specs()
    db = 2 if args.dual == "bf16" else 4
    store = geo.GEO_STORE_BF16 if db == 2 else geo.GEO_STORE_F32
    dims, ps, vs, wss = [], [], [], []
    for spec in specs:
        c = make_cube(spec)
        v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
        d = geo.dims_of(v.shape)
        p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"], dual_storage=store)
        dims.append(d)
        ps.append(p)
        vs.append(v)
        wss.append(geo.Workspace(geo.geo_workspace_size(d, p)))
    total = sum(v.numel() for v in vs)
    table = geo.Workspace(geo.geo_batch_table_size(len(vs)))
    kc, tune_ms = tune_band_chunk(dims, ps, vs, wss, table, candidates="auto")
    K, W = args.steps, args.warmup

    # per-cube loop: each cube alone, one after the other, at the band chunk
    # the library picks for a cube alone (the batch's tuned chunk suits the
    # batch, not the single cubes)
    solo = [geo.params(p.eps, p.alpha, p.beta, p.mu_lo, p.mu_hi, p.omega,
                       dual_storage=p.dual_storage) for p in ps]
    for d, p, v, ws in zip(dims, solo, vs, wss):
        geo.geo_state_init(d, p, v, ws)
        geo.geo_step(d, p, v, ws, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, p, v, ws in zip(dims, solo, vs, wss):
        geo.geo_step(d, p, v, ws, K)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0

    # batched: every cube in one launch sequence per iteration
    for d, p, v, ws in zip(dims, ps, vs, wss):
        geo.geo_state_init(d, p, v, ws)
    geo.geo_batch_step(dims, ps, vs, wss, table, W, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, res = geo.geo_batch_step(dims, ps, vs, wss, table, K, use_graph=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    assert all(r.iters == K for r in res)
    value = total * K / t_batch
    out = {
        "metric": "P-PDS voxel-iterations/s",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * t_batch / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"P-PDS (Alg. 1) on a batch of {len(vs)} uneven cubes "
                               "(N1, N2 in 64..256, N3 in 32..190), batched launches with "
                               "HIP graph replay", "cubes": len(vs), "voxels": total,
                   "dual_storage": args.dual, "band_chunk": kc},
        "roofline": {"bound": "hbm", "kernel": "whole iteration",
                     "achieved": algo_bytes_iter(db) * value / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": algo_bytes_iter(db) * value / HBM_PEAK,
                     "traffic": None, "bytes_per_voxel": algo_bytes_iter(db)},
        "per_cube_loop": {"value": total * K / t_loop, "ms_per_step": 1e3 * t_loop / K},
        "speedup_vs_per_cube_loop": t_loop / t_batch,
        "tuner_ms_per_iteration": tune_ms,
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """A request stream (Poisson arrivals at --rate per second for --seconds,
    four cube sizes, tolerance 1e-4, cap 5000) served in real time by the
    request loop, then drained: latency from arrival to result on the host,
    throughput and the offered load (rho). The same jobs are then solved one
    after another alone (copy in, init, iterate to the rule, copy out) for
    the rate the loop has to beat. Request q takes its cube from a pool of
    --pool cubes per size (generating thousands of distinct cubes would take
    the host longer than serving them); each request is still a job of its
    own, solved from its initial point in its own workspace."""
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from paper_2510_00562_amd.serve import Job, run_stream
    from synth.cubes import like, make_cube, serving_specs

    store = geo.GEO_STORE_BF16 if args.dual == "bf16" else geo.GEO_STORE_F32
    n_req = args.requests if args.requests > 0 else int(round(args.rate * args.seconds * 1.2)) + 8
    specs = [(t, sp) for t, sp in serving_specs(n_req, args.rate) if t <= args.seconds]
    pool = {}
    jobs = []
    for q, (arr, spec) in enumerate(specs):
        key = (spec.n1, spec.n2, spec.n3, q % args.pool)
        if key not in pool:
            c = make_cube(like(spec, seed=40000 + len(pool)))
            pool[key] = (np.ascontiguousarray(c["v"], dtype=np.float32), c["eps"], c["alpha"],
                         c["beta"], c["omega"])
        v, eps, alpha, beta, omega = pool[key]
        jobs.append(Job(q, v, eps, alpha, beta, omega=omega, tol=1e-4, cap=5000, arrival=arr))
    print(f"serve: {len(jobs)} requests in {args.seconds:.0f} s at {args.rate}/s, "
          f"{len(pool)} distinct cubes", flush=True)
    torch.cuda.synchronize()
    cap = int(args.active_mvoxels * 1e6) if args.active_mvoxels > 0 else None
    rep = run_stream(jobs, int(args.hbm_budget_gb * 2 ** 30), round_iters=25, dual_storage=store,
                     active_voxels=cap, keep_results=False,
                     on_progress=lambda st: print("serve: " + ", ".join(
                         f"{k} {v:.0f}" for k, v in st.items()), flush=True))
    done = rep.pop("jobs")
    print(f"serve: stream done in {rep['span_s']:.1f} s", flush=True)
    mean_vox = float(np.mean([j.v.size for j in done]))
    offered = args.rate * mean_vox * rep["mean_iterations"]
    sustainable = rep["busy_voxel_iterations_per_s"] / (mean_vox * rep["mean_iterations"])
    # the same jobs alone, one after another: every distinct cube once, each
    # weighted by how many requests used it
    solo_t, solo_vi = 0.0, 0.0
    uses = {}
    for j in done:
        uses.setdefault(id(j.v), [j, 0])[1] += 1
    for j, k in uses.values():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vd = torch.from_numpy(j.v).cuda()
        dims = geo.dims_of(vd.shape)
        p = geo.params(j.eps, j.alpha, j.beta, omega=j.omega, tol=j.tol, max_iter=j.cap,
                       dual_storage=store)
        ws = geo.Workspace(geo.geo_workspace_size(dims, p))
        u, s_, t_ = (torch.empty_like(vd) for _ in range(3))
        r = geo.geo_solve(dims, p, vd, u, s_, t_, ws)
        host = [x.cpu() for x in (u, s_, t_)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert r.iters == j.iters, (r.iters, j.iters)
        solo_t += k * el
        solo_vi += k * r.iters * vd.numel()
        del host, ws
    solo_rate = solo_vi / solo_t
    out = {
        "metric": "P-PDS request loop latency",
        "value": rep["latency_p50_s"],
        "unit": "s (p50, arrival to result on host)",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "config": {"workload": f"Poisson {args.rate}/s for {args.seconds:.0f} s ({len(done)} requests), "
                               "sizes 128x128x64 / 256x256x128 / 256x256x190 / 512x512x224 "
                               "(0.4/0.3/0.2/0.1), tol 1e-4, cap 5000, FIFO admission by HBM "
                               "footprint, copies overlapped with the rounds",
                   "hbm_budget_gb": args.hbm_budget_gb, "active_mvoxels": args.active_mvoxels,
                   "dual_storage": args.dual, "cube_pool_per_size": args.pool},
        "latency_p50_s": rep["latency_p50_s"],
        "latency_p99_s": rep["latency_p99_s"],
        "latency_mean_s": rep["latency_mean_s"],
        "requests_per_s": rep["requests_per_s"],
        "voxel_iterations_per_s": rep["voxel_iterations_per_s"],
        "busy_voxel_iterations_per_s": rep["busy_voxel_iterations_per_s"],
        "solo_voxel_iterations_per_s": solo_rate,
        "served_over_solo": rep["busy_voxel_iterations_per_s"] / solo_rate,
        "mean_iterations": rep["mean_iterations"],
        "converged": rep["converged"],
        "errors": rep["errors"],
        "offered_voxel_iterations_per_s": offered,
        "rho": offered / rep["busy_voxel_iterations_per_s"],
        "sustainable_requests_per_s": sustainable,
        "span_s": rep["span_s"],
        "busy_s": rep["busy_s"],
    }
    print(json.dumps(out), flush=True)


def bench_quality(args):
    """Restoration quality in the paper's protocol on synthetic stand-ins:
    cubes of the shapes of its two simulated-noise images (120x120x99 and
    100x100x198), noise cases 1-5 with the radius rule of eqs. (25)-(27),
    omega in {0.01, 0.03, 0.05}, stopping rule eq. (28) at 1e-5; MPSNR and
    MSSIM (eqs. (29), (30)). All 30 solves run as one batch."""
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from synth.cubes import CASES, JASPER_SHAPE, PAVIA_SHAPE, paper_case
    from synth.quality import mpsnr, mssim

    runs = []
    for name, (n1, n2, n3) in (("pavia_shape", PAVIA_SHAPE), ("jasper_shape", JASPER_SHAPE)):
        for case in sorted(CASES):
            c = paper_case(case, n1, n2, n3, seed=100 * case + n3)
            for omega in (0.01, 0.03, 0.05):
                runs.append((name, case, omega, c))
    dims, ps, vs, wss = [], [], [], []
    for name, case, omega, c in runs:
        v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
        d = geo.dims_of(v.shape)
        p = geo.params(c["eps"], c["alpha"], c["beta"], omega=omega, tol=1e-5)
        ws = geo.Workspace(geo.geo_workspace_size(d, p))
        geo.geo_state_init(d, p, v, ws)
        dims.append(d)
        ps.append(p)
        vs.append(v)
        wss.append(ws)
    table = geo.Workspace(geo.geo_batch_table_size(len(vs)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, res = geo.geo_batch_step(dims, ps, vs, wss, table, 20000, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rows = []
    for (name, case, omega, c), d, p, v, ws, r in zip(runs, dims, ps, vs, wss, res):
        u = torch.empty_like(v)
        geo.geo_state_get(d, p, ws, "u", v, u)
        uh = u.cpu().numpy().astype(np.float64)
        rows.append({"image": name, "case": case, "omega": omega, "iters": r.iters,
                     "converged": bool(r.converged), "mpsnr": mpsnr(uh, c["u_clean"]),
                     "mssim": mssim(uh, c["u_clean"]),
                     "input_mpsnr": mpsnr(c["v"], c["u_clean"])})
    best = {}
    for row in rows:
        key = f"{row['image']}/case{row['case']}"
        if key not in best or row["mpsnr"] > best[key]["mpsnr"]:
            best[key] = {k: row[k] for k in ("omega", "mpsnr", "mssim", "iters")}
    vox_it = sum(v.numel() * r.iters for v, r in zip(vs, res))
    out = {
        "metric": "restoration quality (MPSNR dB, MSSIM) of the paper's protocol",
        "value": float(np.mean([b["mpsnr"] for b in best.values()])),
        "unit": "dB (mean of the best-omega MPSNR over images and cases)",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic stand-ins of the two image shapes (the datasets are not available)",
        "config": {"workload": "cases 1-5 of Sec. IV-A, radii of eqs. (25)-(27), omega in "
                               "{0.01, 0.03, 0.05}, tol 1e-5, cap 20000, one batch of 30 solves"},
        "best_per_case": best,
        "runs": rows,
        "seconds": el,
        "voxel_iterations_per_s": vox_it / el,
    }
    if args.compare:
        out["comparison"] = quality_comparison(runs, best)
    print(json.dumps(out), flush=True)


def quality_comparison(runs, best):
    """The comparison of Sec. IV-A on the same cubes: SSTV, HSSTV1 and
    HSSTV2 in place of GeoSSTV in the same problem, solved by the same P-PDS
    to the same stopping rule (geo_solve, one cube at a time), each with
    the best MPSNR over one omega grid (the paper's {0.01, 0.03, 0.05}
    widened upward to 0.5: the paper does not state HSSTV's weight, and on
    these cubes both methods' best sits at the top of the paper's grid;
    SSTV has none). GeoSSTV is reported on the paper's grid (the batched
    runs above) and on the wide grid."""
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from synth.quality import mpsnr, mssim

    cubes = {}
    for name, case, omega, c in runs:
        cubes[(name, case)] = c
    wide = (0.01, 0.03, 0.05, 0.1, 0.2, 0.5)
    methods = (("geosstv_wide", 0, (0.1, 0.2, 0.5)),  # with the paper's grid below
               ("sstv", geo.REGULARIZERS["sstv"], (0.0,)),
               ("hsstv1", geo.REGULARIZERS["hsstv1"], wide),
               ("hsstv2", geo.REGULARIZERS["hsstv2"], wide))
    per_case = {}
    t0 = time.perf_counter()
    for (name, case), c in cubes.items():
        key = f"{name}/case{case}"
        v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
        d = geo.dims_of(v.shape)
        ent = {"geosstv": best[key]}
        for mname, reg, omegas in methods:
            top = dict(best[key]) if mname == "geosstv_wide" else None
            for omega in omegas:
                p = geo.params(c["eps"], c["alpha"], c["beta"], omega=omega, tol=1e-5, max_iter=20000,
                               regularizer=reg)
                ws = geo.Workspace(geo.geo_workspace_size(d, p))
                u, s, t = (torch.empty_like(v) for _ in range(3))
                r = geo.geo_solve(d, p, v, u, s, t, ws)
                uh = u.cpu().numpy().astype(np.float64)
                row = {"omega": omega, "iters": r.iters, "converged": bool(r.converged),
                       "mpsnr": mpsnr(uh, c["u_clean"]), "mssim": mssim(uh, c["u_clean"])}
                if top is None or row["mpsnr"] > top["mpsnr"]:
                    top = row
                del ws, u, s, t
            ent[mname] = top
        per_case[key] = ent
        print(f"[quality] {key}: " + ", ".join(f"{m} {e['mpsnr']:.2f} dB" for m, e in ent.items()),
              file=sys.stderr, flush=True)
    names = ("geosstv", "geosstv_wide", "sstv", "hsstv1", "hsstv2")
    return {"per_case": per_case,
            "mean_mpsnr": {m: float(np.mean([e[m]["mpsnr"] for e in per_case.values()])) for m in names},
            "mean_mssim": {m: float(np.mean([e[m]["mssim"] for e in per_case.values()])) for m in names},
            # among the methods on the same (wide) grid
            "cases_won_mpsnr": {m: sum(1 for e in per_case.values()
                                       if max(names[1:], key=lambda x: e[x]["mpsnr"]) == m) for m in names[1:]},
            "seconds": time.perf_counter() - t0}


def bench_realshape(args):
    """The shapes and fixed radii of the paper's real-image experiment
    (120x120x198 with (200, 100, 30), 100x100x360 with (800, 5000, 100),
    omega 0.01) on synthetic stand-ins, each solved to the stopping rule at
    1e-5: iterations, seconds and voxel-iterations/s, with the band chunk
    from the autotuner next to the default one."""
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from paper_2510_00562_amd.tune import tune_band_chunk
    from synth.cubes import REAL_SHAPES, real_shape_case
    from synth.quality import mpsnr, mssim

    rows = {}
    for name in REAL_SHAPES:
        c = real_shape_case(name)
        v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
        d = geo.dims_of(v.shape)
        p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"], tol=1e-5)
        ws = geo.Workspace(geo.geo_workspace_size(d, p))
        table = geo.Workspace(geo.geo_batch_table_size(1))
        kc, tune_ms = tune_band_chunk([d], [p], [v], [ws], table, candidates="auto")
        res = {}
        # tuned; the library's per-cube default (band_chunk 0); a fixed 32
        for label, chunk in (("tuned", kc), ("default", 0), ("fixed_32", 32)):
            p.band_chunk = chunk
            used = geo.geo_sweep_geometry(d, chunk, geo.geo_sweep_blocks(p.dual_storage),
                                          p.dual_storage)[0]
            geo.geo_state_init(d, p, v, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = geo.geo_step(d, p, v, ws, 20000)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            res[label] = {"band_chunk": used, "iters": r.iters, "seconds": el,
                          "voxel_iterations_per_s": v.numel() * r.iters / el,
                          "converged": bool(r.converged)}
        u = torch.empty_like(v)
        geo.geo_state_get(d, p, ws, "u", v, u)
        uh = u.cpu().numpy().astype(np.float64)
        rows[name] = {"shape": list(c["shape"]), "radii": [c["alpha"], c["beta"], c["eps"]],
                      "omega": c["omega"], **res, "tuner_ms_per_iteration": tune_ms,
                      "mpsnr_vs_synthetic_clean": mpsnr(uh, c["u_clean"]),
                      "mssim_vs_synthetic_clean": mssim(uh, c["u_clean"])}
    tot_vox_it = sum(r["tuned"]["iters"] * np.prod(r["shape"]) for r in rows.values())
    tot_s = sum(r["tuned"]["seconds"] for r in rows.values())
    out = {
        "metric": "P-PDS voxel-iterations/s",
        "value": float(tot_vox_it / tot_s),
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic stand-ins of the real images' shapes, noise matched to the fixed radii",
        "config": {"workload": "120x120x198 (200, 100, 30) and 100x100x360 (800, 5000, 100), "
                               "omega 0.01, solved to tol 1e-5"},
        "cubes": rows,
    }
    print(json.dumps(out), flush=True)


def bench_regularizer(args):
    """The benchmark cube solved with SSTV, HSSTV1 or HSSTV2 (Sec. IV-A) in
    place of GeoSSTV, through the same P-PDS (eq. (7)): voxel-iterations/s
    over the timed steps and the roofline of the variant path's dominant
    kernel, its dual kernel (HIP events around every 8th launch)."""
    import numpy as np
    import torch

    import paper_2510_00562_amd as geo
    from synth.cubes import CUBE_256x256x128, CUBE_512x512x224, like, make_cube

    n1, n2, n3 = (int(x) for x in args.cube.lower().split("x"))
    named = {(256, 256, 128): CUBE_256x256x128, (512, 512, 224): CUBE_512x512x224}
    c = make_cube(named.get((n1, n2, n3)) or like(CUBE_256x256x128, n1=n1, n2=n2, n3=n3))
    v = torch.from_numpy(np.ascontiguousarray(c["v"], dtype=np.float32)).cuda()
    N = v.numel()
    reg = geo.REGULARIZERS[args.regularizer]
    P = geo.var_planes("y1", reg)
    dims = geo.dims_of(v.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"], regularizer=reg)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, v, ws)
    geo.geo_step(dims, p, v, ws, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, dual_ms = geo.geo_step_timed(dims, p, v, ws, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    K = args.steps
    value = N * K / el
    # dual kernel, per voxel: reads s, t, u+, u, the P planes of y1, y3, the
    # y4 residual and v (z_s, z_t evaluated from them again); writes s, t+,
    # y3, y1 and the residual
    dual_bytes = 4 * (11 + 2 * P)
    # the iteration's state (u, s, t, y1, y3, y4) read and written once, v read
    iter_bytes = 2 * 4 * (5 + P) + 4
    avg_s = dual_ms / K / 1e3
    achieved = dual_bytes * N / avg_s
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
        "config": {"workload": f"P-PDS (eq. (7)) with the {args.regularizer.upper()} regularizer "
                               f"of Sec. IV-A on one {n1}x{n2}x{n3} cube, synthetic mixed noise, "
                               "FP32 iterates, FP64 reductions",
                   "n1": n1, "n2": n2, "n3": n3, "voxels": N, "omega": c["omega"],
                   "regularizer": args.regularizer},
        "roofline": {"bound": "hbm", "kernel": "var_dual", "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK if avg_s * K <= el else None,
                     "traffic": None, "bytes_per_voxel": dual_bytes,
                     "avg_launch_ms": 1e3 * avg_s},
        "iteration_bytes_per_voxel": iter_bytes,
        "iteration_hbm_frac": iter_bytes * value / HBM_PEAK,
        "last": {"rel_change": res.rel_change, "r": res.r, "tau_s": res.tau_s,
                 "tau_t": res.tau_t, "iters": res.total_iters},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds, reg=reg,
                                           what=f"the FP64 oracle ({args.regularizer})")
    print(json.dumps(out), flush=True)


# the sources sweep A is compiled from (its file and the headers it includes)
SWEEP_A_SOURCES = ("sweep.hip", "common.hpp", "radix.hpp", "solver.hpp")


def geo_source_hash():
    """Hash of sweep A's sources: its traffic counters go stale when they
    change."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2510_00562_amd", "csrc")
    for f in SWEEP_A_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
