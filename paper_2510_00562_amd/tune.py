"""Autotuner of the fused sweep's tile depth (bands per tile, `band_chunk`).

The sweep streams each TI x TJ pixel tile through a chunk of bands. Deeper
chunks amortise the tile's fixed costs: the halo band of y and the tile's
partial sums. Shallower chunks
give more tiles to spread over the 256 compute units. The best depth depends
on the cube sizes, so this tuner times a few candidates on the caller's own
states, in steady state, and returns the fastest one. It uses only the C
ABI (geo_batch_step) and leaves every state back at Alg. 1's initial point.
"""
from __future__ import annotations

from . import geo_batch_step, geo_state_init, geo_sweep_blocks, geo_sweep_geometry

CANDIDATES = (16, 32, 64)


def _busiest_block(cost, G):
    """Longest per-block total when G persistent blocks take the tiles of
    `cost` (in the sweep's order) as the sweep hands them out: each of the 8
    XCDs a contiguous eighth of the list, its blocks every (G/8)-th tile."""
    import numpy as np
    T = cost.size
    if T == 0:
        return 0.0
    g = min(G, T)
    if g >= 8 and g % 8 == 0:
        per = g // 8
        load = np.zeros(g)
        for x in range(8):
            seg = cost[x * T // 8:(x + 1) * T // 8]
            load[x + 8 * np.arange(per)] = np.bincount(np.arange(seg.size) % per, weights=seg,
                                                       minlength=per)
    else:
        load = np.bincount(np.arange(T) % g, weights=cost, minlength=g)
    return float(load.max())


def model_candidates(dims, dual_storage=0, n=4, c0=2.0, lo=8, hi=64):
    """The n band chunks in [lo, hi] that a load-balance model of the
    persistent sweep ranks fastest for these cubes.

    A tile costs its bands plus c0 band-equivalents of fixed work (its halo
    band, the pipeline fill, its partial sums). The model lays the tiles of
    the cubes out in the sweep's order, hands them to the G persistent
    blocks as the sweep does, and takes the busiest block's total as the
    sweep's length; cubes of the two tile shapes run in two launches one
    after the other, so their lengths add. Deep chunks leave blocks idle
    when there are few tiles, shallow ones pay the fixed work more often,
    and a tile count just past a multiple of G costs almost a whole extra
    round. Chunks that cut every cube into the same number of chunks are one
    candidate (the smallest, whose chunks are the most even)."""
    import numpy as np
    G = geo_sweep_blocks(dual_storage)
    est, seen = {}, set()
    for kc in range(lo, hi + 1):
        costs, key = {}, []
        for d in dims:
            used, tiles, rows, _ = geo_sweep_geometry(d, kc, dual_storage=dual_storage)
            chunks = -(-d.n3 // used)
            bands = np.minimum(used, d.n3 - used * np.arange(chunks))
            # tile order within a cube: pixel tiles fastest, band chunks slowest
            costs.setdefault(rows, []).append(np.repeat(bands + c0, tiles // chunks))
            key.append(chunks)
        key = tuple(key)
        if key in seen:
            continue
        seen.add(key)
        est[kc] = sum(_busiest_block(np.concatenate(c), G) for c in costs.values())
    return sorted(est, key=est.get)[:n]


def tune_band_chunk(dims, ps, vs, wss, table, candidates=CANDIDATES, warm=40, timed=10,
                    use_graph=True):
    """Pick the band chunk (one value for every cube of the batch) with the
    shortest time for `timed` iterations after `warm` iterations, which leave
    the start-up threshold searches behind. candidates: the chunks to time,
    or "auto" for the four that model_candidates ranks first. Returns (best,
    {candidate: milliseconds per iteration}). The states are re-initialised
    afterwards."""
    import torch
    if candidates == "auto":
        candidates = model_candidates(dims, ps[0].dual_storage)
    times = {}
    for kc in candidates:
        for p in ps:
            p.band_chunk = kc
        for d, p, v, ws in zip(dims, ps, vs, wss):
            geo_state_init(d, p, v, ws)
        geo_batch_step(dims, ps, vs, wss, table, warm, use_graph=use_graph)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        geo_batch_step(dims, ps, vs, wss, table, timed, use_graph=use_graph)
        e1.record()
        torch.cuda.synchronize()
        times[kc] = e0.elapsed_time(e1) / timed
    best = min(times, key=times.get)
    for p in ps:
        p.band_chunk = best
    for d, p, v, ws in zip(dims, ps, vs, wss):
        geo_state_init(d, p, v, ws)
    return best, times
