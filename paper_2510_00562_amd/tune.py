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

from . import geo_batch_step, geo_state_init

CANDIDATES = (16, 32, 64)


def tune_band_chunk(dims, ps, vs, wss, table, candidates=CANDIDATES, warm=40, timed=10,
                    use_graph=True):
    """Pick the band chunk (one value for every cube of the batch) with the
    shortest time for `timed` iterations after `warm` iterations, which leave
    the start-up threshold searches behind. Returns (best, {candidate:
    milliseconds per iteration}). The states are re-initialised afterwards."""
    import torch
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
