"""The threshold search of the two l1-ball projections (steps 2 and 3 of
Alg. 1, the cited projection's threshold) when its predicted window holds
more values than fit in LDS at once.

Cubes of the uneven batch whose s-field threshold sinks toward 0 put
hundreds of thousands of |z| values inside the window in some iterations.
The search then streams them through LDS in chunks and compacts the
candidates of a deeper radix level. In one of them the window overflows the
candidate slots of the tiles, which sends those iterations to the full
radix search. Every iteration's thresholds must still
equal the FP64 oracle's, and the iterates must follow it."""
import numpy as np
import pytest

from gpu_helpers import announce, f32, rel_l2
from synth.cubes import batch_specs, make_cube
from test_gpu_step import STATE, get_state, gpu_solver

pytestmark = pytest.mark.gpu

CAND_LDS = 28672  # candidates the search holds in LDS at once


@pytest.mark.parametrize("which", [5, 28])
def test_window_search_beyond_lds(ora, which):
    c = make_cube(batch_specs()[which])
    v = f32(c["v"])
    iters = 12
    announce(f"window search beyond LDS: batch cube {which} {v.shape}, {iters} iterations")
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=c["omega"])
    geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
    taus, cands, fallbacks = [], [], 0
    for _ in range(iters):
        res = geo.geo_step(dims, p, vd, ws, 1)
        taus.append((res.tau_s, res.tau_t))
        cands.append(max(res.cand_s, res.cand_t))
        fallbacks += res.fallback_passes
    print("candidates per iteration:", cands, "full searches:", fallbacks, flush=True)
    assert max(cands) > CAND_LDS  # the streamed search ran
    if which == 28:
        # tiles ran out of candidate slots (N/16 in all): the search fell
        # back to the full radix search over the cube in those iterations
        assert max(cands) >= (v.size // 16) * 0.99 and fallbacks > 2
    g = get_state(geo, dims, p, ws, vd, v.shape)
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"])
    S.step(iters)
    for k, (gt, ot) in enumerate(zip(taus, S.trace)):
        assert gt[0] == pytest.approx(ot[2], rel=1e-5), (k, "tau_s")
        assert gt[1] == pytest.approx(ot[3], rel=1e-5), (k, "tau_t")
    errs = {n: rel_l2(g[n], S.state[n]) for n in STATE}
    print("rel L2:", {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    assert errs["u"] <= 1e-5 and max(errs.values()) <= 1e-4
