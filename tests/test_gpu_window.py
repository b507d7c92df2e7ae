"""The threshold search of the two l1-ball projections (constraint sets (16),
(17); the cited projection's threshold) in the first iterations of a solve,
where the threshold moves fast.

Two kinds of iteration are pinned against the FP64 oracle:
  * windows holding more values than fit in LDS at once (the search streams
    them through LDS in chunks and compacts a deeper radix level): cubes
    large enough that the candidate budget of a window (N/256) exceeds what
    LDS holds;
  * windows that miss (the first iterations after the threshold leaves 0):
    the three histogram passes of the same launch slot find the threshold,
    so each one-iteration call completes its iteration.
Every iteration's thresholds must equal the oracle's, and the iterates must
follow it."""
import numpy as np
import pytest

from gpu_helpers import announce, f32, rel_l2
from synth.cubes import batch_specs, make_cube
from test_gpu_step import STATE, get_state, gpu_solver

pytestmark = pytest.mark.gpu

CAND_LDS = 28672  # candidates the search holds in LDS at once


@pytest.mark.parametrize("which", [0, 28])
def test_window_search_and_missed_windows(ora, which):
    c = make_cube(batch_specs()[which])
    v = f32(c["v"])
    iters = 14
    announce(f"threshold search, early iterations: batch cube {which} {v.shape}, {iters} iterations")
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=c["omega"])
    geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
    taus, cands, misses = [], [], []
    for _ in range(iters):
        res = geo.geo_step(dims, p, vd, ws, 1)
        assert res.iters == 1 and res.slots == 1  # a missed window costs no extra slot
        taus.append((res.tau_s, res.tau_t))
        cands.append(max(res.cand_s, res.cand_t))
        misses.append(res.fallback_passes)
    print("candidates per iteration:", cands, "missed windows:", misses, flush=True)
    assert max(cands) > CAND_LDS  # the streamed search ran
    assert sum(misses) >= 2  # and the histogram passes did
    assert max(cands) <= 2 * v.size // 128  # windows kept near their budget
    g = get_state(geo, dims, p, ws, vd, v.shape)
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"])
    S.step(iters)
    for k, (gt, ot) in enumerate(zip(taus, S.trace)):
        assert gt[0] == pytest.approx(ot[2], rel=1e-5), (k, "tau_s")
        assert gt[1] == pytest.approx(ot[3], rel=1e-5), (k, "tau_t")
    errs = {n: rel_l2(g[n], S.state[n]) for n in STATE}
    print("rel L2:", {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    assert errs["u"] <= 1e-5 and max(errs.values()) <= 1e-4


def test_late_miss_evaluates_z_from_the_state(ora):
    """A window that misses long after the start (here: after the radii of
    (16), (17) change between calls, which moves both thresholds) is found
    by histogram passes that evaluate z_s and z_t from the state again
    (sweep A stores them only in the first iterations and after recent
    misses); the thresholds and iterates must still follow the oracle."""
    c = make_cube(batch_specs()[0])
    v = f32(c["v"])
    announce(f"late missed windows: batch cube 0 {v.shape}")
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=c["omega"])
    geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
    res = geo.geo_step(dims, p, vd, ws, 30)
    assert res.iters == 30
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"])
    S.step(30)
    p.alpha, p.beta = 0.5 * prm["alpha"], 0.6 * prm["beta"]
    S.params.alpha, S.params.beta = p.alpha, p.beta
    misses, taus = [], []
    for _ in range(3):
        r = geo.geo_step(dims, p, vd, ws, 1)
        misses.append(r.fallback_passes)
        taus.append((r.tau_s, r.tau_t))
    S.step(3)
    print("missed windows after the change:", misses, flush=True)
    assert misses[0] >= 1
    for k, (gt, ot) in enumerate(zip(taus, S.trace[30:])):
        assert gt[0] == pytest.approx(ot[2], rel=1e-5), (k, "tau_s")
        assert gt[1] == pytest.approx(ot[3], rel=1e-5), (k, "tau_t")
    g = get_state(geo, dims, p, ws, vd, v.shape)
    errs = {n: rel_l2(g[n], S.state[n]) for n in STATE}
    assert errs["u"] <= 1e-5 and max(errs.values()) <= 1e-4, errs
