"""The request loop: jobs of different sizes arriving over time, admitted by
HBM footprint and advanced in batched rounds, each finish with exactly the
iterates (and iteration count) of the same job run alone by geo_step."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, torch_cuda
from synth.cubes import SMALL_64x64x16, like, make_cube

pytestmark = pytest.mark.gpu


def jobs():
    from paper_2510_00562_amd.serve import Job
    shapes = [(12, 40, 70), (6, 17, 33), (20, 64, 64), (9, 31, 130), (3, 8, 8), (15, 50, 20)]
    out = []
    for q, (n3, n1, n2) in enumerate(shapes):
        c = make_cube(like(SMALL_64x64x16, n1=n1, n2=n2, n3=n3, seed=700 + q, cells=5))
        out.append(Job(q, f32(c["v"]).astype(np.float32), c["eps"], c["alpha"], c["beta"],
                       tol=2e-3, cap=150 + 40 * q, arrival=0.05 * q))
    return out


def test_stream_results_equal_solo_runs():
    announce("request loop: 6 jobs, footprint budget for about two at a time")
    torch_cuda()
    import paper_2510_00562_amd as geo
    from paper_2510_00562_amd.serve import footprint, run_stream
    js = jobs()
    budget = 2 * max(footprint(j.v.shape) for j in js) + 1
    rep = run_stream(js, budget, round_iters=16)
    assert len(rep["jobs"]) == len(js)
    for j in rep["jobs"]:
        assert j.finished >= j.admitted >= j.arrival
        dims = geo.dims_of(j.v.shape)
        p = geo.params(j.eps, j.alpha, j.beta, omega=j.omega, tol=j.tol)
        ws = geo.Workspace(geo.geo_workspace_size(dims, p))
        vd = dev(j.v)
        geo.geo_state_init(dims, p, vd, ws)
        r = geo.geo_step(dims, p, vd, ws, j.cap)
        assert r.iters == j.iters and bool(r.converged) == j.converged
        u = __import__("torch").empty_like(vd)
        geo.geo_state_get(dims, p, ws, "u", vd, u)
        assert np.array_equal(u.cpu().numpy(), j.u), j.job_id
    assert rep["latency_p99_s"] >= rep["latency_p50_s"] > 0


def test_non_finite_job_is_retired_and_the_others_go_on():
    """One job's cube holds a NaN: its iterates turn non-finite, the loop
    retires it with an error and no result, and every other job of the same
    batched rounds still finishes with its solo iterates."""
    announce("request loop: a NaN cube among 4 jobs")
    torch = torch_cuda()
    import paper_2510_00562_amd as geo
    from paper_2510_00562_amd.serve import footprint, run_stream
    js = jobs()[:4]
    js[1].v = js[1].v.copy()
    js[1].v[1, 3, 4] = np.nan
    budget = 4 * max(footprint(j.v.shape) for j in js) + 1
    rep = run_stream(js, budget, round_iters=16)
    assert rep["errors"] == 1
    bad = [j for j in rep["jobs"] if j.error is not None]
    assert [j.job_id for j in bad] == [1] and bad[0].u is None
    for j in rep["jobs"]:
        if j.error is not None:
            continue
        dims = geo.dims_of(j.v.shape)
        p = geo.params(j.eps, j.alpha, j.beta, omega=j.omega, tol=j.tol)
        ws = geo.Workspace(geo.geo_workspace_size(dims, p))
        vd = dev(j.v)
        geo.geo_state_init(dims, p, vd, ws)
        r = geo.geo_step(dims, p, vd, ws, j.cap)
        assert r.iters == j.iters and bool(r.converged) == j.converged
        u = torch.empty_like(vd)
        geo.geo_state_get(dims, p, ws, "u", vd, u)
        assert np.array_equal(u.cpu().numpy(), j.u), j.job_id
