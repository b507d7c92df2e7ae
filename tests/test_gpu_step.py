"""GPU parity of one and a few P-PDS iterations (Alg. 1) against the FP64
oracle, from the initial point and from random states, on shapes that span
several tiles and band chunks with ragged tails: relative L2 <= 1e-6 per
state array after one step, scalars tau_s, tau_t, r within 1e-6."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, host, rel_l2, torch_cuda
from synth.cubes import SMALL_64x64x16, like, make_cube, random_state

pytestmark = pytest.mark.gpu

STATE = ("u", "s", "t", "w1", "w2", "y1", "y2", "y3", "y4")


def gpu_solver(shape, v, prm, dual_storage=0):
    import paper_2510_00562_amd as geo
    dims = geo.dims_of(shape)
    p = geo.params(prm["eps"], prm["alpha"], prm["beta"], prm.get("mu_lo", 0.0),
                   prm.get("mu_hi", 1.0), prm["omega"], tol=prm.get("tol", 0.0),
                   dual_storage=dual_storage)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    vd = dev(v)
    geo.geo_state_init(dims, p, vd, ws)
    return geo, dims, p, ws, vd


def get_state(geo, dims, p, ws, vd, shape):
    torch = torch_cuda()
    out = {}
    for name in STATE:
        pl = geo.VAR_PLANES[name]
        t = torch.empty(((pl,) if pl > 1 else ()) + tuple(shape), dtype=torch.float32, device="cuda")
        geo.geo_state_get(dims, p, ws, name, vd, t)
        out[name] = t
    torch.cuda.synchronize()
    return {k: host(t) for k, t in out.items()}


def set_state(geo, dims, p, ws, vd, st):
    for name in STATE:
        geo.geo_state_set(dims, p, ws, name, vd, dev(st[name]))


def compare(gpu, ora_state, tol, names=STATE):
    errs = {n: rel_l2(gpu[n], ora_state[n]) for n in names}
    bad = {n: e for n, e in errs.items() if e > tol}
    assert not bad, errs


def problem(shape, seed):
    n3, n1, n2 = shape
    c = make_cube(like(SMALL_64x64x16, n1=n1, n2=n2, n3=n3, seed=seed, cells=5))
    c["v"] = f32(c["v"])
    return c


# (N3, N1, N2). 8 x 128 tiles: (5, 13, 70), (1, 1, 1), (3, 1, 5), (2, 7, 1);
# 16 x 64 tiles: (17, 9, 130), (33, 20, 64), (16, 64, 64), and (12, 40, 150),
# whose 3 x 3 pixel tiles per band chunk give one tile neighbours on all sides.
@pytest.mark.parametrize("shape", [(5, 13, 70), (17, 9, 130), (1, 1, 1), (3, 1, 5), (2, 7, 1),
                                   (33, 20, 64), (16, 64, 64), (12, 40, 150)])
def test_one_step_from_random_state(ora, shape):
    announce(f"one step random state {shape}")
    c = problem(shape, 3)
    st = {k: f32(v) for k, v in random_state(shape, 7).items()}
    N = int(np.prod(shape))
    # radii that make both l1 projections and the l2 ball active
    prm = dict(eps=0.5 * np.sqrt(N) * 0.1, alpha=0.3 * 0.1 * N, beta=0.2 * 0.1 * N, omega=0.07)
    geo, dims, p, ws, vd = gpu_solver(shape, c["v"], prm)
    set_state(geo, dims, p, ws, vd, st)
    res = geo.geo_step(dims, p, vd, ws, 1)
    S = ora.Solver(c["v"], prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"], state=st)
    S.step(1)
    compare(get_state(geo, dims, p, ws, vd, shape), S.state, 1e-6)
    rel, r, ts, tt = S.trace[-1]
    assert res.r == pytest.approx(r, rel=1e-6)
    assert res.tau_s == pytest.approx(ts, rel=1e-6)
    assert res.tau_t == pytest.approx(tt, rel=1e-6)
    assert res.rel_change == pytest.approx(rel, rel=1e-5)
    assert ts > 0 and tt > 0 and r > prm["eps"]


@pytest.mark.parametrize("shape", [(5, 13, 70), (17, 9, 130), (12, 40, 150)])
def test_few_steps_from_initial_point(ora, shape):
    announce(f"10 steps from init {shape}")
    c = problem(shape, 4)
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=0.03)
    geo, dims, p, ws, vd = gpu_solver(shape, c["v"], prm)
    geo.geo_step(dims, p, vd, ws, 10)
    S = ora.Solver(c["v"], prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"])
    S.step(10)
    compare(get_state(geo, dims, p, ws, vd, shape), S.state, 1e-5)


def test_small_cube_200_iterations(ora):
    """64 x 64 x 16 cube with the paper's mixed noise: after 200 iterations the
    FP32 GPU u is within 1e-4 relative L2 of the FP64 oracle and the MPSNR
    (eq. (29)) gap is below 0.01 dB."""
    announce("64x64x16, 200 iterations")
    c = make_cube(SMALL_64x64x16)
    v = f32(c["v"])
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=0.03)
    geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
    res = geo.geo_step(dims, p, vd, ws, 200)
    assert res.iters == 200 and res.total_iters == 200
    g = get_state(geo, dims, p, ws, vd, v.shape)
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"])
    S.step(200)
    assert rel_l2(g["u"], S.u) <= 1e-4
    assert abs(ora.mpsnr(g["u"], c["u_clean"]) - ora.mpsnr(S.u, c["u_clean"])) <= 0.01
    for n in ("s", "t"):
        assert rel_l2(g[n], S.state[n]) <= 1e-3


def test_stopping_rule_is_exact(ora):
    """The device stops after the first iteration whose ||u+ - u|| / ||u|| is
    below tol (eq. (28); from the second iteration on, reading C14), at the
    oracle's iteration exactly; the count does not depend on how often the
    host looks. tol sits at the geometric middle of the gap between the
    oracle's first relative change below 2e-3 and the smallest one before
    it, so that FP32 rounding of the GPU's relative change (about 1e-6 of
    it) cannot move the decision."""
    announce("stopping rule")
    c = make_cube(like(SMALL_64x64x16, n1=32, n2=40, n3=8, seed=9))
    v = f32(c["v"])
    S0 = ora.Solver(v, c["eps"], c["alpha"], c["beta"], omega=0.03)
    S0.step(500)
    rel = [t[0] for t in S0.trace]  # rel[j]: iteration j + 1
    k = next(j for j in range(1, len(rel)) if rel[j] < 2e-3)
    lo, hi = rel[k], min(rel[1:k])
    tol = float(np.sqrt(lo * hi))
    assert min(hi / tol, tol / lo) > 1 + 1e-4  # a gap the rounding cannot bridge
    expected = k + 1
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=0.03, tol=tol)
    for every in (1, 7, 64):
        geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
        p.check_every = every
        res = geo.geo_step(dims, p, vd, ws, 500)
        assert res.converged == 1 and res.iters == expected, (every, res.iters, expected)
        assert res.rel_change == pytest.approx(lo, rel=1e-4)
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=0.03)
    assert S.step(500, tol=tol) == expected


def test_constant_cube_fixed_point_on_gpu():
    announce("constant cube")
    torch = torch_cuda()
    shape = (20, 17, 70)
    v = np.full(shape, 0.37)
    geo, dims, p, ws, vd = gpu_solver(shape, v, dict(eps=0.5, alpha=1.0, beta=1.0, omega=0.03))
    geo.geo_step(dims, p, vd, ws, 30)
    g = get_state(geo, dims, p, ws, vd, shape)
    np.testing.assert_allclose(g["u"], f32(v), atol=1e-7)
    for n in ("s", "t", "w1", "w2", "y1", "y2", "y3"):
        assert np.abs(g[n]).max() < 1e-6, n


def test_stopping_rule_starts_at_the_second_iteration(ora):
    """A cube inside the box: the first iteration leaves u = v exactly, and
    both sides apply eq. (28) from the second iteration on."""
    announce("stopping rule, first iteration exempt")
    c = make_cube(like(SMALL_64x64x16, n1=30, n2=41, n3=6, seed=12, sigma=0.01, p_s=0.0, p_t=0.02))
    v = np.clip(f32(c["v"]), 0.05, 0.95)
    prm = dict(eps=c["eps"], alpha=c["alpha"] + 1.0, beta=c["beta"], omega=0.03, tol=1e-3)
    geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
    res = geo.geo_step(dims, p, vd, ws, 300)
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=0.03)
    done = S.step(300, tol=1e-3)
    assert S.trace[0][0] == 0.0
    assert res.iters > 1 and abs(done - res.iters) <= 1
