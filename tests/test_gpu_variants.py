"""GPU parity in the special cases of the method and on the shape of the
paper's long-spectrum real image: beta = 0 (no stripe term: t stays 0),
alpha = 0, omega = 0 (no first-order term), N3 = 1 (2-D Condat-TV
denoising, D_s = 0), and a 100 x 100 x 360 cube with the paper's fixed radii
(800, 5000, 100) and omega 0.01, whose 360 bands span several band chunks
with a ragged last one."""
import numpy as np
import pytest

from gpu_helpers import announce, f32, rel_l2
from synth.cubes import SMALL_64x64x16, like, make_cube, real_shape_case
from test_gpu_step import STATE, get_state, gpu_solver

pytestmark = pytest.mark.gpu


def run_both(ora, v, prm, n):
    geo, dims, p, ws, vd = gpu_solver(v.shape, v, prm)
    geo.geo_step(dims, p, vd, ws, n)
    g = get_state(geo, dims, p, ws, vd, v.shape)
    S = ora.Solver(v, prm["eps"], prm["alpha"], prm["beta"], omega=prm["omega"])
    S.step(n)
    return g, S


def check(g, S, tol_u=1e-5, tol=1e-4):
    errs = {n: rel_l2(g[n], S.state[n]) for n in STATE if np.linalg.norm(S.state[n]) > 0}
    assert errs["u"] <= tol_u, errs
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("case", ["beta0", "alpha0", "omega0", "bands1"])
def test_special_cases(ora, case):
    announce(f"special case {case}")
    shape = (1, 50, 70) if case == "bands1" else (12, 37, 70)
    n3, n1, n2 = shape
    c = make_cube(like(SMALL_64x64x16, n1=n1, n2=n2, n3=n3, seed=31, cells=6))
    v = f32(c["v"])
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=0.03)
    if case == "beta0":
        prm["beta"] = 0.0
    if case == "alpha0":
        prm["alpha"] = 0.0
    if case == "omega0":
        prm["omega"] = 0.0
    g, S = run_both(ora, v, prm, 40)
    check(g, S)
    if case == "beta0":
        assert np.all(g["t"] == 0.0) and np.all(S.t == 0.0)
    if case == "alpha0":
        assert np.all(g["s"] == 0.0)


def test_long_spectrum_real_image_shape(ora):
    c = real_shape_case("suwannee_shape")
    v = f32(c["v"])
    announce(f"100x100x360 cube, radii (800, 5000, 100), omega 0.01: 20 iterations")
    prm = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], omega=c["omega"])
    g, S = run_both(ora, v, prm, 20)
    check(g, S)
