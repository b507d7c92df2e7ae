"""GPU parity of the operators and proximal tools behind the C ABI against
the FP64 oracle (same FP32-rounded inputs on both sides): relative L2 error
<= 1e-6 per array; exact thresholds on identical inputs."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, host, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu

SHAPES = [(5, 13, 70), (17, 9, 130), (1, 1, 1), (3, 1, 5), (2, 7, 1), (16, 64, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("op", ["dv", "dh", "ds", "d", "dds", "l_ud", "l_lr", "l_c", "l", "k"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_operator_parity(ora, op, shape, adjoint):
    import paper_2510_00562_amd as geo
    torch = torch_cuda()
    announce(f"op {op} adj={adjoint} shape={shape}")
    pin, pout = geo.OP_PLANES[op]
    if adjoint:
        pin, pout = pout, pin
    N = int(np.prod(shape))
    x = f32(np.random.default_rng(hash((op, shape, adjoint)) % 2**32).normal(size=pin * N))
    out = torch.empty(pout * N, dtype=torch.float32, device="cuda")
    geo.geo_apply_op(op, adjoint, geo.dims_of(shape), dev(x), out)
    torch.cuda.synchronize()
    xin = x if op == "k" else (x.reshape((pin,) + shape) if pin > 1 else x.reshape(shape))
    want = ora.apply(op, xin, shape, adjoint=adjoint).ravel()
    assert rel_l2(host(out), want) <= 1e-6


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (1000, 2), (65536, 3), (3_000_001, 4)])
@pytest.mark.parametrize("frac", [0.0, 0.02, 0.5, 0.999, 1.5])
def test_l1_projection_parity(ora, n, seed, frac):
    import paper_2510_00562_amd as geo
    torch = torch_cuda()
    announce(f"l1 n={n} frac={frac}")
    rng = np.random.default_rng(seed)
    x = rng.laplace(size=n) * rng.uniform(0.01, 10)
    x[rng.uniform(size=n) < 0.1] = 0.0
    if n > 10:
        x[: n // 10] = np.round(x[: n // 10], 1)  # many ties
    x = f32(x)
    radius = frac * np.abs(x).sum()
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    tau = geo.geo_project_l1(dev(x), radius, out)
    want, tau_o = ora.proj_l1(x, radius)
    if radius == 0:
        assert tau == np.inf and not host(out).any()
        return
    if tau_o == 0:
        assert tau == 0
    else:
        # same FP32 values on both sides; only FP64 summation order differs
        assert tau == pytest.approx(tau_o, rel=1e-7)
    assert rel_l2(host(out), want) <= 1e-6 or np.abs(host(out) - want).max() <= 1e-6 * max(tau_o, 1e-30)


def test_l1_projection_special_values(ora):
    import paper_2510_00562_amd as geo
    torch = torch_cuda()
    for x, radius in (([3.0, 0.0, 0.0], 1.0), ([-2.0] * 6, 3.0), ([0.0] * 5, 1.0),
                      ([1e-40, -2e-40, 5.0], 4.0), ([7.0], 2.0)):
        x = f32(x)
        out = torch.empty(len(x), dtype=torch.float32, device="cuda")
        tau = geo.geo_project_l1(dev(x), radius, out)
        want, tau_o = ora.proj_l1(x, radius)
        assert tau == pytest.approx(tau_o, rel=1e-9, abs=0)
        np.testing.assert_allclose(host(out), want, rtol=1e-6, atol=1e-30)


@pytest.mark.parametrize("n", [1, 1000, 1_000_003])
def test_l2_box_group_prox_parity(ora, n):
    import paper_2510_00562_amd as geo
    torch = torch_cuda()
    announce(f"l2/box/prox n={n}")
    rng = np.random.default_rng(n)
    x, c = f32(rng.normal(size=n)), f32(rng.normal(size=n))
    for scale in (0.5, 2.0):
        eps = scale * np.linalg.norm(x - c)
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        r = geo.geo_project_l2(dev(x), dev(c), eps, out)
        want, r_o = ora.proj_l2(x, c, eps)
        assert r == pytest.approx(r_o, rel=1e-9)
        assert rel_l2(host(out), want) <= 1e-6
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    geo.geo_project_box(dev(x), -0.3, 0.7, out)
    np.testing.assert_array_equal(host(out), ora.proj_box(x, -0.3, 0.7).astype(np.float32))
    xb = f32(rng.normal(size=n))
    oa = torch.empty(n, dtype=torch.float32, device="cuda")
    ob = torch.empty(n, dtype=torch.float32, device="cuda")
    geo.geo_prox_l12(dev(x), dev(xb), 0.8, oa, ob)
    wa, wb = ora.prox_l12(x, xb, 0.8)
    assert rel_l2(np.concatenate([host(oa), host(ob)]), np.concatenate([wa, wb])) <= 1e-6
