"""Parity at the full iteration count of the benchmark workload: 5000
iterations of Alg. 1 on the 256 x 256 x 128 cube, in the launch
configuration the benchmark times, against the FP64 oracle's run stored by
tests/golden/make_long_runs.py (sampled u, s, t; MPSNR; last trace entry).
Bounds: u, s and t within 1e-4 relative L2 on the samples, MPSNR within
0.01 dB."""
import json
import os

import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, rel_l2, torch_cuda
from synth.cubes import CUBE_256x256x128, make_cube

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "long_256x256x128_5000.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle long run not generated")
def test_benchmark_cube_5000_iterations():
    announce("256x256x128, 5000 iterations vs the stored FP64 oracle run")
    torch = torch_cuda()
    import paper_2510_00562_amd as geo
    from synth.quality import mpsnr
    g = json.load(open(GOLDEN))
    c = make_cube(CUBE_256x256x128)
    v = f32(c["v"])
    vd = dev(v)
    dims = geo.dims_of(v.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"])
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, vd, ws)
    res = geo.geo_step(dims, p, vd, ws, g["iterations"])
    assert res.iters == g["iterations"]
    idx = np.asarray(g["sample_index"])
    got = {}
    for name in ("u", "s", "t"):
        x = torch.empty_like(vd)
        geo.geo_state_get(dims, p, ws, name, vd, x)
        got[name] = x.cpu().numpy().astype(np.float64)
    eu = rel_l2(got["u"].ravel()[idx], np.asarray(g["u"]))
    es = rel_l2(got["s"].ravel()[idx], np.asarray(g["s"]))
    et = rel_l2(got["t"].ravel()[idx], np.asarray(g["t"]))
    gap = abs(mpsnr(got["u"], c["u_clean"]) - g["mpsnr"])
    band = rel_l2(got["u"].reshape(v.shape[0], -1).mean(axis=1), np.asarray(g["band_mean_u"]))
    print(f"u {eu:.2e}  s {es:.2e}  t {et:.2e}  band means {band:.2e}  MPSNR gap {gap:.2e} dB  "
          f"tau_s {res.tau_s:.6g}/{g['last_trace']['tau_s']:.6g}", flush=True)
    assert eu <= 1e-4 and band <= 1e-4
    assert es <= 1e-4 and et <= 1e-4
    assert gap <= 0.01
    assert res.r == pytest.approx(g["last_trace"]["r"], rel=1e-4)


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle long run not generated")
def test_benchmark_cube_5000_iterations_bf16_duals():
    """BF16 storage of the duals over the same 5000 iterations, against the
    same FP64 oracle run: reported, with loose bounds (the storage rounding
    accumulates; it is not expected to reach the FP32 bounds)."""
    announce("256x256x128, 5000 iterations with BF16 duals vs the stored FP64 oracle run")
    torch = torch_cuda()
    import paper_2510_00562_amd as geo
    from synth.quality import mpsnr
    g = json.load(open(GOLDEN))
    c = make_cube(CUBE_256x256x128)
    vd = dev(f32(c["v"]))
    dims = geo.dims_of(vd.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"], dual_storage=geo.GEO_STORE_BF16)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, vd, ws)
    res = geo.geo_step(dims, p, vd, ws, g["iterations"])
    assert res.iters == g["iterations"]
    u = torch.empty_like(vd)
    geo.geo_state_get(dims, p, ws, "u", vd, u)
    u = u.cpu().numpy().astype(np.float64)
    eu = rel_l2(u.ravel()[np.asarray(g["sample_index"])], np.asarray(g["u"]))
    gap = mpsnr(u, c["u_clean"]) - g["mpsnr"]
    print(f"BF16 duals: u {eu:.2e} relative L2, MPSNR {gap:+.3f} dB against the FP64 oracle", flush=True)
    assert eu <= 3e-2 and abs(gap) <= 0.5
