"""The quality harness on the GPU path: the paper's noise cases 1 (Gaussian
only) and 5 (Gaussian, salt and pepper, stripes, deadlines) of Sec. IV-A on a
synthetic cube of the shape of its first image (120 x 120 x 99), radii by
eqs. (25)-(27), omega in {0.01, 0.03, 0.05}: the six solves in one batched
call (geo_batch_step), 300 iterations, against the FP64 oracle's runs stored
by tests/golden/make_long_runs.py. Bounds: u within 1e-4 relative L2 on the
samples, MPSNR (eq. (29)) within 0.01 dB and MSSIM (eq. (30)) within 1e-4."""
import json
import os

import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quality_cases_300.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle quality runs not generated")
def test_paper_cases_through_the_batched_path():
    torch = torch_cuda()
    import paper_2510_00562_amd as geo
    from synth.cubes import PAVIA_SHAPE, paper_case
    from synth.quality import mpsnr, mssim
    g = json.load(open(GOLDEN))
    announce(f"noise cases {sorted({s['case'] for s in g['solves']})} at {PAVIA_SHAPE}, omega "
             f"{sorted({s['omega'] for s in g['solves']})}, {g['iterations']} iterations, one batch")
    n1, n2, n3 = PAVIA_SHAPE
    cs = [paper_case(s["case"], n1, n2, n3, seed=0, omega=s["omega"]) for s in g["solves"]]
    vs = [dev(f32(c["v"])) for c in cs]
    dims = [geo.dims_of(v.shape) for v in vs]
    ps = [geo.params(c["eps"], c["alpha"], c["beta"], omega=c["omega"]) for c in cs]
    wss = [geo.Workspace(geo.geo_workspace_size(d, p)) for d, p in zip(dims, ps)]
    for d, p, v, ws in zip(dims, ps, vs, wss):
        geo.geo_state_init(d, p, v, ws)
    table = geo.Workspace(geo.geo_batch_table_size(len(vs)))
    rc, res = geo.geo_batch_step(dims, ps, vs, wss, table, g["iterations"], use_graph=True)
    assert rc == 0 and all(r.iters == g["iterations"] for r in res)
    for s, c, d, p, v, ws in zip(g["solves"], cs, dims, ps, vs, wss):
        u = torch.empty_like(v)
        geo.geo_state_get(d, p, ws, "u", v, u)
        u = u.cpu().numpy().astype(np.float64)
        eu = rel_l2(u.ravel()[np.asarray(s["sample_index"])], np.asarray(s["u"]))
        dp = mpsnr(u, c["u_clean"]) - s["mpsnr"]
        ds = mssim(u, c["u_clean"]) - s["mssim"]
        print(f"case {s['case']} omega {s['omega']}: MPSNR {s['mpsnr']:.3f} dB, MSSIM "
              f"{s['mssim']:.4f} (oracle); u {eu:.2e}, MPSNR gap {dp:+.2e} dB, MSSIM gap {ds:+.2e}",
              flush=True)
        assert eu <= 1e-4 and abs(dp) <= 0.01 and abs(ds) <= 1e-4
