"""Batched iterations (geo_batch_step): uneven cubes advanced together in one
launch sequence per iteration. Every cube's iterates must be exactly those
of the same cube iterated alone with geo_step (the per-tile FP64 partials
and the per-cube sweep B blocks make the summation order independent of the
batch), with and without the HIP graph replay, and each cube stops by its
own rule. The single-cube path itself is held to the FP64 oracle by the
other GPU tests; one batched cube is checked against the oracle here too."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, rel_l2, torch_cuda
from synth.cubes import CUBE_512x512x224, SMALL_64x64x16, like, make_cube
from test_gpu_step import STATE, get_state

pytestmark = pytest.mark.gpu

SHAPES = [(16, 64, 64), (5, 13, 70), (1, 1, 1), (33, 20, 64), (7, 130, 9), (40, 17, 66)]


def cubes(shapes, seed0=100):
    out = []
    for q, (n3, n1, n2) in enumerate(shapes):
        c = make_cube(like(SMALL_64x64x16, n1=n1, n2=n2, n3=n3, seed=seed0 + q, cells=6,
                           sigma=0.02 + 0.02 * q))
        c["v"] = f32(c["v"])
        out.append(c)
    return out


def setup(geo, c, tol=0.0, dual_storage=0, band_chunk=0):
    shape = c["v"].shape
    dims = geo.dims_of(shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"], omega=0.03, tol=tol, dual_storage=dual_storage,
                   band_chunk=band_chunk)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    vd = dev(c["v"])
    geo.geo_state_init(dims, p, vd, ws)
    return dims, p, vd, ws


def run_batch(geo, cs, n_iter, tol=0.0, dual_storage=0, use_graph=False, band_chunk=0):
    st = [setup(geo, c, tol, dual_storage, band_chunk) for c in cs]
    table = geo.Workspace(geo.geo_batch_table_size(len(cs)))
    rc, res = geo.geo_batch_step([x[0] for x in st], [x[1] for x in st], [x[2] for x in st],
                                 [x[3] for x in st], table, n_iter, use_graph=use_graph)
    states = [get_state(geo, d, p, ws, vd, c["v"].shape) for (d, p, vd, ws), c in zip(st, cs)]
    return rc, res, states


def run_solo(geo, c, n_iter, tol=0.0, dual_storage=0, band_chunk=0):
    d, p, vd, ws = setup(geo, c, tol, dual_storage, band_chunk)
    res = geo.geo_step(d, p, vd, ws, n_iter)
    return res, get_state(geo, d, p, ws, vd, c["v"].shape)


def same(a, b):
    for n in STATE:
        assert np.array_equal(a[n], b[n]), n


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_each_cube_alone(use_graph):
    announce(f"batch of {len(SHAPES)} uneven cubes, 25 iterations, graph={use_graph}")
    torch_cuda()
    import paper_2510_00562_amd as geo
    cs = cubes(SHAPES)
    rc, res, states = run_batch(geo, cs, 25, use_graph=use_graph)
    assert rc == 0
    for c, r, s in zip(cs, res, states):
        r1, s1 = run_solo(geo, c, 25)
        assert r.iters == r1.iters == 25
        assert r.tau_s == r1.tau_s and r.tau_t == r1.tau_t and r.r == r1.r
        same(s, s1)


def test_batch_cubes_stop_by_their_own_rule():
    announce("batch with tolerance: cubes stop at different iterations")
    torch_cuda()
    import paper_2510_00562_amd as geo
    cs = cubes(SHAPES[:4], seed0=200)
    rc, res, states = run_batch(geo, cs, 400, tol=3e-3)
    iters = [r.iters for r in res]
    for c, r, s in zip(cs, res, states):
        r1, s1 = run_solo(geo, c, 400, tol=3e-3)
        assert r.iters == r1.iters and r.converged == r1.converged
        same(s, s1)
    assert len(set(iters)) > 1, iters


def test_batch_bf16_and_band_chunk():
    announce("batch with BF16 duals and 8-band tiles")
    torch_cuda()
    import paper_2510_00562_amd as geo
    cs = cubes(SHAPES[:3], seed0=300)
    rc, res, states = run_batch(geo, cs, 12, dual_storage=1, band_chunk=8)
    for c, r, s in zip(cs, res, states):
        r1, s1 = run_solo(geo, c, 12, dual_storage=1, band_chunk=8)
        same(s, s1)


def test_band_chunk_does_not_change_the_iterates(ora):
    """The tile depth is a performance knob: iterates agree with the oracle
    whatever it is (FP64 sums are reordered, so not bit for bit)."""
    announce("band chunk 8 / 32 / 64 vs oracle, 40x33x70, 15 iterations")
    torch_cuda()
    import paper_2510_00562_amd as geo
    c = cubes([(40, 33, 70)], seed0=400)[0]
    S = ora.Solver(c["v"], c["eps"], c["alpha"], c["beta"], omega=0.03)
    S.step(15)
    for kc in (8, 32, 64):
        _, s = run_solo(geo, c, 15, band_chunk=kc)
        for n in STATE:
            assert rel_l2(s[n], S.state[n]) <= 1e-5, (kc, n)


def test_batched_cube_matches_oracle(ora):
    announce("batched 64x64x16 cube vs oracle, 60 iterations")
    torch_cuda()
    import paper_2510_00562_amd as geo
    cs = cubes([(16, 64, 64), (9, 31, 77)], seed0=500)
    rc, res, states = run_batch(geo, cs, 60)
    for c, s in zip(cs, states):
        S = ora.Solver(c["v"], c["eps"], c["alpha"], c["beta"], omega=0.03)
        S.step(60)
        assert rel_l2(s["u"], S.u) <= 1e-5


def test_band_chunk_raised_at_the_tile_limit():
    """512 x 512 x 224 with 8-band tiles would need 7168 tiles, beyond the
    4096 a launch supports: the library doubles the chunk to 16 bands, so the
    request for 8 and the request for 16 run the same tiles and give the same
    bits; 32-band tiles differ only by FP64 summation order."""
    announce("band chunk 8 on 512x512x224: raised to 16")
    torch = torch_cuda()
    import paper_2510_00562_amd as geo
    c = make_cube(CUBE_512x512x224)
    out = {}
    for kc in (8, 16, 32):
        d, p, vd, ws = setup(geo, c, band_chunk=kc)
        geo.geo_step(d, p, vd, ws, 3)
        u = torch.empty_like(vd)
        geo.geo_state_get(d, p, ws, "u", vd, u)
        out[kc] = u.cpu().numpy()
        del ws
    assert np.array_equal(out[8], out[16])
    assert rel_l2(out[32], out[16]) <= 1e-6


def test_working_cubes_share_the_persistent_blocks():
    """Three cubes of 128 tiles each (8 x 128 pixels, 8 bands) and one of
    240 (16 x 64 pixels: its width of 160 fills 64-wide tiles better): more
    tiles than resident sweep A blocks in the 8 x 128 launch, so the blocks
    take XCD-ordered tile ranges, and a second launch for the 16 x 64 cube.
    One cube meets its stopping rule early; from then on only the other
    cubes' tiles are in the list the blocks share. Every cube's iterates,
    iteration count and stopping flag must still be those of the cube run
    alone."""
    shapes = [(64, 64, 256), (64, 64, 250), (64, 60, 256), (64, 160, 160)]
    tols = [3e-3, 0.0, 0.0, 0.0]
    n_iter = 80
    announce(f"batch {shapes}, tolerances {tols}, {n_iter} iterations, 8-band tiles")
    torch_cuda()
    import paper_2510_00562_amd as geo
    cs = cubes(shapes, seed0=600)
    st = [setup(geo, c, tol, band_chunk=8) for c, tol in zip(cs, tols)]
    table = geo.Workspace(geo.geo_batch_table_size(len(cs)))
    rc, res = geo.geo_batch_step([x[0] for x in st], [x[1] for x in st], [x[2] for x in st],
                                 [x[3] for x in st], table, n_iter, use_graph=True)
    states = [get_state(geo, d, p, ws, vd, c["v"].shape) for (d, p, vd, ws), c in zip(st, cs)]
    assert res[0].converged and res[0].iters < n_iter - 20, res[0].iters  # stops near 37
    assert [r.iters for r in res[1:]] == [n_iter] * 3
    assert [geo.geo_sweep_geometry(d, 8)[2:] for d, _, _, _ in st] == [(8, 128)] * 3 + [(16, 64)]
    for c, tol, r, s in zip(cs, tols, res, states):
        r1, s1 = run_solo(geo, c, n_iter, tol=tol, band_chunk=8)
        assert r.iters == r1.iters and r.converged == r1.converged
        assert r.tau_s == r1.tau_s and r.tau_t == r1.tau_t and r.r == r1.r
        same(s, s1)


def test_graph_kept_across_calls_reads_the_new_table():
    """Two batches of different cubes with the same sizes, one after the
    other through the same table: the second call replays the graph kept
    from the first (same table address and launch shape), and its cubes'
    iterates must be their own, equal to each cube run alone."""
    announce("graph reuse: two batches of equal sizes through one table")
    torch_cuda()
    import paper_2510_00562_amd as geo
    shapes = [(16, 64, 64), (9, 31, 77)]
    first, second = cubes(shapes, seed0=700), cubes(shapes, seed0=800)
    table = geo.Workspace(geo.geo_batch_table_size(len(shapes)))
    for cs in (first, second, first):
        st = [setup(geo, c) for c in cs]
        rc, res = geo.geo_batch_step([x[0] for x in st], [x[1] for x in st], [x[2] for x in st],
                                     [x[3] for x in st], table, 15, use_graph=True)
        assert rc == 0
        for (d, p, vd, ws), c, r in zip(st, cs, res):
            s = get_state(geo, d, p, ws, vd, c["v"].shape)
            r1, s1 = run_solo(geo, c, 15)
            assert r.tau_s == r1.tau_s and r.tau_t == r1.tau_t and r.r == r1.r
            same(s, s1)
