"""The band-chunk tuner's load-balance model on the host (no GPU): its
ranking for single cubes, and the busiest-block simulation of the sweep's
tile hand-out."""
import numpy as np
import pytest


@pytest.fixture
def tune(monkeypatch):
    import paper_2510_00562_amd.tune as t
    monkeypatch.setattr(t, "geo_sweep_blocks", lambda dual_storage=0: 256)
    return t


def test_busiest_block_matches_a_direct_hand_out(tune):
    """8 XCDs, each a contiguous eighth of the tiles; block b = x + 8 * slot
    takes tiles lo_x + slot, lo_x + slot + G/8, ... of its XCD's eighth."""
    rng = np.random.default_rng(0)
    for T, G in [(1000, 256), (256, 256), (37, 256), (5000, 64), (300, 12)]:
        cost = rng.uniform(1, 10, size=T)
        g = min(G, T)
        load = np.zeros(g)
        if g >= 8 and g % 8 == 0:
            per = g // 8
            for b in range(g):
                x, slot = b % 8, b // 8
                lo, hi = x * T // 8, (x + 1) * T // 8
                load[b] = cost[lo + slot:hi:per].sum()
        else:
            for b in range(g):
                load[b] = cost[b::g].sum()
        assert tune._busiest_block(cost, G) == pytest.approx(load.max())


@pytest.mark.parametrize("shape, best", [
    # (N3, N1, N2): one round of tiles at the most bands per tile
    ((360, 100, 100), (19, 20)),
    ((198, 120, 120), (12,)),
    ((128, 256, 256), (32,)),
])
def test_model_ranks_the_balanced_chunk_first(tune, shape, best):
    import paper_2510_00562_amd as geo
    ranked = tune.model_candidates([geo.dims_of(shape)], n=4)
    assert ranked[0] in best and len(ranked) == 4 and len(set(ranked)) == 4


def test_model_sums_the_two_tile_shapes(tune):
    """A 16 x 64-tile cube and an 8 x 128-tile cube run in two launches: the
    model's estimate is the sum of the two busiest blocks."""
    import paper_2510_00562_amd as geo
    a, b = geo.dims_of((64, 160, 160)), geo.dims_of((64, 128, 128))
    assert geo.geo_sweep_geometry(a, 16)[2:] == (16, 64)
    assert geo.geo_sweep_geometry(b, 16)[2:] == (8, 128)
    # each cube alone at 16 bands: 4 chunks; 10 x 3 and 16 x 1 pixel tiles
    ta = np.repeat(np.full(4, 16 + 2.0), 30)
    tb = np.repeat(np.full(4, 16 + 2.0), 16)
    want = tune._busiest_block(ta, 256) + tune._busiest_block(tb, 256)
    got = {}
    orig = tune._busiest_block

    def spy(cost, G):
        got.setdefault("calls", []).append(cost.size)
        return orig(cost, G)
    tune._busiest_block = spy
    try:
        tune.model_candidates([a, b], n=64, lo=16, hi=16)
    finally:
        tune._busiest_block = orig
    assert sorted(got["calls"]) == sorted([ta.size, tb.size])
    assert want == pytest.approx(2 * 18.0)
