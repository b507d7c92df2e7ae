"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/geosstv.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "geosstv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(geo_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    import paper_2510_00562_amd as geo
    names = declared()
    assert len(names) >= 14
    L = ctypes.CDLL(geo.library_path)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_abi():
    import paper_2510_00562_amd as geo
    for n in declared():
        if n.endswith("_workspace_size") and n != "geo_workspace_size":
            continue  # wrapped inside the projection calls
        assert hasattr(geo, n), n


def test_strerror_and_argument_checks_without_gpu():
    import paper_2510_00562_amd as geo
    L = geo.lib()
    assert geo.geo_strerror(0) == "success"
    assert "invalid" in geo.geo_strerror(-1)
    n = ctypes.c_size_t()
    assert L.geo_workspace_size(geo.geo_dims(0, 4, 4), None, ctypes.byref(n)) == -1
    assert L.geo_workspace_size(geo.geo_dims(64, 64, 16), None, ctypes.byref(n)) == 0
    # 21 state planes twice, plus the y4 intermediate: at least 43 words per voxel
    assert n.value >= 43 * 4 * 64 * 64 * 16
    # batch argument checks need no device
    assert L.geo_batch_table_size(0, ctypes.byref(n)) == -1
    assert L.geo_batch_table_size(65, ctypes.byref(n)) == -1
    assert L.geo_batch_table_size(3, ctypes.byref(n)) == 0 and n.value % 256 == 0
    p = geo.params(1.0, 1.0, 1.0, mu_lo=1.0, mu_hi=0.0)
    assert L.geo_state_init(geo.geo_dims(4, 4, 4), ctypes.byref(p), None, None, 0, None) == -1
    p = geo.params(1.0, 1.0, 1.0)
    fake = ctypes.c_void_p(256)
    assert L.geo_state_init(geo.geo_dims(4, 4, 4), ctypes.byref(p), fake, None, 0, None) == -2
    assert L.geo_apply_op(42, 0, geo.geo_dims(4, 4, 4), fake, fake, None) == -1


def test_sweep_geometry_is_host_side():
    """Tile counts of the fused sweep (8 x 128 pixel tiles): 256 x 256 x 128
    at 32 bands gives 32 x 2 x 4 tiles; 512 x 512 x 224 at 8 bands would
    need 7168 tiles, beyond the 4096 a cube may have, so the chunk is
    doubled to 16 (3584 tiles); requests below 8 bands use 8."""
    import paper_2510_00562_amd as geo
    g = geo.geo_sweep_geometry(geo.dims_of((128, 256, 256)), 32)
    assert g == (32, 256, 8, 128)
    assert geo.geo_sweep_geometry(geo.dims_of((224, 512, 512)), 8)[:2] == (16, 3584)
    assert geo.geo_sweep_geometry(geo.dims_of((360, 100, 100)), 3)[:2] == (8, 13 * 1 * 45)
    L = geo.lib()
    x = ctypes.c_int32()
    assert L.geo_sweep_geometry(geo.geo_dims(0, 4, 4), 0, 8, 256, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4, 4, 4), 5, 8, 256, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4, 4, 4), 0, -1, 256, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4, 4, 4), 0, 0, 0, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4, 4, 4), 0, 8, 256, None, *[ctypes.byref(x)] * 3) == -1
    assert L.geo_sweep_blocks(7, ctypes.byref(x)) == -1
    assert L.geo_sweep_blocks(0, None) == -1
    import torch
    if not torch.cuda.is_available():  # no device: the block count is a device query
        assert L.geo_sweep_blocks(0, ctypes.byref(x)) == -3


@pytest.mark.parametrize("shape, blocks, chunk", [
    # (N3, N1, N2): 256 tiles at 32 bands fill 256 blocks in one round
    ((128, 256, 256), 256, 32),
    # 7 rounds of 32 + 2 band-equivalents; 28 bands would need 8 of 30
    ((224, 512, 512), 256, 32),
    # 384 tiles at 32 bands are 1.5 rounds: 24 bands give 2 rounds of 512
    # tiles of 24 + 2 (27 bands would give 2 rounds of 29, with a last
    # chunk of one band)
    ((190, 256, 256), 256, 24),
    # 32 tiles at 32 bands on 256 blocks: 8 bands give 128 tiles, each 4x shorter
    ((64, 128, 128), 256, 8),
    # 13 tile rows: 19 chunks of at most 19 bands give 247 tiles, one round
    ((360, 100, 100), 256, 19),
    # 15 tile rows: 17 chunks of at most 12 bands give 255 tiles, one round
    ((198, 120, 120), 256, 12),
    # 8 tile rows, 16 bands: 8 tiles of 16 (+2) or 16 tiles of 8 (+2)
    ((16, 64, 64), 256, 8),
    # a single 5-band tile at any depth: ties keep 32
    ((5, 8, 100), 256, 32),
    # fewer blocks: 256 x 256 x 128 on 64 blocks still prefers 32 bands
    ((128, 256, 256), 64, 32),
])
def test_default_band_chunk_balances_the_blocks(shape, blocks, chunk):
    """The library's default depth (band_chunk 0) minimises
    ceil(tiles / blocks) x (min(kc, N3) + 2) over kc in 8..32, ties to the
    deeper chunk."""
    import paper_2510_00562_amd as geo
    d = geo.dims_of(shape)
    used = geo.geo_sweep_geometry(d, 0, blocks)[0]
    assert used == chunk
    # brute force of the same rule from the tile counts the library reports
    cost = {}
    for kc in range(32, 7, -1):
        u, tiles, _, _ = geo.geo_sweep_geometry(d, kc)
        if u == kc:  # a raised chunk repeats a deeper one
            cost[kc] = -(-tiles // min(blocks, tiles)) * (min(kc, shape[0]) + 2)
    assert used == min(cost, key=lambda kc: (cost[kc], -kc))


@pytest.mark.parametrize("shape, rows_cols", [
    # (N3, N1, N2): a width of 160 fills two 128-wide tiles to 62.5% and
    # three 64-wide ones to 83%: 16 x 64 tiles
    ((111, 160, 160), (16, 64)),
    # widths that 128-wide tiles fill as well as 64-wide ones keep 8 x 128
    ((128, 256, 256), (8, 128)),
    ((111, 128, 100), (8, 128)),
    ((198, 120, 120), (8, 128)),
    # 64 columns fill one 64-wide tile, half a 128-wide one
    ((16, 64, 64), (16, 64)),
    # 16-row tiles would leave half the rows of an 8-row cube empty
    ((5, 8, 100), (8, 128)),
    # 190 columns: 74% of two 128-wide tiles, 99% of three 64-wide ones
    ((50, 96, 190), (16, 64)),
])
def test_tile_shape_follows_the_fill(shape, rows_cols):
    """A cube gets 16 x 64 tiles when their share of points inside the cube
    beats that of 8 x 128 tiles by more than 3%; with BF16 duals always
    8 x 128. The tile count follows the shape."""
    import paper_2510_00562_amd as geo
    n3, n1, n2 = shape
    d = geo.dims_of(shape)
    kc, tiles, ti, tj = geo.geo_sweep_geometry(d, 16)
    assert (ti, tj) == rows_cols
    assert tiles == -(-n1 // ti) * -(-n2 // tj) * -(-n3 // kc)
    assert geo.geo_sweep_geometry(d, 16, dual_storage=geo.GEO_STORE_BF16)[2:] == (8, 128)


def test_workspace_holds_every_band_chunk():
    """The per-tile regions of a solver workspace hold the tiles of every
    band chunk the library can pick: any request (512 x 512 x 224 at 14
    bands has 4096 tiles, more than the 3584 of the doubled minimum chunk)
    and the default chunk for any block count (160 x 864 x 300 on 256 blocks
    picks 15 bands: 2800 tiles). Host-only."""
    import numpy as np

    import paper_2510_00562_amd as geo
    big = geo.dims_of((224, 512, 512))
    assert geo.geo_sweep_geometry(big, 14)[:2] == (14, 4096)
    assert geo.geo_sweep_geometry(big, 15)[:2] == (15, 3840)
    assert geo.geo_workspace_tiles(big) >= 4096
    odd = geo.dims_of((300, 160, 864))
    kc, tiles, _, _ = geo.geo_sweep_geometry(odd, 0, 256)
    assert tiles <= geo.geo_workspace_tiles(odd), (kc, tiles)
    rng = np.random.default_rng(5)
    shapes = [(int(rng.integers(1, 400)), int(rng.integers(1, 700)), int(rng.integers(1, 900)))
              for _ in range(40)] + [(224, 512, 512), (300, 160, 864), (1, 2048, 2048)]
    for shape in shapes:
        d = geo.dims_of(shape)
        for ds in (geo.GEO_STORE_F32, geo.GEO_STORE_BF16):
            cap = geo.geo_workspace_tiles(d, ds)
            worst = max(geo.geo_sweep_geometry(d, kc, dual_storage=ds)[1]
                        for kc in range(1, shape[0] + 2))
            worst = max([worst] + [geo.geo_sweep_geometry(d, 0, b, dual_storage=ds)[1]
                                   for b in (8, 64, 200, 256, 512, 1024)])
            assert worst <= cap, (shape, ds, worst, cap)


def test_bands_beyond_the_tile_limit_are_rejected():
    """One band of more than 4096 tiles (here 4096 x 4096 pixels) cannot be
    swept: the solver entry points refuse it instead of looping on the band
    chunk; 2048 x 2048 is the largest square band."""
    import paper_2510_00562_amd as geo
    L = geo.lib()
    n = ctypes.c_size_t()
    x = ctypes.c_int32()
    assert L.geo_workspace_size(geo.geo_dims(4096, 4096, 1), None, ctypes.byref(n)) == -1
    assert L.geo_workspace_tiles(geo.geo_dims(4096, 4096, 1), 0, ctypes.byref(x)) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4096, 4096, 1), 0, 8, 256, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_workspace_size(geo.geo_dims(2048, 2048, 3), None, ctypes.byref(n)) == 0
    assert geo.geo_sweep_geometry(geo.geo_dims(2048, 2048, 3), 8)[:2] == (8, 4096)


def test_regularizer_argument_checks_without_gpu():
    """The comparison regularizers: the workspace size is host-side and takes
    any dims with N < 2^31 (no tile limit); FP32 duals only; an unknown
    regularizer, the batched and the profiled entry points give GEO_EINVAL
    before any device work (fake non-null pointers are never dereferenced)."""
    geo = pytest.importorskip("paper_2510_00562_amd")
    L = geo.lib()
    n = ctypes.c_size_t()
    for reg in (1, 2, 3):
        p = geo.params(1.0, 1.0, 1.0, regularizer=reg)
        assert L.geo_workspace_size(geo.geo_dims(4096, 4096, 1), ctypes.byref(p), ctypes.byref(n)) == 0
        N = 4096 * 4096
        assert n.value >= (11 + (2 if reg == 1 else 4)) * 4 * N  # 11 arrays + the planes of y1
        assert L.geo_workspace_size(geo.geo_dims(4, 5, 6), ctypes.byref(p), ctypes.byref(n)) == 0
        small = n.value
        assert L.geo_workspace_size(geo.geo_dims(0, 5, 6), ctypes.byref(p), ctypes.byref(n)) == -1
        pb = geo.params(1.0, 1.0, 1.0, regularizer=reg, dual_storage=geo.GEO_STORE_BF16)
        assert L.geo_workspace_size(geo.geo_dims(4, 5, 6), ctypes.byref(pb), ctypes.byref(n)) == -1
        fake = ctypes.c_void_p(256)
        d = geo.geo_dims(4, 5, 6)
        assert L.geo_state_init(d, ctypes.byref(p), fake, fake, small - 1, None) == -2
        ms = (ctypes.c_double * 3)()
        assert L.geo_step_profiled(d, ctypes.byref(p), fake, fake, small, 1, None, None, ms) == -1
        D = (geo.geo_dims * 1)(d)
        Pa = (geo.geo_params * 1)(p)
        V = (ctypes.c_void_p * 1)(256)
        B = (ctypes.c_size_t * 1)(small)
        assert L.geo_batch_step(1, D, Pa, V, V, B, fake, 1 << 20, 1, 0, None, None) == -1
    bad = geo.params(1.0, 1.0, 1.0, regularizer=4)
    assert L.geo_workspace_size(geo.geo_dims(4, 5, 6), ctypes.byref(bad), ctypes.byref(n)) == -1
    assert geo.var_planes("y1", 1) == 2 and geo.var_planes("y1", 3) == 4 and geo.var_planes("y1") == 2
    with pytest.raises(KeyError):
        geo.var_planes("w1", 2)
