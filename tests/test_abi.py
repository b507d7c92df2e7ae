"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/geosstv.h declares (no compute calls here)."""
import ctypes
import os
import re

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
    at the default 32 bands gives 32 x 2 x 4 tiles; 512 x 512 x 224 at 8
    bands would need 7168 tiles, beyond the 4096 a cube may have, so the
    chunk is doubled to 16 (3584 tiles); requests below 8 bands use 8."""
    import paper_2510_00562_amd as geo
    g = geo.geo_sweep_geometry(geo.dims_of((128, 256, 256)))
    assert g == (32, 256, 8, 128)
    assert geo.geo_sweep_geometry(geo.dims_of((224, 512, 512)), 8)[:2] == (16, 3584)
    assert geo.geo_sweep_geometry(geo.dims_of((360, 100, 100)), 3)[:2] == (8, 13 * 1 * 45)
    assert geo.geo_sweep_geometry(geo.dims_of((1, 1, 1)), 0)[:2] == (32, 1)
    L = geo.lib()
    x = ctypes.c_int32()
    assert L.geo_sweep_geometry(geo.geo_dims(0, 4, 4), 0, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4, 4, 4), -1, *[ctypes.byref(x)] * 4) == -1
    assert L.geo_sweep_geometry(geo.geo_dims(4, 4, 4), 0, None, *[ctypes.byref(x)] * 3) == -1
    assert L.geo_sweep_blocks(7, ctypes.byref(x)) == -1
    assert L.geo_sweep_blocks(0, None) == -1
