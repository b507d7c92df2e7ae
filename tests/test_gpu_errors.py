"""Error paths of the C ABI on a GPU: every failure comes back as a status
code and leaves nothing running. Workspace checks, batch argument checks, a
cap reached before the tolerance, and NaN in the observed cube (the device
flags the non-finite iterate and idles; the threshold searches still end)."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import announce, dev, f32, torch_cuda
from synth.cubes import SMALL_64x64x16, like, make_cube

pytestmark = pytest.mark.gpu
EINVAL, EWORKSPACE, ENONFINITE, MAXITER = -1, -2, -4, 1


def small(seed=0, shape=(6, 20, 33)):
    n3, n1, n2 = shape
    c = make_cube(like(SMALL_64x64x16, n1=n1, n2=n2, n3=n3, seed=seed, cells=4))
    return f32(c["v"]), c


def test_workspace_checks():
    announce("workspace size and alignment")
    torch_cuda()
    import paper_2510_00562_amd as geo
    v, c = small()
    L = geo.lib()
    dims = geo.dims_of(v.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"])
    need = geo.geo_workspace_size(dims, p)
    ws = geo.Workspace(need + 512)
    vd = dev(v)
    vp = ctypes.c_void_p(vd.data_ptr())
    out = geo.geo_result()
    assert L.geo_state_init(dims, ctypes.byref(p), vp, ws.ptr, need - 256, None) == EWORKSPACE
    odd = ctypes.c_void_p(ws.tensor.data_ptr() + 4)
    assert L.geo_state_init(dims, ctypes.byref(p), vp, odd, need, None) == EWORKSPACE
    assert L.geo_step(dims, ctypes.byref(p), vp, ws.ptr, need - 1, 5, None, ctypes.byref(out)) == EWORKSPACE
    assert L.geo_step(dims, ctypes.byref(p), vp, ws.ptr, need, -1, None, ctypes.byref(out)) == EINVAL
    geo.geo_state_init(dims, p, vd, ws)
    r = geo.geo_step(dims, p, vd, ws, 0)
    assert r.iters == 0 and r.total_iters == 0


def test_batch_argument_checks():
    announce("batch argument checks")
    torch_cuda()
    import paper_2510_00562_amd as geo
    v, c = small(1)
    vd = dev(v)
    dims = geo.dims_of(v.shape)
    p32 = geo.params(c["eps"], c["alpha"], c["beta"])
    p16 = geo.params(c["eps"], c["alpha"], c["beta"], dual_storage=geo.GEO_STORE_BF16)
    w32 = geo.Workspace(geo.geo_workspace_size(dims, p32))
    w16 = geo.Workspace(geo.geo_workspace_size(dims, p16))
    geo.geo_state_init(dims, p32, vd, w32)
    geo.geo_state_init(dims, p16, vd, w16)
    table = geo.Workspace(geo.geo_batch_table_size(2))
    with pytest.raises(geo.GeoError) as e:
        geo.geo_batch_step([dims, dims], [p32, p16], [vd, vd], [w32, w16], table, 3)
    assert e.value.status == EINVAL
    small_table = geo.Workspace(geo.geo_batch_table_size(1))
    with pytest.raises(geo.GeoError) as e:
        geo.geo_batch_step([dims, dims], [p32, p32], [vd, vd], [w32, w32], small_table, 3)
    assert e.value.status == EWORKSPACE
    n = ctypes.c_size_t()
    assert geo.lib().geo_batch_table_size(65, ctypes.byref(n)) == EINVAL
    assert geo.lib().geo_batch_table_size(0, ctypes.byref(n)) == EINVAL


def test_cap_before_tolerance():
    announce("iteration cap before the tolerance")
    torch_cuda()
    import paper_2510_00562_amd as geo
    v, c = small(2)
    vd = dev(v)
    dims = geo.dims_of(v.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"], tol=1e-12)
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, vd, ws)
    rc = geo.lib().geo_step(dims, ctypes.byref(p), ctypes.c_void_p(vd.data_ptr()), ws.ptr,
                            ws.nbytes, 7, None, ctypes.byref(out := geo.geo_result()))
    assert rc == MAXITER and out.iters == 7 and out.converged == 0


@pytest.mark.parametrize("where", ["nan", "inf"])
def test_non_finite_input_is_reported(where):
    announce(f"{where} in the observed cube")
    torch_cuda()
    import paper_2510_00562_amd as geo
    v, c = small(3)
    v = v.copy()
    v[2, 5, 7] = np.nan if where == "nan" else np.inf
    vd = dev(v)
    dims = geo.dims_of(v.shape)
    p = geo.params(c["eps"], c["alpha"], c["beta"])
    ws = geo.Workspace(geo.geo_workspace_size(dims, p))
    geo.geo_state_init(dims, p, vd, ws)
    out = geo.geo_result()
    rc = geo.lib().geo_step(dims, ctypes.byref(p), ctypes.c_void_p(vd.data_ptr()), ws.ptr,
                            ws.nbytes, 20, None, ctypes.byref(out))
    assert rc == ENONFINITE
    assert out.iters < 20
    # the state stays flagged: a later call returns at once
    rc2 = geo.lib().geo_step(dims, ctypes.byref(p), ctypes.c_void_p(vd.data_ptr()), ws.ptr,
                             ws.nbytes, 5, None, ctypes.byref(out))
    assert rc2 == ENONFINITE and out.iters == 0
