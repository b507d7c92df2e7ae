"""GeoSSTV hyperspectral denoising and destriping on AMD MI355X (gfx950).

Python binding of the C ABI in ``include/geosstv.h`` (library
``libgeosstv.so`` next to this file). The functions carry the C names and
only marshal arguments: torch tensors on the GPU become device pointers, the
current torch stream becomes the HIP stream. Every step of the solver runs in
the library's HIP kernels; there is no Python or CPU fallback, and importing
any entry point without the built library raises.

Cube layout: band-sequential float32 tensors of shape (N3, N1, N2), i.e.
element (i, j, k) of the paper's N1 x N2 x N3 cube at [k, i, j].
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "geo_dims", "geo_params", "geo_result", "GeoError", "lib", "library_path",
    "geo_workspace_size", "geo_state_init", "geo_step", "geo_step_profiled", "geo_solve", "geo_state_get",
    "geo_state_set", "geo_apply_op", "geo_project_l1", "geo_project_l2", "geo_prox_l12",
    "geo_project_box", "geo_strerror", "OPS", "VARS", "VAR_PLANES", "REGULARIZERS", "var_planes",
    "Workspace",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libgeosstv.so")

GEO_OK, GEO_MAXITER = 0, 1
GEO_EINVAL, GEO_EWORKSPACE, GEO_EHIP, GEO_ENONFINITE = -1, -2, -3, -4
GEO_STORE_F32, GEO_STORE_BF16 = 0, 1
OPS = dict(dv=0, dh=1, ds=2, d=3, dds=4, l_ud=5, l_lr=6, l_c=7, l=8, k=9)
OP_PLANES = dict(dv=(1, 1), dh=(1, 1), ds=(1, 1), d=(1, 2), dds=(1, 2), l_ud=(2, 2),
                 l_lr=(2, 2), l_c=(2, 2), l=(2, 6), k=(15, 6))
VARS = dict(u=0, s=1, t=2, w1=3, w2=4, y1=5, y2=6, y3=7, y4=8)
VAR_PLANES = dict(u=1, s=1, t=1, w1=6, w2=6, y1=2, y2=2, y3=1, y4=1)
# the comparison regularizers of Sec. IV-A (GEO_REG_*); 0 is GeoSSTV
REGULARIZERS = dict(geosstv=0, sstv=1, hsstv1=2, hsstv2=3)


def var_planes(var: str, regularizer: int = 0) -> int:
    """Planes of a state variable: y1 has 2 (SSTV) or 4 (HSSTV1/2) planes
    for the comparison regularizers, which have no w1, w2 or y2."""
    if regularizer and var in ("w1", "w2", "y2"):
        raise KeyError(f"{var} does not exist for regularizer {regularizer}")
    if regularizer and var == "y1":
        return 2 if regularizer == REGULARIZERS["sstv"] else 4
    return VAR_PLANES[var]


class geo_dims(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32)]


class geo_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("mu_lo", ctypes.c_double), ("mu_hi", ctypes.c_double),
                ("omega", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("dual_storage", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("band_chunk", ctypes.c_int32),
                ("regularizer", ctypes.c_int32)]


class geo_result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_change", ctypes.c_double), ("r", ctypes.c_double),
                ("tau_s", ctypes.c_double), ("tau_t", ctypes.c_double),
                ("total_iters", ctypes.c_int32), ("fallback_passes", ctypes.c_int32),
                ("cand_s", ctypes.c_int32), ("cand_t", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("status", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class GeoError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {geo_strerror(status)} (status {status})")
        self.status = status


_lib = None
_vp, _sz = ctypes.c_void_p, ctypes.c_size_t


def lib():
    """The loaded library; raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing: build it with "
                              "`python paper_2510_00562_amd/build.py`")
        # torch ships its own HIP runtime with the same soname; load it first
        # so that the library binds to it and the process holds one runtime
        # (two HSA runtimes in one process do not share the device).
        import torch  # noqa: F401
        L = ctypes.CDLL(library_path)
        i32, i64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P, R = ctypes.POINTER(geo_params), ctypes.POINTER(geo_result)
        sig = {
            "geo_workspace_size": [geo_dims, P, ctypes.POINTER(_sz)],
            "geo_state_init": [geo_dims, P, _vp, _vp, _sz, _vp],
            "geo_step": [geo_dims, P, _vp, _vp, _sz, i32, _vp, R],
            "geo_solve": [geo_dims, P, _vp, _vp, _vp, _vp, _vp, _sz, _vp, R],
            "geo_step_profiled": [geo_dims, P, _vp, _vp, _sz, i32, _vp, R,
                                  ctypes.POINTER(ctypes.c_double)],
            "geo_step_timed": [geo_dims, P, _vp, _vp, _sz, i32, _vp, R,
                               ctypes.POINTER(ctypes.c_double)],
            "geo_state_get": [geo_dims, P, _vp, _sz, i32, _vp, _vp, _vp],
            "geo_state_set": [geo_dims, P, _vp, _sz, i32, _vp, _vp, _vp],
            "geo_apply_op": [i32, i32, geo_dims, _vp, _vp, _vp],
            "geo_project_l1_workspace_size": [i64, ctypes.POINTER(_sz)],
            "geo_project_l1": [_vp, i64, d, _vp, ctypes.POINTER(d), _vp, _sz, _vp],
            "geo_project_l1_noalloc": [_vp, i64, d, _vp, _vp, _vp],
            "geo_project_l2_workspace_size": [i64, ctypes.POINTER(_sz)],
            "geo_project_l2": [_vp, _vp, i64, d, _vp, ctypes.POINTER(d), _vp, _sz, _vp],
            "geo_prox_l12": [_vp, _vp, i64, d, _vp, _vp, _vp],
            "geo_project_box": [_vp, i64, d, d, _vp, _vp],
            "geo_strerror": [ctypes.c_int],
            "geo_batch_table_size": [i32, ctypes.POINTER(_sz)],
            "geo_sweep_geometry": [geo_dims, i32, i32, i32] + [ctypes.POINTER(i32)] * 4,
            "geo_sweep_blocks": [i32, ctypes.POINTER(i32)],
            "geo_workspace_tiles": [geo_dims, i32, ctypes.POINTER(i32)],
            "geo_batch_step": [i32, ctypes.POINTER(geo_dims), P, ctypes.POINTER(_vp),
                               ctypes.POINTER(_vp), ctypes.POINTER(_sz), _vp, _sz, i32, i32, _vp,
                               R],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "geo_strerror" else ctypes.c_int
        _lib = L
    return _lib


def geo_strerror(status: int) -> str:
    return lib().geo_strerror(status).decode()


# ---------------------------------------------------------------- marshalling
def _torch():
    import torch
    return torch


def _ptr(t, dtype=None):
    if t is None:
        return None
    torch = _torch()
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t):
    return _ptr(t, _torch().float32)


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def dims_of(shape) -> geo_dims:
    """geo_dims from a BSQ shape (N3, N1, N2) (a leading plane axis allowed)."""
    n3, n1, n2 = shape[-3:]
    return geo_dims(n1, n2, n3)


def params(eps, alpha, beta, mu_lo=0.0, mu_hi=1.0, omega=0.03, max_iter=1000, tol=0.0,
           dual_storage=GEO_STORE_F32, check_every=0, band_chunk=0, regularizer=0) -> geo_params:
    """regularizer: 0 (GeoSSTV), a GEO_REG_* value or a name of REGULARIZERS."""
    if isinstance(regularizer, str):
        regularizer = REGULARIZERS[regularizer]
    return geo_params(eps, alpha, beta, mu_lo, mu_hi, omega, max_iter, tol, dual_storage,
                      check_every, band_chunk, regularizer)


def _check(rc, where, allow_maxiter=False):
    if rc < 0 or (rc > 0 and not allow_maxiter):
        raise GeoError(rc, where)
    return rc


# ---------------------------------------------------------------- entry points
def geo_workspace_size(dims: geo_dims, p: geo_params | None = None) -> int:
    n = _sz()
    _check(lib().geo_workspace_size(dims, ctypes.byref(p) if p is not None else None,
                                    ctypes.byref(n)), "geo_workspace_size")
    return n.value


class Workspace:
    """A device buffer of the size the library asks for (torch allocates it;
    256-byte alignment is guaranteed by the caching allocator)."""

    def __init__(self, nbytes: int, device="cuda"):
        torch = _torch()
        self.tensor = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        self.nbytes = int(nbytes)
        assert self.tensor.data_ptr() % 256 == 0

    @property
    def ptr(self):
        return ctypes.c_void_p(self.tensor.data_ptr())


def geo_state_init(dims, p, v, ws: Workspace, stream=None):
    _check(lib().geo_state_init(dims, ctypes.byref(p), _f32(v), ws.ptr, ws.nbytes,
                                _stream(stream)), "geo_state_init")


def geo_step(dims, p, v, ws: Workspace, n_iter: int, stream=None) -> geo_result:
    out = geo_result()
    _check(lib().geo_step(dims, ctypes.byref(p), _f32(v), ws.ptr, ws.nbytes, int(n_iter),
                          _stream(stream), ctypes.byref(out)), "geo_step", allow_maxiter=True)
    return out


PHASES = ("sweep_a", "l1_select", "sweep_b")


def geo_step_profiled(dims, p, v, ws: Workspace, n_iter: int, stream=None):
    """geo_step with per-phase GPU times (HIP events): returns
    (geo_result, {phase: summed milliseconds})."""
    out = geo_result()
    ms = (ctypes.c_double * len(PHASES))()
    _check(lib().geo_step_profiled(dims, ctypes.byref(p), _f32(v), ws.ptr, ws.nbytes, int(n_iter),
                                   _stream(stream), ctypes.byref(out), ms),
           "geo_step_profiled", allow_maxiter=True)
    return out, dict(zip(PHASES, list(ms)))


def geo_step_timed(dims, p, v, ws: Workspace, n_iter: int, stream=None):
    """geo_step with HIP events around the fused sweep (the dual kernel for
    the comparison regularizers) of every 8th slot: returns (geo_result, that
    kernel's milliseconds summed over the call, estimated from the sampled
    launches)."""
    out = geo_result()
    ms = ctypes.c_double()
    _check(lib().geo_step_timed(dims, ctypes.byref(p), _f32(v), ws.ptr, ws.nbytes, int(n_iter),
                                _stream(stream), ctypes.byref(out), ctypes.byref(ms)),
           "geo_step_timed", allow_maxiter=True)
    return out, ms.value


def geo_solve(dims, p, v, u, s, t, ws: Workspace, stream=None) -> geo_result:
    out = geo_result()
    _check(lib().geo_solve(dims, ctypes.byref(p), _f32(v), _f32(u), _f32(s), _f32(t), ws.ptr,
                           ws.nbytes, _stream(stream), ctypes.byref(out)), "geo_solve",
           allow_maxiter=True)
    return out


def geo_batch_table_size(n_cubes: int) -> int:
    n = _sz()
    _check(lib().geo_batch_table_size(int(n_cubes), ctypes.byref(n)), "geo_batch_table_size")
    return n.value


def geo_sweep_geometry(dims, requested: int = 0, blocks: int = 0,
                       dual_storage: int = GEO_STORE_F32):
    """(bands per tile used, tiles, tile rows, tile columns) of the fused
    sweep for one cube at the requested band chunk (0 = the library's
    default for `blocks` persistent blocks)."""
    out = [ctypes.c_int32() for _ in range(4)]
    _check(lib().geo_sweep_geometry(dims, int(dual_storage), int(requested), int(blocks),
                                    *[ctypes.byref(x) for x in out]), "geo_sweep_geometry")
    return tuple(x.value for x in out)


def geo_workspace_tiles(dims, dual_storage: int = GEO_STORE_F32) -> int:
    """Tiles the per-tile regions of a solver workspace hold for these dims."""
    n = ctypes.c_int32()
    _check(lib().geo_workspace_tiles(dims, int(dual_storage), ctypes.byref(n)),
           "geo_workspace_tiles")
    return n.value


def geo_sweep_blocks(dual_storage: int = GEO_STORE_F32) -> int:
    """Persistent blocks of the fused sweep on the current device."""
    n = ctypes.c_int32()
    _check(lib().geo_sweep_blocks(int(dual_storage), ctypes.byref(n)), "geo_sweep_blocks")
    return n.value


def geo_batch_step(dims, ps, vs, wss, table: Workspace, n_iter: int, use_graph=False,
                   stream=None, raise_nonfinite=True):
    """n_iter iterations of every cube of a batch in one launch sequence per
    iteration. dims, ps, vs, wss: lists (geo_dims, geo_params, device cube,
    Workspace) of equal length; table: a Workspace of geo_batch_table_size
    bytes. Returns (status, [geo_result per cube]). raise_nonfinite=False
    returns GEO_ENONFINITE with the results (each cube's own status in
    .status) instead of raising."""
    n = len(dims)
    if not (len(ps) == len(vs) == len(wss) == n):
        raise ValueError("dims, ps, vs and wss must have one entry per cube")
    D = (geo_dims * n)(*dims)
    Pa = (geo_params * n)(*ps)
    V = (_vp * n)(*[_f32(v) for v in vs])
    W = (_vp * n)(*[w.ptr for w in wss])
    B = (_sz * n)(*[w.nbytes for w in wss])
    out = (geo_result * n)()
    rc = lib().geo_batch_step(n, D, Pa, V, W, B, table.ptr, table.nbytes, int(n_iter),
                              1 if use_graph else 0, _stream(stream), out)
    if not (rc == GEO_ENONFINITE and not raise_nonfinite):
        rc = _check(rc, "geo_batch_step", allow_maxiter=True)
    return rc, list(out)


def geo_state_get(dims, p, ws: Workspace, var: str, v, out, stream=None):
    _check(lib().geo_state_get(dims, ctypes.byref(p), ws.ptr, ws.nbytes, VARS[var], _f32(v),
                               _f32(out), _stream(stream)), "geo_state_get")
    return out


def geo_state_set(dims, p, ws: Workspace, var: str, v, x, stream=None):
    _check(lib().geo_state_set(dims, ctypes.byref(p), ws.ptr, ws.nbytes, VARS[var], _f32(v),
                               _f32(x), _stream(stream)), "geo_state_set")


def geo_apply_op(op: str, adjoint: bool, dims, x, out, stream=None):
    _check(lib().geo_apply_op(OPS[op], 1 if adjoint else 0, dims, _f32(x), _f32(out),
                              _stream(stream)), "geo_apply_op")
    return out


def geo_project_l1(x, radius: float, out, ws: Workspace | None = None, stream=None) -> float:
    n = x.numel()
    if ws is None:
        need = _sz()
        _check(lib().geo_project_l1_workspace_size(n, ctypes.byref(need)), "workspace")
        ws = Workspace(need.value, device=x.device)
    tau = ctypes.c_double()
    _check(lib().geo_project_l1(_f32(x), n, float(radius), _f32(out), ctypes.byref(tau), ws.ptr,
                                ws.nbytes, _stream(stream)), "geo_project_l1")
    return tau.value


def geo_project_l1_noalloc(x, radius: float, out, tau_dev=None, stream=None):
    """geo_project_l1 with the library's fixed scratch: no allocation, no
    host copy, no synchronisation. tau_dev: a float64 device tensor of one
    element receiving the level, or None."""
    n = x.numel()
    tp = ctypes.c_void_p(tau_dev.data_ptr()) if tau_dev is not None else None
    _check(lib().geo_project_l1_noalloc(_f32(x), n, float(radius), _f32(out), tp, _stream(stream)),
           "geo_project_l1_noalloc")


def geo_project_l2(x, center, eps: float, out, ws: Workspace | None = None, stream=None) -> float:
    n = x.numel()
    if ws is None:
        need = _sz()
        _check(lib().geo_project_l2_workspace_size(n, ctypes.byref(need)), "workspace")
        ws = Workspace(need.value, device=x.device)
    r = ctypes.c_double()
    _check(lib().geo_project_l2(_f32(x), _f32(center), n, float(eps), _f32(out), ctypes.byref(r),
                                ws.ptr, ws.nbytes, _stream(stream)), "geo_project_l2")
    return r.value


def geo_prox_l12(xa, xb, gamma: float, oa, ob, stream=None):
    _check(lib().geo_prox_l12(_f32(xa), _f32(xb), xa.numel(), float(gamma), _f32(oa), _f32(ob),
                              _stream(stream)), "geo_prox_l12")


def geo_project_box(x, lo: float, hi: float, out, stream=None):
    _check(lib().geo_project_box(_f32(x), x.numel(), float(lo), float(hi), _f32(out),
                                 _stream(stream)), "geo_project_box")
    return out
