"""FP64 CPU oracle for the GeoSSTV P-PDS solver.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package. The GPU product path shares no code
with it and never calls it.

A ctypes wrapper around ``geosstv_oracle.c`` (plain double-precision loops,
one per operator; the generic P-PDS update of eq. (7) applied to problem (20)
block by block). Arrays are numpy
float64 in band-sequential layout: shape (N3, N1, N2), element (i, j, k) at
[k, i, j]. Multi-plane fields carry a leading plane axis: D x and the duals
y1, y2 have 2 planes (vertical, horizontal); L y and w1, w2 have 6 planes
(ud_v, ud_h, lr_v, lr_h, c_v, c_h).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "geosstv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Step sizes printed after eq. (24) of the paper.
STEP_U, STEP_W1, STEP_W2, STEP_S, STEP_T, STEP_Y = 1 / 13, 1 / 4, 1 / 4, 1.0, 1 / 3, 1 / 5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no -march=native: the library travels to
    other hosts). Returns the path of the shared library."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _setup(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("mu_lo", ctypes.c_double),
                ("mu_hi", ctypes.c_double), ("omega", ctypes.c_double)]


def _setup(L):
    i, I64, d = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    for name in ("ora_dv", "ora_dv_t", "ora_dh", "ora_dh_t", "ora_ds", "ora_ds_t",
                 "ora_d", "ora_d_t", "ora_l_ud", "ora_l_ud_t", "ora_l_lr",
                 "ora_l_lr_t", "ora_l_c", "ora_l_c_t", "ora_l", "ora_l_t"):
        getattr(L, name).argtypes = [i, i, i, _dp, _dp]
        getattr(L, name).restype = None
    L.ora_proj_box.argtypes = [_dp, I64, d, d, _dp]
    L.ora_proj_l2.argtypes = [_dp, _dp, I64, d, _dp]
    L.ora_proj_l2.restype = d
    L.ora_proj_l1.argtypes = [_dp, I64, d, _dp]
    L.ora_proj_l1.restype = d
    L.ora_prox_l12.argtypes = [_dp, _dp, I64, d, _dp, _dp]
    st = [_dp] * 9
    L.ora_init.argtypes = [i, i, i, _dp] + st
    L.ora_step.argtypes = [i, i, i, ctypes.POINTER(Params), _dp] + st + [_dp]
    L.ora_run.argtypes = [i, i, i, ctypes.POINTER(Params), _dp] + st + [i, d, i, _dp]
    L.ora_run.restype = i
    L.ora_step_sizes.argtypes = [_dp]
    L.ora_set_threads.argtypes = [i]
    L.ora_get_threads.restype = i
    L.ora_var_planes.argtypes = [i]
    L.ora_var_planes.restype = i
    L.ora_var_step_sizes.argtypes = [i, d, _dp]
    L.ora_var_apply_k.argtypes = [i, i, i, i, d, i, _dp, _dp]
    L.ora_var_init.argtypes = [i, i, i, i, _dp] + [_dp] * 6
    L.ora_var_run.argtypes = [i, i, i, ctypes.POINTER(Params), i, _dp] + [_dp] * 6 + [i, d, i, _dp]
    L.ora_var_run.restype = i
    global _max_threads
    _max_threads = L.ora_get_threads()


_max_threads = 1


def threads_for(n_voxels: int) -> int:
    """Thread count used for a cube of n voxels: one thread below 32K voxels
    (the OpenMP fork costs more than the loop), all host threads above."""
    return 1 if n_voxels < 32768 else _max_threads


def step_sizes():
    """Step sizes compiled into the oracle: (u, w1, w2, s, t, y)."""
    out = np.zeros(6)
    lib().ora_step_sizes(_p(out))
    return tuple(out)


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# operator name -> (C function, input planes, output planes)
_OPS = {
    "dv": ("ora_dv", "ora_dv_t", 1, 1),
    "dh": ("ora_dh", "ora_dh_t", 1, 1),
    "ds": ("ora_ds", "ora_ds_t", 1, 1),
    "d": ("ora_d", "ora_d_t", 1, 2),
    "l_ud": ("ora_l_ud", "ora_l_ud_t", 2, 2),
    "l_lr": ("ora_l_lr", "ora_l_lr_t", 2, 2),
    "l_c": ("ora_l_c", "ora_l_c_t", 2, 2),
    "l": ("ora_l", "ora_l_t", 2, 6),
}
OPS = tuple(_OPS) + ("dds", "k")


def apply(op: str, x, shape, adjoint: bool = False):
    """Apply a linear operator of the problem (or its adjoint).

    ``shape`` = (N3, N1, N2). Inputs with p planes have shape (p, N3, N1, N2)
    (a single plane may drop the leading axis). ``dds`` is D D_s; ``k`` is the
    stacked operator of problem (20), mapping (u, s, t, w1, w2) to
    (y1, y2, y3, y4) as a flat vector of 15N entries to 6N entries."""
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    if op == "dds":
        if not adjoint:
            t = apply("ds", x, shape)
            return apply("d", t, shape)
        t = apply("d", x, shape, adjoint=True)
        return apply("ds", t, shape, adjoint=True)
    if op == "k":
        return _apply_k(np.asarray(x, dtype=np.float64).ravel(), shape, adjoint)
    fwd, adj, pin, pout = _OPS[op]
    if adjoint:
        pin, pout = pout, pin
    xin = _c(x).reshape(-1)
    assert xin.size == pin * N, (op, xin.size, pin * N)
    out = np.empty(pout * N)
    getattr(lib(), adj if adjoint else fwd)(n1, n2, n3, _p(xin), _p(out))
    return out.reshape((pout, n3, n1, n2) if pout > 1 else (n3, n1, n2))


def _apply_k(x, shape, adjoint):
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    if not adjoint:
        u, s, t = x[:N], x[N:2 * N], x[2 * N:3 * N]
        w1, w2 = x[3 * N:9 * N], x[9 * N:15 * N]
        y1 = apply("d", u, shape).ravel() - apply("l", w1, shape, adjoint=True).ravel()
        y2 = apply("dds", u, shape).ravel() - apply("l", w2, shape, adjoint=True).ravel()
        y3 = apply("dv", t, shape).ravel()
        y4 = u + s + t
        return np.concatenate([y1, y2, y3, y4])
    y1, y2, y3, y4 = x[:2 * N], x[2 * N:4 * N], x[4 * N:5 * N], x[5 * N:6 * N]
    u = apply("d", y1, shape, True).ravel() + apply("dds", y2, shape, True).ravel() + y4
    s = y4.copy()
    t = apply("dv", y3, shape, True).ravel() + y4
    w1 = -apply("l", y1, shape).ravel()
    w2 = -apply("l", y2, shape).ravel()
    return np.concatenate([u, s, t, w1, w2])


def proj_box(x, lo, hi):
    x = _c(x)
    out = np.empty_like(x)
    lib().ora_proj_box(_p(x), x.size, lo, hi, _p(out))
    return out


def proj_l2(x, center, eps):
    """Projection onto the eps-ball around ``center`` (eq. (23)); returns
    (projection, ||x - center||)."""
    x, c = _c(x), _c(center)
    out = np.empty_like(x)
    r = lib().ora_proj_l2(_p(x), _p(c), x.size, eps, _p(out))
    return out, r


def proj_l1(x, radius):
    """Projection onto the l1 ball of the given radius; returns (projection,
    tau) with tau the soft-threshold level (0 inside the ball, inf for a zero
    radius)."""
    x = _c(x)
    out = np.empty_like(x)
    tau = lib().ora_proj_l1(_p(x), x.size, radius, _p(out))
    return out, tau


def prox_l12(xa, xb, gamma):
    """Group soft-shrink of eq. (24) over pairs (xa[q], xb[q])."""
    xa, xb = _c(xa), _c(xb)
    oa, ob = np.empty_like(xa), np.empty_like(xb)
    lib().ora_prox_l12(_p(xa), _p(xb), xa.size, gamma, _p(oa), _p(ob))
    return oa, ob


STATE = ("u", "s", "t", "w1", "w2", "y1", "y2", "y3", "y4")
PLANES = dict(u=1, s=1, t=1, w1=6, w2=6, y1=2, y2=2, y3=1, y4=1)


class Solver:
    """P-PDS (eq. (7), the iteration of Alg. 1) for problem (20) on one cube,
    in double precision."""

    def __init__(self, v, eps, alpha, beta, mu_lo=0.0, mu_hi=1.0, omega=0.03, state=None):
        self.v = _c(v)
        self.shape = self.v.shape
        n3, n1, n2 = self.shape
        self.dims = (n1, n2, n3)
        self.params = Params(eps, alpha, beta, mu_lo, mu_hi, omega)
        self.state = {}
        for name in STATE:
            p = PLANES[name]
            self.state[name] = np.zeros(((p,) if p > 1 else ()) + self.shape)
        if state is None:
            lib().ora_init(*self.dims, _p(self.v), *self._ptrs())
        else:
            for name in STATE:
                self.state[name][...] = state[name]
        self.trace = []

    def _ptrs(self):
        return [_p(self.state[n]) for n in STATE]

    def step(self, n: int = 1, tol: float = 0.0) -> int:
        lib().ora_set_threads(threads_for(self.v.size))
        tr = np.zeros(4 * max(n, 1))
        done = lib().ora_run(*self.dims, ctypes.byref(self.params), _p(self.v), *self._ptrs(),
                             n, tol, len(self.trace), _p(tr))
        self.trace.extend(tuple(tr[4 * q:4 * q + 4]) for q in range(done))
        return done

    def __getattr__(self, name):
        st = self.__dict__.get("state")
        if st is not None and name in st:
            return st[name]
        raise AttributeError(name)


# The comparison regularizers of Sec. IV-A, solved by the same P-PDS.
SSTV, HSSTV1, HSSTV2 = 1, 2, 3
VARIANTS = {"sstv": SSTV, "hsstv1": HSSTV1, "hsstv2": HSSTV2}


def var_planes(variant: int) -> int:
    """Entries of A u per voxel: 2 for SSTV (D D_s u), 4 for HSSTV
    (D D_s u and omega D u)."""
    return lib().ora_var_planes(int(variant))


def var_step_sizes(variant: int, omega: float):
    """Step sizes (u, s, t, y) of a variant: eq. (8) with the operator-norm
    bounds of D_v, D, D D_s and omega D."""
    out = np.zeros(4)
    lib().ora_var_step_sizes(int(variant), float(omega), _p(out))
    return tuple(out)


def var_apply_k(variant: int, omega: float, x, shape, adjoint: bool = False):
    """The stacked operator of a variant's problem, (u, s, t) -> (A u, D_v t,
    u + s + t), or its adjoint, on flat vectors."""
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    P = var_planes(variant)
    x = _c(x).ravel()
    assert x.size == ((P + 2) * N if adjoint else 3 * N)
    out = np.empty(3 * N if adjoint else (P + 2) * N)
    lib().ora_var_apply_k(n1, n2, n3, int(variant), float(omega), 1 if adjoint else 0, _p(x), _p(out))
    return out


VAR_STATE = ("u", "s", "t", "y1", "y3", "y4")


class VariantSolver:
    """P-PDS (eq. (7)) for problem (15) with the GeoSSTV term replaced by a
    comparison regularizer (SSTV, HSSTV1, HSSTV2), in double precision. y1
    holds var_planes(variant) planes."""

    def __init__(self, v, eps, alpha, beta, variant, mu_lo=0.0, mu_hi=1.0, omega=0.03, state=None):
        self.v = _c(v)
        self.shape = self.v.shape
        n3, n1, n2 = self.shape
        self.dims = (n1, n2, n3)
        self.variant = int(variant)
        self.params = Params(eps, alpha, beta, mu_lo, mu_hi, omega)
        P = var_planes(self.variant)
        self.state = {n: np.zeros(((P,) if n == "y1" else ()) + self.shape) for n in VAR_STATE}
        if state is None:
            lib().ora_var_init(*self.dims, self.variant, _p(self.v), *self._ptrs())
        else:
            for n in VAR_STATE:
                self.state[n][...] = state[n]
        self.trace = []

    def _ptrs(self):
        return [_p(self.state[n]) for n in VAR_STATE]

    def step(self, n: int = 1, tol: float = 0.0) -> int:
        lib().ora_set_threads(threads_for(self.v.size))
        tr = np.zeros(4 * max(n, 1))
        done = lib().ora_var_run(*self.dims, ctypes.byref(self.params), self.variant, _p(self.v),
                                 *self._ptrs(), n, tol, len(self.trace), _p(tr))
        self.trace.extend(tuple(tr[4 * q:4 * q + 4]) for q in range(done))
        return done

    def __getattr__(self, name):
        st = self.__dict__.get("state")
        if st is not None and name in st:
            return st[name]
        raise AttributeError(name)


def mpsnr(u, u_clean):
    """Mean PSNR over bands, eq. (29), with peak 1 (intensities in [0, 1]):
    mean_k 10 log10(N1 N2 / ||u_k - u_clean_k||^2)."""
    u = np.asarray(u, dtype=np.float64)
    c = np.asarray(u_clean, dtype=np.float64)
    n3 = u.shape[0]
    npix = u[0].size
    err = ((u - c) ** 2).reshape(n3, -1).sum(axis=1)
    return float(np.mean(10.0 * np.log10(npix / err)))
