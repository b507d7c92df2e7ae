"""Seeded synthetic hyperspectral cubes with the paper's mixed-noise model.

This module is shared by the FP64 oracle, the GPU tests and the benchmark. It
holds only input generation: a clean cube, the four noise components of the
observation model (Sec. III-B, the model v = u + s + t + n) and the radii of
the constraint sets. None of the solver's arithmetic lives here.

Layout of every cube: band-sequential (BSQ), a C-contiguous array of shape
(N3, N1, N2); element (i, j, k) of the paper's N1 x N2 x N3 cube (vertical
pixel i, horizontal pixel j, band k) sits at index (k * N1 + i) * N2 + j.

Recipe (the paper's datasets are not available; these cubes stand in for
them with the same value range and noise types, Sec. IV-A):
  G1 endmembers: E spectra, each a sum of 3 Gaussians in band index,
     amplitude ~ U[0.2, 1], centre ~ U[0, N3-1], width ~ U[0.05 N3, 0.25 N3],
     each min-max scaled to [0.1, 0.9].
  G2 abundances: C Voronoi seeds uniform over the image plane; every pixel
     takes its nearest seed (ties to the lower seed index); each cell draws
     r ~ U(0, 1]^E normalised to sum to 1.
  G3 clean cube: u[i, j, k] = sum_e A[i, j, e] f_e(k), inside [0.1, 0.9].
  G4 Gaussian noise n ~ N(0, sigma^2), iid.
  G5 stripes: in each band, round(p_t N2) distinct columns get one offset
     ~ U[-0.5, 0.5] added down the whole column, so the stripe cube has zero
     vertical difference.
  G6 salt and pepper: each voxel with probability p_s is set to 0 or 1.
  G7 dead columns: round(c_d N3) bands; in each, round(p_d N2) columns of
     width 1 are set to 0.
  G8 composition: v = u + t + n, then overwritten by G6 and G7; at an
     overwritten voxel n := 0 and the sparse component s := v - u - t.
  G9 radii: eps = r ||n||_2, alpha = r ||s||_1, beta = r ||t||_1 with
     r = 0.98; box [0, 1]; omega = 0.03.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass(frozen=True)
class CubeSpec:
    n1: int
    n2: int
    n3: int
    endmembers: int = 4
    cells: int = 12
    sigma: float = 0.1
    p_s: float = 0.05
    p_t: float = 0.05
    p_d: float = 0.0
    c_d: float = 0.0
    seed: int = 0
    radius_scale: float = 0.98
    omega: float = 0.03


# Workloads (sizes, noise mix and seeds of the five measured configurations).
SMALL_64x64x16 = CubeSpec(64, 64, 16, endmembers=4, cells=12, sigma=0.1,
                          p_s=0.05, p_t=0.05, seed=0)
CUBE_256x256x128 = CubeSpec(256, 256, 128, endmembers=8, cells=64, sigma=0.05,
                            p_s=0.05, p_t=0.1, p_d=0.02, c_d=0.10, seed=1)
CUBE_512x512x224 = CubeSpec(512, 512, 224, endmembers=8, cells=64, sigma=0.05,
                            p_s=0.05, p_t=0.1, p_d=0.02, c_d=0.10, seed=3)


def like(spec: CubeSpec, **kw) -> CubeSpec:
    return dataclasses.replace(spec, **kw)


def _endmembers(rng, e, n3):
    k = np.arange(n3, dtype=np.float64)
    out = np.empty((e, n3))
    for m in range(e):
        f = np.zeros(n3)
        for _ in range(3):
            amp = rng.uniform(0.2, 1.0)
            ctr = rng.uniform(0.0, max(n3 - 1, 0))
            wid = rng.uniform(0.05 * n3, 0.25 * n3)
            f += amp * np.exp(-((k - ctr) ** 2) / (2.0 * wid * wid))
        lo, hi = f.min(), f.max()
        f = (f - lo) / (hi - lo) if hi > lo else np.zeros(n3)
        out[m] = 0.1 + 0.8 * f
    return out


def _abundances(rng, n1, n2, e, c):
    seeds = np.stack([rng.uniform(0, n1, c), rng.uniform(0, n2, c)], axis=1)
    ii, jj = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    best = np.full((n1, n2), np.inf)
    label = np.zeros((n1, n2), dtype=np.int64)
    for q in range(c):  # strict '<' keeps the lower seed index on ties
        d = (ii - seeds[q, 0]) ** 2 + (jj - seeds[q, 1]) ** 2
        take = d < best
        best[take] = d[take]
        label[take] = q
    r = 1.0 - rng.uniform(0.0, 1.0, size=(c, e))  # in (0, 1]
    r /= r.sum(axis=1, keepdims=True)
    return r[label]  # (n1, n2, e)


def make_cube(spec: CubeSpec) -> dict:
    """Return a dict with float64 BSQ arrays u_clean, v, n, s_bar, t_bar and
    the radii eps, alpha, beta, the box and omega."""
    rng = np.random.default_rng(spec.seed)
    n1, n2, n3 = spec.n1, spec.n2, spec.n3
    f = _endmembers(rng, spec.endmembers, n3)                 # (E, n3)
    a = _abundances(rng, n1, n2, spec.endmembers, spec.cells)  # (n1, n2, E)
    u = np.einsum("ije,ek->kij", a, f)                       # BSQ
    n = rng.normal(0.0, spec.sigma, size=u.shape)
    t = np.zeros_like(u)
    n_str = int(round(spec.p_t * n2))
    for k in range(n3):
        if n_str:
            cols = rng.choice(n2, size=n_str, replace=False)
            t[k][:, cols] += rng.uniform(-0.5, 0.5, size=n_str)[None, :]
    v = u + t + n
    hit = np.zeros(u.shape, dtype=bool)
    if spec.p_s > 0:
        sp = rng.uniform(size=u.shape) < spec.p_s
        val = (rng.uniform(size=u.shape) < 0.5).astype(np.float64)
        v[sp] = val[sp]
        hit |= sp
    n_dead_bands = int(round(spec.c_d * n3))
    n_dead_cols = int(round(spec.p_d * n2))
    if n_dead_bands and n_dead_cols:
        bands = rng.choice(n3, size=n_dead_bands, replace=False)
        for k in bands:
            cols = rng.choice(n2, size=n_dead_cols, replace=False)
            v[k][:, cols] = 0.0
            hit[k][:, cols] = True
    n = np.where(hit, 0.0, n)
    s = np.where(hit, v - u - t, 0.0)
    rs = spec.radius_scale
    return dict(
        u_clean=u, v=v, n=n, s_bar=s, t_bar=t,
        eps=rs * float(np.sqrt(np.sum(n * n))),
        alpha=rs * float(np.sum(np.abs(s))),
        beta=rs * float(np.sum(np.abs(t))),
        mu_lo=0.0, mu_hi=1.0, omega=spec.omega,
        shape=(n3, n1, n2),
    )


def random_state(shape, seed, scale=0.1):
    """Independent seeded random arrays for every state variable of the
    iteration (for single-step parity from a non-trivial state). Plane counts
    follow the variables' sizes: u, s, t one plane; w1, w2 six; y1, y2 two;
    y3, y4 one."""
    rng = np.random.default_rng(seed)
    n3, n1, n2 = shape
    planes = dict(u=1, s=1, t=1, w1=6, w2=6, y1=2, y2=2, y3=1, y4=1)
    out = {}
    for name, p in planes.items():
        arr = rng.normal(0.0, scale, size=(p, n3, n1, n2))
        out[name] = arr[0] if p == 1 else arr
    out["u"] = rng.uniform(0.0, 1.0, size=shape)
    return out


def random_cube(shape, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def batch_specs(n: int = 32, seed: int = 2):
    """The uneven batch: n cubes with N1, N2 ~ U{64..256}, N3 ~ U{32..190},
    Gaussian sigma ~ U[0.02, 0.15], the other noise parts as for the
    256 x 256 x 128 cube; dimensions and sigmas from rng(seed), cube c
    generated from seed 2000 + c."""
    rng = np.random.default_rng(seed)
    n1 = rng.integers(64, 257, size=n)
    n2 = rng.integers(64, 257, size=n)
    n3 = rng.integers(32, 191, size=n)
    sig = rng.uniform(0.02, 0.15, size=n)
    return [like(CUBE_256x256x128, n1=int(n1[c]), n2=int(n2[c]), n3=int(n3[c]),
                 sigma=float(sig[c]), seed=2000 + c) for c in range(n)]


def serving_specs(n: int, rate: float, seed: int = 4):
    """A request stream: Poisson arrivals at `rate` per second, sizes drawn
    from {128x128x64, 256x256x128, 256x256x190, 512x512x224} with weights
    {0.4, 0.3, 0.2, 0.1}, noise as for the 256 x 256 x 128 cube; arrivals and
    sizes from rng(seed), request q generated from seed 40000 + q. Returns
    [(arrival seconds, CubeSpec)]."""
    rng = np.random.default_rng(seed)
    sizes = [(128, 128, 64), (256, 256, 128), (256, 256, 190), (512, 512, 224)]
    pick = rng.choice(len(sizes), size=n, p=[0.4, 0.3, 0.2, 0.1])
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for q in range(n):
        a, b, k = sizes[pick[q]]
        out.append((float(t[q]), like(CUBE_256x256x128, n1=a, n2=b, n3=k, seed=40000 + q)))
    return out


# ---- the paper's five noise cases (Sec. IV-A) on a synthetic clean cube ----
CASES = {
    1: dict(gauss=True, sparse=False, stripe=False, dead=False),
    2: dict(gauss=True, sparse=True, stripe=False, dead=False),
    3: dict(gauss=True, sparse=False, stripe=True, dead=False),
    4: dict(gauss=True, sparse=False, stripe=False, dead=True),
    5: dict(gauss=True, sparse=True, stripe=True, dead=True),
}
CASE_SIGMA, CASE_PS, CASE_PT, CASE_PD = 0.1, 0.05, 0.05, 0.01
CASE_WIDTHS = (1, 2, 3)


def paper_case(case: int, n1: int, n2: int, n3: int, seed: int = 0, omega: float = 0.03,
               endmembers: int = 6, cells: int = 24) -> dict:
    """A cube with noise case 1..5 of Sec. IV-A and the radii of eqs.
    (25)-(27):
      Gaussian sigma 0.1 (every case); salt and pepper at rate 0.05 (cases
      2, 5); vertical stripes, each column of each band with probability
      0.05 offset by U[-0.5, 0.5] (cases 3, 5); deadlines (cases 4, 5): in
      every band each column starts with probability 0.01 a run of zero
      columns of width U{1, 2, 3}.
      alpha = rho N (0.5 p_s + mean(v) c_d), beta = rho 0.5 N p_t (1 - p_s)
      (1 - c_d) / 2, eps = rho sqrt(sigma^2 N (1 - p_s)(1 - c_d)), with the
      deadline coverage c_d = 1 - exp(-mean width * p_d) and rho = 0.98,
      0.95, 0.90 for one, two, three nonzero radii (cases 1, 2-4, 5).
    The clean cube follows G1-G3. Returns the dict of make_cube."""
    flags = CASES[case]
    rng = np.random.default_rng(seed)
    f = _endmembers(rng, endmembers, n3)
    a = _abundances(rng, n1, n2, endmembers, cells)
    u = np.einsum("ije,ek->kij", a, f)
    n = rng.normal(0.0, CASE_SIGMA, size=u.shape)
    t = np.zeros_like(u)
    p_s = CASE_PS if flags["sparse"] else 0.0
    p_t = CASE_PT if flags["stripe"] else 0.0
    p_d = CASE_PD if flags["dead"] else 0.0
    if p_t:
        hit_col = rng.uniform(size=(n3, n2)) < p_t
        off = rng.uniform(-0.5, 0.5, size=(n3, n2))
        t += (hit_col * off)[:, None, :]
    v = u + t + n
    hit = np.zeros(u.shape, dtype=bool)
    if p_s:
        sp = rng.uniform(size=u.shape) < p_s
        val = (rng.uniform(size=u.shape) < 0.5).astype(np.float64)
        v[sp] = val[sp]
        hit |= sp
    if p_d:
        start = rng.uniform(size=(n3, n2)) < p_d
        width = rng.choice(CASE_WIDTHS, size=(n3, n2))
        dead = np.zeros((n3, n2), dtype=bool)
        for k, j in zip(*np.nonzero(start)):
            dead[k, j:j + width[k, j]] = True
        v = np.where(dead[:, None, :], 0.0, v)
        hit |= np.broadcast_to(dead[:, None, :], u.shape)
    n = np.where(hit, 0.0, n)
    s = np.where(hit, v - u - t, 0.0)
    N = u.size
    c_d = 1.0 - np.exp(-np.mean(CASE_WIDTHS) * p_d)
    nonzero = 1 + (p_s > 0 or p_d > 0) + (p_t > 0)
    rho = {1: 0.98, 2: 0.95, 3: 0.90}[nonzero]
    alpha = rho * N * (0.5 * p_s + float(v.mean()) * c_d)
    beta = rho * 0.5 * N * p_t * (1 - p_s) * (1 - c_d) / 2
    eps = rho * np.sqrt(CASE_SIGMA ** 2 * N * (1 - p_s) * (1 - c_d))
    return dict(u_clean=u, v=v, n=n, s_bar=s, t_bar=t, eps=float(eps), alpha=float(alpha),
                beta=float(beta), mu_lo=0.0, mu_hi=1.0, omega=omega, shape=(n3, n1, n2),
                case=case, rho=rho, c_d=c_d)


# Shapes of the paper's two simulated-noise images (Sec. IV-A).
PAVIA_SHAPE = (120, 120, 99)    # N1, N2, N3
JASPER_SHAPE = (100, 100, 198)


# ---- the paper's real-image experiment (Sec. IV-B), synthetic stand-ins ----
# (N1, N2, N3), fixed radii (alpha, beta, eps), omega
REAL_SHAPES = {
    "indian_pines_shape": ((120, 120, 198), (200.0, 100.0, 30.0), 0.01),
    "suwannee_shape": ((100, 100, 360), (800.0, 5000.0, 100.0), 0.01),
}


def real_shape_case(name: str, seed: int = 9) -> dict:
    """A synthetic cube of the shape of one of the paper's real images, with
    its fixed radii (the data itself is not available). The noise levels are
    chosen so that those radii are 0.98 of the noise norms: Gaussian sigma =
    eps / (0.98 sqrt(N)), salt and pepper at rate 2 alpha / (0.98 N), stripes
    on a fraction beta / (0.98 * 0.25 N) of the columns."""
    (n1, n2, n3), (alpha, beta, eps), omega = REAL_SHAPES[name]
    N = n1 * n2 * n3
    spec = like(CUBE_256x256x128, n1=n1, n2=n2, n3=n3, sigma=eps / (0.98 * np.sqrt(N)),
                p_s=2 * alpha / (0.98 * N), p_t=beta / (0.98 * 0.25 * N), p_d=0.0, c_d=0.0,
                seed=seed, omega=omega)
    c = make_cube(spec)
    c.update(eps=eps, alpha=alpha, beta=beta, omega=omega)
    return c
