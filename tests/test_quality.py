"""Pins of the quality metrics and of the paper's noise-case generator
(Sec. IV-A, eqs. (25)-(30)): SSIM against a direct evaluation of its
definition on tiny images, its closed forms (identical images, a constant
shift), MPSNR against the oracle's independent implementation, and the
radius rule and noise structure of the five cases."""
import numpy as np
import pytest

from synth import quality as Q
from synth.cubes import CASES, paper_case


def ssim_direct(x, y):
    """Wang et al.'s index evaluated window by window with explicit sums."""
    g1 = Q.gaussian_window_1d()
    w = np.outer(g1, g1)
    c1, c2 = (0.01) ** 2, (0.03) ** 2
    h = 5
    vals = []
    for i in range(h, x.shape[0] - h):
        for j in range(h, x.shape[1] - h):
            px = x[i - h:i + h + 1, j - h:j + h + 1]
            py = y[i - h:i + h + 1, j - h:j + h + 1]
            mx, my = (w * px).sum(), (w * py).sum()
            sx = (w * (px - mx) ** 2).sum()
            sy = (w * (py - my) ** 2).sum()
            sxy = (w * (px - mx) * (py - my)).sum()
            vals.append(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sx + sy + c2)))
    return np.mean(vals)


def test_gaussian_window():
    g = Q.gaussian_window_1d()
    assert g.shape == (11,) and g.sum() == pytest.approx(1.0)
    assert np.allclose(g, g[::-1])
    assert g[5] / g[4] == pytest.approx(np.exp(1 / (2 * 1.5 ** 2)))


def test_ssim_matches_direct_evaluation():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(17, 15))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    assert Q.ssim(x, y) == pytest.approx(ssim_direct(x, y), rel=1e-10)
    assert Q.ssim(x, y) == pytest.approx(Q.ssim(y, x), rel=1e-12)


def test_ssim_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(20, 23))
    assert Q.ssim(x, x) == pytest.approx(1.0, abs=1e-12)
    # constant shift: equal variances and covariance, only the luminance term
    c = 0.2
    m = Q._local_mean(x, Q.gaussian_window_1d())
    lum = (2 * m * (m + c) + 1e-4) / (m * m + (m + c) ** 2 + 1e-4)
    assert np.allclose(Q.ssim_map(x, x + c), lum, rtol=1e-9)


def test_mpsnr_matches_oracle(ora):
    rng = np.random.default_rng(2)
    u = rng.uniform(size=(4, 9, 13))
    v = u + rng.normal(0, 0.05, size=u.shape)
    assert Q.mpsnr(v, u) == pytest.approx(ora.mpsnr(v, u), rel=1e-12)


@pytest.mark.parametrize("case", sorted(CASES))
def test_paper_cases(case):
    c = paper_case(case, 40, 48, 30, seed=case)
    N = c["v"].size
    assert c["rho"] == {1: 0.98, 2: 0.95, 3: 0.95, 4: 0.95, 5: 0.90}[case]
    f = CASES[case]
    assert (c["alpha"] > 0) == (f["sparse"] or f["dead"])
    assert (c["beta"] > 0) == f["stripe"]
    # decomposition and the stripe cube's zero vertical difference
    assert np.allclose(c["v"], c["u_clean"] + c["t_bar"] + c["n"] + c["s_bar"])
    assert np.allclose(np.diff(c["t_bar"], axis=1), 0.0)
    # eq. (27) with the Gaussian part of the observation
    pd = 0.01 if f["dead"] else 0.0
    cd = 1 - np.exp(-2.0 * pd)
    ps = 0.05 if f["sparse"] else 0.0
    assert c["eps"] == pytest.approx(c["rho"] * np.sqrt(0.01 * N * (1 - ps) * (1 - cd)))
    if f["dead"]:
        zero_cols = np.all(c["v"] == 0.0, axis=1)  # (n3, n2)
        assert zero_cols.mean() == pytest.approx(cd, abs=0.02)
