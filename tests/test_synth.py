"""The seeded cube generator: layout, value ranges and the noise structure
the constraints of problem (15) rely on."""
import numpy as np

from synth.cubes import SMALL_64x64x16, like, make_cube


def test_generator_structure():
    spec = like(SMALL_64x64x16, n1=20, n2=24, n3=10, p_d=0.1, c_d=0.3, seed=5)
    c = make_cube(spec)
    assert c["v"].shape == (10, 20, 24) == c["shape"]
    u = c["u_clean"]
    assert 0.1 - 1e-12 <= u.min() and u.max() <= 0.9 + 1e-12
    # stripes are constant down every column: zero vertical difference
    assert np.abs(np.diff(c["t_bar"], axis=1)).max() == 0.0
    # observation model v = u + s + t + n holds exactly
    np.testing.assert_allclose(c["v"], u + c["s_bar"] + c["t_bar"] + c["n"], atol=1e-15)
    # radii from the true components at 0.98x
    assert c["eps"] == np.float64(0.98) * np.linalg.norm(c["n"])
    assert np.isclose(c["alpha"], 0.98 * np.abs(c["s_bar"]).sum())
    assert np.isclose(c["beta"], 0.98 * np.abs(c["t_bar"]).sum())
    # determinism
    np.testing.assert_array_equal(make_cube(spec)["v"], c["v"])
    # dead columns and salt-and-pepper overwrite: values 0 or 1 there
    hit = c["s_bar"] != 0
    assert set(np.unique(c["v"][hit])).issubset({0.0, 1.0})


def test_oracle_mpsnr_closed_form(ora):
    """eq. (29) with peak 1: an error of constant size d in every voxel gives
    10 log10(1 / d^2)."""
    u = np.random.default_rng(0).uniform(size=(3, 4, 5))
    assert np.isclose(ora.mpsnr(u + 0.01, u), 40.0)
