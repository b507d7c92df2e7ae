"""Pins of the oracle's proximal tools (Sec. II-B, III-B): the l1-ball
projection against a sort-based formula and brute-force enumeration, with the
vertex certificate; the l2-ball projection and the group prox of eq. (24)
against their variational definitions (eq. (1), (5)) solved numerically, and
the Moreau identity of eq. (3)."""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize


def sort_projection_tau(x, radius):
    """tau from sorting |x| in decreasing order: rho = the largest k with
    a_k > (S_k - radius) / k, tau = (S_rho - radius) / rho."""
    a = np.sort(np.abs(x))[::-1]
    S = np.cumsum(a)
    k = np.arange(1, len(a) + 1)
    ok = a > (S - radius) / k
    rho = np.nonzero(ok)[0].max() + 1
    return (S[rho - 1] - radius) / rho


def brute_force_l1(x, radius):
    """Enumerate every active set A; keep the one whose tau is consistent
    (|x_i| > tau exactly on A) and return the projection."""
    a = np.abs(x)
    n = len(x)
    found = []
    for m in range(1, n + 1):
        for A in itertools.combinations(range(n), m):
            A = list(A)
            tau = (a[A].sum() - radius) / m
            if tau <= 0:
                continue
            inside = np.zeros(n, bool)
            inside[A] = True
            if (a[inside] > tau).all() and (a[~inside] <= tau).all():
                found.append(tau)
    assert len(found) >= 1
    tau = found[0]
    assert np.allclose(found, tau)
    return np.sign(x) * np.maximum(a - tau, 0), tau


@pytest.mark.parametrize("seed", range(12))
def test_l1_against_brute_force_and_sort(ora, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    x = rng.normal(size=n) * rng.uniform(0.1, 3)
    if seed % 3 == 0:  # duplicates and zeros
        x[: n // 2] = np.round(x[: n // 2])
    radius = rng.uniform(0.05, 0.95) * np.abs(x).sum()
    if np.abs(x).sum() == 0:
        return
    z, tau = ora.proj_l1(x, radius)
    zb, taub = brute_force_l1(x, radius)
    np.testing.assert_allclose(z, zb, atol=1e-13)
    assert tau == pytest.approx(taub, rel=1e-12)
    assert tau == pytest.approx(sort_projection_tau(x, radius), rel=1e-12)


@pytest.mark.parametrize("n,seed", [(1000, 1), (20000, 2), (7, 3)])
def test_l1_certificate_and_idempotence(ora, n, seed):
    """For x outside the ball, z = P(x) lies on the sphere ||z||_1 = radius and
    satisfies the vertex certificate radius ||x - z||_inf <= <x - z, z>, which
    characterises the projection because the l1 ball is the convex hull of
    the points +-radius e_i."""
    rng = np.random.default_rng(seed)
    x = rng.laplace(size=n)
    x[rng.uniform(size=n) < 0.1] = 0.0
    x[:5] = x[5]  # ties
    radius = 0.3 * np.abs(x).sum()
    z, tau = ora.proj_l1(x, radius)
    assert np.abs(z).sum() == pytest.approx(radius, rel=1e-12)
    d = x - z
    assert radius * np.abs(d).max() <= d @ z + 1e-9 * radius
    z2, tau2 = ora.proj_l1(z, radius)
    np.testing.assert_allclose(z2, z, atol=1e-12)
    assert tau == pytest.approx(sort_projection_tau(x, radius), rel=1e-12)


def test_l1_special_cases(ora):
    x = np.array([0.5, -1.0, 0.25, 0.0])
    z, tau = ora.proj_l1(x, 10.0)  # inside: identity, tau = 0
    np.testing.assert_array_equal(z, x)
    assert tau == 0.0
    z, tau = ora.proj_l1(x, 0.0)  # zero radius: the ball is {0}
    assert not z.any() and tau == np.inf
    z, tau = ora.proj_l1(np.full(6, -2.0), 3.0)  # all equal: spread evenly
    np.testing.assert_allclose(z, np.full(6, -0.5))
    z, tau = ora.proj_l1(np.array([3.0, 0.0, 0.0]), 1.0)  # one active entry
    np.testing.assert_allclose(z, [1.0, 0.0, 0.0])
    assert tau == pytest.approx(2.0)


@pytest.mark.parametrize("seed", range(4))
def test_l2_ball_against_variational_definition(ora, seed):
    rng = np.random.default_rng(seed)
    n = 5
    x, c = rng.normal(size=n), rng.normal(size=n)
    eps = 0.5 * np.linalg.norm(x - c) if seed % 2 == 0 else 2.0 * np.linalg.norm(x - c)
    p, r = ora.proj_l2(x, c, eps)
    assert r == pytest.approx(np.linalg.norm(x - c))
    res = minimize(lambda y: 0.5 * np.sum((y - x) ** 2), c, jac=lambda y: y - x,
                   constraints=[{"type": "ineq", "fun": lambda y: eps ** 2 - np.sum((y - c) ** 2),
                                 "jac": lambda y: -2 * (y - c)}],
                   method="SLSQP", options=dict(ftol=1e-14, maxiter=500))
    np.testing.assert_allclose(p, res.x, atol=1e-6)
    p2, _ = ora.proj_l2(p, c, eps)
    np.testing.assert_allclose(p2, p, atol=1e-14)
    assert np.linalg.norm(p - c) <= eps * (1 + 1e-14)


@pytest.mark.parametrize("seed", range(6))
def test_group_prox_variational_and_moreau(ora, seed):
    rng = np.random.default_rng(seed)
    n = 50
    xa, xb = rng.normal(size=n), rng.normal(size=n)
    gamma = [0.1, 0.5, 1.0, 2.0, 0.0, 0.7][seed]
    oa, ob = ora.prox_l12(xa, xb, gamma)
    # Moreau, eq. (3) with f = ||.||_2 on R^2: prox_{g f}(x) = x - g P_{B(0,1)}(x / g)
    if gamma > 0:
        X = np.stack([xa, xb], 1) / gamma
        nr = np.linalg.norm(X, axis=1, keepdims=True)
        P = X / np.maximum(nr, 1.0)
        want = np.stack([xa, xb], 1) - gamma * P
        np.testing.assert_allclose(np.stack([oa, ob], 1), want, atol=1e-13)
    else:
        np.testing.assert_array_equal(oa, xa)
    # eq. (1) solved numerically for a few groups
    for q in range(5):
        x = np.array([xa[q], xb[q]])
        f = lambda y: gamma * np.linalg.norm(y) + 0.5 * np.sum((x - y) ** 2)
        best = min((minimize(f, y0, method="Nelder-Mead",
                             options=dict(xatol=1e-12, fatol=1e-14, maxiter=4000))
                    for y0 in (x, np.zeros(2), 0.5 * x)), key=lambda r: r.fun)
        assert f(np.array([oa[q], ob[q]])) <= best.fun + 1e-10
    z, _ = ora.prox_l12(np.zeros(3), np.zeros(3), 0.3)
    assert not z.any()


def test_box(ora):
    x = np.array([-0.5, 0.0, 0.3, 1.0, 1.7])
    np.testing.assert_array_equal(ora.proj_box(x, 0.0, 1.0), [0.0, 0.0, 0.3, 1.0, 1.0])
