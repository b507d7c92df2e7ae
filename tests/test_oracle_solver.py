"""Pins of the oracle's Alg. 1 against properties the problem fixes:
fixed points, symmetries, the monotone primal-dual residual of the
preconditioned iteration, and the optimum of problem (15) computed by an
unrelated general-purpose solver (SLSQP) on tiny cubes."""
import numpy as np
import pytest
from scipy.optimize import minimize

from synth.cubes import SMALL_64x64x16, like, make_cube


def small_problem(seed=0, shape=(3, 6, 5)):
    n3, n1, n2 = shape
    c = make_cube(like(SMALL_64x64x16, n1=n1, n2=n2, n3=n3, seed=seed, cells=3))
    return c


def run(ora, c, iters, v=None, **kw):
    p = dict(eps=c["eps"], alpha=c["alpha"], beta=c["beta"], mu_lo=c["mu_lo"],
             mu_hi=c["mu_hi"], omega=c["omega"])
    p.update(kw)
    S = ora.Solver(c["v"] if v is None else v, **p)
    S.step(iters)
    return S


def test_constant_cube_is_a_fixed_point(ora):
    """A constant cube inside the box has zero GeoSSTV and lies in every
    constraint set: starting from u = v, every iterate keeps u = v and all
    other variables at zero (up to rounding in the y4 step)."""
    v = np.full((4, 5, 6), 0.37)
    S = ora.Solver(v, eps=0.5, alpha=1.0, beta=1.0, omega=0.03)
    S.step(40)
    np.testing.assert_allclose(S.u, v, rtol=0, atol=1e-15)
    for name in ("s", "t", "w1", "w2", "y1", "y2", "y3"):
        assert not np.asarray(S.state[name]).any(), name
    assert np.abs(S.y4).max() < 1e-15


def test_translation_covariance(ora):
    """Shifting v and the box by a constant shifts u by it and leaves s, t
    and every auxiliary and dual variable unchanged (differences annihilate
    constants, the fidelity ball moves with v)."""
    c = small_problem(1)
    a = run(ora, c, 30)
    b = run(ora, c, 30, v=c["v"] + 0.25, mu_lo=0.25, mu_hi=1.25)
    np.testing.assert_allclose(b.u, a.u + 0.25, atol=1e-12)
    for name in ("s", "t", "w1", "w2", "y1", "y2", "y3", "y4"):
        np.testing.assert_allclose(b.state[name], a.state[name], atol=1e-11)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_equivariance(ora, axis):
    """Mirroring v along any axis mirrors u, s and t: reading R1 of the
    interpolation operators maps every grid onto itself under a flip."""
    c = small_problem(2)
    a = run(ora, c, 25)
    b = run(ora, c, 25, v=np.flip(c["v"], axis).copy())
    for name in ("u", "s", "t"):
        np.testing.assert_allclose(b.state[name], np.flip(a.state[name], axis), atol=1e-12)


def _primal(S):
    return np.concatenate([np.ravel(S.state[n]) for n in ("u", "s", "t", "w1", "w2")])


def _dual(S):
    return np.concatenate([np.ravel(S.state[n]) for n in ("y1", "y2", "y3", "y4")])


def test_primal_dual_residual_is_monotone(ora):
    """Alg. 1 is a proximal-point iteration in the metric
    M = [[T^-1, -K^T], [-K, Sigma^-1]] (T, Sigma the step sizes, K the stacked
    operator of problem (20)), so ||z_{k+1} - z_k||_M never increases."""
    c = small_problem(3)
    S = ora.Solver(c["v"], c["eps"], c["alpha"], c["beta"], omega=c["omega"])
    shape = S.shape
    N = int(np.prod(shape))
    tinv = np.concatenate([np.full(N, 13.0), np.full(N, 1.0), np.full(N, 3.0),
                           np.full(12 * N, 4.0)])
    x0, y0 = _primal(S), _dual(S)
    res = []
    for _ in range(150):
        S.step(1)
        x1, y1 = _primal(S), _dual(S)
        dx, dy = x1 - x0, y1 - y0
        kdx = ora.apply("k", dx, shape)
        res.append(dx @ (tinv * dx) + 5.0 * (dy @ dy) - 2.0 * (kdx @ dy))
        x0, y0 = x1, y1
    res = np.array(res)
    assert (res >= -1e-12 * res[0]).all()
    assert (np.diff(res) <= 1e-10 * res[:-1] + 1e-300).all()
    assert res[-1] < 0.5 * res[0]


def test_one_dimensional_reduction(ora):
    """With N2 = N3 = 1 and zero l1 radii the problem becomes
    min omega * TV1D(u) s.t. ||u - v|| <= eps, u in [0, 1] (Condat's TV of a
    1-D signal is the anisotropic TV). Its minimiser is unique when the ball
    is active; compare with SLSQP on the smooth epigraph form, and check that
    the optimal omega ||w1||_{1,2} equals omega * sum |u_{i+1} - u_i|."""
    rng = np.random.default_rng(7)
    n = 7
    v = np.clip(np.linspace(0.2, 0.8, n) + rng.normal(0, 0.15, n), 0, 1)
    eps = 0.45 * np.linalg.norm(v - v.mean())
    S = ora.Solver(v.reshape(1, n, 1), eps=eps, alpha=0.0, beta=0.0, omega=0.5)
    S.step(60000)
    u = S.u.ravel()

    def obj(z):
        return np.sum(z[n:])
    cons = [{"type": "ineq", "fun": lambda z: z[n:] - np.diff(z[:n])},
            {"type": "ineq", "fun": lambda z: z[n:] + np.diff(z[:n])},
            {"type": "ineq", "fun": lambda z: eps ** 2 - np.sum((z[:n] - v) ** 2)}]
    z0 = np.concatenate([v, np.abs(np.diff(v)) + 0.1])
    r = minimize(obj, z0, constraints=cons, bounds=[(0, 1)] * n + [(0, None)] * (n - 1),
                 method="SLSQP", options=dict(ftol=1e-12, maxiter=2000))
    assert r.success or r.status == 8  # 8: converged to the line-search limit
    assert np.sum((r.x[:n] - v) ** 2) <= eps ** 2 * (1 + 1e-9)
    np.testing.assert_allclose(u, r.x[:n], atol=2e-6)
    w = S.w1
    tvc = np.sum(np.sqrt(w[0::2] ** 2 + w[1::2] ** 2))
    assert tvc == pytest.approx(np.sum(np.abs(np.diff(u))), rel=1e-6)
    assert not S.s.any() and not S.t.any()


def _assembled(ora, shape):
    N = int(np.prod(shape))

    def mat(op, pin):
        cols = []
        for q in range(pin * N):
            e = np.zeros(pin * N)
            e[q] = 1
            cols.append(ora.apply(op, e.reshape((pin,) + shape) if pin > 1 else e.reshape(shape),
                                  shape).ravel())
        return np.stack(cols, 1)
    return mat("d", 1), mat("dds", 1), mat("dv", 1), mat("l", 2)


def _check_l1_normal(g, x, radius, tol):
    """g in the normal cone of {||x||_1 <= radius} at x."""
    if np.abs(x).sum() < radius * (1 - 1e-6):
        assert np.abs(g).max() < tol
        return
    lam = np.abs(g).max()
    nz = np.abs(x) > 1e-9
    np.testing.assert_allclose(g[nz], lam * np.sign(x[nz]), atol=tol)
    assert (np.abs(g[~nz]) <= lam + tol).all()


def _check_group_subgradient(g, w, thr, N, tol):
    """g in thr * subdifferential of ||.||_{1,2} at w (groups of 2)."""
    g, w = g.reshape(6, N), w.reshape(6, N)
    for a in range(3):
        ga, gb, wa, wb = g[2 * a], g[2 * a + 1], w[2 * a], w[2 * a + 1]
        nw = np.sqrt(wa ** 2 + wb ** 2)
        on = nw > 1e-7
        np.testing.assert_allclose(ga[on], thr * wa[on] / nw[on], atol=tol)
        np.testing.assert_allclose(gb[on], thr * wb[on] / nw[on], atol=tol)
        assert (np.sqrt(ga[~on] ** 2 + gb[~on] ** 2) <= thr + tol).all()


@pytest.mark.parametrize("seed", [11, 12])
def test_limit_satisfies_optimality_conditions(ora, seed):
    """Problem (15) is convex, so a feasible point with multipliers that
    satisfy the subgradient conditions is a global minimiser. On a small
    cube the limit of Alg. 1 must be such a point, with the duals as
    multipliers: feasibility of every constraint; L y1 in omega d||w1||_{1,2};
    L y2 in d||w2||_{1,2}; -(D^T y1 + D_s^T D^T y2 + y4) in the normal cone of
    the box at u; -y4 and -(D_v^T y3 + y4) in the normal cones of the l1
    balls at s and t; y4 in the normal cone of the fidelity ball at u+s+t.
    These conditions come from the problem statement alone, so a wrong sign
    or operand anywhere in the iteration leaves them unmet."""
    shape = (2, 4, 3)  # (N3, N1, N2)
    N = int(np.prod(shape))
    c = make_cube(like(SMALL_64x64x16, n1=4, n2=3, n3=2, seed=seed, cells=2, p_s=0.15, p_t=0.34))
    eps, alpha, beta, omega = 0.8 * c["eps"], 0.7 * c["alpha"], 0.7 * c["beta"], 0.3
    S = ora.Solver(c["v"], eps=eps, alpha=alpha, beta=beta, omega=omega)
    S.step(400000, tol=1e-15)
    D, DDs, Dv, L = _assembled(ora, shape)
    u, s, t = S.u.ravel(), S.s.ravel(), S.t.ravel()
    w1, w2 = S.w1.ravel(), S.w2.ravel()
    y1, y2, y3, y4 = S.y1.ravel(), S.y2.ravel(), S.y3.ravel(), S.y4.ravel()
    v = c["v"].ravel()
    tol = 1e-6
    # feasibility
    assert np.linalg.norm(D @ u - L.T @ w1) < tol
    assert np.linalg.norm(DDs @ u - L.T @ w2) < tol
    assert np.linalg.norm(Dv @ t) < tol
    r = u + s + t - v
    assert np.linalg.norm(r) <= eps + tol
    assert np.abs(s).sum() <= alpha + tol and np.abs(t).sum() <= beta + tol
    assert (u >= -tol).all() and (u <= 1 + tol).all()
    # the constraints of interest are active (otherwise the test is weak)
    assert np.linalg.norm(r) > eps - tol
    assert np.abs(s).sum() > alpha - tol and np.abs(t).sum() > beta - tol
    # stationarity
    _check_group_subgradient(L @ y1, w1, omega, N, tol)
    _check_group_subgradient(L @ y2, w2, 1.0, N, tol)
    gu = -(D.T @ y1 + DDs.T @ y2 + y4)
    inner = (u > 1e-7) & (u < 1 - 1e-7)
    assert np.abs(gu[inner]).max() < tol
    assert (gu[u <= 1e-7] <= tol).all() and (gu[u >= 1 - 1e-7] >= -tol).all()
    _check_l1_normal(-y4, s, alpha, tol)
    _check_l1_normal(-(Dv.T @ y3 + y4), t, beta, tol)
    # y4 = mu (u + s + t - v), mu >= 0
    mu = (y4 @ r) / (r @ r)
    assert mu > 0
    np.testing.assert_allclose(y4, mu * r, atol=tol)


def test_stopping_rule_skips_the_first_iteration(ora):
    """Reading of eq. (28) with the initial point u = v and zero duals: the
    first iteration only projects u onto the box, so for a cube inside the box
    ||u1 - u0|| = 0; the rule starts with the second iteration (the loop
    would otherwise return v unchanged)."""
    rng = np.random.default_rng(5)
    v = rng.uniform(0.2, 0.8, size=(3, 6, 7))
    S = ora.Solver(v, 0.5, 1.0, 1.0, omega=0.03)
    assert S.step(50, tol=0.5) == 2
    assert S.trace[0][0] == 0.0 and S.trace[1][0] > 0.0
    # split calls count iterations since the initial point
    S2 = ora.Solver(v, 0.5, 1.0, 1.0, omega=0.03)
    assert S2.step(1, tol=0.5) == 1
    assert S2.step(50, tol=0.5) == 1
