"""The FP64 oracle of the comparison regularizers (SSTV, HSSTV1, HSSTV2 of
Sec. IV-A, problem (15) with the GeoSSTV term replaced), pinned against
things it does not compute itself:

  * its stacked operator equals a sparse matrix assembled here from
    Kronecker products of 1-D forward differences (Neumann), so a wrong
    operand, sign or weight fails; and its adjoint is the transpose;
  * its step sizes satisfy the convergence condition of the preconditioned
    iteration: ||Sigma^1/2 K T^1/2||^2 <= 1 (power iteration);
  * a constant cube inside the box is a fixed point from the initial point;
  * after many iterations on tiny cubes its objective equals the optimum
    that SLSQP finds on the smooth epigraph form of the l1 problems (SSTV,
    HSSTV1), and the limit of every variant, primal and dual, meets the
    optimality conditions of its problem (HSSTV2's group norms are not
    smooth where groups vanish, which SLSQP does not resolve)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize

VARIANTS = [1, 2, 3]  # SSTV, HSSTV1, HSSTV2


def _diff(n):
    m = sp.lil_matrix((n, n))
    for i in range(n - 1):
        m[i, i], m[i, i + 1] = -1.0, 1.0
    return m.tocsr()


def _assembled_k(shape, variant, omega):
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    I1, I2, I3 = sp.identity(n1), sp.identity(n2), sp.identity(n3)
    Dv = sp.kron(sp.kron(I3, _diff(n1)), I2)   # element (k, i, j) at (k*n1 + i)*n2 + j
    Dh = sp.kron(sp.kron(I3, I1), _diff(n2))
    Ds = sp.kron(sp.kron(_diff(n3), I1), I2)
    blocks = [Dv @ Ds, Dh @ Ds]
    if variant != 1:
        blocks += [omega * Dv, omega * Dh]
    A = sp.vstack(blocks)
    Z = sp.csr_matrix((N, N))
    I = sp.identity(N)
    return sp.bmat([[A, sp.csr_matrix((A.shape[0], N)), sp.csr_matrix((A.shape[0], N))],
                    [Z, Z, Dv], [I, I, I]]).tocsr(), A, Dv


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(4, 5, 6), (1, 3, 7), (3, 1, 1), (2, 2, 2)])
def test_operator_is_the_assembled_matrix(ora, variant, shape):
    omega = 0.07
    K, _, _ = _assembled_k(shape, variant, omega)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(K.shape[1])
    y = rng.standard_normal(K.shape[0])
    np.testing.assert_allclose(ora.var_apply_k(variant, omega, x, shape), K @ x, atol=1e-12)
    np.testing.assert_allclose(ora.var_apply_k(variant, omega, y, shape, adjoint=True), K.T @ y,
                               atol=1e-12)


@pytest.mark.parametrize("variant", VARIANTS)
def test_step_sizes_meet_the_convergence_condition(ora, variant):
    """||Sigma^1/2 K T^1/2||^2 <= 1 with T = diag(g_u, g_s, g_t), Sigma = g_y I:
    power iteration on the oracle's own operator."""
    shape, omega = (6, 7, 5), 0.05
    gu, gs, gt, gy = ora.var_step_sizes(variant, omega)
    N = int(np.prod(shape))
    assert (gs, gt, gy) == (1.0, 0.2, pytest.approx(1 / 3))
    assert gu == pytest.approx(1 / (33 + (0 if variant == 1 else 8 * omega ** 2)))
    T = np.concatenate([np.full(N, gu), np.full(N, gs), np.full(N, gt)])
    x = np.random.default_rng(1).standard_normal(3 * N)
    lam = 0.0
    for _ in range(300):
        z = np.sqrt(gy) * ora.var_apply_k(variant, omega, np.sqrt(T) * x, shape)
        x = np.sqrt(T) * ora.var_apply_k(variant, omega, np.sqrt(gy) * z, shape, adjoint=True)
        lam = np.linalg.norm(x)
        x /= lam
    assert 0.3 < lam <= 1.0


@pytest.mark.parametrize("variant", VARIANTS)
def test_constant_cube_is_a_fixed_point(ora, variant):
    v = np.full((3, 4, 5), 0.37)
    S = ora.VariantSolver(v, eps=0.3, alpha=0.5, beta=0.5, variant=variant, omega=0.05)
    S.step(25)
    assert np.array_equal(S.u, v)
    for n in ("s", "t", "y1", "y3", "y4"):
        assert not np.any(S.state[n]), n


def _regularizer(A, u, variant, N):
    a = A @ u
    if variant in (1, 2):
        return np.abs(a).sum()
    return np.sqrt((a.reshape(4, N) ** 2).sum(axis=0)).sum()


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("with_sparse", [False, True])
def test_limit_is_the_optimum(ora, variant, with_sparse):
    """min R(u) s.t. ||u + s - v|| <= eps, ||s||_1 <= alpha, u in [0, 1]
    (beta = 0, so t = 0) on a 3 x 2 x 3 cube: the oracle after many
    iterations against SLSQP on the epigraph form (R's absolute values or
    group norms bounded by auxiliary variables; s split into its positive
    and negative parts)."""
    shape, omega = (3, 2, 3), 0.5
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    rng = np.random.default_rng(20 + variant)
    base = np.linspace(0.3, 0.7, n3)[:, None, None] + 0.1 * rng.standard_normal(shape)
    v = np.clip(base, 0.05, 0.95)
    if with_sparse:
        v.ravel()[[2, 11]] = [1.0, 0.0]
    alpha = 0.6 if with_sparse else 0.0
    eps = 0.25
    _, A, _ = _assembled_k(shape, variant, omega)
    A = A.toarray()
    S = ora.VariantSolver(v, eps=eps, alpha=alpha, beta=0.0, variant=variant, omega=omega)
    S.step(120000)
    u, s = S.u.ravel(), S.s.ravel()
    assert not S.t.any()
    assert np.linalg.norm(u + s - v.ravel()) <= eps * (1 + 1e-6)
    assert np.abs(s).sum() <= alpha * (1 + 1e-6) + 1e-12
    got = _regularizer(A, u, variant, N)

    P = A.shape[0]
    G = P if variant in (1, 2) else N  # epigraph variables: entries or groups
    vv = v.ravel()

    def split(z):
        return z[:N], z[N:2 * N], z[2 * N:3 * N], z[3 * N:]

    def obj(z):
        return np.sum(split(z)[3])

    def epi(z):
        uu, _, _, pp = split(z)
        a = A @ uu
        if variant in (1, 2):
            return np.concatenate([pp - a, pp + a])
        return pp - np.sqrt((a.reshape(4, N) ** 2).sum(axis=0) + 1e-30)

    cons = [{"type": "ineq", "fun": epi},
            {"type": "ineq", "fun": lambda z: eps ** 2 - np.sum((split(z)[0] + split(z)[1] - split(z)[2] - vv) ** 2)},
            {"type": "ineq", "fun": lambda z: alpha - np.sum(split(z)[1] + split(z)[2])}]
    a0 = A @ vv
    p0 = np.abs(a0) + 0.1 if variant in (1, 2) else np.sqrt((a0.reshape(4, N) ** 2).sum(axis=0)) + 0.1
    z0 = np.concatenate([vv, np.zeros(2 * N), p0])
    bounds = [(0, 1)] * N + [(0, None)] * (2 * N) + [(0, None)] * G
    r = minimize(obj, z0, constraints=cons, bounds=bounds, method="SLSQP",
                 options=dict(ftol=1e-13, maxiter=5000))
    assert r.success or r.status == 8
    assert got == pytest.approx(r.fun, rel=2e-5, abs=1e-7)


@pytest.mark.parametrize("variant", VARIANTS)
def test_limit_meets_the_optimality_conditions(ora, variant):
    """At the limit (u, s; y1, y4) of min R(u) s.t. ||u + s - v|| <= eps,
    ||s||_1 <= alpha, u in [0, 1]: y1 is a subgradient of R's norm at A u
    (entries in [-1, 1], equal to sign(A u) where A u != 0; for HSSTV2 groups
    in the unit ball, equal to the group's direction where it is nonzero);
    -(A^T y1 + y4) is in the box's normal cone at u; y4 = lambda (u + s - v)
    with lambda >= 0 (the fidelity ball, active); -y4 is in the l1 ball's
    normal cone at s. A and the differences are assembled here."""
    shape, omega = (3, 3, 4), 0.5
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    rng = np.random.default_rng(40 + variant)
    v = np.clip(np.linspace(0.3, 0.7, n3)[:, None, None] + 0.12 * rng.standard_normal(shape), 0.05, 0.95)
    v.ravel()[[3, 17]] = [1.0, 0.0]
    eps, alpha = 0.3, 0.5
    _, A, _ = _assembled_k(shape, variant, omega)
    A = A.toarray()
    S = ora.VariantSolver(v, eps=eps, alpha=alpha, beta=0.0, variant=variant, omega=omega)
    S.step(150000)
    u, s, y1, y4 = S.u.ravel(), S.s.ravel(), S.y1.ravel(), S.y4.ravel()
    tol = 1e-6
    a = A @ u
    if variant in (1, 2):
        assert np.abs(y1).max() <= 1 + tol
        nz = np.abs(a) > 1e-7
        np.testing.assert_allclose(y1[nz], np.sign(a[nz]), atol=1e-5)
    else:
        g, yg = a.reshape(4, N), y1.reshape(4, N)
        assert np.sqrt((yg ** 2).sum(axis=0)).max() <= 1 + tol
        nrm = np.sqrt((g ** 2).sum(axis=0))
        nz = nrm > 1e-7
        np.testing.assert_allclose(yg[:, nz], g[:, nz] / nrm[nz], atol=1e-5)
    grad = A.T @ y1 + y4
    inner = (u > 1e-9) & (u < 1 - 1e-9)
    assert np.abs(grad[inner]).max() < 1e-5
    assert (grad[u <= 1e-9] >= -1e-5).all() and (grad[u >= 1 - 1e-9] <= 1e-5).all()
    res = u + s - v.ravel()
    assert np.linalg.norm(res) == pytest.approx(eps, rel=1e-6)  # the ball is active
    lam = y4 @ res / (res @ res)
    assert lam > 0
    np.testing.assert_allclose(y4, lam * res, atol=1e-5)
    # -y4 in the normal cone of {||s||_1 <= alpha} at s
    g = -y4
    if np.abs(s).sum() < alpha * (1 - 1e-6):
        assert np.abs(g).max() < 1e-5
    else:
        mu = np.abs(g).max()
        snz = np.abs(s) > 1e-9
        np.testing.assert_allclose(g[snz], mu * np.sign(s[snz]), atol=1e-5)
