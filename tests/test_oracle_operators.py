"""Pins of the oracle's linear operators (Sec. II-A, II-D, III-A) and of the
printed step sizes (Sec. III-B), against mathematics rather than against the
oracle itself: adjoint identities, matrices assembled column by column and
checked for their closed-form absolute sums, mirror symmetry, and the
convergence condition of the preconditioned iteration."""
import os

import numpy as np
import pytest

SHAPES = [(4, 5, 6), (3, 7, 5), (1, 4, 1), (1, 1, 6), (2, 1, 1), (1, 1, 1), (5, 6, 7)]
PLANES_IN = dict(dv=1, dh=1, ds=1, d=1, dds=1, l_ud=2, l_lr=2, l_c=2, l=2)
PLANES_OUT = dict(dv=1, dh=1, ds=1, d=2, dds=2, l_ud=2, l_lr=2, l_c=2, l=6)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("op", list(PLANES_IN) + ["k"])
def test_adjoint_identity(ora, op, shape):
    rng = np.random.default_rng(hash((op, shape)) % 2**32)
    n = int(np.prod(shape))
    pin, pout = (15, 6) if op == "k" else (PLANES_IN[op], PLANES_OUT[op])
    x = rng.normal(size=pin * n)
    y = rng.normal(size=pout * n)
    ax = ora.apply(op, x.reshape((pin,) + shape) if pin > 1 else x.reshape(shape), shape).ravel()
    aty = ora.apply(op, y.reshape((pout,) + shape) if pout > 1 else y.reshape(shape), shape,
                    adjoint=True).ravel()
    lhs, rhs = float(ax @ y), float(x @ aty)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs), np.linalg.norm(ax) * np.linalg.norm(y))


def assemble(ora, op, shape, adjoint=False):
    """Dense matrix of an operator, one column per unit input vector."""
    n = int(np.prod(shape))
    pin, pout = (15, 6) if op == "k" else (PLANES_IN[op], PLANES_OUT[op])
    if adjoint:
        pin, pout = pout, pin
    cols = []
    for q in range(pin * n):
        e = np.zeros(pin * n)
        e[q] = 1.0
        xin = e if op == "k" else (e.reshape((pin,) + shape) if pin > 1 else e.reshape(shape))
        cols.append(ora.apply(op, xin, shape, adjoint=adjoint).ravel())
    return np.stack(cols, axis=1)


def test_difference_matrices_closed_form(ora):
    """Forward differences with the Neumann boundary of Sec. II-A: each row is
    e_{next} - e_{self}, and the last index of the axis gives a zero row."""
    shape = (3, 4, 5)  # (N3, N1, N2)
    n3, n1, n2 = shape
    idx = np.arange(n3 * n1 * n2).reshape(shape)
    for op, axis, nmax in (("dv", 1, n1), ("dh", 2, n2), ("ds", 0, n3)):
        A = assemble(ora, op, shape)
        for k in range(n3):
            for i in range(n1):
                for j in range(n2):
                    r = idx[k, i, j]
                    pos = [k, i, j]
                    want = np.zeros(A.shape[1])
                    if pos[axis] <= nmax - 2:
                        nxt = list(pos)
                        nxt[axis] += 1
                        want[idx[tuple(nxt)]] = 1.0
                        want[r] = -1.0
                    np.testing.assert_array_equal(A[r], want)


def test_interpolation_rows_are_averages(ora):
    """Each row of L_ud, L_lr, L_c is a 1-, 2- or 4-point average (points that
    fall off the interior edges read as zero): nonnegative, equal weights of
    1, 1/2 or 1/4 in a row, at most four nonzeros, row sums at most 1 and
    exactly 1 away from the border; every column also sums to at most 1."""
    shape = (2, 5, 6)
    for op in ("l_ud", "l_lr", "l_c"):
        A = assemble(ora, op, shape)
        assert (A >= 0).all()
        nnz = (A != 0).sum(axis=1)
        assert nnz.max() <= 4
        for r in np.nonzero(nnz)[0]:
            vals = A[r][A[r] != 0]
            assert len(set(vals.tolist())) == 1 and vals[0] in (1.0, 0.5, 0.25)
            assert len(vals) * vals[0] <= 1.0
        assert A.sum(axis=1).max() == 1.0
        assert A.sum(axis=0).max() <= 1.0 + 1e-15
    L = assemble(ora, "l", shape)
    assert (L != 0).sum(axis=1).max() == 4
    assert np.abs(L).sum(axis=1).max() == pytest.approx(1.0)
    # interior rows of the six planes have 1, 4, 4, 1, 2, 2 nonzeros
    n3, n1, n2 = shape
    N = n1 * n2 * n3
    r0 = (0 * n1 + 2) * n2 + 2
    assert [int((L[p * N + r0] != 0).sum()) for p in range(6)] == [1, 4, 4, 1, 2, 2]


def test_interpolation_norm_bound(ora):
    """||L||^2 <= 3 (three averaging operators, each of norm <= 1), and the
    bound is nearly met on a large enough grid."""
    L = assemble(ora, "l", (1, 8, 8))
    s = np.linalg.norm(L, 2) ** 2
    assert 2.5 < s <= 3.0 + 1e-12


def test_masked_entries(ora):
    """Dual edge fields live on interior edges: L ignores the last row of the
    vertical field and the last column of the horizontal field, and L^T never
    writes there (reading R1 of Condat's operators)."""
    shape = (2, 4, 5)
    n3, n1, n2 = shape
    rng = np.random.default_rng(3)
    y = rng.normal(size=(2,) + shape)
    y2 = y.copy()
    y2[0][:, n1 - 1, :] = rng.normal(size=(n3, n2))
    y2[1][:, :, n2 - 1] = rng.normal(size=(n3, n1))
    np.testing.assert_array_equal(ora.apply("l", y, shape), ora.apply("l", y2, shape))
    w = rng.normal(size=(6,) + shape)
    p = ora.apply("l", w, shape, adjoint=True)
    assert not p[0][:, n1 - 1, :].any() and not p[1][:, :, n2 - 1].any()
    d = ora.apply("d", rng.normal(size=shape), shape)
    assert not d[0][:, n1 - 1, :].any() and not d[1][:, :, n2 - 1].any()
    dds = ora.apply("dds", rng.normal(size=shape), shape)
    assert not dds[:, n3 - 1].any()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_of_gram_operators(ora, axis):
    """Mirroring the cube maps every grid of reading R1 onto itself, so the
    self-adjoint compositions L^T L, D^T D and (D D_s)^T (D D_s) commute with
    a flip of any axis."""
    shape = (4, 5, 6)
    rng = np.random.default_rng(axis)
    x = rng.normal(size=shape)
    for op in ("d", "dds"):
        g = ora.apply(op, ora.apply(op, x, shape), shape, adjoint=True)
        gf = ora.apply(op, ora.apply(op, np.flip(x, axis).copy(), shape), shape, adjoint=True)
        np.testing.assert_allclose(np.flip(g, axis), gf, atol=1e-13)
    # L^T L on a dual edge field: flipping along i (axis 1) maps the vertical
    # edge at row i to the one at row N1-2-i, so the vertical plane is flipped
    # within rows 0..N1-2 only (likewise the horizontal plane along j).
    if axis == 0:
        y = rng.normal(size=(2,) + shape)
        g = ora.apply("l", ora.apply("l", y, shape), shape, adjoint=True)
        gf = ora.apply("l", ora.apply("l", np.flip(y, 1).copy(), shape), shape, adjoint=True)
        np.testing.assert_allclose(np.flip(g, 1), gf, atol=1e-13)
    else:
        n3, n1, n2 = shape
        y = rng.normal(size=(2,) + shape)
        y[0][:, n1 - 1, :] = 0
        y[1][:, :, n2 - 1] = 0

        def flip_edges(a):
            a = a.copy()
            if axis == 1:
                a[0][:, :n1 - 1, :] = a[0][:, n1 - 2::-1, :]
                a[1] = a[1][:, ::-1, :]
            else:
                a[0] = a[0][:, :, ::-1]
                a[1][:, :, :n2 - 1] = a[1][:, :, n2 - 2::-1]
            return a
        g = ora.apply("l", ora.apply("l", y, shape), shape, adjoint=True)
        gf = ora.apply("l", ora.apply("l", flip_edges(y), shape), shape, adjoint=True)
        np.testing.assert_allclose(flip_edges(g), gf, atol=1e-13)


def _golden_steps():
    path = os.path.join(os.path.dirname(__file__), "golden", "step_sizes.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, a, b = line.split()
            out[name] = int(a) / int(b)
    return out


def test_printed_step_sizes(ora):
    g = _golden_steps()
    assert ora.STEP_U == g["u"] and ora.STEP_S == g["s"] and ora.STEP_T == g["t"]
    assert ora.STEP_W1 == g["w1"] and ora.STEP_W2 == g["w2"]
    assert all(g[f"y{q}"] == ora.STEP_Y for q in (1, 2, 3, 4))
    assert ora.step_sizes() == (g["u"], g["w1"], g["w2"], g["s"], g["t"], g["y1"])


def test_step_sizes_are_column_sums(ora):
    """The printed primal steps of u, s and t are the reciprocals of the
    largest absolute column sums of the corresponding blocks of the stacked
    operator K of problem (20) (13 = 4 + 8 + 1 for u, 3 = 2 + 1 for t, 1 for
    s); the dual step 1/5 is 1/(number of primal blocks), as in eq. (8)."""
    shape = (4, 5, 6)
    K = assemble(ora, "k", shape)
    N = int(np.prod(shape))
    col = np.abs(K).sum(axis=0)
    g = _golden_steps()
    assert col[:N].max() == pytest.approx(1 / g["u"])
    assert col[N:2 * N].max() == pytest.approx(1 / g["s"])
    assert col[2 * N:3 * N].max() == pytest.approx(1 / g["t"])
    assert 5 == len(("u", "s", "t", "w1", "w2")) == round(1 / g["y1"])


def test_convergence_condition(ora):
    """With T = diag of the primal steps and Sigma = (1/5) I, the
    preconditioned operator satisfies ||Sigma^1/2 K T^1/2||^2 < 1, the
    condition under which the iteration of eq. (7) converges."""
    shape = (3, 5, 6)
    N = int(np.prod(shape))
    K = assemble(ora, "k", shape)
    tdiag = np.concatenate([np.full(N, ora.STEP_U), np.full(N, ora.STEP_S),
                            np.full(N, ora.STEP_T), np.full(6 * N, ora.STEP_W1),
                            np.full(6 * N, ora.STEP_W2)])
    M = np.sqrt(ora.STEP_Y) * K * np.sqrt(tdiag)[None, :]
    s2 = np.linalg.norm(M, 2) ** 2
    assert s2 < 1.0
    assert s2 > 0.3  # not vacuous
