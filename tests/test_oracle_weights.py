"""Oracle RBF-FD weights (Sec. 2.1) pinned by exactness and invariances."""
import numpy as np
import pytest

import nodecloud as nc
import oracle as O

MONO = [lambda x, y, z: np.ones_like(x), lambda x, y, z: x, lambda x, y, z: y, lambda x, y, z: z,
        lambda x, y, z: x * x, lambda x, y, z: x * y, lambda x, y, z: x * z, lambda x, y, z: y * y,
        lambda x, y, z: y * z, lambda x, y, z: z * z]


def target(op, vec):
    """(L p_l)(0) for the ten monomials, written from calculus."""
    if op == "dx":
        return np.array([0, 1, 0, 0, 0, 0, 0, 0, 0, 0.0])
    if op == "dy":
        return np.array([0, 0, 1, 0, 0, 0, 0, 0, 0, 0.0])
    if op == "dz":
        return np.array([0, 0, 0, 1, 0, 0, 0, 0, 0, 0.0])
    if op == "lap":
        return np.array([0, 0, 0, 0, 2, 0, 0, 2, 0, 2.0])
    if op in ("dir", "dn"):
        return np.array([0, vec[0], vec[1], vec[2], 0, 0, 0, 0, 0, 0.0])
    if op in ("shift", "shift_row"):
        s = np.asarray(vec, dtype=float)
        return np.array([f(s[0], s[1], s[2]) for f in MONO])
    if op == "taylor":  # p(0) + vec . grad p(0): the constant and the linear monomials only
        return np.array([1, vec[0], vec[1], vec[2], 0, 0, 0, 0, 0, 0.0])
    raise ValueError(op)


def check_exact(pos, S, w, ops, rowvec=None, tol=1e-11):
    worst = 0.0
    for i in range(S.shape[0]):
        X = nc.min_image(pos[S[i]] - pos[S[i, 0]])
        P = np.stack([f(X[:, 0], X[:, 1], X[:, 2]) for f in MONO])  # [10][nl]
        for o, op in enumerate(ops):
            vec = rowvec[i] if op[0] in ("dn", "shift_row") else (op[1] if len(op) > 1 else None)
            got = P @ w[i, o]
            scale = np.abs(P * w[i, o]).sum(1) + np.abs(target(op[0], vec))
            err = np.abs(got - target(op[0], vec)) / np.maximum(scale, 1e-300)
            worst = max(worst, err.max())
    assert worst < tol, worst


def test_monomial_exactness_all_operators(small_cloud, small_stencils):
    c, S = small_cloud, small_stencils
    rows = np.r_[np.arange(0, c.n_int, 37), np.arange(c.n_int, c.n, 11)]
    Sr = S[rows]
    rng = np.random.default_rng(0)
    rowvec = rng.normal(size=(len(rows), 3)) * 0.01
    e = np.array([0.3, -0.5, 0.8])
    ops = [("dx",), ("dy",), ("dz",), ("lap",), ("dir", e), ("shift", (0.004, -0.003, 0.0)), ("dn",),
           ("taylor", (0.004, -0.003, 0.002))]
    w, info = O.weights(c.pos, Sr, ops, rowvec=rowvec)
    assert not info.any()
    check_exact(c.pos, Sr, w, ops, rowvec=rowvec)
    w2, info = O.weights(c.pos, Sr, [("shift_row",)], rowvec=rowvec)
    check_exact(c.pos, Sr, w2, [("shift_row",)], rowvec=rowvec)


def test_shift_to_nodes_is_kronecker(small_cloud, small_stencils):
    c, S = small_cloud, small_stencils
    rows = np.arange(0, c.n, 101)
    Sr = S[rows]
    for j in (0, 1, 7, 29):
        s = nc.min_image(c.pos[Sr[:, j]] - c.pos[Sr[:, 0]])
        w, info = O.weights(c.pos, Sr, [("shift_row",)], rowvec=s)
        expect = np.zeros(30)
        expect[j] = 1.0
        assert np.abs(w[:, 0, :] - expect).max() < 1e-9


def test_taylor_is_identity_plus_directional_derivative(small_cloud, small_stencils):
    """The first-order Taylor row is linear in its functional: the weights of
    value-at-x_i (the unit vector e_1) plus those of s . grad."""
    c, S = small_cloud, small_stencils
    Sr = S[::53]
    s = (-0.003, 0.002, 0.004)
    w, info = O.weights(c.pos, Sr, [("taylor", s), ("dir", s)])
    assert not info.any()
    expect = w[:, 1, :].copy()
    expect[:, 0] += 1.0
    assert np.abs(w[:, 0, :] - expect).max() < 1e-10 * np.abs(expect).max()


def local_cluster(seed=0, n=60, spread=0.05):
    rng = np.random.default_rng(seed)
    pts = 0.5 + rng.uniform(-spread, spread, size=(n, 3))
    pts[0] = 0.5
    S = nc.stencils(pts, 30)[:1]
    return pts, S


def test_rotation_and_scale_invariance():
    pts, S = local_cluster()
    ops = [("dx",), ("dy",), ("dz",), ("lap",), ("shift", (0.01, 0.0, -0.005))]
    w, _ = O.weights(pts, S, ops)
    # rotation about the centre
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    rp = 0.5 + (pts - 0.5) @ Q.T
    s_rot = Q @ np.array([0.01, 0.0, -0.005])
    wr, _ = O.weights(rp, S, [("dx",), ("dy",), ("dz",), ("lap",), ("shift", tuple(s_rot))])
    grad = w[0, :3]            # [3][nl]: d/dx_a weights
    grad_r = wr[0, :3]
    assert np.abs(grad_r - Q @ grad).max() < 1e-9 * np.abs(grad).max()
    assert np.abs(wr[0, 3] - w[0, 3]).max() < 1e-9 * np.abs(w[0, 3]).max()
    assert np.abs(wr[0, 4] - w[0, 4]).max() < 1e-9
    # scaling about the centre: d/dx ~ 1/lam, lap ~ 1/lam^2, shift invariant
    lam = 0.5
    sp = 0.5 + lam * (pts - 0.5)
    ws, _ = O.weights(sp, S, [("dx",), ("dy",), ("dz",), ("lap",), ("shift", (0.005, 0.0, -0.0025))])
    assert np.abs(ws[0, :3] * lam - w[0, :3]).max() < 1e-9 * np.abs(w[0, :3]).max()
    assert np.abs(ws[0, 3] * lam * lam - w[0, 3]).max() < 1e-9 * np.abs(w[0, 3]).max()
    assert np.abs(ws[0, 4] - w[0, 4]).max() < 1e-9


def test_translation_invariance(small_cloud, small_stencils):
    c, S = small_cloud, small_stencils
    rows = np.arange(0, c.n, 97)
    w, _ = O.weights(c.pos, S[rows], [("dx",), ("lap",)])
    wt, _ = O.weights((c.pos + np.array([0.123, 0.456, 0.789])) % 1.0, S[rows], [("dx",), ("lap",)])
    assert np.abs(w - wt).max() < 1e-8 * np.abs(w).max()


def test_cartesian_stencil_symmetry():
    h = 0.01
    g = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], dtype=float)
    order = np.argsort((g * g).sum(1), kind="stable")
    g = g[order]
    pts = 0.5 + h * g
    S = np.arange(27, dtype=np.int32)[None, :]
    w, info = O.weights(pts, S, [("dx",), ("lap",)], )
    assert not info.any()
    mirror = np.array([np.flatnonzero((g == [-a, b, c]).all(1))[0] for a, b, c in g])
    assert np.abs(w[0, 0] + w[0, 0][mirror]).max() < 1e-9 * np.abs(w[0, 0]).max()
    assert np.abs(w[0, 1] - w[0, 1][mirror]).max() < 1e-9 * np.abs(w[0, 1]).max()


def test_singular_system_flagged():
    pts, S = local_cluster()
    pts = pts.copy()
    pts[S[0, 5]] = pts[S[0, 6]]  # two coincident stencil nodes: identical rows
    w, info = O.weights(pts, S, [("dx",)])
    assert info[0] > 0


def null_space_weights(X, op):
    """Weights of one row by a second algorithm: the null-space method for the
    saddle system [A P; P^T 0][w; lam] = [b; c] (Sec. 2.1, PHS r^3 plus the ten
    monomials), in the row's own minimum-image coordinates X [nl][3] (the
    weights do not depend on a scaling).  P = Q R; w = Q1 R^-T c + Q2 z with
    (Q2^T A Q2) z = Q2^T (b - A Q1 R^-T c); no factorisation of the full saddle
    matrix is involved.  b_j is L applied to |x - x_j|^3 at x = 0, written from
    calculus: d/dx gives -3 |x_j| x_j,x; the Laplacian gives 12 |x_j|."""
    r = np.sqrt((X * X).sum(1))
    A = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(2)) ** 3
    P = np.stack([f(X[:, 0], X[:, 1], X[:, 2]) for f in MONO], 1)  # [nl][10]
    b = -3.0 * r * X[:, 0] if op == "dx" else 12.0 * r
    c = target(op, None)
    Q, R = np.linalg.qr(P, mode="complete")
    m = P.shape[1]
    Q1, Q2, R1 = Q[:, :m], Q[:, m:], R[:m, :]
    w0 = Q1 @ np.linalg.solve(R1.T, c)
    z = np.linalg.solve(Q2.T @ A @ Q2, Q2.T @ (b - A @ w0))
    return w0 + Q2 @ z


def test_null_space_method_agrees(small_cloud, small_stencils):
    """The oracle's weights (LU with partial pivoting of the full saddle
    matrix) against the null-space method on every 40th row, for the x
    derivative and the Laplacian: they agree to the systems' conditioning."""
    pos, S = small_cloud.pos, small_stencils
    rows = np.arange(0, S.shape[0], 40)
    ops = [("dx",), ("lap",)]
    w, info = O.weights(pos, S[rows], ops)
    assert not info.any()
    worst = 0.0
    for k, i in enumerate(rows):
        X = nc.min_image(pos[S[i]] - pos[S[i, 0]])
        for o, (op,) in enumerate(ops):
            ref = null_space_weights(X, op)
            worst = max(worst, np.abs(w[k, o] - ref).max() / np.abs(ref).max())
    assert worst < 1e-11, worst  # measured 1e-13
