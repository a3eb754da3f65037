"""Pins of the FP64 PCA and soft-label oracles.

PCA: paper Section 2 (PCA paragraph: centre, covariance, eigenvectors,
orthonormal).  Soft-label CVA is not in the paper; its definition reduces to
the paper's CVA (Section 2, canonical variates paragraph) for one-hot
weights, which is one of the pins below.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.cva import _rows


# ------------------------------------------------------------------- PCA

def test_pca_trace_orthonormal_and_numpy_cov():
    from synth import make_case
    c = make_case(2, scale=0.08)
    fit = oracle.pca_fit(c.cube, n_comp=c.B)
    V = fit["V"]
    assert np.max(np.abs(V.T @ V - np.eye(c.B))) <= 1e-12
    assert abs(np.trace(fit["cov"]) - fit["all_eigvals"].sum()) <= 1e-12 * np.trace(fit["cov"])
    X = _rows(c.cube).astype(np.float64)
    ref = np.cov(X, rowvar=False)
    assert np.max(np.abs(fit["cov"] - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert (np.diff(fit["eigvals"]) <= 0).all()


def test_pca_brute_force_loop_and_mask():
    rng = np.random.default_rng(21)
    cube = rng.integers(0, 4096, size=(5, 4, 3)).astype(np.uint16)
    mask = rng.integers(0, 2, size=(5, 4)).astype(np.uint8)
    mask[0, 0] = mask[0, 1] = 1
    rows = [[int(v) for v in cube[i, j]] for i in range(5) for j in range(4) if mask[i, j]]
    P = len(rows)
    mu = [Fraction(sum(r[b] for r in rows), P) for b in range(3)]
    cov = [[sum((r[a] - mu[a]) * (r[b] - mu[b]) for r in rows) / (P - 1) for b in range(3)]
           for a in range(3)]
    _, cv, _ = oracle.pca.pca_moments(cube, mask)
    ref = np.array([[float(v) for v in r] for r in cov])
    assert np.max(np.abs(cv - ref)) <= 1e-14 * np.max(np.abs(ref))


def _scores(fit, X):
    return (X - fit["mean"]) @ fit["V"]


def test_pca_standardized_scale_invariance_and_definition():
    """Standardised PCA: the eigenvalues are those of the correlation matrix
    (summing to B, each band contributing 1); multiplying bands by positive
    constants leaves the scores unchanged (the vectors scale inversely);
    and the scores equal the covariance-PCA scores of data standardised
    beforehand (the plain definition), up to the arbitrary sign."""
    rng = np.random.default_rng(23)
    P, B = 2000, 6
    X = rng.standard_normal((P, B)) @ rng.standard_normal((B, B)) * [1, 10, 100, 0.5, 3, 40] + 500
    f = oracle.pca_fit(X[:, None, :], n_comp=3, standardize=True)
    assert abs(f["all_eigvals"].sum() - B) <= 1e-12 * B
    M = f["metric"]
    assert np.max(np.abs(f["V"].T @ M @ f["V"] - np.eye(3))) <= 1e-12
    assert np.max(np.abs(f["V"].T @ f["cov"] @ f["V"] - np.diag(f["eigvals"]))) <= 1e-12 * f["eigvals"][0]
    a = np.array([3.0, 0.01, 7.0, 250.0, 1.0, 0.2])
    g = oracle.pca_fit((X * a)[:, None, :], n_comp=3, standardize=True)
    assert np.max(np.abs(g["eigvals"] - f["eigvals"])) <= 1e-10 * B
    sf, sg = _scores(f, X), _scores(g, X * a)
    for j in range(3):
        s = np.sign(sf[:, j] @ sg[:, j])
        assert np.max(np.abs(s * sg[:, j] - sf[:, j])) <= 1e-9 * np.max(np.abs(sf[:, j]))
    mu = X.mean(0)
    Z = (X - mu) / X.std(0, ddof=1)
    h = oracle.pca_fit(Z[:, None, :], n_comp=3)
    assert np.max(np.abs(h["eigvals"] - f["eigvals"])) <= 1e-10 * B
    sh = _scores(h, Z)
    for j in range(3):
        s = np.sign(sf[:, j] @ sh[:, j])
        assert np.max(np.abs(s * sh[:, j] - sf[:, j])) <= 1e-9 * np.max(np.abs(sf[:, j]))
    # the default stays covariance PCA: not scale invariant
    c = oracle.pca_fit(X[:, None, :], n_comp=3)
    d = oracle.pca_fit((X * a)[:, None, :], n_comp=3)
    assert np.max(np.abs(c["eigvals"] - d["eigvals"])) > 1.0
    with pytest.raises(ValueError):
        Y = X.copy()
        Y[:, 2] = 7.0
        oracle.pca_fit(Y[:, None, :], n_comp=2, standardize=True)


def test_pca_constructed_eigenvalues():
    rng = np.random.default_rng(22)
    P, B = 500, 5
    Z = rng.standard_normal((P, B))
    Z -= Z.mean(0)
    ev, U = np.linalg.eigh(Z.T @ Z)
    Z = Z @ (U / np.sqrt(ev)) @ U.T * np.sqrt(P - 1)      # sample covariance = I
    Q, _ = np.linalg.qr(rng.standard_normal((B, B)))
    lam = np.array([50.0, 20.0, 7.0, 2.0, 0.5])
    X = Z @ (Q * np.sqrt(lam)) .T + rng.uniform(100, 200, B)
    fit = oracle.pca_fit(X[:, None, :], n_comp=B)
    assert np.max(np.abs(fit["eigvals"] - lam)) <= 1e-10 * lam.max()
    for j in range(B):
        assert abs(abs(fit["V"][:, j] @ Q[:, j]) - 1) <= 1e-9


# ------------------------------------------------------------------ soft

def _soft_small(seed=31, N=400, B=4, K=3):
    rng = np.random.default_rng(seed)
    mus = rng.uniform(800, 3500, size=(K, B))
    cls = rng.integers(0, K, N)
    cls[:K] = np.arange(K)
    X = mus[cls] + rng.normal(0, 60, size=(N, B))
    w = np.zeros((N, K))
    w[np.arange(N), cls] = 1.0
    soft = rng.random(N) < 0.3
    w[soft] = rng.dirichlet(np.full(K, 0.5), size=int(soft.sum()))
    return X, w, cls


def test_one_hot_weights_reproduce_hard_cva():
    X, w, cls = _soft_small()
    onehot = np.zeros_like(w)
    onehot[np.arange(len(cls)), cls] = 1.0
    s = oracle.soft_fit(X, onehot)
    h = oracle.cva_fit(X[:, None, :], cls.astype(np.int8)[:, None], w.shape[1])
    assert abs(s["J"] - h["eigvals"].sum()) <= 1e-12 * s["J"]
    assert np.max(np.abs(s["Sw"] - h["Sw"])) <= 1e-12 * np.max(np.abs(h["Sw"]))
    assert np.max(np.abs(s["Sb"] - h["Sb"])) <= 1e-12 * np.max(np.abs(h["Sb"]))
    assert abs(s["J"] - s["trace_form"]) <= 1e-10 * s["J"]


def test_gradient_matches_central_differences_of_exact_change():
    X, w, _ = _soft_small(seed=32, N=600, B=5, K=4)
    g = oracle.soft_grad(X, w)
    rng = np.random.default_rng(4)
    h = 1e-3
    gmax = np.max(np.abs(g))
    for _ in range(64):
        p = int(rng.integers(0, X.shape[0]))
        c = int(rng.integers(0, w.shape[1]))
        fd = (oracle.soft_delta_J(X, w, p, c, h) - oracle.soft_delta_J(X, w, p, c, -h)) / (2 * h)
        assert abs(fd - g[p, c]) <= 1e-6 * gmax


def test_delta_J_matches_full_recompute():
    X, w, _ = _soft_small(seed=33, N=80, B=3, K=3)
    p, c, h = 5, 1, 0.25
    w2 = w.copy()
    w2[p, c] += h
    J1 = oracle.soft_fit(X, w)["trace_form"]
    J2 = oracle.soft_fit(X, w2)["trace_form"]
    assert abs((J2 - J1) - oracle.soft_delta_J(X, w, p, c, h)) <= 1e-9 * abs(J1)


def _exact_J(X, w):
    """trace(S_w^-1 S_b) in exact rationals (tiny sizes)."""
    N, B = len(X), len(X[0])
    K = len(w[0])
    n = [sum(w[p][c] for p in range(N)) for c in range(K)]
    mc = [[sum(w[p][c] * X[p][i] for p in range(N)) / n[c] for i in range(B)] for c in range(K)]
    Nt = sum(n)
    m = [sum(n[c] * mc[c][i] for c in range(K)) / Nt for i in range(B)]
    Sw = [[sum(w[p][c] * (X[p][i] - mc[c][i]) * (X[p][j] - mc[c][j])
               for p in range(N) for c in range(K)) for j in range(B)] for i in range(B)]
    Sb = [[sum(n[c] * (mc[c][i] - m[i]) * (mc[c][j] - m[j]) for c in range(K))
           for j in range(B)] for i in range(B)]
    # solve Sw Y = Sb by Gauss-Jordan, then trace(Y)
    A = [row[:] + Sb[i][:] for i, row in enumerate(Sw)]
    for col in range(B):
        piv = next(r for r in range(col, B) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(B):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return sum(A[i][B + i] for i in range(B))


def test_gradient_against_exact_rational_differences():
    rng = np.random.default_rng(34)
    N, B, K = 9, 2, 3
    Xi = rng.integers(0, 50, size=(N, B))
    wq = rng.integers(1, 9, size=(N, K))
    X = [[Fraction(int(v)) for v in r] for r in Xi]
    w = [[Fraction(int(v), 8) for v in r] for r in wq]
    g = oracle.soft_grad(Xi.astype(np.float64), wq / 8.0)
    h = Fraction(1, 10 ** 6)
    for p, c in [(0, 0), (3, 1), (8, 2), (5, 0)]:
        wp = [r[:] for r in w]
        wm = [r[:] for r in w]
        wp[p][c] += h
        wm[p][c] -= h
        fd = (_exact_J(X, wp) - _exact_J(X, wm)) / (2 * h)
        assert abs(float(fd) - g[p, c]) <= 1e-8 * max(1.0, abs(float(fd)))


def test_euler_identity():
    X, w, _ = _soft_small(seed=35)
    g = oracle.soft_grad(X, w)
    s = np.sum(w * g)
    assert abs(s) <= 1e-10 * np.sum(np.abs(w * g))


def test_soft_weights_generator_shapes():
    from synth import make_soft_case
    X, w, cls, idx, case = make_soft_case(4, scale=0.05)
    assert X.shape == (idx.size, case.B) and w.shape == (idx.size, case.K)
    assert np.allclose(w.sum(1), 1.0, atol=1e-5)
    assert (w >= 0).all()
    assert ((w.max(1) < 1).sum()) > 0          # some pixels lie near a border


# ------------------------------------------------ mask refinement step

def _kkt_ok(v, w, tol=1e-12):
    """w is the Euclidean projection of v onto the simplex iff w >= 0,
    sum w = 1, and for some theta: v_c - w_c = theta where w_c > 0 and
    v_c <= theta where w_c = 0 (the optimality conditions)."""
    if np.any(w < 0) or abs(w.sum() - 1.0) > tol:
        return False
    sup = w > 0
    theta = np.mean(v[sup] - w[sup])
    return bool(np.all(np.abs(v[sup] - w[sup] - theta) <= tol) and np.all(v[~sup] <= theta + tol))


def test_simplex_projection_optimality_conditions():
    rng = np.random.default_rng(40)
    for K in (2, 3, 5, 8, 32):
        V = rng.normal(0, 2, (200, K))
        W = oracle.simplex_projection(V)
        for v, w in zip(V, W):
            assert _kkt_ok(v, w)


def test_simplex_projection_fixes_simplex_points():
    rng = np.random.default_rng(41)
    W0 = rng.dirichlet(np.full(6, 0.7), 100)
    W0[:10] = np.eye(6)[rng.integers(0, 6, 10)]
    assert np.allclose(oracle.simplex_projection(W0), W0, atol=1e-15)


def test_simplex_projection_brute_force_small_k():
    rng = np.random.default_rng(42)
    # K = 2: the segment w = (t, 1 - t), t in [0, 1]; K = 3: a fine triangle grid
    t = np.linspace(0, 1, 20001)
    seg = np.stack([t, 1 - t], 1)
    a, b = np.meshgrid(np.linspace(0, 1, 401), np.linspace(0, 1, 401))
    tri = np.stack([a.ravel(), b.ravel(), 1 - a.ravel() - b.ravel()], 1)
    tri = tri[tri[:, 2] >= -1e-12]
    for grid in (seg, tri):
        K = grid.shape[1]
        for _ in range(20):
            v = rng.normal(0, 1.5, K)
            best = grid[np.argmin(((grid - v) ** 2).sum(1))]
            w = oracle.simplex_projection(v[None, :])[0]
            assert np.max(np.abs(w - best)) <= 2.0 / (len(t) - 1 if K == 2 else 400)
            assert ((w - v) ** 2).sum() <= ((best - v) ** 2).sum() + 1e-12


def test_refinement_step_moves_mislabelled_pixels_only():
    """Two well separated classes: a pixel drawn from class 0 but labelled
    1 moves towards class 0; correctly labelled one-hot pixels stay put."""
    rng = np.random.default_rng(43)
    N, B = 400, 3
    cls = np.arange(N) % 2
    X = np.where(cls[:, None] == 0, 0.0, 10.0) + rng.normal(0, 1, (N, B))
    lab = cls.copy()
    lab[:20:2] = 1                              # ten class-0 pixels labelled 1
    w = np.eye(2)[lab]
    g = oracle.soft_grad(X, w)
    w1 = oracle.soft_update(w, g, 0.5)
    assert np.allclose(w1.sum(1), 1.0) and (w1 >= 0).all()
    bad = np.zeros(N, bool)
    bad[:20:2] = True
    assert np.all(w1[bad, 0] > 0.4)             # moved by the full step towards class 0
    assert np.allclose(w1[~bad], w[~bad])       # the rest stay one-hot
    # the direction lies in the simplex's plane: a zero step changes nothing
    assert np.allclose(oracle.soft_update(w, g, 0.0), w)
