"""Pins of the FP64 CVA oracle to things other than itself.

Paper: Section 2 (canonical variates paragraph; regression-coefficient and
rescale paragraphs), Section 4 (generalized symmetric-definite eigensolver;
eigenvector signs differ between correct solvers, Figure 5).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.cva import _rows


def _tiny_case(rng, H=7, W=5, B=3, K=3, hi=4096, ensure=2):
    cube = rng.integers(0, hi, size=(H, W, B)).astype(np.uint16)
    labels = rng.integers(-1, K, size=(H, W)).astype(np.int8)
    flat = labels.reshape(-1)
    for k in range(K):          # every class gets at least `ensure` pixels
        for j in range(ensure):
            flat[(k * ensure + j) % flat.size] = k
    return cube, labels


# --------------------------------------------------------------- P1 counts

def test_counts_and_index_lists_brute_force():
    rng = np.random.default_rng(11)
    for K in (2, 3, 5):
        lab = rng.integers(-1, K, size=(13, 17)).astype(np.int8)
        counts = [0] * K
        lists = [[] for _ in range(K)]
        for i, v in enumerate(lab.reshape(-1).tolist()):
            if v >= 0:
                counts[v] += 1
                lists[v].append(i)
        assert oracle.class_counts(lab, K).tolist() == counts
        got = oracle.class_index_lists(lab, K)
        assert [g.tolist() for g in got] == lists


def test_counts_reject_out_of_range_labels():
    with pytest.raises(ValueError):
        oracle.class_counts(np.array([0, 1, 3], dtype=np.int8), 3)
    with pytest.raises(ValueError):
        oracle.class_counts(np.array([0, -2], dtype=np.int8), 3)


# ------------------------------------------- P2 brute force + exact rationals

def _exact_scatter(cube, labels, K):
    """Double loops over pixels and bands in exact rational arithmetic."""
    X = _rows(cube).tolist()
    lab = labels.reshape(-1).tolist()
    B = len(X[0])
    n = [0] * K
    s = [[0] * B for _ in range(K)]
    for x, k in zip(X, lab):
        if k < 0:
            continue
        n[k] += 1
        for i in range(B):
            s[k][i] += int(x[i])
    m = [[Fraction(s[k][i], n[k]) for i in range(B)] for k in range(K)]
    N = sum(n)
    g = [Fraction(sum(s[k][i] for k in range(K)), N) for i in range(B)]
    Sw = [[Fraction(0)] * B for _ in range(B)]
    for x, k in zip(X, lab):
        if k < 0:
            continue
        for i in range(B):
            di = int(x[i]) - m[k][i]
            for j in range(B):
                Sw[i][j] += di * (int(x[j]) - m[k][j])
    Sb = [[sum(n[k] * (m[k][i] - g[i]) * (m[k][j] - g[j]) for k in range(K))
           for j in range(B)] for i in range(B)]
    return n, s, Sw, Sb


@pytest.mark.parametrize("seed,H,W,B,K", [(1, 7, 5, 3, 3), (2, 6, 6, 4, 2), (3, 9, 4, 5, 4)])
def test_moments_and_scatter_match_exact_rationals(seed, H, W, B, K):
    rng = np.random.default_rng(seed)
    cube, labels = _tiny_case(rng, H, W, B, K)
    n, s, Sw_x, Sb_x = _exact_scatter(cube, labels, K)
    counts, sums, means = oracle.class_moments(cube, labels, K)
    assert counts.tolist() == n
    assert sums.tolist() == s                        # exact integer sums
    Sw = oracle.within_scatter(cube, labels, K, means)
    Sb = oracle.between_scatter(counts, means)
    Swx = np.array([[float(v) for v in r] for r in Sw_x])
    Sbx = np.array([[float(v) for v in r] for r in Sb_x])
    assert np.max(np.abs(Sw - Swx)) <= 1e-14 * np.max(np.abs(Swx))
    assert np.max(np.abs(Sb - Sbx)) <= 1e-14 * np.max(np.abs(Sbx))


def test_float_page_brute_force_loops():
    rng = np.random.default_rng(5)
    cube = rng.normal(1000.0, 50.0, size=(6, 5, 3)).astype(np.float32)
    labels = rng.integers(0, 3, size=(6, 5)).astype(np.int8)
    X = _rows(cube).astype(np.float64)
    lab = labels.reshape(-1)
    B, K = 3, 3
    Sw = np.zeros((B, B))
    for k in range(K):
        rows = [X[p] for p in range(X.shape[0]) if lab[p] == k]
        mk = [sum(r[i] for r in rows) / len(rows) for i in range(B)]
        for r in rows:
            for i in range(B):
                for j in range(B):
                    Sw[i, j] += (r[i] - mk[i]) * (r[j] - mk[j])
    counts, sums, means = oracle.class_moments(cube, labels, K)
    got = oracle.within_scatter(cube, labels, K, means)
    assert np.max(np.abs(got - Sw)) <= 1e-12 * np.max(np.abs(Sw))


# ------------------------------------------------------------- P3 S_w+S_b=S_t

def test_within_plus_between_is_total_scatter():
    from synth import make_case
    c = make_case(1, scale=0.25)
    counts, sums, means = oracle.class_moments(c.cube, c.labels, c.K)
    Sw = oracle.within_scatter(c.cube, c.labels, c.K, means)
    Sb = oracle.between_scatter(counts, means)
    St = oracle.total_scatter(c.cube, c.labels)
    assert np.max(np.abs(Sw + Sb - St)) <= 1e-12 * np.max(np.abs(St))


# --------------------------------------------------- P4 eigen normalisation

def test_eigvec_normalisation_and_null_space():
    from synth import make_case
    c = make_case(2, scale=0.1)
    fit = oracle.cva_fit(c.cube, c.labels, c.K)
    W, lam, Sw, Sb = fit["W"], fit["eigvals"], fit["Sw"], fit["Sb"]
    C = c.K - 1
    assert W.shape == (c.B, C)
    I = W.T @ Sw @ W
    assert np.max(np.abs(I - np.eye(C))) <= 1e-10
    D = W.T @ Sb @ W
    assert np.max(np.abs(D - np.diag(lam))) <= 1e-10 * lam.max()
    assert (lam > 0).all() and (np.diff(lam) <= 0).all()
    lam_all, _ = oracle.generalized_eig(Sb, Sw)
    assert np.max(np.abs(lam_all[C:])) <= 1e-10 * lam_all[0]


# ------------------------------------------------------------- P5 LDA, K=2

def test_two_classes_reduce_to_fisher_lda():
    rng = np.random.default_rng(7)
    from synth import make_case
    c = make_case(1, scale=0.2)
    lab = c.labels.copy()
    lab[lab == 2] = -1                       # keep parchment vs overtext
    fit = oracle.cva_fit(c.cube, lab, 2)
    X = _rows(c.cube).astype(np.float64)
    f = lab.reshape(-1)
    X0, X1 = X[f == 0], X[f == 1]
    m0, m1 = X0.mean(0), X1.mean(0)
    Sw = (X0 - m0).T @ (X0 - m0) + (X1 - m1).T @ (X1 - m1)
    d = m1 - m0
    w_lda = np.linalg.solve(Sw, d)
    n0, n1 = len(X0), len(X1)
    lam_lda = n0 * n1 / (n0 + n1) * d @ w_lda
    w = fit["W"][:, 0]
    cosang = abs(w @ w_lda) / (np.linalg.norm(w) * np.linalg.norm(w_lda))
    assert abs(1 - cosang) <= 1e-10
    assert abs(fit["eigvals"][0] - lam_lda) <= 1e-10 * lam_lda
    del rng


# --------------------------------------- P6 Fisher ratios known by construction

def _constructed(rng, n, B, mus, Sigma):
    """Classes with exact sample means mus[k] and pooled within-class scatter
    exactly (N-K) Sigma."""
    K = len(mus)
    Z = [rng.standard_normal((n, B)) for _ in range(K)]
    Z = [z - z.mean(0) for z in Z]
    M = sum(z.T @ z for z in Z)
    ev, U = np.linalg.eigh(M)
    Mih = (U / np.sqrt(ev)) @ U.T
    N = n * K
    L = np.linalg.cholesky((N - K) * Sigma)
    Xs = [z @ Mih @ L.T + mu for z, mu in zip(Z, mus)]
    cube = np.concatenate(Xs, 0)[:, None, :]
    labels = np.repeat(np.arange(K), n).astype(np.int8)[:, None]
    return cube, labels


def test_fisher_ratios_known_by_construction():
    rng = np.random.default_rng(3)
    B, n = 6, 40
    G = rng.standard_normal((B, B))
    Sigma = G @ G.T + B * np.eye(B)
    L = np.linalg.cholesky(Sigma)
    a, b = 3.0, 1.0
    f = np.array([[a, b], [-a, b], [0.0, -2 * b]])       # sums to zero
    F = np.zeros((3, B))
    F[:, :2] = f
    c0 = rng.uniform(800, 3500, B)
    mus = [c0 + L @ F[k] for k in range(3)]
    cube, labels = _constructed(rng, n, B, mus, Sigma)
    fit = oracle.cva_fit(cube, labels, 3)
    N, K = 3 * n, 3
    expect = np.sort(np.array([n * 2 * a * a, n * 6 * b * b]) / (N - K))[::-1]
    assert np.max(np.abs(fit["eigvals"] - expect)) <= 1e-10 * expect.max()
    # in whitened coordinates the canonical vectors are e1 (ratio 2a^2 n/(N-K),
    # the larger one here) and e2, so W's columns are parallel to L^-T e1, L^-T e2
    Linv_T = np.linalg.inv(L).T
    for j in range(2):
        ref = Linv_T[:, j]
        w = fit["W"][:, j]
        cosang = abs(w @ ref) / np.linalg.norm(w) / np.linalg.norm(ref)
        assert abs(1 - cosang) <= 1e-9


def test_fisher_ratios_equilateral_degenerate_pair():
    rng = np.random.default_rng(4)
    B, n, r = 5, 30, 2.5
    Sigma = np.diag(rng.uniform(1, 4, B))
    L = np.linalg.cholesky(Sigma)
    F = np.zeros((3, B))
    for k in range(3):
        F[k, 0] = r * np.cos(2 * np.pi * k / 3)
        F[k, 1] = r * np.sin(2 * np.pi * k / 3)
    c0 = rng.uniform(800, 3500, B)
    cube, labels = _constructed(rng, n, B, [c0 + L @ F[k] for k in range(3)], Sigma)
    fit = oracle.cva_fit(cube, labels, 3)
    lam = 3 * n * r * r / (2 * (3 * n - 3))
    assert np.max(np.abs(fit["eigvals"] - lam)) <= 1e-10 * lam


# ------------------------------------------------------ P7 affine invariance

def test_affine_invariance_of_projection_and_pca_negative_control():
    from synth import make_case
    c = make_case(1, scale=0.15)
    X = _rows(c.cube).astype(np.float64)
    rng = np.random.default_rng(9)
    A = rng.standard_normal((c.B, c.B)) + 3 * np.eye(c.B)
    t = rng.uniform(-100, 100, c.B)
    Y = X @ A.T + t
    cube2 = Y.reshape(c.H, c.W, c.B)
    f1 = oracle.cva_fit(c.cube, c.labels, c.K)
    f2 = oracle.cva_fit(cube2, c.labels, c.K)
    y1 = oracle.project(c.cube, f1["W"], f1["mean"])
    y2 = oracle.project(cube2, f2["W"], f2["mean"])
    for j in range(y1.shape[1]):
        s = np.sign(y1[:, j] @ y2[:, j])
        rng_j = np.ptp(y1[:, j])
        assert np.max(np.abs(y1[:, j] - s * y2[:, j])) <= 1e-9 * rng_j
    assert np.max(np.abs(f1["eigvals"] - f2["eigvals"])) <= 1e-9 * f1["eigvals"].max()
    q1, _ = oracle.cva_project(c.cube, f1["W"], f1["mean"])
    q2, _ = oracle.cva_project(cube2, f2["W"], f2["mean"])
    for j in range(q1.shape[0]):
        a = q1[j].astype(int)
        b = q2[j].astype(int)
        d = min(np.max(np.abs(a - b)), np.max(np.abs(a - (255 - b))))
        assert d <= 1
    # PCA is not affine invariant: the leading component changes
    p1 = oracle.pca_fit(c.cube, n_comp=1)
    p2 = oracle.pca_fit(cube2, n_comp=1)
    z1 = oracle.project(c.cube, p1["V"], p1["mean"])[:, 0]
    z2 = oracle.project(cube2, p2["V"], p2["mean"])[:, 0]
    corr = abs(np.corrcoef(z1, z2)[0, 1])
    assert corr < 0.999


# -------------------------------------------------------------- P8 stretch

def test_stretch_properties_and_brute_force():
    rng = np.random.default_rng(12)
    y = rng.normal(0, 3, size=(5000, 3))
    q, a, b = oracle.stretch_minmax(y)
    for j in range(3):
        assert q[np.argmin(y[:, j]), j] == 0
        assert q[np.argmax(y[:, j]), j] == 255
        order = np.argsort(y[:, j], kind="stable")
        assert (np.diff(q[order, j].astype(int)) >= 0).all()
    q2, _, _ = oracle.stretch_minmax(7.5 * y + 3.0)
    assert np.max(np.abs(q2.astype(int) - q.astype(int))) <= 1
    q3, _, _ = oracle.stretch_minmax(-y)
    assert np.max(np.abs(q3.astype(int) - (255 - q.astype(int)))) <= 1
    # brute force element loop on a slice
    for j in range(3):
        lo, hi = min(y[:, j]), max(y[:, j])
        for p in range(0, 5000, 97):
            v = int(np.floor(255.0 * (y[p, j] - lo) / (hi - lo) + 0.5))
            v = 0 if v < 0 else (255 if v > 255 else v)
            assert q[p, j] == v
    # constant component maps to zero
    qc, _, _ = oracle.stretch_minmax(np.ones((10, 1)))
    assert (qc == 0).all()


def test_stretch_modes_two_and_three():
    rng = np.random.default_rng(13)
    y = rng.normal(0, 1, size=(20000, 2))
    yt = y[:200]
    q, a, b = oracle.stretch_training_range(y, yt)
    assert np.allclose(a, yt.min(0)) and np.allclose(b, yt.max(0))
    assert q[np.argmin(y[:, 0]), 0] == 0 and q[np.argmax(y[:, 0]), 0] == 255
    q5, a5, b5 = oracle.stretch_percentile(y, 5.0)
    frac_lo = (q5[:, 0] == 0).mean()
    assert 0.04 <= frac_lo <= 0.06
    srt = np.sort(y[:, 0])
    pos = 0.05 * (srt.size - 1)
    i = int(np.floor(pos))
    assert abs(a5[0] - (srt[i] + (pos - i) * (srt[i + 1] - srt[i]))) <= 1e-12


def test_stretch_sixteen_bits():
    rng = np.random.default_rng(14)
    y = rng.normal(0, 2, size=(6000, 2))
    q16, a, b = oracle.stretch_minmax(y, levels=65535)
    assert q16.dtype == np.uint16
    q8, _, _ = oracle.stretch_minmax(y)
    for j in range(2):
        assert q16[np.argmin(y[:, j]), j] == 0 and q16[np.argmax(y[:, j]), j] == 65535
        # 65535 = 255 * 257: the two maps agree within one 8-bit level
        assert np.max(np.abs(np.rint(q16[:, j] / 257.0) - q8[:, j])) <= 1
        lo, hi = y[:, j].min(), y[:, j].max()
        for p in range(0, 6000, 131):
            v = int(np.floor(65535.0 * (y[p, j] - lo) / (hi - lo) + 0.5))
            assert q16[p, j] == min(max(v, 0), 65535)
    # modes 2 and 3 clamp at the 16-bit top as well
    qt, _, _ = oracle.stretch_training_range(y, y[:50], levels=65535)
    assert qt.max() == 65535 and qt.min() == 0


def test_percentiles_closed_forms():
    rng = np.random.default_rng(15)
    # a shuffled arithmetic sequence 0, 1, ..., 100: the p-th percentile is p
    y = rng.permutation(np.arange(101.0))[:, None]
    for pct in (0.0, 1.0, 5.0, 12.5):
        _, a, b = oracle.stretch_percentile(y, pct)
        assert a[0] == pct and b[0] == 100.0 - pct
    # the 0-th percentile is the minimum: mode 3 at 0 is mode 1
    z = rng.normal(size=(997, 3))
    q0, a0, b0 = oracle.stretch_percentile(z, 0.0)
    q1, a1, b1 = oracle.stretch_minmax(z)
    assert (a0 == a1).all() and (b0 == b1).all() and (q0 == q1).all()
    # 0.01 % of 10001 values sits exactly on the second order statistic
    w = rng.permutation(np.arange(10001.0) * 0.5)[:, None]
    _, a, b = oracle.stretch_percentile(w, 0.01)
    assert a[0] == 0.5 and abs(b[0] - 4999.5) <= 1e-9   # 99.99 / 100 is inexact
    # between two order statistics: 10 values 0, 10, ..., 90, 5 % -> 0.45
    v = rng.permutation(np.arange(10) * 10.0)[:, None]
    _, a, b = oracle.stretch_percentile(v, 5.0)
    assert abs(a[0] - 4.5) <= 1e-12 and abs(b[0] - 85.5) <= 1e-12


def test_compose_rgb_layout():
    rng = np.random.default_rng(16)
    r, g = rng.integers(0, 256, (2, 7, 9), dtype=np.uint8)
    rgb = oracle.compose_rgb(r, g, None)
    assert rgb.shape == (7, 9, 3)
    for y in range(7):
        for x in range(9):
            assert tuple(rgb[y, x]) == (r[y, x], g[y, x], 0)
    two = oracle.compose_rgb(g, r, r)          # one image in two channels
    assert (two[..., 1] == two[..., 2]).all() and (two[..., 0] == g).all()


# ------------------------------------------------- DB and Dunn indices (Sec. 3)

def test_cluster_indices_two_clusters_closed_form():
    # {0, 2} and {10, 12}: centroids 1 and 11, scatters 1 and 1, M = 10
    img = np.array([[0, 2, 10, 12, 99]], dtype=np.uint8)
    r = oracle.cluster_indices(img, [0, 1, 2, 3, 4], [0, 0, 1, 1, -1], 2)
    assert r["centroids"].tolist() == [[1.0], [11.0]]
    assert r["scatter"].tolist() == [1.0, 1.0]
    assert r["dist"][0, 1] == 10.0 and r["dist"][1, 0] == 10.0
    assert r["dbi_pairs"][0, 1] == 0.2 and r["dbi"] == 0.2            # (1 + 1) / 10
    assert r["dunn_pairs"][0, 1] == 8.0 and r["dunn"] == 8.0          # (10 - 1 - 1) / 1
    assert r["counts"].tolist() == [2, 2]


def test_cluster_indices_three_clusters_by_hand():
    # centroids 0, 10, 30 with scatters 1, 2, 3 (points c - s, c + s)
    vals = [-1, 1, 8, 12, 27, 33]
    r = oracle.cluster_indices(np.array([vals], dtype=np.float64), range(6), [0, 0, 1, 1, 2, 2], 3)
    assert np.allclose(r["scatter"], [1, 2, 3], rtol=0, atol=1e-15)
    R = r["dbi_pairs"]
    assert abs(R[0, 1] - 3 / 10) < 1e-15 and abs(R[0, 2] - 4 / 30) < 1e-15 and abs(R[1, 2] - 5 / 20) < 1e-15
    assert abs(r["dbi"] - (0.3 + 0.3 + 0.25) / 3) < 1e-15
    assert abs(r["dunn"] - min(10 - 3, 30 - 4, 20 - 5) / 3) < 1e-15
    assert abs(r["dunn_pairs"][1, 2] - (20 - 5) / 3) < 1e-15


def test_cluster_indices_brute_force_norms_and_invariance():
    rng = np.random.default_rng(21)
    img = rng.normal(size=(3, 40, 30))
    pix = rng.choice(1200, 300, replace=False)
    cls = rng.integers(-1, 4, 300)
    for p in (1.0, 2.0, 3.0):
        r = oracle.cluster_indices(img, pix, cls, 4, p=p)
        flat = img.reshape(3, -1)
        for k in range(4):
            pts = [flat[:, q] for q, c in zip(pix, cls) if c == k]
            A = [sum(v[f] for v in pts) / len(pts) for f in range(3)]
            S = sum(sum(abs(v[f] - A[f]) ** p for f in range(3)) ** (1 / p) for v in pts) / len(pts)
            assert abs(r["scatter"][k] - S) <= 1e-12 * S
        a0, a1 = r["centroids"][0], r["centroids"][1]
        assert abs(r["dist"][0, 1] - sum(abs(a0 - a1) ** p) ** (1 / p)) <= 1e-12 * r["dist"][0, 1]
        # scale and shift of every feature leave the ratios unchanged
        r2 = oracle.cluster_indices(7.0 * img - 3.0, pix, cls, 4, p=p)
        assert np.allclose(r2["dbi_pairs"], r["dbi_pairs"], rtol=1e-12, atol=0)
        assert np.allclose(r2["dunn_pairs"], r["dunn_pairs"], rtol=1e-12, atol=1e-12)
    # p = 1 and p = 2 on two-dimensional points (0, 0), (2, 2): A = (1, 1)
    img2 = np.array([[0, 2, 5, 5], [0, 2, 9, 9]], dtype=np.float64)
    assert oracle.cluster_indices(img2, [0, 1, 2, 3], [0, 0, 1, 1], 2, p=1.0)["scatter"][0] == 2.0
    assert abs(oracle.cluster_indices(img2, [0, 1, 2, 3], [0, 0, 1, 1], 2)["scatter"][0] - np.sqrt(2)) < 1e-15


def test_cluster_indices_errors():
    img = np.zeros((1, 10))
    with pytest.raises(ValueError):
        oracle.cluster_indices(img, [0, 1], [0, 2], 2)          # class outside
    with pytest.raises(ValueError):
        oracle.cluster_indices(img, [0, 10], [0, 1], 2)         # pixel outside
    with pytest.raises(ValueError):
        oracle.cluster_indices(img, [0, 1], [0, 0], 2)          # empty class


# ----------------------------------------------------------- sign and errors

def test_sign_rule():
    W = np.array([[0.1, -3.0, 2.0], [-0.5, 1.0, -2.0], [0.2, 2.9, 0.0]])
    S = oracle.sign_rule(W)
    assert S[1, 0] > 0 and S[0, 1] > 0
    assert S[0, 2] == 2.0 and S[1, 2] == -2.0        # tie -> lowest index positive


def test_fit_errors():
    rng = np.random.default_rng(1)
    cube, labels = _tiny_case(rng, 8, 8, 3, 3)
    lab = labels.copy()
    lab[lab == 2] = -1
    with pytest.raises(ValueError):
        oracle.cva_fit(cube, lab, 3)                  # empty class
    c2 = cube.copy()
    c2[..., 2] = c2[..., 1]                           # duplicated band -> singular S_w
    with pytest.raises(ValueError):
        oracle.cva_fit(c2, labels, 3)
    with pytest.raises(ValueError):
        oracle.cva_fit(cube, labels, 3, n_comp=3)


def test_fit_from_points_matches_label_map_in_any_order():
    """A list of the labelled pixels, in any order, gives the label-map fit;
    entries marked -1 are skipped."""
    rng = np.random.default_rng(61)
    cube = rng.integers(0, 4096, size=(9, 11, 5)).astype(np.uint16)
    labels = rng.integers(-1, 3, size=(9, 11)).astype(np.int8)
    ref = oracle.cva_fit(cube, labels, 3)
    pix = np.flatnonzero(labels.reshape(-1) >= 0)
    cls = labels.reshape(-1)[pix]
    order = rng.permutation(pix.size)
    extra = rng.integers(0, 99, size=7)                  # skipped entries
    pts = np.concatenate([pix[order], extra])
    cl = np.concatenate([cls[order], np.full(7, -1, np.int8)])
    got = oracle.cva_fit_points(cube, pts, cl, 3)
    np.testing.assert_array_equal(got["counts"], ref["counts"])
    np.testing.assert_allclose(got["Sw"], ref["Sw"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(got["Sb"], ref["Sb"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(got["eigvals"], ref["eigvals"], rtol=1e-10)
    np.testing.assert_allclose(got["W"], ref["W"], rtol=1e-8, atol=1e-12)


def test_fit_from_points_repeated_list_doubles_the_scatters():
    """Listing every point twice doubles n_k, S_w and S_b: the eigenvalues of
    S_b w = lambda S_w w are unchanged and W (with w^T S_w w = 1) shrinks by
    1/sqrt(2)."""
    rng = np.random.default_rng(62)
    cube = rng.normal(1000.0, 50.0, size=(6, 8, 4))
    pix = rng.permutation(48)[:30]
    cls = rng.integers(0, 3, size=30).astype(np.int8)
    cls[:3] = [0, 1, 2]
    one = oracle.cva_fit_points(cube, pix, cls, 3)
    two = oracle.cva_fit_points(cube, np.concatenate([pix, pix]), np.concatenate([cls, cls]), 3)
    np.testing.assert_array_equal(two["counts"], 2 * one["counts"])
    np.testing.assert_allclose(two["Sw"], 2 * one["Sw"], rtol=1e-12)
    np.testing.assert_allclose(two["Sb"], 2 * one["Sb"], rtol=1e-12)
    np.testing.assert_allclose(two["eigvals"], one["eigvals"], rtol=1e-10)
    np.testing.assert_allclose(two["W"], one["W"] / np.sqrt(2.0), rtol=1e-8, atol=1e-14)


def test_fit_from_points_rejects_pixels_outside_the_page():
    cube = np.zeros((4, 4, 3), np.uint16)
    with pytest.raises(ValueError):
        oracle.cva_fit_points(cube, np.array([0, 16]), np.array([0, 1], np.int8), 2)
