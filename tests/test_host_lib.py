"""CPU tests of the C ABI library: it loads, exports every declared symbol,
its FP64 finisher agrees with LAPACK, and argument checking returns the
documented status codes without touching a GPU (context with device -1).
"""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cvamx.h")


def _lib():
    from paper_1612_06457_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcvamx.so not built")
    return L


def test_library_exports_every_declared_symbol():
    L = _lib()
    text = open(HEADER).read()
    names = re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(\w+)\s*\(", text, re.M)
    assert len(names) >= 12
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_sym_eig_matches_lapack():
    _lib()
    from paper_1612_06457_amd import sym_eig
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 7, 16, 23, 33, 64):
        G = rng.standard_normal((n, n))
        A = G + G.T
        w, V = sym_eig(A)
        ref = np.sort(np.linalg.eigvalsh(A))[::-1]
        assert np.max(np.abs(w - ref)) <= 1e-12 * max(1, np.abs(ref).max())
        assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-12
        assert np.max(np.abs(A @ V - V * w)) <= 1e-11 * max(1, np.abs(ref).max())
        for j in range(n):                          # sign rule
            i = int(np.argmax(np.abs(V[:, j])))
            assert V[i, j] > 0


def _check_top(A, k, w, V, tol_r=1e-11):
    """Eigenvalues against LAPACK, orthonormal columns, small residuals, the
    sign rule, and each cluster's span against LAPACK's."""
    n = A.shape[0]
    ref_w, ref_V = np.linalg.eigh(A)
    ref_w, ref_V = ref_w[::-1], ref_V[:, ::-1]
    scale = max(1.0, np.abs(ref_w).max())
    assert np.max(np.abs(w - ref_w)) <= 1e-12 * scale
    assert V.shape == (n, k)
    assert np.max(np.abs(V.T @ V - np.eye(k))) <= 1e-11
    assert np.max(np.abs(A @ V - V * w[:k])) <= tol_r * scale
    for j in range(k):
        i = int(np.argmax(np.abs(V[:, j])))
        assert V[i, j] > 0
    # the span of the leading k vectors (when w[k-1] is apart from w[k])
    if k < n and ref_w[k - 1] - ref_w[k] > 1e-6 * scale:
        P = V @ V.T - ref_V[:, :k] @ ref_V[:, :k].T
        assert np.max(np.abs(P)) <= 1e-8


def test_sym_eig_top_matches_lapack():
    """The leading eigenpairs: random symmetric matrices, covariance-like
    spectra over eight decades, an exactly threefold eigenvalue, a pair
    1e-9 apart, diagonal matrices (one with a threefold entry), a
    block-diagonal matrix (the tridiagonal form splits), a multiple of the
    identity, the all-ones matrix and the zero matrix."""
    _lib()
    from paper_1612_06457_amd import sym_eig_top
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 8, 16, 23, 33, 47, 64):
        G = rng.standard_normal((n, n))
        A = G + G.T
        for k in sorted({1, 2, 3, min(n, 8), n} & set(range(1, n + 1))):
            w, V = sym_eig_top(A, k)
            _check_top(A, k, w, V)
    for n in (23, 33, 47):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        for ev in (np.logspace(6, -2, n), np.r_[[10.0, 10.0, 10.0, 5.0], np.linspace(1, 1e-3, n - 4)],
                   np.r_[[10.0, 10.0 + 1e-9, 9.0], np.linspace(2, 1, n - 3)]):
            A = (Q * ev) @ Q.T
            A = 0.5 * (A + A.T)
            for k in (1, 3, 4):
                w, V = sym_eig_top(A, k)
                _check_top(A, k, w, V)
    D = np.diag(rng.uniform(1, 5, 33))
    B2 = np.zeros((33, 33))
    B2[:16, :16] = D[:16, :16] + 0.1
    B2[16:, 16:] = D[16:, 16:] - 0.2
    for A in (D, B2, np.zeros((33, 33)), 7.0 * np.eye(33), np.ones((33, 33)),
              np.diag([3.0, 3.0, 3.0] + [1.0] * 30)):
        w, V = sym_eig_top(A, 3)
        if np.abs(A).max() == 0:
            assert np.all(w == 0) and np.allclose(V.T @ V, np.eye(3))
        else:
            _check_top(A, 3, w, V)


def _scatter_case(rng, K, B, cond=1e2):
    counts = rng.integers(1, 5000, K)
    cm = rng.uniform(800, 3500, (K, B))
    Q, _ = np.linalg.qr(rng.standard_normal((B, B)))
    ev = np.logspace(0, np.log10(cond), B) * 1e4
    Sw = (Q * ev) @ Q.T
    return counts, cm, 0.5 * (Sw + Sw.T)


@pytest.mark.parametrize("K,B", [(2, 3), (3, 16), (4, 23), (8, 33), (5, 4), (12, 5), (40, 33), (3, 64)])
def test_cva_solve_moments_matches_lapack(K, B):
    _lib()
    import oracle
    from paper_1612_06457_amd import cva_solve_moments
    rng = np.random.default_rng(K * 100 + B)
    for cond in (1e1, 1e4):
        counts, cm, Sw = _scatter_case(rng, K, B, cond)
        C = min(K - 1, B)
        W, lam, mean = cva_solve_moments(counts, cm, Sw)
        Sb = oracle.between_scatter(counts, cm)
        lam_r, W_r = oracle.generalized_eig(Sb, Sw)
        W_r = oracle.sign_rule(W_r[:, :C])
        assert np.max(np.abs(lam - lam_r[:C])) <= 1e-10 * lam_r[0]
        assert np.max(np.abs(W.T @ Sw @ W - np.eye(C))) <= 1e-9
        # eigenvectors of distinct eigenvalues agree (sign rule applied on both)
        lr = lam_r[:C + 1] if C < B else np.append(lam_r[:C], -np.inf)
        gaps = np.abs(np.diff(lr)) / lam_r[0]
        for j in range(C):
            lo = gaps[j - 1] if j > 0 else 1.0
            if min(lo, gaps[j]) > 1e-6:
                assert np.max(np.abs(W[:, j] - W_r[:, j])) <= 1e-8 * np.max(np.abs(W_r[:, j]))
        n = counts.astype(float)
        assert np.allclose(mean, (n[:, None] * cm).sum(0) / n.sum(), rtol=1e-14, atol=0)


def test_cva_solve_moments_error_codes():
    L = _lib()
    from paper_1612_06457_amd import cva_solve_moments, CvamxError
    rng = np.random.default_rng(3)
    counts, cm, Sw = _scatter_case(rng, 4, 6)
    Sw2 = Sw.copy()
    Sw2[:, 1] = Sw2[:, 0]
    Sw2[1, :] = Sw2[0, :]
    with pytest.raises(CvamxError) as e:
        cva_solve_moments(counts, cm, Sw2)
    assert e.value.status == L.E_NOT_PD
    c0 = counts.copy()
    c0[2] = 0
    with pytest.raises(CvamxError) as e:
        cva_solve_moments(c0, cm, Sw)
    assert e.value.status == L.E_EMPTY_CLASS
    with pytest.raises(CvamxError) as e:
        cva_solve_moments(counts, cm, Sw, n_comp=4)
    assert e.value.status == L.E_INVALID_ARG
    # a ridge makes a singular S_w solvable
    W, lam, _ = cva_solve_moments(counts, cm, Sw2, ridge=1.0)
    assert np.isfinite(W).all() and (lam >= 0).all()


def test_argument_checks_without_a_device():
    L = _lib()
    lib = L.lib()
    ctx = ctypes.c_void_p()
    assert lib.cvamx_create(ctypes.byref(ctx), -1) == L.OK
    try:
        buf = (ctypes.c_double * 4096)()
        i64 = (ctypes.c_int64 * 128)()
        aligned = ctypes.c_void_p(0x10000)           # never dereferenced: checks come first
        lab = ctypes.c_void_p(0x20000)

        def fit(cube, labels=lab, K=3, prec=0, ridge=0.0, n_comp=2, W=buf):
            return lib.cva_fit(ctx, ctypes.byref(cube) if cube is not None else None, labels, K,
                               prec, ridge, n_comp, W, buf, buf, i64, None, None, None, None)

        good = L.Cube(aligned.value, 16, 16, 8, L.DT_U16)
        assert fit(None) == L.E_INVALID_ARG
        assert fit(L.Cube(None, 16, 16, 8, 0)) == L.E_INVALID_ARG
        assert fit(L.Cube(aligned.value, 0, 16, 8, 0)) == L.E_INVALID_ARG
        assert fit(L.Cube(aligned.value, 16, 16, 65, 0)) == L.E_UNSUPPORTED
        assert fit(L.Cube(aligned.value, 16, 16, 8, 9)) == L.E_UNSUPPORTED
        assert fit(L.Cube(aligned.value + 2, 16, 16, 8, 0)) == L.E_UNSUPPORTED
        assert fit(L.Cube(aligned.value, 1 << 16, 1 << 16, 8, 0)) == L.E_UNSUPPORTED
        assert fit(good, labels=None) == L.E_INVALID_ARG
        assert fit(good, labels=ctypes.c_void_p(0x20001)) == L.E_UNSUPPORTED
        assert fit(good, labels=ctypes.c_void_p(0x20004)) == L.E_UNSUPPORTED
        assert fit(good, K=1) == L.E_INVALID_ARG
        assert fit(good, K=128) == L.E_INVALID_ARG
        assert fit(good, prec=7) == L.E_INVALID_ARG
        assert fit(good, ridge=-1.0) == L.E_INVALID_ARG
        assert fit(good, ridge=float("nan")) == L.E_INVALID_ARG
        assert fit(good, n_comp=3) == L.E_INVALID_ARG
        assert fit(good, n_comp=0) == L.E_INVALID_ARG
        assert fit(good, W=None) == L.E_INVALID_ARG
        assert fit(good) == L.E_DEVICE
        assert b"no device" in lib.cvamx_last_error(ctx)
        # projection
        W = np.zeros((8, 2))
        c = np.zeros(8)
        assert lib.cva_project(ctx, ctypes.byref(good), W.ctypes.data, c.ctypes.data, 0, aligned,
                               None, None) == L.E_INVALID_ARG
        W[0, 0] = np.nan
        assert lib.cva_project(ctx, ctypes.byref(good), W.ctypes.data, c.ctypes.data, 2, aligned,
                               None, None) == L.E_INVALID_ARG
        W[0, 0] = 0
        assert lib.cva_project(ctx, ctypes.byref(good), W.ctypes.data, c.ctypes.data, 2, aligned,
                               None, None) == L.E_DEVICE
        assert lib.cva_fit_project(ctx, ctypes.byref(good), lab, 3, 0, 0.0, 2, buf, buf, buf, i64, None, None,
                                   None) == L.E_INVALID_ARG
        assert lib.cva_fit_project(ctx, ctypes.byref(good), lab, 3, 0, 0.0, 3, buf, buf, buf, i64, aligned, None,
                                   None) == L.E_INVALID_ARG
        assert lib.cva_fit_project(ctx, ctypes.byref(good), lab, 3, 0, 0.0, 2, buf, buf, buf, i64, aligned, None,
                                   None) == L.E_DEVICE
        # CVA and PCA in one call: the checks of both halves
        def both(labels=lab, K=3, n_cva=2, cva_img=aligned, n_pca=3, V=buf, pca_img=aligned):
            return lib.cvamx_cva_pca(ctx, ctypes.byref(good), labels, K, 0, 0.0, n_cva, buf, buf, buf, i64,
                                     cva_img, None, n_pca, V, buf, buf, pca_img, None)
        assert both(K=1) == L.E_INVALID_ARG
        assert both(n_cva=3) == L.E_INVALID_ARG
        assert both(labels=None) == L.E_INVALID_ARG
        assert both(labels=ctypes.c_void_p(0x20004)) == L.E_UNSUPPORTED
        assert both(n_pca=0) == L.E_INVALID_ARG
        assert both(n_pca=9) == L.E_INVALID_ARG
        assert both(V=None) == L.E_INVALID_ARG
        assert both(cva_img=None) == L.E_INVALID_ARG
        assert both(pca_img=None) == L.E_INVALID_ARG
        assert both() == L.E_DEVICE
        assert lib.cvamx_cva_pca(None, ctypes.byref(good), lab, 3, 0, 0.0, 2, buf, buf, buf, i64, aligned, None, 3,
                                 buf, buf, buf, aligned, None) == L.E_INVALID_ARG
        # pca
        assert lib.pca_fit(ctx, ctypes.byref(good), None, 9, 0, buf, buf, buf, None, None) == L.E_INVALID_ARG
        assert lib.pca_fit(ctx, ctypes.byref(good), None, 3, 0, buf, buf, buf, None, None) == L.E_DEVICE
        # soft
        X = ctypes.c_void_p(0x30000)
        assert lib.cva_soft_forward(ctx, X, X, 100, 8, 1, 0, 0.0, buf, buf, buf, buf, buf, None) == L.E_INVALID_ARG
        assert lib.cva_soft_forward(ctx, X, X, 100, 8, 33, 0, 0.0, buf, buf, buf, buf, buf, None) == L.E_INVALID_ARG
        assert lib.cva_soft_forward(ctx, ctypes.c_void_p(0x30004), X, 100, 8, 3, 0, 0.0, buf, buf, buf, buf,
                                    buf, None) == L.E_UNSUPPORTED
        assert lib.cva_soft_forward(ctx, X, X, 100, 8, 3, 0, 0.0, buf, buf, buf, buf, buf, None) == L.E_DEVICE
        assert lib.cva_soft_backward(ctx, X, buf, buf, buf, buf, 100, 8, 3, float("inf"), X, None) == L.E_INVALID_ARG
        assert lib.cva_soft_backward(ctx, X, buf, buf, buf, buf, 100, 8, 3, 1.0, X, None) == L.E_DEVICE
        assert lib.cva_soft_forward(ctx, X, ctypes.c_void_p(0x30008), 100, 8, 3, 0, 0.0, buf, buf, buf, buf,
                                    buf, None) == L.E_UNSUPPORTED
        # fit from a point list
        pts, cls = ctypes.c_void_p(0x40000), ctypes.c_void_p(0x50000)

        def fitp(pixels=pts, classes=cls, N=100, K=3, n_comp=2):
            return lib.cva_fit_points(ctx, ctypes.byref(good), pixels, classes, N, K, 0, 0.0, n_comp,
                                      buf, buf, buf, i64, None, None, None, None)

        assert fitp(pixels=None) == L.E_INVALID_ARG
        assert fitp(classes=None) == L.E_INVALID_ARG
        assert fitp(N=0) == L.E_INVALID_ARG
        assert fitp(N=1 << 31) == L.E_INVALID_ARG
        assert fitp(K=1) == L.E_INVALID_ARG
        assert fitp(n_comp=3) == L.E_INVALID_ARG
        assert fitp(classes=ctypes.c_void_p(0x50008)) == L.E_UNSUPPORTED
        assert fitp(pixels=ctypes.c_void_p(0x40004)) == L.E_UNSUPPORTED
        assert fitp() == L.E_DEVICE
        # float images, rescaling, colour
        assert lib.cvamx_project_float(ctx, ctypes.byref(good), W.ctypes.data, c.ctypes.data, 2, None,
                                       None) == L.E_INVALID_ARG
        assert lib.cvamx_project_float(ctx, ctypes.byref(good), W.ctypes.data, c.ctypes.data, 2,
                                       ctypes.c_void_p(0x10002), None) == L.E_UNSUPPORTED
        assert lib.cvamx_project_float(ctx, ctypes.byref(good), W.ctypes.data, c.ctypes.data, 2, aligned,
                                       None) == L.E_DEVICE
        y, out, tp = ctypes.c_void_p(0x60000), ctypes.c_void_p(0x70000), ctypes.c_void_p(0x80000)

        def st(y=y, P=256, n=2, mode=1, pct=1.0, train=None, n_train=0, bits=8, out=out):
            return lib.cvamx_stretch(ctx, y, P, n, mode, pct, train, n_train, bits, out, None, None)

        assert st(y=None) == L.E_INVALID_ARG
        assert st(out=None) == L.E_INVALID_ARG
        assert st(P=0) == L.E_INVALID_ARG
        assert st(n=0) == L.E_INVALID_ARG
        assert st(n=65) == L.E_INVALID_ARG
        assert st(mode=0) == L.E_INVALID_ARG
        assert st(mode=4) == L.E_INVALID_ARG
        assert st(bits=12) == L.E_INVALID_ARG
        assert st(mode=2) == L.E_INVALID_ARG                      # no pixel list
        assert st(mode=2, train=tp, n_train=0) == L.E_INVALID_ARG
        assert st(mode=3, pct=50.0) == L.E_INVALID_ARG
        assert st(mode=3, pct=-0.5) == L.E_INVALID_ARG
        assert st(mode=3, pct=float("nan")) == L.E_INVALID_ARG
        assert st(y=ctypes.c_void_p(0x60002)) == L.E_UNSUPPORTED
        assert st(bits=16, out=ctypes.c_void_p(0x70001)) == L.E_UNSUPPORTED
        assert st(mode=2, train=ctypes.c_void_p(0x80004), n_train=5) == L.E_UNSUPPORTED
        assert st(mode=2, train=tp, n_train=5) == L.E_DEVICE
        assert st(mode=3, pct=0.0) == L.E_DEVICE
        assert st(bits=16, out=ctypes.c_void_p(0x70002)) == L.E_DEVICE
        assert lib.cvamx_compose_rgb(ctx, y, y, y, 10, None, None) == L.E_INVALID_ARG
        assert lib.cvamx_compose_rgb(ctx, y, y, y, 0, out, None) == L.E_INVALID_ARG
        assert lib.cvamx_compose_rgb(ctx, None, y, None, 10, out, None) == L.E_DEVICE
        # cluster indices
        sc = np.empty(2)

        def ci(img=y, dt=L.DT_U8, P=64, n=1, pix=pts, cl=cls, N=10, K=2, p=2.0, scores=sc.ctypes.data):
            return lib.cvamx_cluster_indices(ctx, img, dt, P, n, pix, cl, N, K, p, None, None, None, None, None,
                                             scores, None)

        assert ci(img=None) == L.E_INVALID_ARG
        assert ci(scores=None) == L.E_INVALID_ARG
        assert ci(dt=9) == L.E_UNSUPPORTED
        assert ci(P=0) == L.E_INVALID_ARG
        assert ci(n=0) == L.E_INVALID_ARG
        assert ci(N=0) == L.E_INVALID_ARG
        assert ci(K=1) == L.E_INVALID_ARG
        assert ci(p=0.5) == L.E_INVALID_ARG
        assert ci(p=float("inf")) == L.E_INVALID_ARG
        assert ci(dt=L.DT_F32, img=ctypes.c_void_p(0x60002)) == L.E_UNSUPPORTED
        assert ci(pix=ctypes.c_void_p(0x40004)) == L.E_UNSUPPORTED
        assert ci(cl=ctypes.c_void_p(0x50008)) == L.E_UNSUPPORTED
        assert ci(img=ctypes.c_void_p(0x60001)) == L.E_DEVICE          # bytes need no alignment
        # the plain FP32 switch is host-only
        assert lib.cvamx_set_plain_fp32(None, 1) == L.E_INVALID_ARG
        assert lib.cvamx_set_plain_fp32(ctx, 1) == L.OK
        assert lib.cvamx_set_plain_fp32(ctx, 0) == L.OK
        assert lib.cvamx_set_pca_standardize(None, 1) == L.E_INVALID_ARG
        assert lib.cvamx_set_pca_standardize(ctx, 1) == L.OK
        assert lib.cvamx_set_pca_standardize(ctx, 0) == L.OK
        # class index lists
        off = (ctypes.c_int32 * 129)()
        ix = ctypes.c_void_p(0xa0000)

        def li(labels=lab, n=100, K=3, idx=ix, counts=i64, offsets=off):
            return lib.cvamx_label_index(ctx, labels, n, K, idx, counts, offsets, None)

        assert li(labels=None) == L.E_INVALID_ARG
        assert li(idx=None) == L.E_INVALID_ARG
        assert li(counts=None) == L.E_INVALID_ARG
        assert li(offsets=None) == L.E_INVALID_ARG
        assert li(n=0) == L.E_INVALID_ARG
        assert li(n=1 << 31) == L.E_INVALID_ARG
        assert li(K=0) == L.E_INVALID_ARG
        assert li(K=128) == L.E_INVALID_ARG
        assert li(labels=ctypes.c_void_p(0x20008)) == L.E_UNSUPPORTED
        assert li(idx=ctypes.c_void_p(0xa0002)) == L.E_UNSUPPORTED
        assert li(K=1) == L.E_DEVICE
        assert li(K=127) == L.E_DEVICE
        # band images and page batches
        cb = ctypes.c_void_p(0x90000)
        assert lib.cvamx_bands_to_cube(ctx, None, L.DT_U8, 8, 64, cb, None) == L.E_INVALID_ARG
        assert lib.cvamx_bands_to_cube(ctx, y, L.DT_BF16, 8, 64, cb, None) == L.E_UNSUPPORTED
        assert lib.cvamx_bands_to_cube(ctx, y, L.DT_U8, 65, 64, cb, None) == L.E_INVALID_ARG
        assert lib.cvamx_bands_to_cube(ctx, y, L.DT_U8, 8, 0, cb, None) == L.E_INVALID_ARG
        assert lib.cvamx_bands_to_cube(ctx, ctypes.c_void_p(0x60001), L.DT_U16, 8, 64, cb, None) == L.E_UNSUPPORTED
        assert lib.cvamx_bands_to_cube(ctx, y, L.DT_U8, 8, 64, ctypes.c_void_p(0x90008), None) == L.E_UNSUPPORTED
        assert lib.cvamx_bands_to_cube(ctx, ctypes.c_void_p(0x60001), L.DT_U8, 8, 64, cb, None) == L.E_DEVICE
        pg = (L.Page * 2)()

        def rp(dt=L.DT_U8, B=8, H=16, W=16, K=3, n_comp=2, mode=1, bits=8, pages=pg, n=2):
            return lib.cvamx_run_pages(ctx, dt, B, H, W, K, n_comp, 0, 0.0, mode, 1.0, bits, pages, n, None)

        assert rp(pages=None) == L.E_INVALID_ARG
        assert rp(n=0) == L.E_INVALID_ARG
        assert rp(dt=L.DT_F16) == L.E_UNSUPPORTED
        assert rp(B=0) == L.E_INVALID_ARG
        assert rp(H=0) == L.E_INVALID_ARG
        assert rp(K=1) == L.E_INVALID_ARG
        assert rp(n_comp=3) == L.E_INVALID_ARG
        assert rp(mode=5) == L.E_INVALID_ARG
        assert rp(bits=4) == L.E_INVALID_ARG
        assert rp() == L.E_DEVICE
        # reference streams
        sk = ctypes.c_void_p(0xb0000)
        a16, b16 = ctypes.c_void_p(0xc0000), ctypes.c_void_p(0xd0000)
        assert lib.cvamx_stream_read(ctx, None, 64, sk, None) == L.E_INVALID_ARG
        assert lib.cvamx_stream_read(ctx, a16, 8, sk, None) == L.E_INVALID_ARG
        assert lib.cvamx_stream_read(ctx, ctypes.c_void_p(0xc0008), 64, sk, None) == L.E_UNSUPPORTED
        assert lib.cvamx_stream_read(ctx, a16, 64, sk, None) == L.E_DEVICE
        assert lib.cvamx_stream_mix(ctx, a16, 64, None, 16, sk, None) == L.E_INVALID_ARG
        assert lib.cvamx_stream_mix(ctx, a16, 64, b16, 0, sk, None) == L.E_INVALID_ARG
        assert lib.cvamx_stream_mix(ctx, a16, 64, b16, 24, sk, None) == L.E_INVALID_ARG
        assert lib.cvamx_stream_mix(ctx, a16, 64, b16, 80, sk, None) == L.E_INVALID_ARG
        assert lib.cvamx_stream_mix(ctx, a16, 64, ctypes.c_void_p(0xd0004), 16, sk, None) == L.E_UNSUPPORTED
        assert lib.cvamx_stream_mix(ctx, a16, 64, b16, 64, sk, None) == L.E_DEVICE
    finally:
        lib.cvamx_destroy(ctx)
    assert lib.cvamx_status_str(L.E_NOT_PD) == b"within-class scatter not positive definite"
