"""GPU parity: the HIP path through the C ABI against the FP64 oracle, on the
same seeded inputs.

Tolerances (FP32 path): class counts bit-exact; S_w, S_b within 1e-5 of the
largest entry; eigenvalues within 1e-5 relative; sign-aligned canonical
vectors within 1e-4; projection ranges within 1e-4 of b - a; 8-bit images
within one grey level.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_case, make_soft_case, to_half_cube
from tests._cases import full_page
from tests._parity import (TOL_LAM, TOL_S, TOL_Y, check_cva_vectors, check_images, check_pca_vectors,
                           check_vectors, rel_max)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_06457_amd  # noqa: F401  (raises if the library is missing)
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    if hasattr(a, "to"):
        return a.contiguous().to(dev)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _fit_parity(cube_host, labels, K, dev, ridge=0.0):
    import paper_1612_06457_amd as cx
    ref = oracle.cva_fit(cube_host, labels, K, ridge=ridge)
    got = cx.cva_fit(_t(cube_host, dev), _t(labels, dev), K, ridge=ridge)
    assert got.counts.tolist() == ref["counts"].tolist()
    assert rel_max(got.class_means, ref["class_means"]) <= 1e-7
    assert rel_max(got.Sw, ref["Sw"]) <= TOL_S
    assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    signs, _ = check_cva_vectors(got.W, ref, ridge=ridge)
    assert rel_max(got.mean, ref["mean"]) <= 1e-7
    return ref, got, signs


def _project_parity(cube_host, W, center, dev, signs=None):
    import paper_1612_06457_amd as cx
    q_ref, ab_ref = oracle.cva_project(cube_host, W, center)
    q, ab = cx.cva_project(_t(cube_host, dev), W, center, return_range=True)
    q = q.cpu().numpy()
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    frac = check_images(q, q_ref, None)
    return q, q_ref, frac


# ------------------------------------------------------------------ workloads

def test_page_512x512x16_fit_and_project(dev):
    say("512x512x16 u16 page, K=3")
    c = make_case(1)
    ref, got, signs = _fit_parity(c.cube, c.labels, c.K, dev)
    # projection with the oracle's own vectors isolates the projection kernel
    _project_parity(c.cube, ref["W"], ref["mean"], dev)
    # end to end: the GPU fit's vectors, compared after sign alignment
    import paper_1612_06457_amd as cx
    q = cx.cva_project(_t(c.cube, dev), got.W, got.mean).cpu().numpy()
    q_ref, _ = oracle.cva_project(c.cube, ref["W"], ref["mean"])
    frac = check_images(q, q_ref, signs)
    say(f"512x512x16 page: differing bytes {frac:.2e}")


def test_page_4096x4096x23_structure_scaled_cva_and_pca(dev):
    say("4096x4096x23 page structure at 1024x1024x23 u16, K=4")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.25)
    ref, got, signs = _fit_parity(c.cube, c.labels, c.K, dev)
    _project_parity(c.cube, ref["W"], ref["mean"], dev)
    pr = oracle.pca_fit(c.cube, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(_t(c.cube, dev), n_comp=3)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert np.max(np.abs(lam - pr["eigvals"]) / pr["eigvals"]) <= TOL_LAM
    assert rel_max(mean, pr["mean"]) <= 1e-9
    s, _ = check_pca_vectors(V, pr)
    _project_parity(c.cube, pr["V"], pr["mean"], dev)


@pytest.mark.parametrize("H,W,B,K", [
    (37, 53, 7, 3), (5, 7, 3, 2), (64, 64, 16, 4), (33, 31, 33, 5), (40, 41, 64, 3),
    (19, 23, 1, 2), (50, 50, 2, 3), (128, 96, 23, 8), (3, 300, 9, 2)])
def test_shapes_and_ragged_tails(dev, H, W, B, K):
    say(f"shape H={H} W={W} B={B} K={K}")
    rng = np.random.default_rng(H * 1000 + W * 10 + B)
    mu = rng.uniform(800, 3500, (K, B))
    cls = rng.integers(0, K, H * W)
    cube = np.clip(np.rint(mu[cls] + rng.normal(0, 60, (H * W, B))), 0, 4095).astype(np.uint16)
    cube = cube.reshape(H, W, B)
    lab = np.where(rng.random(H * W) < 0.5, cls, -1).astype(np.int8)
    for k in range(K):                         # at least B + 2 pixels per class
        idx = np.flatnonzero(cls == k)
        if idx.size < B + 2:
            extra = rng.choice(H * W, B + 2, replace=False)
            cls[extra] = k
            cube.reshape(-1, B)[extra] = np.clip(np.rint(mu[k] + rng.normal(0, 60, (B + 2, B))), 0, 4095)
            idx = extra
        lab[idx[: B + 2]] = k
    labels = lab.reshape(H, W)
    ref, got, signs = _fit_parity(cube, labels, K, dev)
    _project_parity(cube, ref["W"], ref["mean"], dev)


def test_fit_project_in_one_call(dev):
    say("cva_fit_project equals cva_fit then cva_project")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.5)
    cube, labels = _t(c.cube, dev), _t(c.labels, dev)
    q1, fit1, r1 = cx.cva_fit_project(cube, labels, c.K, return_range=True)
    fit0 = cx.cva_fit(cube, labels, c.K)
    q0, r0 = cx.cva_project(cube, fit0.W, fit0.mean, return_range=True)
    assert np.array_equal(fit1.W, fit0.W) and np.array_equal(fit1.eigvals, fit0.eigvals)
    assert np.array_equal(fit1.counts, fit0.counts) and np.array_equal(fit1.mean, fit0.mean)
    assert np.array_equal(q1.cpu().numpy(), q0.cpu().numpy()) and np.array_equal(r1, r0)
    q2, _ = cx.cva_fit_project(cube, labels, c.K, n_comp=1)
    assert np.array_equal(q2.cpu().numpy()[0], q0.cpu().numpy()[0])


def test_single_pixel_class(dev):
    say("class with one training pixel")
    c = make_case(1, scale=0.25)
    lab = c.labels.copy()
    k2 = np.flatnonzero(lab.reshape(-1) == 2)
    lab.reshape(-1)[k2[1:]] = -1
    _fit_parity(c.cube, lab, 3, dev)


@pytest.mark.parametrize("kind", ["f32", "bf16", "f16"])
def test_float_pages(dev, kind):
    say(f"float page {kind}")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.12)
    if kind == "f32":
        cube = c.cube.astype(np.float32) / np.float32(4095.0)
    else:
        cube = to_half_cube(c.cube, kind)
    host = cube if kind == "f32" else cube.float().numpy()
    ref = oracle.cva_fit(host, c.labels, c.K)
    got = cx.cva_fit(_t(cube, dev), _t(c.labels, dev), c.K)
    assert got.counts.tolist() == ref["counts"].tolist()
    assert rel_max(got.Sw, ref["Sw"]) <= TOL_S
    assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    check_cva_vectors(got.W, ref)
    q_ref, ab_ref = oracle.cva_project(host, ref["W"], ref["mean"])
    q, ab = cx.cva_project(_t(cube, dev), ref["W"], ref["mean"], return_range=True)
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    check_images(q.cpu().numpy(), q_ref)
    pr = oracle.pca_fit(host, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(_t(cube, dev), n_comp=3)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    check_pca_vectors(V, pr)


def test_pca_mask(dev):
    say("pca with mask")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.5)
    rng = np.random.default_rng(7)
    mask = (rng.random((c.H, c.W)) < 0.3).astype(np.uint8)
    pr = oracle.pca_fit(c.cube, mask=mask, n_comp=4)
    V, lam, mean, cov = cx.pca_fit(_t(c.cube, dev), mask=_t(mask, dev), n_comp=4)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert rel_max(mean, pr["mean"]) <= 1e-9
    check_pca_vectors(V, pr)


@pytest.mark.parametrize("case,dtype,masked,prec", [
    (1, "u16", False, "fp32"), (1, "u16", True, "fp32"), (2, "u16", False, "fp32"), (2, "f32", False, "fp32"),
    (2, "bf16", False, "bf16x3"), (1, "u16", False, "plain")])
def test_pca_standardized(dev, case, dtype, masked, prec):
    """Standardised PCA (the bands scaled to unit variance over the selected
    pixels) against the oracle: the correlation eigenvalues, the projection
    vectors D^-1/2 u checked through C v = lambda D v and v^T D v = 1 (every
    column) and against the oracle's vectors where the eigenvalues are
    apart, and the images of pca_project with the oracle's vectors, within
    one level."""
    say(f"standardised pca: config {case} {dtype} masked={masked} {prec}")
    import paper_1612_06457_amd as cx
    c = make_case(case, scale=0.5 if case == 1 else 0.08)
    if dtype == "u16":
        host, dcube = c.cube, _t(c.cube, dev)
    elif dtype == "f32":
        host = (c.cube.astype(np.float32) / 4095.0).astype(np.float32)
        dcube = _t(host, dev)
    else:
        half = to_half_cube(c.cube, dtype)
        host, dcube = half.float().numpy(), half.contiguous().to(dev)
    rng = np.random.default_rng(case)
    mask = (rng.random((c.H, c.W)) < 0.5).astype(np.uint8) if masked else None
    pr = oracle.pca_fit(host, mask=mask, n_comp=3, standardize=True)
    cx.set_plain_fp32(prec == "plain")
    try:
        V, lam, mean, cov = cx.pca_fit(dcube, mask=None if mask is None else _t(mask, dev), n_comp=3,
                                       precision="fp32" if prec == "plain" else prec, standardize=True)
    finally:
        cx.set_plain_fp32(False)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert np.max(np.abs(lam - pr["eigvals"]) / pr["eigvals"]) <= TOL_LAM
    check_vectors(V, pr["V"], pr["eigvals"], A_ref=pr["cov"], M_ref=pr["metric"], lam_next=pr["all_eigvals"][3])
    # the oracle's projection vectors through the device projection
    q = cx.pca_project(dcube, pr["V"], pr["mean"]).cpu().numpy()
    q_ref, _ = oracle.pca_project(host, pr["V"], pr["mean"])
    check_images(q, q_ref)
    # and the default stays covariance PCA
    V0, lam0, _, _ = cx.pca_fit(dcube, mask=None if mask is None else _t(mask, dev), n_comp=3,
                                precision="fp32" if prec == "plain" else prec)
    p0 = oracle.pca_fit(host, mask=mask, n_comp=3)
    assert np.max(np.abs(lam0 - p0["eigvals"]) / p0["eigvals"]) <= TOL_LAM


def test_pca_standardized_zero_variance_band(dev):
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(5)
    cube = rng.integers(0, 4096, (40, 30, 6)).astype(np.uint16)
    cube[:, :, 2] = 1234
    with pytest.raises(cx.CvamxError):
        cx.pca_fit(_t(cube, dev), n_comp=2, standardize=True)
    V, lam, _, _ = cx.pca_fit(_t(cube, dev), n_comp=2)   # covariance PCA is fine
    assert lam[0] > 0


@pytest.mark.parametrize("H,W,B,masked", [
    (61, 67, 33, False), (29, 31, 64, False), (17, 19, 5, False), (40, 40, 16, True), (45, 47, 47, True)])
def test_pca_u16_full_range(dev, H, W, B, masked):
    """uint16 values over the whole 16-bit range (two populations, near 0
    and near 65535, so both bytes of a value take every size).  The page
    covariance of a uint16 page is built from exact integer sums, so it
    matches the FP64 oracle to rounding."""
    say(f"pca full 16-bit range H={H} W={W} B={B} masked={masked}")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(H * 100 + B)
    hi = rng.random(H * W) < 0.4
    mu = np.where(hi[:, None], rng.uniform(60000, 65000, B), rng.uniform(50, 3000, B))
    cube = np.clip(np.rint(mu + rng.normal(0, 900, (H * W, B))), 0, 65535).astype(np.uint16).reshape(H, W, B)
    mask = (rng.random((H, W)) < 0.6).astype(np.uint8) if masked else None
    pr = oracle.pca_fit(cube, mask=mask, n_comp=2)
    V, lam, mean, cov = cx.pca_fit(_t(cube, dev), mask=None if mask is None else _t(mask, dev), n_comp=2)
    assert rel_max(cov, pr["cov"]) <= 1e-11
    assert rel_max(mean, pr["mean"]) <= 1e-12
    check_pca_vectors(V, pr)


def test_many_components_and_groups(dev):
    say("projection with 11 components (two groups)")
    rng = np.random.default_rng(3)
    cube = rng.integers(0, 4096, (61, 47, 23)).astype(np.uint16)
    W = rng.standard_normal((23, 11))
    center = rng.uniform(1000, 3000, 23)
    _project_parity(cube, W, center, dev)


def test_errors(dev):
    say("error paths")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.2)
    cube = _t(c.cube, dev)
    bad = c.labels.copy()
    bad[0, 0] = 5
    with pytest.raises(cx.CvamxError) as e:
        cx.cva_fit(cube, _t(bad, dev), 3)
    assert e.value.status == -1
    lab = c.labels.copy()
    lab[lab == 1] = -1
    with pytest.raises(cx.CvamxError) as e:
        cx.cva_fit(cube, _t(lab, dev), 3)
    assert e.value.status == -3
    dup = c.cube.copy()
    dup[..., 5] = dup[..., 4]
    with pytest.raises(cx.CvamxError) as e:
        cx.cva_fit(_t(dup, dev), _t(c.labels, dev), 3)
    assert e.value.status == -4
    # the library still works after errors
    _fit_parity(c.cube, c.labels, 3, dev)


def test_repeatable(dev):
    say("bitwise repeatability")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.1)
    cube, lab = _t(c.cube, dev), _t(c.labels, dev)
    a = cx.cva_fit(cube, lab, c.K)
    b = cx.cva_fit(cube, lab, c.K)
    assert np.array_equal(a.W, b.W) and np.array_equal(a.Sw, b.Sw)
    qa, ra = cx.cva_project(cube, a.W, a.mean, return_range=True)
    qb, rb = cx.cva_project(cube, a.W, a.mean, return_range=True)
    assert np.array_equal(ra, rb)
    assert bool((qa == qb).all())
    p1 = cx.pca_fit(cube, n_comp=3)
    p2 = cx.pca_fit(cube, n_comp=3)
    assert np.array_equal(p1[3], p2[3])


# ------------------------------------------------------ fit from point lists

def _points(c, rng, n_dup=500, n_skip=37):
    """The labelled pixels of a case as a shuffled point list, with some
    points listed twice and some entries marked -1."""
    flat = c.labels.reshape(-1)
    pix = np.flatnonzero(flat >= 0)
    cls = flat[pix]
    order = rng.permutation(pix.size)
    dup = rng.choice(pix.size, size=n_dup, replace=False)
    skip = rng.integers(0, flat.size, size=n_skip)
    pts = np.concatenate([pix[order], pix[dup], skip]).astype(np.int64)
    cl = np.concatenate([cls[order], cls[dup], np.full(n_skip, -1)]).astype(np.int8)
    return pts, cl


@pytest.mark.parametrize("cfg,scale", [(1, 1.0), (5, 0.05)])
def test_fit_points(dev, cfg, scale):
    say(f"fit from a point list, cfg{cfg} at scale {scale}")
    import paper_1612_06457_amd as cx
    c = make_case(cfg, scale=scale)
    pts, cl = _points(c, np.random.default_rng(cfg))
    ref = oracle.cva_fit_points(c.cube, pts, cl, c.K)
    got = cx.cva_fit_points(_t(c.cube, dev), _t(pts, dev), _t(cl, dev), c.K)
    assert got.counts.tolist() == ref["counts"].tolist()
    assert rel_max(got.class_means, ref["class_means"]) <= 1e-7
    assert rel_max(got.Sw, ref["Sw"]) <= TOL_S
    assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    check_cva_vectors(got.W, ref)


def test_fit_points_errors(dev):
    say("fit from a point list: errors")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.2)
    pts, cl = _points(c, np.random.default_rng(3), n_dup=10, n_skip=5)
    cube = _t(c.cube, dev)
    out = pts.copy()
    out[7] = c.H * c.W                       # one past the last pixel
    with pytest.raises(cx.CvamxError) as e:
        cx.cva_fit_points(cube, _t(out, dev), _t(cl, dev), c.K)
    assert e.value.status == -1
    badc = cl.copy()
    badc[3] = c.K
    with pytest.raises(cx.CvamxError) as e:
        cx.cva_fit_points(cube, _t(pts, dev), _t(badc, dev), c.K)
    assert e.value.status == -1
    # a class that no entry names
    none = cl.copy()
    none[none == 2] = -1
    with pytest.raises(cx.CvamxError) as e:
        cx.cva_fit_points(cube, _t(pts, dev), _t(none, dev), c.K)
    assert e.value.status == -3


# ---------------------------------------------------------------- soft label

def _soft_parity(X, w, dev, gtol=1e-4):
    import paper_1612_06457_amd as cx
    ref = oracle.soft_fit(X, w)
    g_ref = oracle.soft_grad(X, w)
    Xd, wd = _t(X, dev), _t(w, dev)
    fit = cx.cva_soft_forward(Xd, wd)
    assert abs(fit.J - ref["J"]) <= TOL_LAM * ref["J"]
    assert np.max(np.abs(fit.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    check_cva_vectors(fit.W, ref)
    g = cx.cva_soft_backward(Xd, fit, 1.0, w.shape[1]).cpu().numpy()
    gmax = np.max(np.abs(g_ref))
    assert np.max(np.abs(g - g_ref)) <= gtol * gmax
    return fit, g, g_ref


def test_soft_label_small(dev):
    say("soft-label CVA, 1M x 23 structure at 1/16 scale")
    X, w, cls, idx, case = make_soft_case(4, scale=0.25)
    _soft_parity(X, w, dev)


def test_soft_label_one_hot_equals_hard_fit(dev):
    say("soft-label with one-hot weights")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.5)
    flat = c.labels.reshape(-1)
    idx = np.flatnonzero(flat >= 0)
    X = c.cube.reshape(-1, c.B)[idx].astype(np.float32)
    w = np.zeros((idx.size, c.K), np.float32)
    w[np.arange(idx.size), flat[idx]] = 1
    fit = cx.cva_soft_forward(_t(X, dev), _t(w, dev))
    hard = cx.cva_fit(_t(c.cube, dev), _t(c.labels, dev), c.K)
    assert abs(fit.J - hard.eigvals.sum()) <= 1e-5 * fit.J


def test_soft_label_autograd(dev):
    say("SoftCVA autograd")
    import torch
    import paper_1612_06457_amd as cx
    X, w, cls, idx, case = make_soft_case(4, scale=0.1)
    Xd = _t(X, dev)
    wd = _t(w, dev).requires_grad_(True)
    J = cx.SoftCVA.apply(Xd, wd)
    (2.5 * J).backward()
    fit = cx.cva_soft_forward(Xd, wd.detach())
    g = cx.cva_soft_backward(Xd, fit, 2.5, w.shape[1])
    assert torch.allclose(wd.grad, g, rtol=0, atol=1e-6 * float(g.abs().max()))
    assert abs(float(J.detach()) - fit.J) <= 1e-12 * fit.J


@pytest.mark.parametrize("N,B,K,xs,ws,neg", [
    (1000, 23, 5, 1.0, 1.0, False), (100, 7, 3, 1.0, 1.0, False), (5000, 64, 32, 1.0, 1.0, False),
    (3000, 1, 2, 1.0, 1.0, False), (4000, 33, 8, 1e5, 1e3, False), (4000, 33, 8, 1e-4, 1e-3, False),
    (6000, 16, 4, 1.0, 1.0, True), (2000, 17, 3, 1.0, 1.0, False), (3000, 32, 6, 1.0, 1.0, True),
    (2500, 48, 5, 1.0, 1.0, False), (2500, 49, 9, 1.0, 1.0, False), (4000, 33, 12, 1.0, 1.0, True),
    (1001, 7, 3, 1.0, 1.0, False), (4003, 33, 11, 1.0, 1.0, False)])
def test_soft_label_shapes_and_scales(dev, N, B, K, xs, ws, neg):
    """Ragged and short row counts, every row-block count, the band counts
    whose one or two trailing columns run on the vector ALU (16, 17, 32, 33,
    48, 49, 64), class groups that leave waves idle, values far outside the
    fp16 range either way, and weights of both signs: J, eigenvalues, class
    means, W^T S_w W = I against the oracle's S_w, and the whole gradient
    against the oracle's closed form, including C = 11 and C = 31, whose
    backward runs as two and four accumulating launches; and last tiles whose
    gradients end inside a 16-byte store (1001 x 3, 4003 x 11)."""
    say(f"soft-label N={N} B={B} K={K} x*{xs} w*{ws} neg={neg}")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(N + B + K)
    mu = rng.uniform(800, 3500, (K, B))
    cls = np.arange(N) % K
    X = (mu[cls] + rng.normal(0, 60, (N, B))) * xs
    w = rng.dirichlet(np.full(K, 0.5), N)
    w = 0.5 * w + 0.5 * np.eye(K)[cls]
    if neg:
        flip = rng.random(N) < 0.1
        w[flip] -= 0.05
    w = w * ws
    X, w = X.astype(np.float32), w.astype(np.float32)
    ref = oracle.soft_fit(X, w)
    fit = cx.cva_soft_forward(_t(X, dev), _t(w, dev))
    assert abs(fit.J - ref["J"]) <= TOL_LAM * ref["J"]
    assert np.max(np.abs(fit.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    assert rel_max(fit.class_means, ref["class_means"]) <= 1e-6
    check_cva_vectors(fit.W, ref)
    G = fit.W.T @ ref["Sw"] @ fit.W
    assert np.max(np.abs(G - np.eye(G.shape[0]))) <= 1e-5
    # the gradient; C = min(K - 1, B) above 8 runs in several launches of
    # eight components that accumulate into dw
    g = cx.cva_soft_backward(_t(X, dev), fit, 1.0, K).cpu().numpy()
    g_ref = oracle.soft_grad(X, w)
    gerr = np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))
    say(f"  gradient error {gerr:.2e} of max |dJ/dw| (C = {min(K - 1, B)})")
    assert gerr <= 1e-4


# ------------------------------------------------------------ full sizes

@pytest.mark.timeout(900)
def test_full_page_7216x5412x33(dev):
    """7216 x 5412 x 33 uint16 page, K = 8, 200k training pixels per class:
    fit parity, every pixel of the 7 projected images, and PCA."""
    say("full page 7216x5412x33 u16 K=8")
    import paper_1612_06457_amd as cx
    c = full_page()
    say("page generated")
    ref, got, signs = _fit_parity(c.cube, c.labels, c.K, dev)
    say("fit ok", got.eigvals)
    cube = _t(c.cube, dev)
    q, ab = cx.cva_project(cube, ref["W"], ref["mean"], return_range=True)
    q = q.cpu().numpy()
    q_ref, ab_ref = oracle.cva_project(c.cube, ref["W"], ref["mean"])
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    frac = check_images(q, q_ref)
    say(f"project ok, differing bytes {frac:.2e}")
    del q, q_ref
    pr = oracle.pca_fit(c.cube, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(cube, n_comp=3)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert np.max(np.abs(lam - pr["eigvals"]) / pr["eigvals"]) <= TOL_LAM
    check_pca_vectors(V, pr)
    say("pca ok")


@pytest.mark.timeout(900)
def test_full_page_4096x4096x23_u16(dev):
    """The FP32 CVA + PCA workload at full size: 4096 x 4096 x 23 uint16,
    four classes of 50,000 training pixels (parchment, over-, under-text and
    both).  The fit against the oracle; every pixel of the three CVA images,
    from the oracle's vectors and end to end from the device's own fit; the
    PCA covariance and vectors; every pixel of the three PCA images."""
    say("full page 4096x4096x23 u16 K=4")
    import paper_1612_06457_amd as cx
    c = make_case(2, threads=16)
    say("page generated")
    ref, got, signs = _fit_parity(c.cube, c.labels, c.K, dev)
    say("fit ok", got.eigvals)
    cube = _t(c.cube, dev)
    q_ref, ab_ref = oracle.cva_project(c.cube, ref["W"], ref["mean"])
    q, ab = cx.cva_project(cube, ref["W"], ref["mean"], return_range=True)
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    frac = check_images(q.cpu().numpy(), q_ref)
    say(f"cva project ok, differing bytes {frac:.2e}")
    q1, fit1 = cx.cva_fit_project(cube, _t(c.labels, dev), c.K)
    assert np.array_equal(fit1.W, got.W)
    frac = check_images(q1.cpu().numpy(), q_ref, signs)
    say(f"cva fit + project end to end ok, differing bytes {frac:.2e}")
    del q, q1, q_ref
    pr = oracle.pca_fit(c.cube, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(cube, n_comp=3)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert np.max(np.abs(lam - pr["eigvals"]) / pr["eigvals"]) <= TOL_LAM
    assert rel_max(mean, pr["mean"]) <= 1e-9
    check_pca_vectors(V, pr)
    q_ref, ab_ref = oracle.cva_project(c.cube, pr["V"], pr["mean"])
    q, ab = cx.pca_project(cube, pr["V"], pr["mean"], return_range=True)
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    frac = check_images(q.cpu().numpy(), q_ref)
    say(f"pca ok, differing bytes {frac:.2e}")


@pytest.mark.timeout(600)
def test_full_soft_1M_x23(dev):
    """1,000,000 x 23 float32 training pixels, K = 5, Dirichlet(0.5) weights
    near class borders: J, gradient against the closed form, and central
    differences of the exact finite change on 64 random pixels."""
    say("soft label 1M x 23, K=5")
    X, w, cls, idx, case = make_soft_case(4)
    fit, g, g_ref = _soft_parity(X, w, dev)
    rng = np.random.default_rng(4)
    gmax = np.max(np.abs(g_ref))
    h = 1e-3
    mom = oracle.soft_moments(X, w)
    for _ in range(64):
        p = int(rng.integers(0, X.shape[0]))
        k = int(rng.integers(0, w.shape[1]))
        fd = (oracle.soft_delta_J(X, w, p, k, h, mom) - oracle.soft_delta_J(X, w, p, k, -h, mom)) / (2 * h)
        assert abs(g[p, k] - fd) <= 1e-4 * gmax


@pytest.mark.timeout(900)
def test_full_soft_page_1600k_x33(dev):
    """The soft-label workload of the benchmark: the 1.6 M training pixels
    of the 7216 x 5412 x 33 page (K = 8), Dirichlet(0.5) weights within two
    pixels of a class border and one-hot weights inside, in the launch shape
    the benchmark uses (33 bands: the last band and the ones column on the
    vector ALU).  J, eigenvalues, vectors and the whole gradient."""
    say("soft label, full page training pixels 1.6M x 33, K=8")
    from synth import border_map, soft_weights
    c = full_page()
    flat = c.labels.reshape(-1)
    idx = np.flatnonzero(flat >= 0)
    cls = flat[idx].astype(np.int64)
    rng = np.random.default_rng([c.seed, 0x50F7])
    nb = border_map(c.class_map)[np.unravel_index(idx, c.labels.shape)]
    w = soft_weights(cls, nb, c.K, rng)
    X = c.cube.reshape(-1, c.B)[idx].astype(np.float32)
    say(f"N={X.shape[0]}")
    _soft_parity(X, w, dev)


# ------------------------------------------------- compensated MFMA scatter

def _abs_gram(cube_host, labels, K):
    """sum over training pixels of |x_i - m_ki| |x_j - m_kj| (FP64), the
    scale of the a-priori rounding bound of a scatter entry."""
    from oracle.cva import _rows
    X = _rows(cube_host).astype(np.float64)
    lab = np.asarray(labels).reshape(-1)
    B = X.shape[1]
    A = np.zeros((B, B))
    for k in range(K):
        D = np.abs(X[lab == k] - X[lab == k].mean(0))
        A += D.T @ D
    return A


def _mixed_fit_check(cube_dev, cube_host, labels, K, dev, prec, rel):
    import paper_1612_06457_amd as cx
    ref = oracle.cva_fit(cube_host, labels, K)
    got = cx.cva_fit(cube_dev, _t(labels, dev), K, precision=prec)
    assert got.counts.tolist() == ref["counts"].tolist()
    bound = rel * _abs_gram(cube_host, labels, K)
    err = np.abs(got.Sw - ref["Sw"])
    worst = float(np.max(err / bound))
    say(f"{prec}: S_w error / stated bound = {worst:.3f}, max rel {rel_max(got.Sw, ref['Sw']):.2e}")
    assert worst <= 1.0
    assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= 10 * rel + TOL_LAM
    check_cva_vectors(got.W, ref, tol_s=max(TOL_S, rel))
    return ref, got


# a-priori bounds on |dS_ij| / sum_p |x_pi||x_pj|: exact split (integer and
# half pages): FP32 accumulation only, (32 + 16) * 2^-24 < 3e-6, stated as
# 1e-5; fp32 pages: plus the split residual 2 u_h^2 (bf16: 2^-15, fp16: 2^-21)
BOUND_EXACT = 1e-5
BOUND_F32 = {"bf16x3": 2.0 ** -15 + 1e-5, "f16x3": 2.0 ** -21 + 1e-5}


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
def test_mixed_cva_and_pca_u16(dev, prec):
    say(f"mixed {prec} on the 4096x4096x23 structure at 1024x1024x23 u16")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.25)
    cube = _t(c.cube, dev)
    ref, got = _mixed_fit_check(cube, c.cube, c.labels, c.K, dev, prec, BOUND_EXACT)
    _project_parity(c.cube, got.W, got.mean, dev)
    pr = oracle.pca_fit(c.cube, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(cube, n_comp=3, precision=prec)
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert np.max(np.abs(lam - pr["eigvals"]) / pr["eigvals"]) <= TOL_LAM
    check_pca_vectors(V, pr)


@pytest.mark.parametrize("kind,prec", [("bf16", "bf16x3"), ("f16", "f16x3"), ("bf16", "f16x3"),
                                       ("f16", "bf16x3")])
def test_mixed_half_pages(dev, kind, prec):
    say(f"mixed {prec} on a {kind} page (4096x4096x23 structure at 1/4 scale)")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.25)
    cube = to_half_cube(c.cube, kind)
    host = cube.float().numpy()
    exact = (kind == "bf16") or (prec == "f16x3")
    rel = BOUND_EXACT if exact else BOUND_F32[prec]
    _mixed_fit_check(_t(cube, dev), host, c.labels, c.K, dev, prec, rel)
    pr = oracle.pca_fit(host, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(_t(cube, dev), n_comp=3, precision=prec)
    assert rel_max(cov, pr["cov"]) <= 10 * rel + TOL_S
    check_pca_vectors(V, pr, tol_s=10 * rel + TOL_S)


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
def test_mixed_f32_page(dev, prec):
    say(f"mixed {prec} on an fp32 page")
    c = make_case(2, scale=0.15)
    cube = (c.cube.astype(np.float32) + np.float32(0.25))
    _mixed_fit_check(_t(cube, dev), cube, c.labels, c.K, dev, prec, BOUND_F32[prec])


@pytest.mark.parametrize("H,W,B,K", [(37, 53, 7, 3), (33, 31, 33, 5), (40, 41, 64, 3), (19, 23, 1, 2),
                                     (50, 50, 47, 3)])
def test_mixed_shapes(dev, H, W, B, K):
    say(f"mixed shapes H={H} W={W} B={B} K={K}")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(H * 7 + B)
    mu = rng.uniform(800, 3500, (K, B))
    cls = rng.integers(0, K, H * W)
    cls[: K * (B + 2)] = np.repeat(np.arange(K), B + 2)
    cube = np.clip(np.rint(mu[cls] + rng.normal(0, 60, (H * W, B))), 0, 4095).astype(np.uint16).reshape(H, W, B)
    labels = np.where(rng.random(H * W) < 0.6, cls, -1).astype(np.int8)
    labels[: K * (B + 2)] = cls[: K * (B + 2)]
    labels = labels.reshape(H, W)
    for prec in ("bf16x3", "f16x3"):
        _mixed_fit_check(_t(cube, dev), cube, labels, K, dev, prec, BOUND_EXACT)
        pr = oracle.pca_fit(cube, n_comp=1)
        V, lam, mean, cov = cx.pca_fit(_t(cube, dev), n_comp=1, precision=prec)
        assert rel_max(cov, pr["cov"]) <= TOL_S


def test_mixed_pca_mask(dev):
    say("mixed pca with mask")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.5)
    rng = np.random.default_rng(8)
    mask = (rng.random((c.H, c.W)) < 0.4).astype(np.uint8)
    pr = oracle.pca_fit(c.cube, mask=mask, n_comp=2)
    V, lam, mean, cov = cx.pca_fit(_t(c.cube, dev), mask=_t(mask, dev), n_comp=2, precision="bf16x3")
    assert rel_max(cov, pr["cov"]) <= TOL_S
    check_pca_vectors(V, pr)


@pytest.mark.timeout(900)
def test_full_page_7216x5412x33_mixed(dev):
    """The benchmark workload: 7216 x 5412 x 33 uint16, K = 8, BF16
    compensated scatter on MFMA, FP64 eigensolve; PCA on all pixels."""
    say("full page 7216x5412x33, bf16x3")
    import paper_1612_06457_amd as cx
    c = full_page()
    cube = _t(c.cube, dev)
    ref, got = _mixed_fit_check(cube, c.cube, c.labels, c.K, dev, "bf16x3", BOUND_EXACT)
    say("mixed fit ok", got.eigvals)
    pr = oracle.pca_fit(c.cube, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(cube, n_comp=3, precision="bf16x3")
    assert rel_max(cov, pr["cov"]) <= TOL_S
    assert np.max(np.abs(lam - pr["eigvals"]) / pr["eigvals"]) <= TOL_LAM
    check_pca_vectors(V, pr)
    say("mixed pca ok")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_full_half_page_4096x4096x23(dev, kind):
    """The 4096 x 4096 x 23 page as bf16 / fp16 values (4 classes, 50,000
    training pixels each), at full size: the FP32 fit and the split fit
    against the oracle on the same 16-bit values, every pixel of the three
    projected images, and the split PCA covariance."""
    say(f"full page 4096x4096x23 {kind}")
    import paper_1612_06457_amd as cx
    c = make_case(3, threads=16)
    cube = to_half_cube(c.cube, kind)
    host = cube.float().numpy()
    del c.cube
    dcube = _t(cube, dev)
    prec = "bf16x3" if kind == "bf16" else "f16x3"
    ref = oracle.cva_fit(host, c.labels, c.K)
    got = cx.cva_fit(dcube, _t(c.labels, dev), c.K)
    assert got.counts.tolist() == ref["counts"].tolist()
    assert rel_max(got.Sw, ref["Sw"]) <= TOL_S
    assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    check_cva_vectors(got.W, ref)
    _mixed_fit_check(dcube, host, c.labels, c.K, dev, prec, BOUND_EXACT)
    say(f"{kind} fits ok")
    q, ab = cx.cva_project(dcube, ref["W"], ref["mean"], return_range=True)
    q_ref, ab_ref = oracle.cva_project(host, ref["W"], ref["mean"])
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    frac = check_images(q.cpu().numpy(), q_ref)
    say(f"{kind} project ok, differing bytes {frac:.2e}")
    del q, q_ref
    pr = oracle.pca_fit(host, n_comp=3)
    V, lam, mean, cov = cx.pca_fit(dcube, n_comp=3, precision=prec)
    assert rel_max(cov, pr["cov"]) <= 10 * BOUND_EXACT + TOL_S
    check_pca_vectors(V, pr, tol_s=10 * BOUND_EXACT + TOL_S)
    say(f"{kind} pca ok")


def test_pca_u16_exact_with_a_one_block_gram(dev):
    """CVAMX_GRAM_BLOCKS=1 on a uint16 page of 4.4 M pixels (over the 2^22
    pixels one block of the exact integer Gram may cover): the library
    raises the grid, and the covariance stays exact (within 1e-11 of the
    oracle's largest entry, as at every other grid).  Run in a fresh process,
    since the variable is read when the context is made."""
    say("PCA u16 with CVAMX_GRAM_BLOCKS=1, 2200 x 2000 x 5")
    import os
    import subprocess
    code = r"""
import sys, numpy as np, torch
sys.path.insert(0, %r)
import oracle, paper_1612_06457_amd as cx
rng = np.random.default_rng(3)
x = rng.integers(0, 65536, (2200, 2000, 5)).astype(np.uint16)
x[:, :, 1] = (x[:, :, 0] // 2 + rng.integers(0, 4000, (2200, 2000))).astype(np.uint16)
pr = oracle.pca_fit(x, n_comp=3)
V, lam, mean, cov = cx.pca_fit(torch.from_numpy(x).cuda(), n_comp=3)
err = np.max(np.abs(cov - pr["cov"])) / np.max(np.abs(pr["cov"]))
print("cov_err", err, flush=True)
assert err <= 1e-11
""" % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CVAMX_GRAM_BLOCKS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    say(r.stdout.strip()[-200:])
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
