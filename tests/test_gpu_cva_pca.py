"""The combined CVA + PCA entry point (cvamx_cva_pca) against the separate
calls it schedules: cva_fit_project, pca_fit and pca_project.  Same kernels
in the same order, so every output must agree bit for bit: W, eigenvalues,
means, counts, and every byte of both image stacks; with and without a PCA
mask, with standardised PCA, with more than eight components (two
projection groups), on bf16 and fp16 pages, and at the full 4096 x 4096 x
23 page."""
import sys

import numpy as np
import pytest

from synth import make_case

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
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _check(dev, cube, labels, K, mask=None, n_pca=3, standardize=False, precision="fp32"):
    import torch
    import paper_1612_06457_amd as cx
    img1, fit1 = cx.cva_fit_project(cube, labels, K, precision=precision)
    V1, lam1, mean1, _ = cx.pca_fit(cube, mask=mask, n_comp=n_pca, standardize=standardize, precision=precision)
    pimg1 = cx.pca_project(cube, V1, mean1)
    torch.cuda.synchronize()
    img2, fit2, pimg2, (V2, lam2, mean2) = cx.cva_pca(cube, labels, K, mask=mask, n_pca=n_pca,
                                                      standardize=standardize, precision=precision)
    torch.cuda.synchronize()
    for a, b in ((fit1.W, fit2.W), (fit1.eigvals, fit2.eigvals), (fit1.mean, fit2.mean), (V1, V2),
                 (lam1, lam2), (mean1, mean2)):
        assert np.array_equal(a, b)
    assert np.array_equal(fit1.counts, fit2.counts)
    assert torch.equal(img1, img2)
    assert torch.equal(pimg1, pimg2)


@pytest.mark.parametrize("case,scale,masked,n_pca,standardize", [
    (1, 0.5, False, 3, False), (1, 0.5, True, 3, False), (2, 0.1, False, 10, False), (1, 0.5, False, 4, True)])
def test_cva_pca_equals_the_separate_calls(dev, case, scale, masked, n_pca, standardize):
    say(f"cva_pca: config {case} scale {scale} masked={masked} n_pca={n_pca} standardize={standardize}")
    c = make_case(case, scale=scale)
    rng = np.random.default_rng(11)
    mask = _t((rng.random((c.H, c.W)) < 0.6).astype(np.uint8), dev) if masked else None
    _check(dev, _t(c.cube, dev), _t(c.labels, dev), c.K, mask=mask, n_pca=n_pca, standardize=standardize)


@pytest.mark.parametrize("kind,precision", [("bf16", "bf16x3"), ("f16", "fp32")])
def test_cva_pca_half_pages(dev, kind, precision):
    say(f"cva_pca: config 2 at 0.15 scale as {kind}, {precision}")
    from synth import to_half_cube
    c = make_case(2, scale=0.15)
    cube = to_half_cube(c.cube, kind).contiguous().to(dev)
    _check(dev, cube, _t(c.labels, dev), c.K, precision=precision)


@pytest.mark.timeout(600)
def test_cva_pca_full_page_4096x4096x23(dev):
    say("cva_pca: full 4096 x 4096 x 23 page")
    c = make_case(2, threads=16)
    _check(dev, _t(c.cube, dev), _t(c.labels, dev), c.K)


def test_cva_pca_errors_leave_the_library_usable(dev):
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.25)
    cube, labels = _t(c.cube, dev), _t(c.labels, dev)
    bad = c.labels.copy()
    bad[0, 0] = c.K
    with pytest.raises(cx.CvamxError):
        cx.cva_pca(cube, _t(bad, dev), c.K)
    _check(dev, cube, labels, c.K)
