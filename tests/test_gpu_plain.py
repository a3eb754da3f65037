"""GPU tests of the plain FP32 reference path (cvamx_set_plain_fp32): the
vector-ALU kernels for the fit moments, the PCA covariance and every
projection, whatever the page type.

Bars: the same FP32 tolerances against the FP64 oracle as the default path
(S within 1e-5 of the largest entry, eigenvalues 1e-5 relative, vectors
1e-4 after sign alignment, ranges 1e-4 of b - a, images within one grey
level); and against the default (matrix-core) path on the same page: equal
counts, eigenvalues within 1e-5 relative, float images within 1e-4 of each
component's range, 8-bit images within one level.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_case, to_half_cube
from tests._parity import TOL_LAM, TOL_S, TOL_Y, check_cva_vectors, check_images, check_pca_vectors, rel_max

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


@pytest.fixture
def plain(dev):
    import paper_1612_06457_amd as cx
    cx.set_plain_fp32(True)
    yield
    cx.set_plain_fp32(False)


def _t(a, dev):
    import torch
    if hasattr(a, "to"):
        return a.contiguous().to(dev)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _page(kind, odd=True):
    """23 bands (odd) or 16 (even)."""
    c = make_case(2, scale=0.1) if odd else make_case(1, scale=0.3)
    if kind == "u16":
        return c, c.cube, c.cube
    cube = to_half_cube(c.cube, kind)
    return c, cube, cube.float().numpy()


def _run(cx, dev, cube, c):
    fit = cx.cva_fit(_t(cube, dev), _t(c.labels, dev), c.K)
    q, ab = cx.cva_project(_t(cube, dev), fit.W, fit.mean, return_range=True)
    y = cx.project_float(_t(cube, dev), fit.W, fit.mean)
    pca = cx.pca_fit(_t(cube, dev), n_comp=3)
    return fit, q.cpu().numpy(), ab, y.cpu().numpy(), pca


@pytest.mark.parametrize("kind,odd", [("u16", True), ("u16", False), ("bf16", True), ("f16", False)])
def test_plain_path_against_oracle(dev, plain, kind, odd):
    """Odd band counts put two pixels in a lane group on the 16-bit pages."""
    say(f"plain FP32 path, {kind} page, odd B = {odd}")
    import paper_1612_06457_amd as cx
    c, cube, host = _page(kind, odd)
    assert (c.B % 2 == 1) == odd
    fit, q, ab, y, pca = _run(cx, dev, cube, c)
    ref = oracle.cva_fit(host, c.labels, c.K)
    assert fit.counts.tolist() == ref["counts"].tolist()
    assert rel_max(fit.Sw, ref["Sw"]) <= TOL_S
    assert rel_max(fit.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(fit.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    signs, _ = check_cva_vectors(fit.W, ref)
    q_ref, ab_ref = oracle.cva_project(host, fit.W, fit.mean)
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab - ab_ref) / span[:, None]) <= TOL_Y
    check_images(q, q_ref)
    y_ref = oracle.project(host, fit.W, fit.mean).T.reshape(y.shape)
    assert np.max(np.abs(y - y_ref).reshape(y.shape[0], -1) / span[:, None]) <= TOL_Y
    pr = oracle.pca_fit(host, n_comp=3)
    assert rel_max(pca[3], pr["cov"]) <= TOL_S
    check_pca_vectors(pca[0], pr)


@pytest.mark.parametrize("kind", ["u16", "bf16"])
def test_plain_equals_default_within_fp32(dev, kind):
    say(f"plain FP32 path against the default path, {kind} page")
    import paper_1612_06457_amd as cx
    c, cube, host = _page(kind)
    base = _run(cx, dev, cube, c)
    cx.set_plain_fp32(True)
    try:
        other = _run(cx, dev, cube, c)
    finally:
        cx.set_plain_fp32(False)
    f0, f1 = base[0], other[0]
    assert f0.counts.tolist() == f1.counts.tolist()
    assert np.max(np.abs(f0.eigvals - f1.eigvals) / f0.eigvals) <= TOL_LAM
    # the same W on both paths: project with the default fit's vectors
    cx.set_plain_fp32(True)
    try:
        q1, ab1 = cx.cva_project(_t(cube, dev), f0.W, f0.mean, return_range=True)
        y1 = cx.project_float(_t(cube, dev), f0.W, f0.mean).cpu().numpy()
    finally:
        cx.set_plain_fp32(False)
    span = base[2][:, 1] - base[2][:, 0]
    assert np.max(np.abs(ab1 - base[2]) / span[:, None]) <= TOL_Y
    assert np.max(np.abs(y1 - base[3]).reshape(y1.shape[0], -1) / span[:, None]) <= TOL_Y
    assert np.max(np.abs(q1.cpu().numpy().astype(int) - base[1].astype(int))) <= 1


def test_kernel_timing_modes(dev):
    """Per-kernel timing: every kernel, or only the page-streaming
    projection passes; the counts match the launches."""
    say("kernel timing modes")
    import paper_1612_06457_amd as cx
    c, cube, _ = _page("u16", odd=True)
    tc, tl = _t(cube, dev), _t(c.labels, dev)
    cx.profile_enable(True)
    try:
        cx.cva_fit_project(tc, tl, c.K)
        rep = cx.profile_report()
    finally:
        cx.profile_enable(False)
    C = c.K - 1
    for name in ("label_count", "label_scan", "label_index", "class_moments_mfma", "reduce_partials",
                 f"project_range_store_nc{C}", f"project_stretch_stored_nc{C}"):
        assert rep.get(name, (0, 0.0))[0] == 1, (name, rep)
        assert rep[name][1] > 0.0
    cx.profile_enable("projection")
    try:
        cx.cva_fit_project(tc, tl, c.K)
        cx.cva_fit_project(tc, tl, c.K)
        rep = cx.profile_report()
    finally:
        cx.profile_enable(False)
    assert sorted(rep) == sorted([f"project_range_store_nc{C}", f"project_stretch_stored_nc{C}"]), rep
    assert all(v[0] == 2 for v in rep.values()), rep
    # the two-read schedule's passes
    cx.set_schedule("two_reads")
    cx.profile_enable("projection")
    try:
        cx.cva_fit_project(tc, tl, c.K)
        rep = cx.profile_report()
    finally:
        cx.profile_enable(False)
        cx.set_schedule("auto")
    assert sorted(rep) == sorted([f"project_range_nc{C}", f"project_stretch_nc{C}"]), rep
    assert all(v[0] == 1 for v in rep.values()), rep
