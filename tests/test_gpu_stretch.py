"""GPU parity of the float images, the three rescaling modes, the 16-bit
output, the RGB composite and the cluster-separation indices, through the
C ABI.

Bars: the float planes within 1e-4 of each component's range of the FP64
oracle's (as for the fused projection), and mode 1 on them finds the fused
projection's range bit for bit; the order statistics behind mode 3 are
exact, so the range equals NumPy's percentile of the device's own FP32
values up to FP64 rounding of the interpolation; the images equal, bit for
bit, the oracle's quantisation of the device's own values on the device's
range (both evaluate the definition in FP64), and lie within one level of
the full FP64 oracle pipeline; the RGB composite is bit-exact; the
Davies-Bouldin and Dunn indices within 1e-12 relative of the FP64 oracle
(FP64 sums in another order).
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_case, to_half_cube
from tests._cases import full_page
from oracle.stretch import _quantise
from tests._parity import TOL_Y, check_images

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


def _levels(bits):
    return 255 if bits == 8 else 65535


def _check_q(q, q_ref, max_diff=1, max_frac=None):
    """Images within max_diff levels (and at most max_frac of the elements
    differing, when given)."""
    q = np.asarray(q).astype(np.int64)
    q_ref = np.asarray(q_ref).astype(np.int64)
    assert q.shape == q_ref.shape
    d = np.abs(q - q_ref)
    assert d.max() <= max_diff, f"max level difference {d.max()} (allowed {max_diff})"
    frac = float((d != 0).mean())
    if max_frac is not None:
        assert frac <= max_frac, f"{frac:.2e} of the elements differ"
    return frac


def _pipeline_check(q, y_dev, y_ref, ab, a_ref, b_ref, levels):
    """Device images against the FP64 pipeline's: the level position
    L (y - a) / (b - a) moves by at most L (|dy| + 2 max(|da|, |db|)) / (b - a)
    between the two, so floors differ by at most one more than that."""
    dy = np.max(np.abs(y_dev - y_ref), axis=0)
    dab = np.maximum(np.abs(ab[:, 0] - a_ref), np.abs(ab[:, 1] - b_ref))
    span = b_ref - a_ref
    assert np.max((dy + dab) / (y_ref.max(0) - y_ref.min(0))) <= TOL_Y
    bound = float(np.max(levels * (dy + 2 * dab) / span))
    return _check_q(q, _quantise(y_ref, a_ref, b_ref, levels), max_diff=1 + int(bound))


def _planes_to_rows(y):
    """n x H x W (torch) -> P x n float64 numpy, the oracle's layout."""
    n = y.shape[0]
    return y.reshape(n, -1).double().cpu().numpy().T.copy()


def _q_rows(q):
    """n x H x W uint8 / uint16 (torch) -> P x n int64 numpy."""
    n = q.shape[0]
    return q.cpu().numpy().reshape(n, -1).T.astype(np.int64)


def _page(kind, H, W, B, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(800, 3500, (3, B))
    cls = rng.integers(0, 3, H * W)
    x = np.clip(np.rint(mu[cls] + rng.normal(0, 60, (H * W, B))), 0, 4095).astype(np.uint16)
    cube = x.reshape(H, W, B)
    if kind == "u16":
        return cube, cube
    if kind == "f32":
        c = cube.astype(np.float32) / np.float32(4095.0)
        return c, c
    h = to_half_cube(cube, kind)
    return h, h.float().numpy()


@pytest.mark.parametrize("kind,H,W,B", [
    ("u16", 37, 53, 33), ("u16", 64, 64, 16), ("u16", 19, 23, 1), ("u16", 41, 40, 64),
    ("f32", 37, 53, 7), ("bf16", 33, 31, 23), ("f16", 40, 41, 9)])
def test_float_planes_and_fused_bytes(dev, kind, H, W, B):
    say(f"float planes {kind} H={H} W={W} B={B}")
    import paper_1612_06457_amd as cx
    cube, host = _page(kind, H, W, B, H * 100 + B)
    rng = np.random.default_rng(B)
    n = min(B, 10)
    Wm = rng.normal(size=(B, n))
    center = np.asarray(host, dtype=np.float64).reshape(-1, B).mean(0)
    y_ref = oracle.project(host, Wm, center)                          # P x n
    span = y_ref.max(0) - y_ref.min(0)
    cd = _t(cube, dev)
    y = cx.project_float(cd, Wm, center)
    yh = _planes_to_rows(y)
    assert np.max(np.abs(yh - y_ref) / span[None, :]) <= TOL_Y
    # mode 1 on the planes: the fused pass's range bit for bit, its bytes
    # within a level, and the oracle's quantisation of these values exactly
    q, ab = cx.stretch(y, "minmax", return_range=True)
    qf, abf = cx.cva_project(cd, Wm, center, return_range=True)
    assert np.array_equal(ab, abf.astype(np.float64))
    check_images(q.cpu().numpy(), qf.cpu().numpy())
    assert np.array_equal(_q_rows(q), _quantise(yh, ab[:, 0], ab[:, 1]))
    check_images(q.cpu().numpy(), oracle.cva_project(host, Wm, center)[0])


def _synthetic_planes(dev, n, H, W, seed):
    """Float planes with a constant plane, a heavily tied plane, a plane
    straddling zero and skewed planes."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    y = torch.randn((n, H, W), generator=g, dtype=torch.float32)
    y[0] = 3.25                                        # constant
    y[1] = torch.round(y[1] * 3.0) * 0.7311 + 0.1234   # ties
    y[2] = y[2] * 1e-3                                 # tiny values around 0
    if n > 3:
        y[3] = torch.exp(y[3] * 2.0) + 100.0           # skewed, positive
    if n > 4:
        y[4] = -torch.exp(y[4])                        # negative
    return y.contiguous().to(dev)


@pytest.mark.parametrize("bits", [8, 16])
@pytest.mark.parametrize("pct", [0.0, 0.01, 1.0, 5.0, 25.0])
def test_percentile_mode(dev, bits, pct):
    say(f"percentile mode pct={pct} bits={bits}")
    import paper_1612_06457_amd as cx
    y = _synthetic_planes(dev, 10, 97, 103, seed=int(pct * 100) + bits)
    q, ab = cx.stretch(y, "percentile", pct=pct, bits=bits, return_range=True)
    import torch
    assert q.dtype == (torch.uint8 if bits == 8 else torch.uint16)
    yh = _planes_to_rows(y)                 # the device's own FP32 values
    q_ref, a, b = oracle.stretch_percentile(yh, pct, levels=_levels(bits))
    tol = 1e-12 * (np.abs(a) + np.abs(b) + 1e-30)
    assert np.all(np.abs(ab[:, 0] - a) <= tol) and np.all(np.abs(ab[:, 1] - b) <= tol)
    assert np.array_equal(_q_rows(q), _quantise(yh, ab[:, 0], ab[:, 1], _levels(bits)))
    _check_q(_q_rows(q), q_ref, max_frac=1e-3)
    if pct == 0.0:   # the 0-th percentile is the minimum
        q1, ab1 = cx.stretch(y, "minmax", bits=bits, return_range=True)
        assert np.array_equal(q.cpu().numpy(), q1.cpu().numpy()) and np.array_equal(ab, ab1)


def test_percentile_order_statistics_exact(dev):
    """Where the virtual index (P - 1) q is an integer the range is an order
    statistic itself: the sorted value, bit for bit (P = 1025 and q a power
    of two keep every step of the index exact)."""
    say("percentile: exact order statistics")
    import paper_1612_06457_amd as cx
    import torch
    P = 1025
    y = torch.randn((9, P), generator=torch.Generator().manual_seed(5))
    y[1] = torch.round(y[1] * 2.0)          # ties
    y = y.to(dev)
    s = np.sort(y.cpu().numpy(), axis=1)
    for pct, rank in ((1.5625, 16), (6.25, 64), (0.0, 0)):
        _, ab = cx.stretch(y, "percentile", pct=pct, return_range=True)
        assert np.array_equal(ab[:, 0], s[:, rank].astype(np.float64))
        assert np.array_equal(ab[:, 1], s[:, P - 1 - rank].astype(np.float64))


@pytest.mark.parametrize("bits", [8, 16])
def test_training_mode_against_oracle(dev, bits):
    say(f"training-range mode bits={bits}")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.5)
    cd = _t(c.cube, dev)
    fit = cx.cva_fit(cd, _t(c.labels, dev), c.K)
    ref = oracle.cva_fit(c.cube, c.labels, c.K)
    y = cx.project_float(cd, ref["W"], ref["mean"])
    train = np.flatnonzero(c.labels.reshape(-1) >= 0).astype(np.int64)
    q, ab = cx.stretch(y, "training", train_pixels=_t(train, dev), bits=bits, return_range=True)
    # against the device's own values
    yh = _planes_to_rows(y)
    q_dev, a, b = oracle.stretch_training_range(yh, yh[train], levels=_levels(bits))
    assert np.array_equal(ab[:, 0], a) and np.array_equal(ab[:, 1], b)
    assert np.array_equal(_q_rows(q), q_dev)
    # against the FP64 oracle pipeline
    y_ref = oracle.project(c.cube, ref["W"], ref["mean"])
    _, a_ref, b_ref = oracle.stretch_training_range(y_ref, y_ref[train], levels=_levels(bits))
    frac = _pipeline_check(_q_rows(q), yh, y_ref, ab, a_ref, b_ref, _levels(bits))
    say(f"  differing from the FP64 pipeline: {frac:.2e}")
    assert fit.counts.tolist() == ref["counts"].tolist()


@pytest.mark.parametrize("pct", [0.1, 5.0])
def test_percentile_against_fp64_pipeline(dev, pct):
    say(f"percentile mode vs the FP64 pipeline pct={pct}")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.25)
    ref = oracle.cva_fit(c.cube, c.labels, c.K)
    y = cx.project_float(_t(c.cube, dev), ref["W"], ref["mean"])
    q, ab = cx.stretch(y, "percentile", pct=pct, return_range=True)
    assert np.array_equal(_q_rows(q), _quantise(_planes_to_rows(y), ab[:, 0], ab[:, 1]))
    y_ref = oracle.project(c.cube, ref["W"], ref["mean"])
    _, a_ref, b_ref = oracle.stretch_percentile(y_ref, pct)
    frac = _pipeline_check(_q_rows(q), _planes_to_rows(y), y_ref, ab, a_ref, b_ref, 255)
    say(f"  differing from the FP64 pipeline: {frac:.2e}")


def test_ragged_and_misaligned_buffers(dev):
    """P not a multiple of 4 and buffers off their 16-byte alignment take
    the element-wise paths; results equal the aligned run's."""
    say("stretch: ragged and misaligned buffers")
    import paper_1612_06457_amd as cx
    import torch
    n, H, W = 5, 29, 31
    y = _synthetic_planes(dev, n, H, W, seed=9)
    for mode, kw in (("minmax", {}), ("percentile", {"pct": 1.0})):
        for bits in (8, 16):
            ref, ab_ref = cx.stretch(y, mode, bits=bits, return_range=True, **kw)
            yb = torch.empty(n * H * W + 1, dtype=torch.float32, device=dev)
            ys = yb[1:].view(n, H, W)
            ys.copy_(y)
            odt = torch.uint8 if bits == 8 else torch.uint16
            ob = torch.empty(n * H * W + 1, dtype=odt, device=dev)
            out = ob[1:].view(n, H, W)
            got, ab = cx.stretch(ys, mode, bits=bits, out=out, return_range=True, **kw)
            assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy()) and np.array_equal(ab, ab_ref)
    # float planes into a misaligned output equal the aligned ones
    c = make_case(1, scale=0.1)
    cd = _t(c.cube, dev)
    rng = np.random.default_rng(4)
    Wm = rng.normal(size=(c.cube.shape[2], 3))
    center = c.cube.reshape(-1, c.cube.shape[2]).mean(0)
    y0 = cx.project_float(cd, Wm, center)
    P = y0[0].numel()
    yb = torch.empty(3 * P + 1, dtype=torch.float32, device=dev)
    y1 = cx.project_float(cd, Wm, center, out=yb[1:].view(y0.shape))
    assert torch.equal(y0, y1)


def test_one_pixel_and_many_planes(dev):
    say("stretch: one pixel, 64 planes")
    import paper_1612_06457_amd as cx
    import torch
    y = torch.randn((64, 1, 1), generator=torch.Generator().manual_seed(2)).to(dev)
    for mode in ("minmax", "percentile"):
        q, ab = cx.stretch(y, mode, pct=5.0, return_range=True)
        assert (q.cpu().numpy() == 0).all()
        assert np.array_equal(ab[:, 0], y.reshape(-1).double().cpu().numpy())
        assert np.array_equal(ab[:, 0], ab[:, 1])
    y = _synthetic_planes(dev, 64, 16, 17, seed=3)
    q, ab = cx.stretch(y, "percentile", pct=5.0, bits=16, return_range=True)
    yh = _planes_to_rows(y)
    q_ref, a, b = oracle.stretch_percentile(yh, 5.0, levels=65535)
    assert np.allclose(ab[:, 0], a, rtol=1e-12, atol=0) and np.allclose(ab[:, 1], b, rtol=1e-12, atol=0)
    assert np.array_equal(_q_rows(q), _quantise(yh, ab[:, 0], ab[:, 1], 65535))
    _check_q(_q_rows(q), q_ref, max_frac=1e-3)


def test_stretch_errors(dev):
    say("stretch: errors")
    import paper_1612_06457_amd as cx
    import torch
    y = torch.zeros((2, 8, 8), dtype=torch.float32, device=dev)
    bad = torch.tensor([0, 5, 64], dtype=torch.int64, device=dev)   # 64 is outside an 8 x 8 page
    with pytest.raises(cx.CvamxError) as e:
        cx.stretch(y, "training", train_pixels=bad)
    assert e.value.status == -1
    with pytest.raises(cx.CvamxError):
        cx.stretch(y, "training", train_pixels=torch.tensor([-1], dtype=torch.int64, device=dev))
    with pytest.raises(cx.CvamxError):
        cx.stretch(y, "percentile", pct=50.0)
    with pytest.raises(cx.CvamxError):
        cx.stretch(y, "percentile", pct=-1.0)
    with pytest.raises(ValueError):
        cx.stretch(y, "training")
    with pytest.raises(ValueError):
        cx.stretch(y, bits=12)
    # the context still works after the errors
    ok = torch.tensor([0, 63], dtype=torch.int64, device=dev)
    q = cx.stretch(y, "training", train_pixels=ok)
    assert (q.cpu().numpy() == 0).all()


@pytest.mark.parametrize("H,W", [(1, 1), (7, 9), (64, 64), (33, 35)])
def test_compose_rgb(dev, H, W):
    say(f"compose rgb {H}x{W}")
    import paper_1612_06457_amd as cx
    import torch
    rng = np.random.default_rng(H * W)
    r, g, b = rng.integers(0, 256, (3, H, W), dtype=np.uint8)
    tr, tg, tb = (_t(a, dev) for a in (r, g, b))
    assert np.array_equal(cx.compose_rgb(tr, tg, tb).cpu().numpy(), oracle.compose_rgb(r, g, b))
    assert np.array_equal(cx.compose_rgb(tr, None, tb).cpu().numpy(), oracle.compose_rgb(r, None, b))
    assert np.array_equal(cx.compose_rgb(None, tg, tg).cpu().numpy(), oracle.compose_rgb(None, g, g))
    # a misaligned channel takes the element-wise path
    big = torch.empty(H * W + 1, dtype=torch.uint8, device=dev)
    mis = big[1:].view(H, W)
    mis.copy_(tg)
    assert np.array_equal(cx.compose_rgb(tr, mis, tb).cpu().numpy(), oracle.compose_rgb(r, g, b))


@pytest.mark.timeout(900)
def test_full_page_percentile_7216x5412x33(dev):
    """7216 x 5412 x 33 uint16 page, the 7 CVA components: the selected order
    statistics against a CPU partition of the same FP32 values, and the
    16-bit images on sampled pixels against the oracle's map."""
    say("full page 7216x5412x33: float planes, percentile and 16-bit stretch")
    import paper_1612_06457_amd as cx
    c = full_page()
    cd = _t(c.cube, dev)
    fit = cx.cva_fit(cd, _t(c.labels, dev), c.K)
    y = cx.project_float(cd, fit.W, fit.mean)
    qf, abf = cx.cva_project(cd, fit.W, fit.mean, return_range=True)
    q1, ab1 = cx.stretch(y, "minmax", return_range=True)
    assert np.array_equal(ab1, abf.astype(np.float64))
    assert int((q1.int() - qf.int()).abs().max()) <= 1
    del qf, q1
    pct = 1.0
    q, ab = cx.stretch(y, "percentile", pct=pct, bits=16, return_range=True)
    yh = y.reshape(y.shape[0], -1).cpu().numpy()
    P = yh.shape[1]
    h = (P - 1) * pct / 100.0
    for j in range(yh.shape[0]):
        lo, hi = int(np.floor(h)), int(np.floor((P - 1) - h))
        part = np.partition(yh[j], [lo, lo + 1, hi, hi + 1])
        a = np.percentile(yh[j].astype(np.float64), pct)
        b = np.percentile(yh[j].astype(np.float64), 100 - pct)
        assert part[lo] <= ab[j, 0] <= part[lo + 1] and part[hi] <= ab[j, 1] <= part[hi + 1]
        assert abs(ab[j, 0] - a) <= 1e-12 * abs(a) + 1e-30 and abs(ab[j, 1] - b) <= 1e-12 * abs(b) + 1e-30
    rng = np.random.default_rng(55)
    sample = rng.choice(P, 200_000, replace=False)
    qs = q.cpu().numpy().reshape(q.shape[0], -1)[:, sample].astype(np.int64)
    q_ref = _quantise(yh[:, sample].T, ab[:, 0], ab[:, 1], 65535)
    assert np.array_equal(qs.T, q_ref)


# ------------------------------------------ Davies-Bouldin and Dunn (Sec. 3)

@pytest.mark.parametrize("dt", ["u8", "u16", "f32", "bf16"])
@pytest.mark.parametrize("p", [2.0, 1.0, 3.0])
def test_cluster_indices(dev, dt, p):
    say(f"cluster indices {dt} p={p}")
    import paper_1612_06457_amd as cx
    import torch
    rng = np.random.default_rng(7)
    n, H, W, K = 3, 61, 47, 4
    base = rng.uniform(0, 200, (n, H, W))
    if dt == "u8":
        img = base.astype(np.uint8)
    elif dt == "u16":
        img = (base * 300).astype(np.uint16)
    elif dt == "f32":
        img = base.astype(np.float32)
    else:
        img = torch.from_numpy(base.astype(np.float32)).to(torch.bfloat16)
    N = 2000
    pix = rng.integers(0, H * W, N).astype(np.int64)
    cls = rng.integers(-1, K, N).astype(np.int8)
    host = img.float() if dt == "bf16" else img
    got = cx.cluster_indices(_t(img, dev), _t(pix, dev), _t(cls, dev), K, p=p)
    ref = oracle.cluster_indices(host.numpy() if dt == "bf16" else host, pix, cls, K, p=p)
    for name in ("centroids", "scatter", "dist", "dbi_pairs", "dunn_pairs"):
        a, b = getattr(got, name), ref[name]
        assert np.max(np.abs(a - b)) <= 1e-12 * max(np.max(np.abs(b)), 1e-300), name
    assert abs(got.dbi - ref["dbi"]) <= 1e-12 * abs(ref["dbi"])
    assert abs(got.dunn - ref["dunn"]) <= 1e-12 * abs(ref["dunn"])
    # bit for bit repeatable
    again = cx.cluster_indices(_t(img, dev), _t(pix, dev), _t(cls, dev), K, p=p)
    assert np.array_equal(again.scatter, got.scatter) and again.dbi == got.dbi


def test_cluster_indices_closed_form_and_one_image(dev):
    say("cluster indices: closed form, one H x W image")
    import paper_1612_06457_amd as cx
    import torch
    img = torch.tensor([[0, 2, 10, 12], [99, 99, 99, 99]], dtype=torch.uint8, device=dev)
    pix = torch.tensor([0, 1, 2, 3, 4], dtype=torch.int64, device=dev)
    cls = torch.tensor([0, 0, 1, 1, -1], dtype=torch.int8, device=dev)
    r = cx.cluster_indices(img, pix, cls, 2)
    assert r.centroids.tolist() == [[1.0], [11.0]] and r.scatter.tolist() == [1.0, 1.0]
    assert r.dbi == 0.2 and r.dunn == 8.0


def test_cluster_indices_on_cva_images(dev):
    """The paper's assessment: 8-bit CVA components of a page, underwriting
    against parchment points; many points per class and several blocks."""
    say("cluster indices on the CVA images of a page")
    import paper_1612_06457_amd as cx
    c = make_case(2, scale=0.25)
    cd = _t(c.cube, dev)
    fit = cx.cva_fit(cd, _t(c.labels, dev), c.K)
    q = cx.cva_project(cd, fit.W, fit.mean)
    flat = c.labels.reshape(-1)
    pix = np.flatnonzero(flat >= 0).astype(np.int64)
    cls = flat[pix].astype(np.int8)
    qh = q.cpu().numpy()
    got = cx.cluster_indices(q, _t(pix, dev), _t(cls, dev), c.K)
    ref = oracle.cluster_indices(qh, pix, cls, c.K)
    assert np.max(np.abs(got.dbi_pairs - ref["dbi_pairs"])) <= 1e-12 * np.max(np.abs(ref["dbi_pairs"]))
    assert abs(got.dbi - ref["dbi"]) <= 1e-12 * ref["dbi"]
    # the components separate the classes better than any single raw band
    raw = np.ascontiguousarray(np.moveaxis(c.cube, -1, 0))
    best_band = min(oracle.cluster_indices(raw[b:b + 1], pix, cls, c.K)["dbi"] for b in range(raw.shape[0]))
    say(f"  DBI: CVA images {got.dbi:.4f}, best raw band {best_band:.4f}")
    assert got.dbi < best_band


def test_cluster_indices_errors(dev):
    say("cluster indices: errors")
    import paper_1612_06457_amd as cx
    import torch
    img = torch.zeros((1, 8, 8), dtype=torch.uint8, device=dev)
    pix = torch.tensor([0, 1, 2], dtype=torch.int64, device=dev)
    with pytest.raises(cx.CvamxError) as e:
        cx.cluster_indices(img, pix, torch.tensor([0, 0, 0], dtype=torch.int8, device=dev), 2)
    assert e.value.status == -3                                      # empty class
    with pytest.raises(cx.CvamxError) as e:
        cx.cluster_indices(img, pix, torch.tensor([0, 1, 5], dtype=torch.int8, device=dev), 2)
    assert e.value.status == -1                                      # class outside
    with pytest.raises(cx.CvamxError) as e:
        cx.cluster_indices(img, torch.tensor([0, 1, 64], dtype=torch.int64, device=dev),
                           torch.tensor([0, 1, 1], dtype=torch.int8, device=dev), 2)
    assert e.value.status == -1                                      # pixel outside
    with pytest.raises(cx.CvamxError):
        cx.cluster_indices(img, pix, torch.tensor([0, 1, 1], dtype=torch.int8, device=dev), 2, p=0.5)
    r = cx.cluster_indices(img, pix, torch.tensor([0, 1, 1], dtype=torch.int8, device=dev), 2)
    assert r.scatter.tolist() == [0.0, 0.0]
