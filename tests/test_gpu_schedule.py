"""The projection schedules through the C ABI: one page read with an fp16
intermediate (the default), two page reads, and the one-read pass 1
followed by its page re-reading fallback; on uint16 pages (matrix cores),
and on float32, bf16 and fp16 pages and the plain FP32 path (vector ALU).

Bars: the ranges equal bit for bit under every schedule (pass 1 is the same
FP32 computation); the forced fallback equals the two-read images bit for
bit (same map, same kernel body); the one-read images lie within one grey
level of the two-read images and of the FP64 oracle's, and the fraction of
bytes that differ from the two-read images stays below the fraction the
error bound allows (the stored values move the map's argument by at most
255 * 2^-11 * max(|a|, |b|) / (b - a) levels, 1/8 of a level when the
centre lies inside the projected range; a byte changes only when its
argument lies that close to an integer).  A centre far outside the page's
range makes the bound exceed half a level: the device then falls back to
re-reading the page by itself, and the images equal the two-read ones.
"""
import sys

import numpy as np
import pytest

import oracle
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


def _page(H, W, B, seed, full_range=False):
    rng = np.random.default_rng(seed)
    if full_range:
        x = rng.integers(0, 65536, (H * W, B)).astype(np.uint16)
    else:
        mu = rng.uniform(800, 3500, (3, B))
        cls = rng.integers(0, 3, H * W)
        x = np.clip(np.rint(mu[cls] + rng.normal(0, 60, (H * W, B))), 0, 4095).astype(np.uint16)
    return x.reshape(H, W, B)


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _run(cx, cube_d, Wm, center, schedule, plain=False):
    cx.set_schedule(schedule)
    cx.set_plain_fp32(plain)
    try:
        q, ab = cx.cva_project(cube_d, Wm, center, return_range=True)
    finally:
        cx.set_schedule("auto")
        cx.set_plain_fp32(False)
    return q.cpu().numpy().astype(np.int32), ab


def _bound_frac(y_ref, ab):
    """Fraction of values whose map argument lies within the stored-value
    error bound of a rounding boundary (an upper estimate of the bytes that
    may differ from the two-read ones)."""
    a, b = ab[:, 0].astype(np.float64), ab[:, 1].astype(np.float64)
    t = 255.0 * (y_ref - a) / (b - a) + 0.5
    bound = 255.0 * 2.0 ** -11 * np.maximum(np.abs(a), np.abs(b)) / (b - a) + 5e-3
    near = np.abs(t - np.rint(t)) <= bound
    return float(near.mean())


@pytest.mark.parametrize("H,W,B,n,seed", [
    (37, 53, 33, 7, 1),     # odd bands: two-pixel rows; ragged last tile
    (64, 64, 16, 3, 2),     # even bands: one-pixel rows
    (19, 23, 1, 1, 3),      # one band, P not a multiple of 16
    (41, 40, 64, 10, 4),    # two groups of components (8 + 2)
    (5, 7, 23, 3, 5),       # a page smaller than one tile
    (301, 257, 33, 8, 6),   # many tiles, 8 components
])
def test_schedules_agree(dev, H, W, B, n, seed):
    say(f"schedules: {H}x{W}x{B} u16, {n} components")
    import paper_1612_06457_amd as cx
    cube = _page(H, W, B, seed)
    rng = np.random.default_rng(seed + 100)
    Wm = rng.normal(size=(B, n))
    center = cube.reshape(-1, B).astype(np.float64).mean(0)
    cd = _t(cube, dev)
    q1, ab1 = _run(cx, cd, Wm, center, "auto")
    q2, ab2 = _run(cx, cd, Wm, center, "two_reads")
    q3, ab3 = _run(cx, cd, Wm, center, "force_reread")
    assert np.array_equal(ab1, ab2) and np.array_equal(ab1, ab3)
    assert np.array_equal(q3, q2), "the forced fallback differs from the two-read images"
    q_ref, ab_ref = oracle.cva_project(cube, Wm, center)
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab1 - ab_ref) / span[:, None]) <= TOL_Y
    frac = check_images(q1, q2)
    check_images(q1, q_ref)
    y_ref = oracle.project(cube, Wm, center)
    allowed = _bound_frac(y_ref, ab1)
    say(f"  one-read bytes differing from two-read: {frac:.3e} (bound allows {allowed:.3e})")
    assert frac <= allowed + 1e-12


def test_full_uint16_range(dev):
    say("schedules: values over the whole 16-bit range, 33 bands")
    import paper_1612_06457_amd as cx
    cube = _page(97, 131, 33, 7, full_range=True)
    rng = np.random.default_rng(7)
    Wm = rng.normal(size=(33, 7)) * np.logspace(-6, 3, 33)[:, None]
    center = cube.reshape(-1, 33).astype(np.float64).mean(0)
    cd = _t(cube, dev)
    q1, ab1 = _run(cx, cd, Wm, center, "auto")
    q2, ab2 = _run(cx, cd, Wm, center, "two_reads")
    assert np.array_equal(ab1, ab2)
    check_images(q1, q2)
    check_images(q1, oracle.cva_project(cube, Wm, center)[0])


def test_far_centre_falls_back(dev):
    say("schedules: centre far outside the projected range -> device fallback")
    import paper_1612_06457_amd as cx
    cube = _page(64, 80, 33, 8)
    rng = np.random.default_rng(8)
    Wm = rng.normal(size=(33, 3))
    mean = cube.reshape(-1, 33).astype(np.float64).mean(0)
    y = oracle.project(cube, Wm, mean)
    span = y.max(0) - y.min(0)
    # move the centre along w_0 so that y_0 sits 20 spans away from zero
    w0 = Wm[:, 0]
    center = mean - 20.0 * span[0] * w0 / (w0 @ w0)
    yc = oracle.project(cube, Wm, center)
    assert np.min(np.abs(yc[:, 0])) >= 19 * span[0]
    cd = _t(cube, dev)
    q1, ab1 = _run(cx, cd, Wm, center, "auto")
    q2, ab2 = _run(cx, cd, Wm, center, "two_reads")
    assert np.array_equal(ab1, ab2)
    assert np.array_equal(q1, q2), "the bound check did not send pass 2 back to the page"


def test_constant_component(dev):
    say("schedules: a zero weight column (constant component) maps to 0")
    import paper_1612_06457_amd as cx
    cube = _page(33, 35, 9, 9)
    rng = np.random.default_rng(9)
    Wm = rng.normal(size=(9, 3))
    Wm[:, 1] = 0.0
    center = cube.reshape(-1, 9).astype(np.float64).mean(0)
    cd = _t(cube, dev)
    q1, ab1 = _run(cx, cd, Wm, center, "auto")
    q2, ab2 = _run(cx, cd, Wm, center, "two_reads")
    assert np.array_equal(ab1, ab2)
    assert (q1[1] == 0).all() and (q2[1] == 0).all()
    check_images(q1, q2)


def _typed(cube, kind, dev):
    """The page as `kind` values (float32, bf16, fp16 scaled to [0, 1]) on the
    device, and the FP64 values the oracle sees."""
    import torch
    from synth import to_half_cube
    if kind == "u16":
        return _t(cube, dev), cube
    if kind == "f32":
        c = (cube.astype(np.float32) / np.float32(4095.0))
        return _t(c, dev), c
    h = to_half_cube(cube, kind)
    return h.to(dev), h.float().numpy()


@pytest.mark.parametrize("kind,plain", [("f32", False), ("bf16", False), ("f16", False), ("u16", True),
                                        ("bf16", True)])
@pytest.mark.parametrize("H,W,B,n", [(37, 53, 23, 3), (64, 64, 16, 8), (19, 23, 1, 1), (41, 40, 64, 10)])
def test_schedules_other_pages(dev, kind, plain, H, W, B, n):
    say(f"schedules: {H}x{W}x{B} {kind}{' plain' if plain else ''}, {n} components")
    import paper_1612_06457_amd as cx
    cube, host = _typed(_page(H, W, B, H + B), kind, dev)
    rng = np.random.default_rng(H + n)
    Wm = rng.normal(size=(B, n))
    center = np.asarray(host, dtype=np.float64).reshape(-1, B).mean(0)
    q1, ab1 = _run(cx, cube, Wm, center, "auto", plain)
    q2, ab2 = _run(cx, cube, Wm, center, "two_reads", plain)
    q3, ab3 = _run(cx, cube, Wm, center, "force_reread", plain)
    assert np.array_equal(ab1, ab2) and np.array_equal(ab1, ab3)
    assert np.array_equal(q3, q2), "the forced fallback differs from the two-read images"
    frac = check_images(q1, q2)
    q_ref, ab_ref = oracle.cva_project(np.asarray(host, dtype=np.float64), Wm, center)
    check_images(q1, q_ref)
    y_ref = oracle.project(np.asarray(host, dtype=np.float64), Wm, center)
    allowed = _bound_frac(y_ref, ab1)
    say(f"  one-read bytes differing from two-read: {frac:.3e} (bound allows {allowed:.3e})")
    assert frac <= allowed + 1e-12


def test_float_page_beyond_the_assumed_range_falls_back(dev):
    say("schedules: float32 values far beyond 1024 (|centre| + 1) -> device fallback")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(11)
    H, W, B = 50, 60, 9
    x = rng.normal(0, 1e6, (H, W, B)).astype(np.float32)          # centre near 0, spread 1e6
    Wm = rng.normal(size=(B, 3))
    center = np.zeros(B)
    cd = _t(x, dev)
    q1, ab1 = _run(cx, cd, Wm, center, "auto")
    q2, ab2 = _run(cx, cd, Wm, center, "two_reads")
    assert np.array_equal(ab1, ab2)
    assert np.array_equal(q1, q2), "the overflow check did not send pass 2 back to the page"


@pytest.mark.parametrize("nr,nw", [(1 << 20, 1 << 20), (3 << 20, 1 << 19), (123456 * 16, 777 * 16), (4096, 16)])
def test_reference_streams(dev, nr, nw):
    """The measurement streams run to completion on any size; with equal
    sizes the mixed stream writes tile t of the output from read tile t,
    i.e. it copies; with fewer write bytes every write tile is written."""
    say(f"reference streams: read {nr} B, write {nw} B")
    import torch
    import paper_1612_06457_amd as cx
    g = torch.Generator(device="cpu").manual_seed(nr ^ nw)
    src = torch.randint(0, 256, (nr,), dtype=torch.uint8, generator=g).to(dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    cx.stream_read(src, sink)
    dst = torch.zeros(nw, dtype=torch.uint8, device=dev)
    cx.stream_mix(src, dst, sink)
    torch.cuda.synchronize()
    if nw == nr:
        assert torch.equal(dst, src)
    else:
        # each written 16-byte chunk is some chunk of the source
        d = dst.view(-1, 16).cpu().numpy()
        s = {bytes(r) for r in src.view(-1, 16).cpu().numpy()}
        assert all(bytes(r) in s for r in d)
    with pytest.raises(ValueError):
        cx.stream_mix(src[:16], dst if nw > 16 else torch.zeros(32, dtype=torch.uint8, device=dev))
