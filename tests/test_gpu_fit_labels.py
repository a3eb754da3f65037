"""CVA fits over label maps of many layouts, through the C ABI, against the
FP64 oracle: the label bookkeeping (counts, per-class lists) and the class
moments that gather those lists.

Bars: class counts bit-exact; class means within 1e-7 and S_w, S_b within
1e-5 of their largest entry; eigenvalues within 1e-5 relative.  The label
maps cover scattered pixels, runs of one class (the usual training masks),
every pixel labelled, a class that appears only at the page's end, a class
dense enough that one 4,096-entry wave tile holds thousands of its rows, K
on both sides of 64, and page sizes around the wave tiles.  A label outside
-1..K-1 anywhere (first entry, tile edges, last entry) is an error.
"""
import sys

import numpy as np
import pytest

import oracle
from tests._parity import TOL_LAM, TOL_S, rel_max

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


def _labels(P, K, kind, rng):
    if kind == "scattered":
        lab = np.where(rng.random(P) < 0.3, rng.integers(0, K, P), -1)
    elif kind == "regions":
        lab = np.empty(P, dtype=np.int64)
        i = 0
        while i < P:
            L = int(rng.integers(1, 3000))
            lab[i:i + L] = rng.integers(-1, K)
            i += L
    elif kind == "all":
        lab = rng.integers(0, K, P)
    elif kind == "late":                       # class K - 1 only in the last tile
        lab = np.where(rng.random(P) < 0.3, rng.integers(0, K - 1, P), -1)
        lab[-min(P, 3000):] = np.where(rng.random(min(P, 3000)) < 0.5, K - 1, -1)
    else:                                      # "dense": 90 % of the pixels in class 0
        lab = np.where(rng.random(P) < 0.9, 0, rng.integers(1, K, P))
    # every class needs more pixels than bands
    for k in range(K):
        if (lab == k).sum() < 12:
            lab[rng.choice(P, 12, replace=False)] = k
    return lab.astype(np.int8)


def _page(lab, B, K, rng):
    mu = rng.uniform(800, 3500, (K, B))
    cls = np.where(lab >= 0, lab, rng.integers(0, K, lab.size))
    x = np.clip(np.rint(mu[cls] + rng.normal(0, 60, (lab.size, B))), 0, 4095).astype(np.uint16)
    return x


@pytest.mark.parametrize("P,K,kind", [
    (4096, 3, "scattered"), (4097, 3, "regions"), (8191, 4, "all"), (100003, 5, "late"),
    (65536, 4, "dense"), (300001, 70, "scattered"), (250000, 127, "all"), (12289, 2, "regions")])
def test_fit_label_maps(dev, P, K, kind):
    say(f"fit over label map: P={P} K={K} {kind}")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(P + K)
    B = 5
    lab = _labels(P, K, kind, rng)
    x = _page(lab, B, K, rng)
    H, W = 1, P
    cube = x.reshape(H, W, B)
    labels = lab.reshape(H, W)
    ref = oracle.cva_fit(cube, labels, K)
    got = cx.cva_fit(_t(cube, dev), _t(labels, dev), K)
    assert got.counts.tolist() == ref["counts"].tolist()
    assert rel_max(got.class_means, ref["class_means"]) <= 1e-7
    assert rel_max(got.Sw, ref["Sw"]) <= TOL_S
    assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
    assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM


def test_fit_label_errors(dev):
    say("fit over label map: a label outside -1..K-1 anywhere in the map")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(5)
    P, K, B = 20000, 3, 4
    lab = _labels(P, K, "scattered", rng)
    x = _page(lab, B, K, rng)
    for at in (0, 4095, 4096, P - 1):
        bad = lab.copy()
        bad[at] = K
        with pytest.raises(cx.CvamxError) as e:
            cx.cva_fit(_t(x.reshape(1, P, B), dev), _t(bad.reshape(1, P), dev), K)
        assert e.value.status == -1
    # and the library still fits after the errors
    got = cx.cva_fit(_t(x.reshape(1, P, B), dev), _t(lab.reshape(1, P), dev), K)
    assert got.counts.tolist() == oracle.class_counts(lab, K).tolist()


@pytest.mark.parametrize("P,B,K,full16", [
    (70001, 33, 8, False), (40000, 47, 5, True), (33333, 31, 3, True), (20000, 32, 4, False),
    (5000, 48, 3, False), (16384, 1, 2, True)])
def test_fit_label_map_bands(dev, P, B, K, full16):
    """uint16 label-map fits at band counts on both sides of the matrix-core
    kernels' 16-band row blocks (31/32, 47/48) and at one band, with values
    over the whole 16-bit range (both bytes of a value take every size) or
    in the 12-bit range; and the point-list fit of the same pixels.  Both
    against the FP64 oracle, with the bars of the other fit tests."""
    say(f"fit over label map: P={P} B={B} K={K} full16={full16}")
    import torch
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(P + B)
    lab = _labels(P, K, "regions", rng)
    if full16:
        hi = rng.random(P) < 0.4
        mu = np.where(hi[:, None], rng.uniform(60000, 65000, B), rng.uniform(50, 3000, B))
        cls = np.where(lab >= 0, lab, 0)
        mu = mu + 300.0 * cls[:, None]
        x = np.clip(np.rint(mu + rng.normal(0, 900, (P, B))), 0, 65535).astype(np.uint16)
    else:
        x = _page(lab, B, K, rng)
    cube = x.reshape(1, P, B)
    labels = lab.reshape(1, P)
    ref = oracle.cva_fit(cube, labels, K)
    pix = np.flatnonzero(lab >= 0).astype(np.int64)
    fits = {"label map": cx.cva_fit(_t(cube, dev), _t(labels, dev), K),
            "point list": cx.cva_fit_points(_t(cube, dev), _t(pix, dev), _t(lab[pix], dev), K)}
    torch.cuda.synchronize()
    for name, got in fits.items():
        say(f"  {name}")
        assert got.counts.tolist() == ref["counts"].tolist()
        assert rel_max(got.class_means, ref["class_means"]) <= 1e-7
        assert rel_max(got.Sw, ref["Sw"]) <= TOL_S
        assert rel_max(got.Sb, ref["Sb"]) <= TOL_S
        assert np.max(np.abs(got.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
