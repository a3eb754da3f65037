"""GPU tests of the class index lists (the training pixels per class that
every fit gathers), through the C ABI.

Bar: bit-exact.  The list of class k is the increasing positions of the
entries equal to k; the classes follow each other in order; counts and
offsets are exact.  Cases span one wave step (1,024 entries), a block tile
(65,536), ragged ends, class maps made of regions (the usual training
masks) and of scattered pixels, and K on both sides of 64 (per-class values
live in two registers per lane, classes l and 64 + l).
"""
import sys

import numpy as np
import pytest

import oracle

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


def _labels(n, K, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "scattered":
        lab = np.where(rng.random(n) < 0.3, rng.integers(0, K, n), -1)
    elif kind == "regions":
        # runs of one class (or of no class) with lengths from 1 to 3000
        lab = np.empty(n, dtype=np.int64)
        i = 0
        while i < n:
            L = int(rng.integers(1, 3000))
            lab[i:i + L] = rng.integers(-1, K)
            i += L
    elif kind == "all":
        lab = rng.integers(0, K, n)
    else:                                                     # "none"
        lab = np.full(n, -1)
    return lab.astype(np.int8)


def _check(dev, lab, K):
    import paper_1612_06457_amd as cx
    import torch
    idx, counts, offsets = cx.label_index(torch.from_numpy(lab).to(dev), K)
    want_counts = oracle.class_counts(lab, K)
    lists = oracle.class_index_lists(lab, K)
    want_off = np.concatenate([[0], np.cumsum(want_counts)]).astype(np.int32)
    assert np.array_equal(counts, want_counts)
    assert np.array_equal(offsets, want_off)
    want = np.concatenate(lists) if lists else np.zeros(0, np.int64)
    assert np.array_equal(idx.cpu().numpy().astype(np.int64), want)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1023, 1024, 1025, 4099, 65536, 65553, 200005])
@pytest.mark.parametrize("kind", ["scattered", "regions", "all", "none"])
def test_label_index_sizes(dev, n, kind):
    say(f"label index n={n} {kind}")
    for K in (1, 3, 8):
        _check(dev, _labels(n, K, kind, n + K), K)


@pytest.mark.parametrize("K", [2, 63, 64, 65, 100, 127])
@pytest.mark.parametrize("kind", ["scattered", "regions"])
def test_label_index_many_classes(dev, K, kind):
    say(f"label index K={K} {kind}")
    _check(dev, _labels(300007, K, kind, K), K)


def test_label_index_page_labels(dev):
    """The training map of the 7216 x 5412 page (8 classes, about 1.6 M
    training pixels in regions), and the same map with every entry labelled."""
    say("label index: full page")
    from tests._cases import full_page
    c = full_page()
    _check(dev, np.ascontiguousarray(c.labels.reshape(-1)), c.K)
    rng = np.random.default_rng(5)
    _check(dev, rng.integers(0, c.K, c.labels.size).astype(np.int8), c.K)


def test_label_index_errors(dev):
    say("label index: labels outside -1..K-1")
    import paper_1612_06457_amd as cx
    import torch
    lab = _labels(5000, 4, "scattered", 1)
    for bad in (4, 100, -2, -128):
        x = lab.copy()
        x[4321] = bad
        with pytest.raises(cx.CvamxError) as e:
            cx.label_index(torch.from_numpy(x).to(dev), 4)
        assert e.value.status == -1
    # the library still works afterwards
    _check(dev, lab, 4)
