"""Mask refinement by the gradient of the Fisher criterion, scored by the
Davies-Bouldin and Dunn indices (paper Section 3, Eqs. 1-5; Section 4, the
call for an automatic choice of training points), through the C ABI.

Bars.  The update kernel against the FP64 oracle's step on the same
weights and gradient: within 1e-5 (FP32 arithmetic of a step of at most
`step` per entry, and an exact projection).  The refinement loop (soft
forward, hand-written backward, update) on training masks with about 20 %
wrong labels: the GPU and the oracle, each running the same loop, end with
weights within 1e-3 of each other and the same hard labels; the
Davies-Bouldin index of the CVA images on held-out true labels improves
(falls) on both, and the GPU's index lies within 2 % of the oracle's (the
8-bit images differ by at most one level).
"""
import sys

import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("N,K,step", [(1000, 2, 0.5), (5000, 5, 0.3), (777, 8, 1.0), (3000, 32, 0.25),
                                      (64, 3, 0.0)])
def test_update_kernel_against_oracle(dev, N, K, step):
    say(f"soft update kernel N={N} K={K} step={step}")
    import paper_1612_06457_amd as cx
    rng = np.random.default_rng(N + K)
    w = rng.dirichlet(np.full(K, 0.5), N)
    w[: N // 4] = np.eye(K)[rng.integers(0, K, N // 4)]          # one-hot rows
    w[N // 4: N // 3] += rng.normal(0, 0.3, (N // 3 - N // 4, K))  # rows off the simplex
    g = rng.normal(0, 1, (N, K)) * 10.0 ** rng.uniform(-3, 3, (N, 1))
    g[: 5] = 7.0                                                  # a gradient equal for every class
    w32, g32 = w.astype(np.float32), g.astype(np.float32)
    want = oracle.soft_update(w32, g32, step)
    wd = _t(w32, dev)
    cx.cva_soft_update(wd, _t(g32, dev), step)
    got = wd.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-5
    assert np.all(got >= 0) and np.max(np.abs(got.sum(1) - 1.0)) <= 1e-5


def _dbi(cx, cube, W, mean, pixels, classes, K, dev):
    q = cx.cva_project(cube, W, mean)
    r = cx.cluster_indices(q, _t(pixels.astype(np.int64), dev), _t(classes.astype(np.int8), dev), K)
    return r, q


def test_refinement_improves_held_out_dbi(dev):
    say("mask refinement: 20 % wrong labels, 3 steps, DBI on held-out true labels")
    import paper_1612_06457_amd as cx
    c = make_case(1, scale=0.5)
    rng = np.random.default_rng(7)
    flat = c.labels.reshape(-1)
    idx = np.flatnonzero(flat >= 0)
    true = flat[idx].astype(np.int64)
    perm = rng.permutation(idx.size)
    ntr = int(0.7 * idx.size)
    tr, ho = perm[:ntr], perm[ntr:]
    X = c.cube.reshape(-1, c.B)[idx[tr]].astype(np.float32)
    lab = true[tr].copy()
    wrong = rng.random(ntr) < 0.2
    lab[wrong] = (lab[wrong] + rng.integers(1, c.K, wrong.sum())) % c.K
    w0 = np.eye(c.K, dtype=np.float32)[lab]
    steps, step = 3, 0.5
    # the oracle's loop, in FP64
    wo = w0.astype(np.float64)
    fo0 = oracle.soft_fit(X, wo)
    for _ in range(steps):
        wo = oracle.soft_update(wo, oracle.soft_grad(X, wo), step)
    fo = oracle.soft_fit(X, wo)
    qo0, _ = oracle.cva_project(c.cube, fo0["W"], fo0["mean"])
    qo, _ = oracle.cva_project(c.cube, fo["W"], fo["mean"])
    ro0 = oracle.cluster_indices(qo0, idx[ho], true[ho], c.K)
    ro = oracle.cluster_indices(qo, idx[ho], true[ho], c.K)
    # the GPU's loop
    cube = _t(c.cube, dev)
    Xd = _t(X, dev)
    wd = _t(w0, dev)
    f0 = cx.cva_soft_forward(Xd, wd)
    r0, _ = _dbi(cx, cube, f0.W, f0.mean, idx[ho], true[ho], c.K, dev)
    f = cx.refine_weights(Xd, wd, steps=steps, step=step)
    r, _ = _dbi(cx, cube, f.W, f.mean, idx[ho], true[ho], c.K, dev)
    wg = wd.cpu().numpy()
    say(f"  held-out DBI: GPU {r0.dbi:.4f} -> {r.dbi:.4f}, oracle {ro0['dbi']:.4f} -> {ro['dbi']:.4f}; "
        f"Dunn GPU {r0.dunn:.2f} -> {r.dunn:.2f}; weights max diff {np.max(np.abs(wg - wo)):.2e}; "
        f"training labels right: before {np.mean(lab == true[tr]):.3f}, after {np.mean(wg.argmax(1) == true[tr]):.3f}")
    assert np.max(np.abs(wg - wo)) <= 1e-3
    assert np.array_equal(wg.argmax(1), wo.argmax(1))
    assert ro["dbi"] < ro0["dbi"] and r.dbi < r0.dbi
    assert abs(r.dbi - ro["dbi"]) <= 0.02 * ro["dbi"]
    assert abs(r0.dbi - ro0["dbi"]) <= 0.02 * ro0["dbi"]


def test_update_errors(dev):
    import torch
    import paper_1612_06457_amd as cx
    w = torch.zeros((10, 3), dtype=torch.float32, device=dev)
    with pytest.raises(ValueError):
        cx.cva_soft_update(w, torch.zeros((10, 4), dtype=torch.float32, device=dev), 0.5)
    with pytest.raises(cx.CvamxError):
        cx.cva_soft_update(w, torch.zeros_like(w), -1.0)
    with pytest.raises(cx.CvamxError):
        cx.cva_soft_update(torch.zeros((10, 1), dtype=torch.float32, device=dev),
                           torch.zeros((10, 1), dtype=torch.float32, device=dev), 0.5)
