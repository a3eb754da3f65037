"""The soft-label forward on its three paths, through the C ABI, against the
FP64 oracle: the default (FP32 products on the FP32 matrix instruction),
the plain FP32 vector-ALU reference (cvamx_set_plain_fp32), and the
compensated bf16 / fp16 split on the 16-bit matrix units.

Bars.  Default and plain: the FP32 bars (J and eigenvalues within 1e-5
relative, class means within 1e-6, W^T S_w W = I within 1e-5 against the
oracle's S_w, the gradient within 1e-4 of max |dJ/dw|).  Split: every S_w
entry is within e M_ij of the exact one, M_ij = sum_c sum_p |w_pc| |d_pi|
|d_pj|, e = 2 u^2 + 512 2^-24 (u = 2^-8 bf16, 2^-11 fp16), and the class
sums of the same Gram carry the split error of w d alone; to first order
an eigenvalue moves by v^T (dS_b - lambda dS_w) v with v the oracle's
vector (v^T S_w v = 1), so by at most (1 + lambda) e |v|^T M |v|, which the
test allows twice over (the factor covering dS_b through the class means);
the class means and the gradient are held to the same relative size.  The
measured errors are printed.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_soft_case
from tests._parity import TOL_LAM, check_cva_vectors, rel_max

pytestmark = pytest.mark.gpu

U = {"bf16x3": 2.0 ** -8, "f16x3": 2.0 ** -11}


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


def _case(N, B, K, seed, xs=1.0, neg=False):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(800, 3500, (K, B))
    cls = np.arange(N) % K
    X = (mu[cls] + rng.normal(0, 60, (N, B))) * xs
    w = rng.dirichlet(np.full(K, 0.5), N)
    w = 0.5 * w + 0.5 * np.eye(K)[cls]
    if neg:
        w[rng.random(N) < 0.1] -= 0.05
    return X.astype(np.float32), w.astype(np.float32)


def _abs_moment(X, w, means):
    """M = sum_c sum_p |w_pc| |d_p| |d_p|^T, d = x_p - m_c (FP64)."""
    X = X.astype(np.float64)
    M = np.zeros((X.shape[1], X.shape[1]))
    for c in range(w.shape[1]):
        D = np.abs(X - means[c])
        M += (D * np.abs(w[:, c:c + 1]).astype(np.float64)).T @ D
    return M


def _allowed(X, w, ref, prec):
    """Per eigenvalue: 2 (1 + lambda) e |v|^T M |v| + 1e-6 lambda."""
    eps = 2 * U[prec] ** 2 + 512 * 2.0 ** -24
    M = _abs_moment(X, w, ref["class_means"])
    V = np.abs(ref["W"])
    lam = ref["eigvals"]
    return 2 * (1 + lam) * eps * np.einsum("ik,ij,jk->k", V, M, V) + 1e-6 * lam


@pytest.mark.parametrize("N,B,K,xs,neg", [
    (20000, 23, 5, 1.0, False), (5000, 33, 8, 1.0, True), (3000, 7, 3, 1e-3, False), (4000, 64, 12, 1e4, False),
    (1001, 16, 2, 1.0, False)])
def test_plain_soft_path(dev, N, B, K, xs, neg):
    say(f"plain FP32 soft path N={N} B={B} K={K} x*{xs}")
    import paper_1612_06457_amd as cx
    X, w = _case(N, B, K, N + B, xs, neg)
    ref = oracle.soft_fit(X, w)
    Xd, wd = _t(X, dev), _t(w, dev)
    cx.set_plain_fp32(True)
    try:
        fit = cx.cva_soft_forward(Xd, wd)
        g = cx.cva_soft_backward(Xd, fit, 1.0, K).cpu().numpy()
    finally:
        cx.set_plain_fp32(False)
    assert abs(fit.J - ref["J"]) <= TOL_LAM * ref["J"]
    assert np.max(np.abs(fit.eigvals - ref["eigvals"]) / ref["eigvals"]) <= TOL_LAM
    assert rel_max(fit.class_means, ref["class_means"]) <= 1e-6
    check_cva_vectors(fit.W, ref)
    G = fit.W.T @ ref["Sw"] @ fit.W
    assert np.max(np.abs(G - np.eye(G.shape[0]))) <= 1e-5
    g_ref = oracle.soft_grad(X, w)
    gerr = np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))
    say(f"  plain: J err {abs(fit.J - ref['J']) / ref['J']:.2e}, gradient err {gerr:.2e}")
    assert gerr <= 1e-4
    # and against the default path on the same inputs
    d = cx.cva_soft_forward(Xd, wd)
    assert np.max(np.abs(fit.eigvals - d.eigvals) / d.eigvals) <= 2 * TOL_LAM


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("N,B,K,xs,neg", [
    (20000, 23, 5, 1.0, False), (5000, 33, 8, 1.0, True), (3000, 7, 3, 1e-3, False), (4000, 64, 12, 1e4, False),
    (1001, 16, 2, 1.0, False), (6000, 48, 6, 1.0, False)])
def test_split_soft_path(dev, prec, N, B, K, xs, neg):
    say(f"{prec} soft path N={N} B={B} K={K} x*{xs}")
    import paper_1612_06457_amd as cx
    X, w = _case(N, B, K, N + 7 * B, xs, neg)
    ref = oracle.soft_fit(X, w)
    Xd, wd = _t(X, dev), _t(w, dev)
    fit = cx.cva_soft_forward(Xd, wd, precision=prec)
    lam, lam_ref = fit.eigvals, ref["eigvals"]
    allowed = _allowed(X, w, ref, prec)
    lerr = np.max(np.abs(lam - lam_ref) / lam_ref)
    merr = rel_max(fit.class_means, ref["class_means"])
    g = cx.cva_soft_backward(Xd, fit, 1.0, K).cpu().numpy()
    g_ref = oracle.soft_grad(X, w)
    gerr = np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))
    say(f"  {prec}: eigenvalue err {lerr:.2e} (bound {np.max(allowed / lam_ref):.2e}), "
        f"class means {merr:.2e}, gradient {gerr:.2e}")
    assert np.all(np.abs(lam - lam_ref) <= allowed)
    assert abs(fit.J - ref["J"]) <= np.sum(allowed)
    rel_bound = float(np.max(allowed / lam_ref))
    assert merr <= max(1e-6, rel_bound)
    assert gerr <= max(1e-4, 10 * rel_bound)


def test_split_soft_config4_scale(dev):
    """The 1,000,000 x 23, K = 5 soft-label workload at 1/16 of its pixels,
    on both splits: the measured errors against the FP64 oracle."""
    say("split soft paths at the 1M x 23 structure, 1/16 scale")
    import paper_1612_06457_amd as cx
    X, w, _, _, _ = make_soft_case(4, scale=0.25)
    ref = oracle.soft_fit(X, w)
    Xd, wd = _t(X, dev), _t(w, dev)
    for prec in ("bf16x3", "f16x3"):
        fit = cx.cva_soft_forward(Xd, wd, precision=prec)
        allowed = _allowed(X, w, ref, prec)
        lerr = np.max(np.abs(fit.eigvals - ref["eigvals"]) / ref["eigvals"])
        say(f"  {prec}: eigenvalue err {lerr:.2e} (bound {np.max(allowed / ref['eigvals']):.2e}), "
            f"J err {abs(fit.J - ref['J']) / ref['J']:.2e}")
        assert np.all(np.abs(fit.eigvals - ref["eigvals"]) <= allowed)


@pytest.mark.parametrize("plain", [False, True])
def test_soft_shift_sample_misses_a_class(dev, plain):
    """The class shifts come from a strided sample of the chunks of 128
    pixels (every 4th chunk here, 2,048 chunks); a class whose weight lies
    only in chunks outside the sample is shifted by the weighted mean of all
    classes, far from its own mean, and the fit still meets the FP32 bars
    (the scatter carries the shifted sums, so any shift is exact)."""
    say(f"soft forward with a class outside the shift sample (plain={plain})")
    import paper_1612_06457_amd as cx
    N, B, K = 2048 * 128, 23, 5
    rng = np.random.default_rng(11)
    mu = rng.uniform(800, 3500, (K, B))
    chunk = np.arange(N) // 128
    cls = rng.integers(0, K - 1, N)
    last = (chunk % 4 == 1) & (rng.random(N) < 0.5)
    cls[last] = K - 1
    X = (mu[cls] + rng.normal(0, 60, (N, B))).astype(np.float32)
    w = 0.8 * np.eye(K)[cls]
    w[:, : K - 1] += 0.2 * rng.dirichlet(np.full(K - 1, 0.5), N) * (~last)[:, None]
    w[last, K - 1] = 1.0
    w = w.astype(np.float32)
    assert np.all(w[chunk % 4 == 0, K - 1] == 0)
    ref = oracle.soft_fit(X, w)
    Xd, wd = _t(X, dev), _t(w, dev)
    cx.set_plain_fp32(plain)
    try:
        fit = cx.cva_soft_forward(Xd, wd)
        g = cx.cva_soft_backward(Xd, fit, 1.0, K).cpu().numpy()
    finally:
        cx.set_plain_fp32(False)
    lerr = np.max(np.abs(fit.eigvals - ref["eigvals"]) / ref["eigvals"])
    g_ref = oracle.soft_grad(X, w)
    gerr = np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))
    say(f"  eigenvalues {lerr:.2e}, class means {rel_max(fit.class_means, ref['class_means']):.2e}, gradient {gerr:.2e}")
    assert abs(fit.J - ref["J"]) <= TOL_LAM * ref["J"]
    assert lerr <= TOL_LAM
    assert rel_max(fit.class_means, ref["class_means"]) <= 1e-6
    check_cva_vectors(fit.W, ref)
    assert gerr <= 1e-4
