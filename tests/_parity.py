"""Comparison helpers shared by the GPU parity tests."""
import numpy as np

# FP32 path tolerances (relative to the largest entry / to the range).
TOL_S = 1e-5        # S_w, S_b: max |dS| / max |S|
TOL_LAM = 1e-5      # eigenvalues, relative
TOL_W = 1e-4        # sign-aligned canonical vectors, relative to max |w_j|
TOL_Y = 1e-4        # projection range (min, max), relative to b - a


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def align_signs(W, W_ref):
    """Flip columns of W to agree in sign with W_ref; returns (W', signs)."""
    W = np.array(W, dtype=np.float64, copy=True)
    s = np.sign(np.sum(W * W_ref, axis=0))
    s[s == 0] = 1
    return W * s[None, :], s


def check_vectors(W, W_ref, lam_ref, tol=TOL_W):
    """Columns with a well separated eigenvalue must match after sign
    alignment; degenerate pairs are compared as subspaces."""
    Wa, s = align_signs(W, W_ref)
    C = W_ref.shape[1]
    worst = 0.0
    for j in range(C):
        gap_lo = abs(lam_ref[j - 1] - lam_ref[j]) if j > 0 else np.inf
        gap_hi = abs(lam_ref[j] - lam_ref[j + 1]) if j + 1 < C else np.inf
        if min(gap_lo, gap_hi) > 1e-3 * abs(lam_ref[0]):
            e = np.max(np.abs(Wa[:, j] - W_ref[:, j])) / np.max(np.abs(W_ref[:, j]))
            worst = max(worst, e)
    assert worst <= tol, f"canonical vectors differ by {worst:.3e} (tol {tol})"
    return s, worst


def check_images(q, q_ref, signs=None, max_diff=1):
    """8-bit images equal within max_diff grey levels; a component whose
    vector has the opposite sign is compared as 255 - q.  Returns the
    fraction of bytes that differ."""
    q = np.asarray(q).astype(np.int32)
    q_ref = np.asarray(q_ref).astype(np.int32)
    assert q.shape == q_ref.shape
    ndiff = 0
    for j in range(q.shape[0]):
        a = q[j]
        if signs is not None and signs[j] < 0:
            a = 255 - a
        d = np.abs(a - q_ref[j])
        assert d.max() <= max_diff, f"component {j}: max grey-level difference {d.max()}"
        ndiff += int((d != 0).sum())
    return ndiff / q.size
