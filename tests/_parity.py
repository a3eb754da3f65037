"""Comparison helpers shared by the GPU parity tests."""
import numpy as np

# FP32 path tolerances (relative to the largest entry / to the range).
TOL_S = 1e-5        # S_w, S_b: max |dS| / max |S|
TOL_LAM = 1e-5      # eigenvalues, relative
TOL_W = 1e-4        # sign-aligned canonical vectors, relative to max |w_j|
TOL_Y = 1e-4        # projection range (min, max), relative to b - a

# Eigenvalues closer than this fraction of the largest one form a cluster
# whose vectors are compared as a subspace.
REL_GAP = 1e-3


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


def eig_clusters(lam, rel_gap=REL_GAP, lam_next=None):
    """Runs of consecutive eigenvalues (descending) whose neighbours lie
    within rel_gap * max |lam| of each other.  Returns (clusters, open_tail):
    a list of index lists covering every column, and whether the last run
    continues into lam_next, the first eigenvalue not returned (its vectors
    are then only fixed together with vectors the caller does not have)."""
    lam = np.asarray(lam, dtype=np.float64)
    scale = float(np.max(np.abs(lam))) if lam.size else 1.0
    clusters = [[0]]
    for j in range(1, lam.size):
        if abs(lam[j - 1] - lam[j]) <= rel_gap * scale:
            clusters[-1].append(j)
        else:
            clusters.append([j])
    open_tail = bool(lam_next is not None and abs(lam[-1] - float(lam_next)) <= rel_gap * scale)
    return clusters, open_tail


def check_vectors(W, W_ref, lam_ref, tol=TOL_W, rel_gap=REL_GAP, A_ref=None, M_ref=None, lam_next=None,
                  tol_s=TOL_S):
    """Check every column of W, eigenvectors of A w = lam M w (M = I when
    M_ref is None), against the reference vectors W_ref.

    A column whose eigenvalue lies more than rel_gap * max |lam| from both
    neighbours is unique up to sign and must equal its reference after sign
    alignment (max |w - w_ref| / max |w_ref| <= tol).  The gap is measured on
    the scale of the largest eigenvalue because that is the size of a
    rounding perturbation of the whitened problem: a vector moves by about
    that perturbation divided by its gap.  A run of nearer eigenvalues fixes
    only the span of its vectors; such a cluster is compared through
    W_c W_c^T, which is the same for every M-orthonormal basis of the span
    (relative to max |W_ref,c W_ref,c^T|).  A run that continues past the
    returned columns (lam_next) cannot be compared as a span and is checked
    only through the reference matrices, which are then required.

    With A_ref: every column is also checked through W^T M W = I and
    W^T A W = diag(lam_ref), which hold for any correct basis whatever the
    gaps.  Their bars are what matrices within tol_s of the references
    (relative to their largest entries, the scatter tolerance) allow:
    tol_s ||M|| ||W||^2 for the first, tol_s (||A|| + max|lam| ||M||)
    ||W||^2 / max|lam| for the second (spectral norms, W the reference
    vectors).

    Returns (signs, worst) with signs the sign alignment of each column
    (meaningful for the singleton columns) and worst the largest vector or
    span difference found."""
    W = np.asarray(W, dtype=np.float64)
    W_ref = np.asarray(W_ref, dtype=np.float64)
    lam_ref = np.asarray(lam_ref, dtype=np.float64)
    assert W.shape == W_ref.shape and W.shape[1] == lam_ref.size
    Wa, s = align_signs(W, W_ref)
    clusters, open_tail = eig_clusters(lam_ref, rel_gap, lam_next)
    worst = 0.0
    checked = np.zeros(W.shape[1], dtype=bool)
    for ci, cl in enumerate(clusters):
        if open_tail and ci == len(clusters) - 1:
            assert A_ref is not None, (
                f"columns {cl} belong to a cluster that continues past the returned vectors; "
                "pass the reference matrices to check them")
            continue
        if len(cl) == 1:
            j = cl[0]
            e = np.max(np.abs(Wa[:, j] - W_ref[:, j])) / np.max(np.abs(W_ref[:, j]))
        else:
            Pg = W[:, cl] @ W[:, cl].T
            Pr = W_ref[:, cl] @ W_ref[:, cl].T
            e = np.max(np.abs(Pg - Pr)) / np.max(np.abs(Pr))
        worst = max(worst, float(e))
        checked[cl] = True
        assert e <= tol, f"canonical vectors {cl} differ by {e:.3e} (tol {tol})"
    if A_ref is not None:
        A_ref = np.asarray(A_ref, dtype=np.float64)
        M = np.eye(W.shape[0]) if M_ref is None else np.asarray(M_ref, dtype=np.float64)
        lmax = float(np.max(np.abs(lam_ref)))
        w2 = np.linalg.norm(W_ref, 2) ** 2
        nM, nA = np.linalg.norm(M, 2), np.linalg.norm(A_ref, 2)
        bar_m = tol_s * nM * w2
        bar_a = tol_s * (nA + lmax * nM) * w2 / lmax
        G = W.T @ M @ W
        eg = float(np.max(np.abs(G - np.eye(G.shape[0]))))
        assert eg <= bar_m, f"W^T M W differs from I by {eg:.3e} (bar {bar_m:.3e})"
        R = W.T @ A_ref @ W
        er = float(np.max(np.abs(R - np.diag(lam_ref))) / lmax)
        assert er <= bar_a, f"W^T A W differs from diag(lam) by {er:.3e} (bar {bar_a:.3e})"
        checked[:] = True
    assert checked.all(), f"columns {np.flatnonzero(~checked).tolist()} were not checked"
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


def check_cva_vectors(W, ref, ridge=0.0, lam_next=None, tol_s=TOL_S):
    """check_vectors for canonical vectors against an oracle CVA fit (hard or
    soft labels): S_b w = lam (S_w + ridge I) w.  When fewer than B vectors
    exist the next eigenvalue is that of the null space of S_b, zero."""
    B, n = np.shape(W)
    if lam_next is None and n == np.size(ref["eigvals"]) and n < B:
        lam_next = 0.0
    M = np.asarray(ref["Sw"]) + ridge * np.eye(B)
    return check_vectors(W, ref["W"], ref["eigvals"], A_ref=ref["Sb"], M_ref=M, lam_next=lam_next, tol_s=tol_s)


def check_pca_vectors(V, pr, tol_s=TOL_S):
    """check_vectors for principal axes against an oracle PCA fit."""
    B, n = np.shape(V)
    lam = pr["all_eigvals"]
    return check_vectors(V, pr["V"], lam[:n], A_ref=pr["cov"], lam_next=lam[n] if n < B else None, tol_s=tol_s)
