"""FP64 cluster-separation indices of labelled points (test infrastructure:
only the tests, the smoke check and the benchmark's CPU baseline use this
package).

Paper, Section 3, Eqs. 1-5: for clusters i and j of feature vectors,
S_i = (1/T_i) sum_j ||X_j - A_i||_p with A_i the centroid (Eq. 1),
M_ij = ||A_i - A_j||_p (Eq. 2), the Davies-Bouldin ratio
R_ij = (S_i + S_j) / M_ij (Eq. 3) and the Dunn index with the paper's
proxies, (M_ij - S_i - S_j) / max(S_i, S_j) (Eqs. 4-5).

Readings (the paper compares two clusters only): for K clusters the
Davies-Bouldin index is the usual (1/K) sum_i max_{j != i} R_ij and the Dunn
index min_{i != j} (M_ij - S_i - S_j) / max_k S_k; both reduce to Eqs. 3
and 5 for K = 2.  A point's feature vector is the values of the given
images at its pixel (the paper: the grayscale image with the clearest
underwriting, one feature).

Pinned by tests/test_oracle_cva.py: two one-dimensional clusters with known
centroids and scatters give R and D in closed form; a three-cluster case
gives both K-cluster indices by hand; a brute-force loop over points gives
the same S and M; R and D are unchanged by scaling and shifting all the
features; p = 1 and p = 2 on two-dimensional points match hand values.
The paper's own index values need its images: parity unpinned for those.
"""
from __future__ import annotations

import numpy as np


def _norm(d: np.ndarray, p: float, axis=-1) -> np.ndarray:
    d = np.abs(np.asarray(d, dtype=np.float64))
    if p == 2.0:
        return np.sqrt(np.sum(d * d, axis=axis))
    if p == 1.0:
        return np.sum(d, axis=axis)
    return np.sum(d ** p, axis=axis) ** (1.0 / p)


def cluster_indices(images, pixels, classes, K: int, p: float = 2.0) -> dict:
    """images: n x ... planes (any numeric type); pixels: flat pixel
    indices; classes: -1 (skip) or 0..K-1 per point."""
    imgs = np.asarray(images)
    n = imgs.shape[0]
    flat = imgs.reshape(n, -1)
    pix = np.asarray(pixels, dtype=np.int64)
    cls = np.asarray(classes, dtype=np.int64)
    if pix.shape != cls.shape:
        raise ValueError("pixels and classes must have the same length")
    if cls.size and (cls.min() < -1 or cls.max() >= K):
        raise ValueError("a class lies outside -1..K-1")
    if pix.size and (pix.min() < 0 or pix.max() >= flat.shape[1]):
        raise ValueError("a point lies outside the page")
    X = flat[:, pix].T.astype(np.float64)          # N x n feature vectors
    A = np.empty((K, n))
    S = np.empty(K)
    counts = np.empty(K, dtype=np.int64)
    for k in range(K):
        Xk = X[cls == k]
        if Xk.shape[0] == 0:
            raise ValueError(f"class {k} has no point")
        counts[k] = Xk.shape[0]
        A[k] = Xk.mean(axis=0)                                     # centroid
        S[k] = _norm(Xk - A[k][None, :], p, axis=1).mean()         # Eq. 1
    M = np.zeros((K, K))
    R = np.zeros((K, K))
    D = np.zeros((K, K))
    for i in range(K):
        for j in range(K):
            if i != j:
                M[i, j] = _norm(A[i] - A[j], p)                    # Eq. 2
                R[i, j] = (S[i] + S[j]) / M[i, j]                  # Eq. 3
                D[i, j] = (M[i, j] - S[i] - S[j]) / max(S[i], S[j])  # Eq. 5
    off = ~np.eye(K, dtype=bool)
    dbi = float(np.mean([R[i][off[i]].max() for i in range(K)]))
    gaps = (M - S[:, None] - S[None, :])[off]
    dunn = float(gaps.min() / S.max())
    return {"centroids": A, "scatter": S, "dist": M, "dbi_pairs": R, "dunn_pairs": D,
            "dbi": dbi, "dunn": dunn, "counts": counts}
