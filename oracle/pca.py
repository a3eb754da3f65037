"""FP64 principal component analysis of a page.

Paper, Section 2 (PCA paragraph): subtract the mean of each variable,
form the covariance matrix, take its eigenvectors and eigenvalues, and keep
them orthonormal.  The unsupervised variants use the entire page (Section 2,
the ImageJ/Matlab paragraph, after cropping to the folio, which the optional
pixel mask expresses); the supervised variant uses only the training pixels.

Readings: covariance PCA on the raw values by default, divided by P - 1;
components sorted by descending eigenvalue; sign as in CVA (largest entry
of each returned vector positive).  With standardize=True each band is
first scaled to unit variance over the selected pixels (the toolbox
methods the paper compares with standardise their inputs, Section 2), so
the eigenproblem is that of the correlation matrix R = D^-1/2 C D^-1/2
(D = diag C), and the returned vectors are the projection vectors
v_j = D^-1/2 u_j: v_j^T (x - mean) is the score of the standardised bands,
C v = lambda D v, v^T D v = 1.

Pinned by tests/test_oracle_pca_soft.py: trace(cov) equals the sum of all
eigenvalues, V is orthonormal, a brute-force loop covariance on tiny pages,
numpy.cov, and constructed data whose covariance eigenvalues are known;
standardised: the eigenvalues sum to B, the scores do not change when a
band is multiplied by a positive constant, and they equal the covariance
PCA scores of data standardised beforehand.
"""
from __future__ import annotations

import numpy as np

from .cva import _rows, _is_int, sign_rule, cva_project


def pca_moments(cube, mask=None, chunk: int = 1 << 20):
    """Mean and covariance (divisor P - 1) of the selected pixels, two-pass."""
    X = _rows(cube)
    if mask is not None:
        X = X[np.asarray(mask).reshape(-1).astype(bool)]
    P, B = X.shape
    if P < 2:
        raise ValueError("need at least two pixels")
    if _is_int(X):
        s = np.zeros(B, dtype=np.int64)
        for i in range(0, P, chunk):
            s += X[i:i + chunk].astype(np.int64).sum(axis=0)
        mean = s.astype(np.float64) / P
    else:
        s = np.zeros(B)
        for i in range(0, P, chunk):
            s += X[i:i + chunk].astype(np.float64).sum(axis=0)
        mean = s / P
    G = np.zeros((B, B))
    for i in range(0, P, chunk):
        D = X[i:i + chunk].astype(np.float64) - mean[None, :]
        G += D.T @ D
    cov = 0.5 * (G + G.T) / (P - 1)
    return mean, cov, P


def pca_fit(cube, mask=None, n_comp: int = 3, standardize: bool = False):
    """Top n_comp principal axes: dict(V B x n, eigvals n, mean B, cov B x B,
    all_eigvals B, metric B x B); metric is the matrix M with V^T M V = I
    (the identity, or D = diag(cov) when standardised)."""
    mean, cov, P = pca_moments(cube, mask)
    B = cov.shape[0]
    if not (1 <= n_comp <= B):
        raise ValueError("n_comp must lie in 1..B")
    if standardize:
        sd = np.sqrt(np.diag(cov))
        if not np.all(sd > 0):
            raise ValueError("a band has zero variance")
        A = cov / np.outer(sd, sd)
    else:
        sd = np.ones(B)
        A = cov
    lam, U = np.linalg.eigh(A)
    order = np.argsort(lam)[::-1]
    lam, U = lam[order], U[:, order]
    V = U[:, :n_comp] / sd[:, None]
    return dict(V=sign_rule(V), eigvals=lam[:n_comp].copy(), mean=mean, cov=cov, all_eigvals=lam,
                metric=np.diag(sd ** 2) if standardize else np.eye(B), n_pixels=P)


def pca_project(cube, V: np.ndarray, mean: np.ndarray):
    """Same projection and min-max stretch as CVA, with (V, mean)."""
    return cva_project(cube, V, mean)
