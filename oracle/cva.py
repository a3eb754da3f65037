"""FP64 canonical variates analysis, written as its definition reads.

Paper, Section 2 (canonical variates paragraph): CVA computes the
covariance within each class and between the classes, and an eigenanalysis
of these two matrices gives the canonical vectors used to make new greyscale
images.  Section 4 (the GSL implementation) names the eigensolver as a
generalized symmetric-definite one, i.e. S_b w = lambda S_w w with S_w
positive definite.  Section 2 (regression coefficients paragraph): the
coefficients multiply every band of the whole page and each resulting float
image is rescaled to 0..255.

Readings where the paper is silent (each also listed in the design notes):

* scatter, not covariance: S_w and S_b are plain sums, without division by
  degrees of freedom (eigenvectors are unchanged; eigenvalues scale);
* the grand mean is the mean of all training pixels (count-weighted), so
  S_w + S_b equals the total scatter of the training pixels;
* eigenvectors are scaled so that w^T S_w w = 1, sorted by descending
  eigenvalue, and only C = min(K-1, B) are kept (the rest span the null
  space of S_b and are not unique);
* sign: the entry of largest magnitude in each eigenvector is made positive,
  ties going to the lowest band index (the paper notes that two correct
  solvers gave opposite signs, Section 4, Figure 5);
* projections are centred on the grand mean before the rescale (the min-max
  rescale is shift invariant, so the 8-bit image does not depend on it).

Pinned by tests/test_oracle_cva.py: brute-force loops and exact rational
arithmetic on tiny pages, S_w + S_b = S_t, W^T S_w W = I and
W^T S_b W = diag(lambda), the two-class closed form of Fisher's
discriminant, constructed samples whose Fisher ratios are known in closed
form, and invariance of the projections under invertible affine band maps.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _rows(cube) -> np.ndarray:
    """View a band-interleaved H x W x B cube as P x B rows (no copy when
    possible).  Torch tensors (bf16/fp16 included) are upcast exactly."""
    if hasattr(cube, "detach"):
        t = cube.detach().cpu()
        if t.dtype in (getattr(__import__("torch"), "bfloat16"),
                       getattr(__import__("torch"), "float16")):
            t = t.float()
        cube = t.numpy()
    cube = np.asarray(cube)
    return cube.reshape(-1, cube.shape[-1])


def _is_int(a: np.ndarray) -> bool:
    return np.issubdtype(a.dtype, np.integer)


def class_counts(labels, K: int) -> np.ndarray:
    """n_k = number of training pixels labelled k (labels -1 are ignored)."""
    lab = np.asarray(labels).reshape(-1)
    if lab.size and (lab.min() < -1 or lab.max() >= K):
        raise ValueError("labels must lie in {-1, 0..K-1}")
    return np.bincount(lab[lab >= 0].astype(np.int64), minlength=K).astype(np.int64)


def class_index_lists(labels, K: int):
    """Raster-ordered pixel indices of each class."""
    lab = np.asarray(labels).reshape(-1)
    return [np.flatnonzero(lab == k) for k in range(K)]


def class_moments(cube, labels, K: int):
    """Counts n_k, class sums s_k and class means m_k = s_k / n_k.

    Sums are exact int64 for integer pages, float64 otherwise."""
    X = _rows(cube)
    B = X.shape[1]
    idx = class_index_lists(labels, K)
    counts = np.array([i.size for i in idx], dtype=np.int64)
    if _is_int(X):
        sums = np.zeros((K, B), dtype=np.int64)
        for k in range(K):
            sums[k] = X[idx[k]].astype(np.int64).sum(axis=0)
    else:
        sums = np.zeros((K, B), dtype=np.float64)
        for k in range(K):
            sums[k] = X[idx[k]].astype(np.float64).sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        means = sums.astype(np.float64) / counts[:, None]
    return counts, sums, means


def within_scatter(cube, labels, K: int, means: np.ndarray) -> np.ndarray:
    """S_w = sum_k sum_{p in k} (x_p - m_k)(x_p - m_k)^T, two-pass centred."""
    X = _rows(cube)
    B = X.shape[1]
    Sw = np.zeros((B, B))
    for k, ix in enumerate(class_index_lists(labels, K)):
        if ix.size == 0:
            continue
        D = X[ix].astype(np.float64) - means[k][None, :]
        Sw += D.T @ D
    return 0.5 * (Sw + Sw.T)


def between_scatter(counts: np.ndarray, means: np.ndarray) -> np.ndarray:
    """S_b = sum_k n_k (m_k - m)(m_k - m)^T with m the count-weighted mean."""
    n = counts.astype(np.float64)
    m = (n[:, None] * means).sum(axis=0) / n.sum()
    D = means - m[None, :]
    Sb = (D * n[:, None]).T @ D
    return 0.5 * (Sb + Sb.T)


def total_scatter(cube, labels) -> np.ndarray:
    """S_t of all training pixels about their mean."""
    X = _rows(cube)
    lab = np.asarray(labels).reshape(-1)
    Y = X[lab >= 0].astype(np.float64)
    D = Y - Y.mean(axis=0)[None, :]
    St = D.T @ D
    return 0.5 * (St + St.T)


def sign_rule(W: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (ties: the
    lowest row index)."""
    W = np.array(W, dtype=np.float64, copy=True)
    for j in range(W.shape[1]):
        i = int(np.argmax(np.abs(W[:, j])))
        if W[i, j] < 0:
            W[:, j] = -W[:, j]
    return W


def generalized_eig(Sb: np.ndarray, Sw: np.ndarray, ridge: float = 0.0):
    """All eigenpairs of S_b w = lambda (S_w + ridge I) w, descending, with
    w^T (S_w + ridge I) w = 1 (LAPACK's symmetric-definite solver)."""
    B = Sw.shape[0]
    A = Sw + ridge * np.eye(B)
    try:
        lam, W = scipy.linalg.eigh(Sb, A)
    except np.linalg.LinAlgError as e:
        raise ValueError("S_w is not positive definite") from e
    order = np.argsort(lam)[::-1]
    return lam[order], W[:, order]


def cva_fit(cube, labels, K: int, ridge: float = 0.0, n_comp: int | None = None):
    """Fit CVA on the labelled pixels of a page.

    Returns a dict with W (B x C), eigvals (C), mean (B, the grand mean used
    to centre projections), counts (K), class_means (K x B), Sw and Sb."""
    X = _rows(cube)
    B = X.shape[1]
    if K < 2:
        raise ValueError("need at least two classes")
    counts, sums, means = class_moments(cube, labels, K)
    if (counts < 1).any():
        raise ValueError("empty class")
    Sw = within_scatter(cube, labels, K, means)
    Sb = between_scatter(counts, means)
    C = min(K - 1, B)
    if n_comp is None:
        n_comp = C
    if not (1 <= n_comp <= C):
        raise ValueError("n_comp must lie in 1..min(K-1, B)")
    lam, W = generalized_eig(Sb, Sw, ridge)
    W = sign_rule(W[:, :n_comp])
    n = counts.astype(np.float64)
    mean = (n[:, None] * means).sum(axis=0) / n.sum()
    return dict(W=W, eigvals=lam[:n_comp].copy(), mean=mean, counts=counts,
                class_sums=sums, class_means=means, Sw=Sw, Sb=Sb)


def cva_fit_points(cube, pixels, classes, K: int, ridge: float = 0.0, n_comp: int | None = None):
    """Fit CVA on a list of training points (paper Section 2: a set of
    points per class, picked by the analyst; Section 4: given as (x, y)
    coordinates).  pixels holds y * width + x; classes holds -1 (skip) or
    0..K-1.  Each entry is one training sample, so a repeated pixel counts
    as often as it is listed.  The fit is the same as cva_fit over the
    listed rows."""
    X = _rows(cube)
    pix = np.asarray(pixels, dtype=np.int64).reshape(-1)
    cls = np.asarray(classes).reshape(-1)
    if pix.shape != cls.shape:
        raise ValueError("pixels and classes must have the same length")
    if pix.size and (pix.min() < 0 or pix.max() >= X.shape[0]):
        raise ValueError("a training point lies outside the page")
    rows = X[pix][None, :, :]                # a 1 x N "page" of the listed rows
    return cva_fit(rows, cls[None, :], K, ridge=ridge, n_comp=n_comp)


def project(cube, W: np.ndarray, center: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """y_p = W^T (x_p - center) for every pixel, float64, P x C."""
    X = _rows(cube)
    P = X.shape[0]
    W = np.asarray(W, dtype=np.float64)
    center = np.asarray(center, dtype=np.float64)
    y = np.empty((P, W.shape[1]))
    for s in range(0, P, chunk):
        y[s:s + chunk] = (X[s:s + chunk].astype(np.float64) - center[None, :]) @ W
    return y


def cva_project(cube, W: np.ndarray, center: np.ndarray):
    """Project the whole page and stretch each component to 8 bits.

    Returns (images C x H x W uint8, ranges C x 2 of (min, max) of y)."""
    from .stretch import stretch_minmax
    shape = np.shape(cube) if not hasattr(cube, "shape") else tuple(cube.shape)
    H, Wd = int(shape[0]), int(shape[1])
    y = project(cube, W, center)
    q, a, b = stretch_minmax(y)
    C = y.shape[1]
    images = np.ascontiguousarray(q.T).reshape(C, H, Wd)
    return images, np.stack([a, b], axis=1)
