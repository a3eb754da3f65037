"""FP64 soft-label CVA: the Fisher criterion and its gradient.

Not in the paper.  It generalises the paper's CVA (Section 2, canonical
variates paragraph) from hard class labels to real per-pixel class weights
w_pc, so that an analyst's rough training masks can be refined by gradient
steps (the paper re-ran pages with different training points, Section 4,
and calls for automatic choice of training points, Section 4).  With
one-hot weights every quantity below equals the hard-label one.

Definitions (float64):
  n_c = sum_p w_pc,  m_c = sum_p w_pc x_p / n_c,  N = sum_c n_c,
  m = sum_c n_c m_c / N,
  S_w = sum_c sum_p w_pc (x_p - m_c)(x_p - m_c)^T,
  S_b = sum_c n_c (m_c - m)(m_c - m)^T,
  J = sum_k lambda_k = trace(S_w^-1 S_b)  (generalized eigenvalues).

Gradient (closed form, derived from dS_w/dw_pc = (x_p-m_c)(x_p-m_c)^T and
dS_b/dw_pc = (x_p-m)(x_p-m)^T - (x_p-m_c)(x_p-m_c)^T, then
dJ = tr(S_w^-1 dS_b) - tr(S_w^-1 dS_w S_w^-1 S_b)):
  dJ/dw_pc = (x_p-m)^T S_w^-1 (x_p-m)
             - (x_p-m_c)^T (S_w^-1 + S_w^-1 S_b S_w^-1) (x_p-m_c).

Pinned by tests/test_oracle_pca_soft.py: one-hot weights reproduce hard-label
CVA; central differences of the exact finite change of J (rank-one moment
updates) on random (p, c); exact rational arithmetic on a tiny case; and
Euler's identity sum_pc w_pc dJ/dw_pc = 0 (J is homogeneous of degree 0).

Mask refinement (a reading: the paper asks for an automatic choice of
training points, Section 4, and scores images by Eqs. 1-5 of Section 3,
but gives no update rule): one step moves each pixel's weights along the
part of its gradient within the simplex's plane, d = g_p - mean_c g_pc,
scaled so that max_c |d_c| = step, and projects the result back onto the
probability simplex {w >= 0, sum_c w_c = 1} (Euclidean projection by the
sort-based rule of Held, Wolfe and Crowder).  Pinned by
tests/test_oracle_pca_soft.py: the projection satisfies its optimality
conditions (entries above the threshold sum to one; v - w is the same on
the support and v <= theta off it), leaves simplex points unchanged, and
equals a brute-force search for K = 2 and 3; the step leaves a correctly
labelled one-hot pixel in place and moves a mislabelled one to the class
its gradient favours.
"""
from __future__ import annotations

import numpy as np

from .cva import generalized_eig, sign_rule


def soft_moments(X, w):
    """n (K), m_c (K x B), m (B), S_w, S_b in float64, two-pass."""
    X = np.asarray(X, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = w.sum(axis=0)
    mc = (w.T @ X) / n[:, None]
    m = (n[:, None] * mc).sum(axis=0) / n.sum()
    B = X.shape[1]
    Sw = np.zeros((B, B))
    for c in range(w.shape[1]):
        D = X - mc[c][None, :]
        Sw += (D * w[:, c][:, None]).T @ D
    D = mc - m[None, :]
    Sb = (D * n[:, None]).T @ D
    return n, mc, m, 0.5 * (Sw + Sw.T), 0.5 * (Sb + Sb.T)


def soft_fit(X, w, ridge: float = 0.0):
    """J and the canonical basis of the weighted problem.

    Returns dict(J, eigvals (C), W (B x C), mean, class_means, n, Sw, Sb,
    trace_form) with C = min(K-1, B); trace_form = trace(S_w^-1 S_b)."""
    n, mc, m, Sw, Sb = soft_moments(X, w)
    K = mc.shape[0]
    B = X.shape[1] if np.ndim(X) == 2 else mc.shape[1]
    C = min(K - 1, B)
    lam, W = generalized_eig(Sb, Sw, ridge)
    A = Sw + ridge * np.eye(B)
    trace_form = float(np.trace(np.linalg.solve(A, Sb)))
    return dict(J=float(lam[:C].sum()), eigvals=lam[:C].copy(),
                W=sign_rule(W[:, :C]), mean=m, class_means=mc, n=n, Sw=Sw, Sb=Sb,
                trace_form=trace_form)


def soft_grad(X, w, chunk: int = 1 << 18):
    """dJ/dw (N x K) by the closed form above."""
    X = np.asarray(X, dtype=np.float64)
    n, mc, m, Sw, Sb = soft_moments(X, w)
    A = np.linalg.inv(Sw)
    A = 0.5 * (A + A.T)
    Q = A + A @ Sb @ A
    Q = 0.5 * (Q + Q.T)
    N, K = np.shape(w)
    g = np.empty((N, K))
    for s in range(0, N, chunk):
        Xs = X[s:s + chunk]
        D = Xs - m[None, :]
        t = np.einsum("pi,ij,pj->p", D, A, D)
        for c in range(K):
            Dc = Xs - mc[c][None, :]
            g[s:s + chunk, c] = t - np.einsum("pi,ij,pj->p", Dc, Q, Dc)
    return g


def soft_delta_J(X, w, p: int, c: int, h: float, moments=None) -> float:
    """Exact change of J = trace(S_w^-1 S_b) when w_pc becomes w_pc + h.

    Uses the weighted rank-one moment updates
      S_w' = S_w + a u u^T,  a = n_c h / (n_c + h),  u = x_p - m_c,
      S_t' = S_t + b v v^T,  b = N h / (N + h),      v = x_p - m,
    with J = trace(S_w^-1 S_t) - B and Sherman-Morrison for S_w'^-1, so the
    O(h) change is formed without subtracting two large traces.  `moments`
    may carry soft_moments(X, w) to avoid recomputing them."""
    X = np.asarray(X, dtype=np.float64)
    n, mc, m, Sw, Sb = soft_moments(X, w) if moments is None else moments
    St = Sw + Sb
    N = n.sum()
    A = np.linalg.inv(Sw)
    u = X[p] - mc[c]
    v = X[p] - m
    a = n[c] * h / (n[c] + h)
    b = N * h / (N + h)
    Au = A @ u
    den = 1.0 + a * (u @ Au)
    term_w = -a * (Au @ St @ Au) / den
    Av = A @ v
    vSv = v @ Av - a * (Au @ v) ** 2 / den
    return float(term_w + b * vSv)


def simplex_projection(V):
    """Rows of V projected onto the probability simplex (Euclidean): sort each
    row descending, take the largest rho with u_rho > (sum_{i<=rho} u_i - 1)
    / rho, and theta = (sum_{i<=rho} u_i - 1) / rho; w = max(v - theta, 0)."""
    V = np.asarray(V, dtype=np.float64)
    K = V.shape[1]
    U = -np.sort(-V, axis=1)
    css = np.cumsum(U, axis=1) - 1.0
    j = np.arange(1, K + 1)
    ok = U - css / j > 0
    rho = K - 1 - np.argmax(ok[:, ::-1], axis=1)
    theta = css[np.arange(V.shape[0]), rho] / (rho + 1)
    return np.maximum(V - theta[:, None], 0.0)


def soft_update(w, g, step: float):
    """One refinement step of the weights w (N x K) along the gradient g."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    d = g - g.mean(axis=1, keepdims=True)
    s = np.abs(d).max(axis=1, keepdims=True)
    d = np.divide(d, s, out=np.zeros_like(d), where=s > 0)
    return simplex_projection(w + step * d)
