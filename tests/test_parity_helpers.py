"""The vector comparison the GPU parity tests rely on, pinned on the CPU:
it must accept every correct basis (any signs, any rotation inside a
cluster of equal or nearly equal eigenvalues) and reject a wrong vector
anywhere, including inside a cluster and among small eigenvalues."""
import numpy as np
import pytest
import scipy.linalg

from tests._parity import check_vectors, eig_clusters


def _problem(lam, B, seed, generalized=True):
    """A and M with A w = lam M w for the given eigenvalues (descending) and
    B - len(lam) zero eigenvalues; returns A, M, W (M-orthonormal)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((B, B)))
    d = np.zeros(B)
    d[: len(lam)] = lam
    if generalized:
        G = rng.standard_normal((B, B))
        M = G @ G.T + B * np.eye(B)
    else:
        M = np.eye(B)
    L = np.linalg.cholesky(M)
    W = scipy.linalg.solve_triangular(L.T, Q)        # W^T M W = I
    A = np.linalg.inv(W).T @ np.diag(d) @ np.linalg.inv(W)
    return 0.5 * (A + A.T), M, W


def test_clusters_follow_the_largest_eigenvalue():
    assert eig_clusters([10.0, 5.0, 1.0])[0] == [[0], [1], [2]]
    assert eig_clusters([1000.0, 1.0, 0.5])[0] == [[0], [1, 2]]
    assert eig_clusters([3.0, 3.0, 3.0 - 1e-9, 1.0])[0] == [[0, 1, 2], [3]]
    assert eig_clusters([5.0, 1.0], lam_next=1.0 - 1e-6)[1] is True
    assert eig_clusters([5.0, 1.0], lam_next=0.0)[1] is False


def test_correct_basis_with_flipped_signs_passes():
    lam = np.array([9.0, 4.0, 1.5])
    A, M, W = _problem(lam, 6, 1)
    Wf = W[:, :3] * np.array([1, -1, -1])
    signs, worst = check_vectors(Wf, W[:, :3], lam, A_ref=A, M_ref=M, lam_next=0.0)
    assert signs.tolist() == [1, -1, -1] and worst < 1e-12


def test_wrong_singleton_vector_fails():
    lam = np.array([9.0, 4.0, 1.5])
    A, M, W = _problem(lam, 6, 2)
    Wb = W[:, :3].copy()
    Wb[2, 1] += 0.01 * np.max(np.abs(Wb[:, 1]))
    with pytest.raises(AssertionError):
        check_vectors(Wb, W[:, :3], lam)
    with pytest.raises(AssertionError):
        check_vectors(Wb, W[:, :3], lam, A_ref=A, M_ref=M, lam_next=0.0, tol=1.0)


def test_rotation_inside_a_degenerate_cluster_passes_and_leaving_it_fails():
    lam = np.array([7.0, 3.0, 3.0, 3.0, 1.0])
    A, M, W = _problem(lam, 8, 3)
    R, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((3, 3)))
    Wr = W[:, :5].copy()
    Wr[:, 1:4] = Wr[:, 1:4] @ R                      # another M-orthonormal basis of the span
    check_vectors(Wr, W[:, :5], lam, A_ref=A, M_ref=M, lam_next=0.0)
    check_vectors(Wr, W[:, :5], lam)                 # the span alone, without the matrices
    c, s = np.cos(0.1), np.sin(0.1)
    Wx = W[:, :5].copy()
    Wx[:, 3], Wx[:, 4] = c * W[:, 3] + s * W[:, 4], -s * W[:, 3] + c * W[:, 4]   # mixes in column 4
    with pytest.raises(AssertionError):
        check_vectors(Wx, W[:, :5], lam)


def test_nearly_degenerate_pair_compared_as_a_span():
    lam = np.array([10.0, 2.0 + 1e-7, 2.0, 0.5])
    A, M, W = _problem(lam, 6, 5)
    c, s = np.cos(0.7), np.sin(0.7)
    Wr = W[:, :4].copy()
    Wr[:, 1], Wr[:, 2] = c * W[:, 1] + s * W[:, 2], -s * W[:, 1] + c * W[:, 2]
    check_vectors(Wr, W[:, :4], lam, A_ref=A, M_ref=M, lam_next=0.0)


def test_small_eigenvalues_are_checked_not_skipped():
    """Eigenvalues far below the largest one sit in one cluster (their
    vectors are as uncertain as that cluster's gap to the largest scale
    allows); a wrong vector there still fails through the span and through
    the reference matrices."""
    lam = np.array([1000.0, 1.0, 0.5])
    A, M, W = _problem(lam, 5, 6)
    Wb = W[:, :3].copy()
    Wb[:, 2] = W[:, 3]                               # a null-space vector in place of the third
    with pytest.raises(AssertionError):
        check_vectors(Wb, W[:, :3], lam)
    with pytest.raises(AssertionError):
        check_vectors(Wb, W[:, :3], lam, A_ref=A, M_ref=M, lam_next=0.0, tol=10.0)


def test_cluster_running_past_the_returned_vectors_needs_the_matrices():
    lam = np.array([5.0, 2.0, 2.0, 2.0])
    A, M, W = _problem(lam, 6, 7, generalized=False)
    with pytest.raises(AssertionError, match="continues past"):
        check_vectors(W[:, :2], W[:, :2], lam[:2], lam_next=lam[2])
    R, _ = np.linalg.qr(np.random.default_rng(8).standard_normal((3, 3)))
    Wr = W.copy()
    Wr[:, 1:4] = W[:, 1:4] @ R
    check_vectors(Wr[:, :2], W[:, :2], lam[:2], A_ref=A, lam_next=lam[2])
    Wb = Wr[:, :2].copy()
    Wb[:, 1] = W[:, 4]
    with pytest.raises(AssertionError):
        check_vectors(Wb, W[:, :2], lam[:2], A_ref=A, lam_next=lam[2])
