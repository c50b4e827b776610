"""Pins for the oracle's accuracy metrics (Section 4: the O(eps) orthogonality target
||I - Q^T Q|| and the backward error ||V - Q R|| / ||V||; Table 1: ||.|| is the l2-norm).

Every reference value here is exact or computed independently of the metric under test:
per-entry ``math.fsum`` (correctly rounded sums), matrices whose Gram matrix is known in
closed form, and residuals planted on rows that Q R does not touch.  The planted
cancellation across row chunks fails the compensated sum if a Neumaier branch is swapped
or the compensation dropped."""
import math

import numpy as np
import pytest

from oracle import metrics


def _fsum_gram(A, B):
    return np.array([[math.fsum(A[:, i] * B[:, j]) for j in range(B.shape[1])] for i in range(A.shape[1])])


def _cancelling_columns(nchunks_small, chunk):
    """Two columns whose row-chunk products are, chunk by chunk: +1 (x nchunks_small), +2^60,
    +1 (x nchunks_small), -2^60.  Every chunk's product sum is exact; the exact total is
    2 * nchunks_small, while a plain running sum of the chunk results returns 0."""
    parts = [1.0] * nchunks_small + [2.0 ** 60] + [1.0] * nchunks_small + [-(2.0 ** 60)]
    a = np.zeros(len(parts) * chunk)
    b = np.zeros(len(parts) * chunk)
    for i, v in enumerate(parts):
        a[i * chunk] = 2.0 ** 30 if abs(v) > 1 else 1.0
        b[i * chunk] = math.copysign(2.0 ** 30, v) if abs(v) > 1 else 1.0
    return a, b


@pytest.mark.parametrize("chunk", [1, 4, 16])
def test_gram_compensates_cancellation_across_chunks(chunk):
    a, b = _cancelling_columns(5, chunk)
    G = metrics.gram(a[:, None], b[:, None], chunk=chunk)
    assert G[0, 0] == 10.0
    # the small terms also arrive after the large one (the other Neumaier branch)
    a2, b2 = a[::-1].copy(), b[::-1].copy()
    assert metrics.gram(a2[:, None], b2[:, None], chunk=chunk)[0, 0] == 10.0
    # a plain sum of the same chunk results loses them
    naive = 0.0
    for i in range(0, a.size, chunk):
        naive += float(a[i:i + chunk] @ b[i:i + chunk])
    assert naive == 0.0


def test_gram_matches_correctly_rounded_sums():
    rng = np.random.default_rng(11)
    n = 20000
    A = rng.standard_normal((n, 5)) * np.exp(rng.uniform(-3, 3, (n, 1)))
    B = rng.standard_normal((n, 3))
    G = metrics.gram(A, B, chunk=512)
    ref = _fsum_gram(A, B)
    scale = np.abs(A).T @ np.abs(B)
    # per-entry error of 512-term chunk dot products, compensated across chunks
    assert np.max(np.abs(G - ref) / scale) <= 600 * 2.0 ** -53
    # the default (one argument) form is A^T A
    GA = metrics.gram(A)
    assert np.max(np.abs(GA - _fsum_gram(A, A)) / (np.abs(A).T @ np.abs(A))) <= 5000 * 2.0 ** -53


@pytest.mark.parametrize("w", [1, 4, 9])
def test_orth_error_of_scaled_orthonormal_columns(w):
    """Q = U diag(1 + d): Q^T Q = diag((1 + d)^2), so ||I - Q^T Q||_2 = max |1 - (1 + d_i)^2|
    and the Frobenius norm is the 2-norm of that vector."""
    n = 3000
    # U: orthonormal columns with exactly representable entries (disjoint supports, +-1/2)
    U = np.zeros((n, w))
    for c in range(w):
        rows = np.arange(4 * c, 4 * c + 4) * 7
        U[rows, c] = np.array([0.5, -0.5, 0.5, 0.5])
    d = np.array([2.0 ** -20 * (c + 1) * (-1) ** c for c in range(w)])
    Q = U * (1.0 + d)
    two, fro = metrics.orth_error(Q)
    exact = np.array([1.0 - (1.0 + x) ** 2 for x in d])
    assert two == pytest.approx(np.max(np.abs(exact)), rel=1e-12)
    assert fro == pytest.approx(np.linalg.norm(exact), rel=1e-12)


def test_orth_error_non_diagonal_gram():
    """Q = U M with U orthonormal and M = P diag(s) P^T (P a rotation): Q^T Q = M^T M has
    eigenvalues s_i^2, so ||I - Q^T Q||_2 = max |1 - s_i^2|.  Taking eigenvalues of Q^T Q
    instead of I - Q^T Q, or dropping the identity, would give about 1."""
    U = np.linalg.qr(np.random.default_rng(3).standard_normal((500, 3)))[0]
    t = 0.3
    P = np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0], [0.0, 0.0, 1.0]])
    s = np.array([1.0 + 1e-9, 1.0 - 3e-9, 1.0 + 2e-10])
    M = P @ np.diag(s) @ P.T
    two, _ = metrics.orth_error(U @ M)
    want = np.max(np.abs(1.0 - s ** 2))
    assert abs(two - want) <= 1e-14
    assert two == pytest.approx(want, rel=1e-4)


def test_orth_error_exact_orthonormal_is_zero():
    Q = np.zeros((64, 4))
    Q[[0, 9, 18, 27], [0, 1, 2, 3]] = 1.0
    assert metrics.orth_error(Q) == (0.0, 0.0)


@pytest.mark.parametrize("chunk", [3, 4096])
def test_backward_error_planted_residual(chunk):
    """V = Q R + E with Q's rows disjoint from E's: ||V - Q R||_F = ||E||_F and
    ||V||_F^2 = ||R||_F^2 + ||E||_F^2 exactly (integer data)."""
    n, w = 1000, 4
    Q = np.zeros((n, w))
    Q[np.arange(w) * 11, np.arange(w)] = 1.0
    R = np.triu(np.arange(1, w * w + 1, dtype=float).reshape(w, w))
    E = np.zeros((n, w))
    E[500:503, :] = np.array([[3.0, 0.0, -1.0, 2.0], [0.0, 4.0, 0.0, 0.0], [1.0, 1.0, 0.0, -2.0]])
    V = Q @ R + E
    got = metrics.backward_error(V, Q, R, chunk=chunk)
    want = math.sqrt(float(np.sum(E * E)) / (float(np.sum(R * R)) + float(np.sum(E * E))))
    assert got == pytest.approx(want, rel=1e-15)
    assert metrics.backward_error(Q @ R, Q, R, chunk=chunk) == 0.0


def test_backward_error_compensates_across_chunks():
    """Residual rows that are tiny next to a huge ||V|| are not lost: the numerator sums
    only the residual, chunk by chunk, with compensation."""
    n, w = 64, 1
    Q = np.zeros((n, w))
    Q[0, 0] = 1.0
    R = np.array([[2.0 ** 40]])
    E = np.zeros((n, w))
    E[8:, 0] = 1.0
    V = Q @ R + E
    got = metrics.backward_error(V, Q, R, chunk=8)
    want = math.sqrt(56.0 / (2.0 ** 80 + 56.0))
    assert got == pytest.approx(want, rel=1e-15)


def test_rel_diff_and_cond2_closed_forms():
    A = np.array([[3.0, 0.0], [0.0, 4.0]])
    B = np.zeros((2, 2))
    assert metrics.rel_diff(A, A) == 0.0
    assert metrics.rel_diff(A + np.array([[0.0, 5.0], [0.0, 0.0]]), A) == 1.0
    assert metrics.rel_diff(A, B) == 5.0          # ||B|| = 0: absolute difference
    assert metrics.cond2(np.diag([2.0, 1e-3, 5.0])) == pytest.approx(5000.0, rel=1e-14)
    assert metrics.cond2(np.array([[1.0, 1.0], [1.0, 1.0]])) >= 1e15
