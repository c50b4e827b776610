"""Pins for the oracle's small dense kernels against LAPACK (numpy/scipy)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense
from oracle.krylov import hessenberg_lsq


def _signfix(Q, R):
    d = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * d, d[:, None] * R


@pytest.mark.parametrize("m,w", [(24, 6), (64, 6), (128, 11), (48, 21), (7, 7)])
def test_householder_matches_lapack(m, w):
    A = np.random.default_rng(m * w).standard_normal((m, w))
    Q, R, info = dense.householder_qr(A)
    assert info == 0
    Ql, Rl = _signfix(*np.linalg.qr(A))
    assert np.all(np.diag(R) >= 0)
    assert np.max(np.abs(R - Rl)) <= 1e-13 * np.abs(Rl).max()
    assert np.max(np.abs(Q - Ql)) <= 1e-13
    assert np.max(np.abs(Q.T @ Q - np.eye(w))) <= 1e-14


def test_householder_zero_column_reports_breakdown():
    A = np.random.default_rng(1).standard_normal((20, 5))
    A[:, 2] = A[:, 0] * 2.0 - A[:, 1] * 0.0  # exact dependence is not exact in floating point
    A[:, 3] = 0.0
    _, _, info = dense.householder_qr(A)
    assert info == 4


@pytest.mark.parametrize("w", [1, 6, 11, 36, 61])
def test_cholesky_matches_lapack(w):
    X = np.random.default_rng(w).standard_normal((3 * w + 5, w))
    G = X.T @ X
    R, info = dense.cholesky_upper(G)
    assert info == 0
    Rl = np.linalg.cholesky(G).T
    assert np.max(np.abs(R - Rl)) <= 1e-13 * np.abs(Rl).max()


@pytest.mark.parametrize("G,col", [
    (np.diag([1.0, -1.0, 1.0]), 2),
    (np.array([[1.0, 1.0], [1.0, 1.0]]), 2),
    (np.array([[0.0, 0.0], [0.0, 1.0]]), 1),
    (np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]]), 2),
    (np.array([[1.0, np.nan], [np.nan, 1.0]]), 2),
])
def test_cholesky_breakdown_column(G, col):
    _, info = dense.cholesky_upper(G)
    assert info == col


@pytest.mark.parametrize("w", [1, 6, 11])
def test_trsm_matches_scipy(w):
    rng = np.random.default_rng(w + 100)
    V = rng.standard_normal((500, w))
    R = np.triu(rng.standard_normal((w, w))) + 3 * np.eye(w)
    X = dense.trsm_right_upper(V, R)
    Xl = sla.solve_triangular(R.T, V.T, lower=True).T
    assert np.max(np.abs(X - Xl)) <= 1e-13 * np.abs(Xl).max()


@pytest.mark.parametrize("k", [1, 5, 30, 60])
def test_hessenberg_lsq_matches_lstsq(k):
    rng = np.random.default_rng(k)
    H = np.triu(rng.standard_normal((k + 1, k)), -1) + 4.0 * np.eye(k + 1, k)
    g = np.zeros(k + 1)
    g[0] = 2.5
    y, res = hessenberg_lsq(H, g)
    yl, *_ = np.linalg.lstsq(H, g, rcond=None)
    assert np.max(np.abs(y - yl)) <= 1e-10 * max(1.0, np.abs(yl).max())
    assert abs(res - np.linalg.norm(g - H @ yl)) <= 1e-12 * 2.5
