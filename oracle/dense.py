"""Small dense kernels of the method, written as textbook loops in float64.

* ``householder_qr`` -- HH(.) of Fig. 4: Householder QR returning an explicit thin
  Q and upper-triangular R, normalised so that diag(R) >= 0 (Fig. 1 caption: the
  QR factorisation is taken with non-negative diagonal).
* ``cholesky_upper`` -- chol(G) of Fig. 2: upper-triangular R with R^T R = G;
  breakdown at the first pivot that is not positive (Section 5.1, recursive
  CholQR discussion) or not finite; the 1-based column is reported.
* ``trsm_right_upper`` -- X = V R^{-1} row by row (the forward substitution of
  Fig. 4a, used by CholQR in Fig. 2b as well).
"""
from __future__ import annotations

import math

import numpy as np


def householder_qr(A: np.ndarray):
    """Return (Q, R, info): A (m x w, m >= w) = Q R, Q^T Q = I, diag(R) >= 0.

    Column j: reflect x = A[j:, j] onto -sign(x_0) ||x|| e_1 with
    H = I - beta v v^T, v = x - alpha e_1, beta = 2 / (v^T v); apply H to the
    trailing columns.  Q is formed by applying the reflectors to [I; 0] in reverse
    order.  info = j+1 if the j-th diagonal of R is exactly zero, else 0.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, w = A.shape
    if m < w:
        raise ValueError("householder_qr needs m >= w")
    refl = []
    for j in range(w):
        x = A[j:, j].copy()
        normx = math.sqrt(float(np.dot(x, x)))
        if normx == 0.0:
            refl.append((None, 0.0))
            continue
        alpha = -math.copysign(normx, x[0])
        v = x
        v[0] -= alpha
        beta = 2.0 / float(np.dot(v, v))
        block = A[j:, j:]
        block -= beta * np.outer(v, v @ block)
        A[j + 1:, j] = 0.0
        refl.append((v, beta))
    R = np.triu(A[:w, :w])
    Q = np.zeros((m, w))
    Q[:w, :w] = np.eye(w)
    for j in reversed(range(w)):
        v, beta = refl[j]
        if v is None:
            continue
        block = Q[j:, :]
        block -= beta * np.outer(v, v @ block)
    d = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    R = d[:, None] * R
    Q = Q * d[None, :]
    info = 0
    for j in range(w):
        if R[j, j] == 0.0:
            info = j + 1
            break
    return Q, R, info


def cholesky_upper(G: np.ndarray):
    """Return (R, info): right-looking Cholesky, R upper with R^T R = G.

    info = 0 on success, else the 1-based column whose pivot was <= 0 or not
    finite (R is then only partially filled).
    """
    A = np.array(G, dtype=np.float64, copy=True)
    w = A.shape[0]
    R = np.zeros((w, w))
    for j in range(w):
        d = A[j, j]
        if not (d > 0.0) or not math.isfinite(d):
            return R, j + 1
        r = math.sqrt(d)
        R[j, j] = r
        R[j, j + 1:] = A[j, j + 1:] / r
        A[j + 1:, j + 1:] -= np.outer(R[j, j + 1:], R[j, j + 1:])
    return R, 0


def trsm_right_upper(V: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X = V R^{-1} for upper-triangular R: x_c = (v_c - sum_{a<c} x_a R[a,c]) / R[c,c].

    Vectorised over rows; the inner sum runs a = 0, 1, ..., c-1 in order.
    """
    V = np.asarray(V, dtype=np.float64)
    n, w = V.shape
    X = np.empty((n, w))
    for c in range(w):
        acc = V[:, c].copy()
        for a in range(c):
            acc -= X[:, a] * R[a, c]
        X[:, c] = acc / R[c, c]
    return X

