"""Accuracy metrics, accumulated so that the measurement error stays near machine precision.

Orthogonality error ||I - Q^T Q|| (Section 4, eq. for the O(eps) target) and the
backward error ||V - Q R|| / ||V|| (Section 4, intra-block conditions).  Sums over
the long dimension n are taken as float64 products over row chunks of 4096 rows,
and the chunk results are combined with Neumaier's compensated summation, so
the error of the metric itself is a few units of rounding even for n = 2^24.
The spectral norm of the small matrix I - Q^T Q is its largest singular value
(the l2-norm of the paper's notation table, Table 1), so no symmetrisation of the computed Gram
matrix is involved.
"""
from __future__ import annotations

import numpy as np

CHUNK = 4096


class _Neumaier:
    def __init__(self, shape):
        self.s = np.zeros(shape)
        self.c = np.zeros(shape)

    def add(self, t):
        s = self.s
        tot = s + t
        big = np.abs(s) >= np.abs(t)
        self.c += np.where(big, (s - tot) + t, (t - tot) + s)
        self.s = tot

    def value(self):
        return self.s + self.c


def gram(A: np.ndarray, B: np.ndarray | None = None, chunk: int = CHUNK) -> np.ndarray:
    """A^T B (float64) with compensated accumulation over row chunks."""
    B = A if B is None else B
    acc = _Neumaier((A.shape[1], B.shape[1]))
    for i in range(0, A.shape[0], chunk):
        a = np.asarray(A[i:i + chunk], dtype=np.float64)
        b = np.asarray(B[i:i + chunk], dtype=np.float64)
        acc.add(a.T @ b)
    return acc.value()


def orth_error(Q: np.ndarray):
    """(||I - Q^T Q||_2, ||I - Q^T Q||_F)."""
    E = np.eye(Q.shape[1]) - gram(Q)
    two = float(np.linalg.svd(E, compute_uv=False)[0]) if E.size else 0.0
    return two, float(np.linalg.norm(E))


def backward_error(V: np.ndarray, Q: np.ndarray, R: np.ndarray, chunk: int = CHUNK) -> float:
    """||V - Q R||_F / ||V||_F."""
    num = _Neumaier(())
    den = _Neumaier(())
    for i in range(0, V.shape[0], chunk):
        v = np.asarray(V[i:i + chunk], dtype=np.float64)
        q = np.asarray(Q[i:i + chunk], dtype=np.float64)
        d = v - q @ R
        num.add(float(np.sum(d * d)))
        den.add(float(np.sum(v * v)))
    return float(np.sqrt(num.value() / den.value()))


def rel_diff(A: np.ndarray, B: np.ndarray) -> float:
    """||A - B||_F / ||B||_F."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / (nb if nb > 0 else 1.0))


def cond2(X: np.ndarray) -> float:
    s = np.linalg.svd(np.asarray(X, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")
