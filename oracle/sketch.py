"""Random sketches Theta (n x k) and their application Y = Theta^T X.

Section 3 of the paper: a sketch is an n x k random matrix applied as
Theta^T X; the Gaussian choice is Theta = G / sqrt(k) with G standard normal.
Section 5.2 (Count sketch): one +-1 per row of Theta, applied as a sparse
product.  The sparse-sign sketch here generalises that to zeta nonzeros per row
of Theta, each +-1/sqrt(zeta); zeta = 1 is the paper's Count sketch.
Section 5.2 (Count-Gaussian sketch): a Count sketch to O(s^2) rows followed by
a Gaussian sketch to O(s) rows, Theta = Theta_c Theta_g, applied as
Theta_g^T (Theta_c^T X) (Theta_c: kc columns, Theta_g: kc x k Gaussian with
N(0, 1/k) entries, drawn by the input generator).

Nonzero placement (the reading used for the unspecified hash, shared with the
GPU side only as this written definition):

* B = k / zeta slots per nonzero (zeta must divide k, B <= 128).  Nonzero t of
  row i lives in the slot block [t*B, (t+1)*B), so the zeta nonzeros of a row
  are in distinct rows of Theta^T.
* Random bits: nw = ceil(zeta/8) 64-bit words per row; word u of row i is the
  output of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) seeded with ``seed``
  after c+1 steps, c = i*nw + u.
* Byte b = bits [8*(t%8), 8*(t%8)+8) of word t//8: the sign is -1 iff bit 0 of b
  is set, the slot is t*B + floor((b >> 1) * B / 128).
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
SPLITMIX_GAMMA = 0x9E3779B97F4A7C15
SPLITMIX_M1 = 0xBF58476D1CE4E5B9
SPLITMIX_M2 = 0x94D049BB133111EB


def splitmix64_scalar(seed: int, c: int) -> int:
    """Output number c+1 (0-based c) of a SplitMix64 stream started at ``seed``.

    Pure Python integers, written from the generator's published definition:
    the state advances by the golden-ratio increment, the output is the state
    passed through the variant-13 finaliser.
    """
    z = (seed + (c + 1) * SPLITMIX_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * SPLITMIX_M1) & MASK64
    z = ((z ^ (z >> 27)) * SPLITMIX_M2) & MASK64
    return z ^ (z >> 31)


def splitmix64(seed: int, c: np.ndarray) -> np.ndarray:
    """Vectorised ``splitmix64_scalar`` over an array of counters (uint64 wrap-around)."""
    c = np.asarray(c, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + (c + np.uint64(1)) * np.uint64(SPLITMIX_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(SPLITMIX_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(SPLITMIX_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def sparse_sign_pattern(rows: np.ndarray, k: int, zeta: int, seed: int):
    """Slots (len(rows) x zeta, int64) and signs (+-1.0) of the given rows of Theta."""
    if zeta < 1 or k % zeta != 0:
        raise ValueError("zeta must divide k")
    B = k // zeta
    if B > 128:
        raise ValueError("k/zeta must be <= 128")
    rows = np.asarray(rows, dtype=np.int64)
    nw = (zeta + 7) // 8
    slots = np.empty((rows.size, zeta), dtype=np.int64)
    signs = np.empty((rows.size, zeta), dtype=np.float64)
    for u in range(nw):
        word = splitmix64(seed, rows.astype(np.uint64) * np.uint64(nw) + np.uint64(u))
        for tt in range(8):
            t = 8 * u + tt
            if t >= zeta:
                break
            b = ((word >> np.uint64(8 * tt)) & np.uint64(0xFF)).astype(np.int64)
            signs[:, t] = np.where(b & 1, -1.0, 1.0)
            slots[:, t] = t * B + (((b >> 1) * B) >> 7)
    return slots, signs


def sparse_sign_dense(n: int, k: int, zeta: int, seed: int) -> np.ndarray:
    """Materialise Theta (n x k) from the definition above (small n only)."""
    slots, signs = sparse_sign_pattern(np.arange(n), k, zeta, seed)
    theta = np.zeros((n, k))
    scale = 1.0 / math.sqrt(zeta)
    for i in range(n):
        for t in range(zeta):
            theta[i, slots[i, t]] = signs[i, t] * scale
    return theta


class Sketch:
    """Description of Theta: ``kind`` is 'gaussian' (explicit n x k array), 'sparse_sign',
    or 'count_gauss' (sparse-sign Theta_c with kc columns times the kc x k array theta)."""

    def __init__(self, kind: str, k: int, zeta: int = 1, seed: int = 0, theta: np.ndarray | None = None,
                 kc: int = 0):
        if kind not in ("gaussian", "sparse_sign", "dense", "count_gauss"):
            raise ValueError(kind)
        self.kind, self.k, self.zeta, self.seed, self.theta = kind, int(k), int(zeta), int(seed), theta
        self.kc = int(kc)

    @staticmethod
    def gaussian(theta: np.ndarray) -> "Sketch":
        return Sketch("gaussian", theta.shape[1], theta=np.asarray(theta, dtype=np.float64))

    @staticmethod
    def sparse_sign(k: int, zeta: int, seed: int) -> "Sketch":
        return Sketch("sparse_sign", k, zeta, seed)

    @staticmethod
    def count_gauss(kc: int, zeta: int, seed: int, theta_g: np.ndarray) -> "Sketch":
        """Count-Gaussian composite (Section 5.2): sparse-sign (kc rows, zeta nonzeros per row
        of Theta_c, stream ``seed``) followed by the Gaussian factor theta_g (kc x k)."""
        theta_g = np.asarray(theta_g, dtype=np.float64)
        if theta_g.shape[0] != kc:
            raise ValueError("the Gaussian factor must have kc rows")
        return Sketch("count_gauss", theta_g.shape[1], zeta, seed, theta=theta_g, kc=kc)

    @staticmethod
    def dense(theta: np.ndarray) -> "Sketch":
        """Any explicit Theta (used by tests, e.g. Theta = I)."""
        return Sketch("dense", theta.shape[1], theta=np.asarray(theta, dtype=np.float64))

    def apply(self, X: np.ndarray) -> np.ndarray:
        return apply_sketch(self, X)


def apply_sketch(sk: Sketch, X: np.ndarray) -> np.ndarray:
    """Y = Theta^T X (k x w) in float64."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    n, w = X.shape
    if sk.kind in ("gaussian", "dense"):
        if sk.theta.shape[0] != n:
            raise ValueError("theta has the wrong number of rows")
        return sk.theta.T @ X
    if sk.kind == "count_gauss":
        # the Count part first, then the Gaussian factor on its kc x w result
        return sk.theta.T @ _apply_sparse_sign(sk.kc, sk.zeta, sk.seed, X)
    return _apply_sparse_sign(sk.k, sk.zeta, sk.seed, X)


def _apply_sparse_sign(k: int, zeta: int, seed: int, X: np.ndarray) -> np.ndarray:
    n, w = X.shape
    slots, signs = sparse_sign_pattern(np.arange(n), k, zeta, seed)
    scale = 1.0 / math.sqrt(zeta)
    Y = np.zeros((k, w))
    for t in range(zeta):
        coef = signs[:, t] * scale
        for c in range(w):
            Y[:, c] += np.bincount(slots[:, t], weights=coef * X[:, c], minlength=k)
    return Y
