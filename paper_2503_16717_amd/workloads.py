"""Seeded synthetic inputs for sketched block orthogonalization and s-step GMRES.

This module only *draws* inputs: sparse matrices in CSR form, right-hand sides,
test blocks with a prescribed condition number and the dense Gaussian sketch
matrix.  It holds none of the method's arithmetic, and both the HIP path and the
CPU oracle receive their inputs from here.

Recipes (all seeded, all float64 on the host, CSR indices int32, columns sorted):

* ``laplacian_2d(N)`` / ``laplacian_3d(N)``: unscaled 5-/7-point stencil
  (2d on the diagonal, -1 per neighbour), zero Dirichlet boundary,
  lexicographic numbering ``i = x + N*y (+ N*N*z)``.  The paper's MPK experiment
  (Section 9, Fig. 12) and strong-scaling runs (Table 5) use Laplace matrices
  without stating the scaling; the integer stencil is the reading used here.
* ``convdiff_2d`` / ``convdiff_3d``: -Lap(u) + b.grad(u) on the unit cube with
  h = 1/(N+1), first-order upwind differences for b >= 0, rows multiplied by h^2:
  centre 2d + h*sum(b), the upwind neighbour in direction d gets -1 - h*b_d,
  the downwind neighbour -1.
* ``glued_blocks``: nb blocks V_j = U_j diag(sigma) W_j^T with U_j (n x w) and
  W_j (w x w) the orthonormal factors of seeded standard normal matrices and
  sigma log-spaced from 1 down to 10^-e.  This stands in for the paper's
  ``glued`` test matrices (Section 9), whose generator is not reproduced.
* ``gaussian_theta``: the n x k dense Gaussian sketch with N(0, 1/k) entries
  (Section 3: Theta = G / sqrt(k)).
* ``rhs_uniform``: entries uniform in [-1, 1].
* ``batched_convdiff``: per-system grid sizes and winds for many independent
  2-D convection-diffusion solves.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CSR", "laplacian_2d", "laplacian_3d", "convdiff_2d", "convdiff_3d",
    "glued_blocks", "glued_block", "gaussian_theta", "rhs_uniform", "batched_convdiff_specs",
]


class CSR:
    """Plain holder for a square CSR matrix (int32 indices, float64 values)."""

    def __init__(self, n: int, rowptr: np.ndarray, colind: np.ndarray, val: np.ndarray):
        self.n = int(n)
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self.colind = np.ascontiguousarray(colind, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))


def _stencil_csr(dims: tuple[int, ...], centre: float, lower: list[float], upper: list[float]) -> CSR:
    """Assemble a constant-coefficient (2*len(dims)+1)-point stencil on a box grid.

    ``lower[d]`` multiplies the neighbour at coordinate x_d - 1, ``upper[d]`` the
    one at x_d + 1.  Neighbours outside the box are dropped (zero Dirichlet).
    Entries of each row come out sorted by column index.
    """
    dims = tuple(int(x) for x in dims)
    n = int(np.prod(dims))
    strides = [int(np.prod(dims[:d])) for d in range(len(dims))]
    coords = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]  # coords[d][i], x fastest
    idx = np.arange(n, dtype=np.int64)
    cols, vals, valid = [], [], []
    # offsets in increasing column order: highest dimension lower neighbour first
    offsets = []
    for d in reversed(range(len(dims))):
        offsets.append((d, -1))
    offsets.append((None, 0))
    for d in range(len(dims)):
        offsets.append((d, +1))
    for d, o in offsets:
        if d is None:
            cols.append(idx)
            vals.append(np.full(n, centre))
            valid.append(np.ones(n, dtype=bool))
        else:
            c = coords[d] + o
            ok = (c >= 0) & (c < dims[d])
            cols.append(idx + o * strides[d])
            vals.append(np.full(n, lower[d] if o < 0 else upper[d]))
            valid.append(ok)
    cols = np.stack(cols, axis=1)
    vals = np.stack(vals, axis=1)
    valid = np.stack(valid, axis=1)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n, rowptr, cols[valid], vals[valid])


def laplacian_2d(N: int) -> CSR:
    return _stencil_csr((N, N), 4.0, [-1.0, -1.0], [-1.0, -1.0])


def laplacian_3d(N: int) -> CSR:
    return _stencil_csr((N, N, N), 6.0, [-1.0] * 3, [-1.0] * 3)


def _convdiff(N: int, wind: tuple[float, ...]) -> CSR:
    d = len(wind)
    h = 1.0 / (N + 1)
    wind = [float(b) for b in wind]
    if min(wind) < 0:
        raise ValueError("upwind recipe assumes non-negative wind components")
    centre = 2.0 * d + h * sum(wind)
    lower = [-1.0 - h * b for b in wind]
    upper = [-1.0] * d
    return _stencil_csr((N,) * d, centre, lower, upper)


def convdiff_2d(N: int, bx: float, by: float) -> CSR:
    return _convdiff(N, (bx, by))


def convdiff_3d(N: int, wind=(10.0, 20.0, 30.0)) -> CSR:
    return _convdiff(N, tuple(wind))


def _orthonormal_factor(g: np.ndarray) -> np.ndarray:
    # Orthonormal basis of a random Gaussian matrix (input generation only; LAPACK
    # Householder QR on the Fortran-ordered copy).
    import scipy.linalg as sla
    q, _ = sla.qr(np.asfortranarray(g), mode="economic", overwrite_a=True, check_finite=False)
    return q


def glued_block(n: int, w: int, log10_cond: float, j: int, dtype=np.float64,
                out: np.ndarray | None = None) -> np.ndarray:
    """Block j of ``glued_blocks``: U diag(sigma) W^T, column-major (Fortran) n x w.

    U and W are the orthonormal factors of default_rng([2, j]) and default_rng([3, j])
    standard normal draws of shape (n, w) and (w, w)."""
    u = _orthonormal_factor(np.random.default_rng([2, j]).standard_normal((n, w)))
    wm = _orthonormal_factor(np.random.default_rng([3, j]).standard_normal((w, w)))
    if w > 1:
        sigma = 10.0 ** (-float(log10_cond) * np.arange(w) / (w - 1))
    else:
        sigma = np.ones(1)
    blk = u @ (sigma[:, None] * wm.T)
    if out is None:
        out = np.empty((n, w), dtype=dtype, order="F")
    out[:, :] = blk
    return out


def glued_blocks(n: int, nb: int, w: int, log10_cond: float = 12.0, dtype=np.float64,
                 threads: int = 1) -> np.ndarray:
    """n x (nb*w) column-major matrix of nb independent blocks of condition 10^log10_cond."""
    V = np.empty((n, nb * w), dtype=dtype, order="F")

    def one(j):
        glued_block(n, w, log10_cond, j, dtype=dtype, out=V[:, j * w:(j + 1) * w])

    if threads > 1 and nb > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(nb)))
    else:
        for j in range(nb):
            one(j)
    return V


def gaussian_theta(n: int, k: int, seed: int = 0) -> np.ndarray:
    """Dense Gaussian sketch: n x k, entries N(0, 1/k), row-major as drawn."""
    return np.random.default_rng(seed).standard_normal((n, k)) / np.sqrt(k)


def rhs_uniform(n: int, seed: int = 1) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def batched_convdiff_specs(nsys: int, log2_lo: float = 12.0, log2_hi: float = 18.0,
                           wind_max: float = 50.0):
    """Per-system (N, bx, by, rhs_seed, sketch_seed) for many independent 2-D solves.

    n = N^2 is log-uniform in [2^log2_lo, 2^log2_hi] (N = round(2^(u/2)), u uniform),
    winds uniform in [0, wind_max]; system i draws from default_rng([4, i]) and its
    right-hand side from default_rng([5, i]).
    """
    specs = []
    for i in range(nsys):
        r = np.random.default_rng([4, i])
        u = r.uniform(log2_lo, log2_hi)
        N = max(2, int(round(2.0 ** (u / 2.0))))
        bx, by = r.uniform(0.0, wind_max, 2)
        specs.append(dict(N=N, bx=float(bx), by=float(by), rhs_seed=[5, i], sketch_seed=i))
    return specs


def batched_rhs(n: int, seed) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)
