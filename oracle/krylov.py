"""CSR SpMV, the monomial matrix-powers kernel and restarted s-step GMRES, in float64.

Follows Section 4 (Fig. 1) for the one-stage solver and Section 6 (Fig. 5) for
the two-stage solver, with right preconditioning M^{-1} (Jacobi: M = diag(A)).

Basis bookkeeping (the paper's Table 1 notation, V_j = [v_{s(j-1)+1}, ...,
v_{sj+1}] including its start vector, which is the last basis vector so far):

* One-stage block j: V_j = [q, (A M^{-1}) q, ..., (A M^{-1})^s q] with q the
  current last basis vector (index k).  V_j is orthogonalised by BCGS2 against
  the first k basis vectors (the basis without its last vector, p = s(j-1)), so
  V_j = Q_{1:k} R_proj + Q_j R_diag; column k of the basis is replaced by the
  first column of Q_j and the other s columns are appended.
* Every MPK input and output is kept as a coefficient vector in the current
  basis: T_in (inputs) and T_out (outputs) satisfy A M^{-1} Q_{1:m} T_in =
  Q_{1:m+1} T_out, hence A M^{-1} Q_{1:m} = Q_{1:m+1} H with H = T_out T_in^{-1}
  (upper Hessenberg).  When a basis vector is replaced, the stored coefficient
  vectors are rewritten with its new representation (only the boundary vector
  of consecutive blocks is ever replaced).
* The least-squares problem min ||g - H y|| (g = beta e_1 in the final basis) is
  solved by Givens rotations; its residual is the implicit residual norm.
* Convergence: relative residual ||b - A x|| / ||b|| <= tol, with x_0 = 0 unless
  given.  The implicit residual is checked after every block (one-stage) or
  every big panel (two-stage, the Hessenberg matrix is only formed once the big
  panel is orthonormal, Section 6); at the end of a cycle, or once the implicit
  check passes, x is updated and the explicit residual decides.
* Newton basis (Section 4 names it as the more stable alternative to the monomial
  basis, after Bai, Hu and Reichel 1994): the first restart cycle runs with the
  monomial basis; the eigenvalues of its square Hessenberg matrix (Ritz values),
  in Leja order, give the shifts of every later cycle.  In real arithmetic step j
  of the matrix-powers kernel is v_{j+1} = (A M^{-1} - a_j) v_j + b_j v_{j-1}: a
  real shift theta gives (a_j, b_j) = (theta, 0); a complex pair alpha +- i beta
  takes two steps, (alpha, 0) then (alpha, beta^2), so that v_{j+2} =
  (A M^{-1} - theta)(A M^{-1} - conj(theta)) v_j.  The outputs are then
  A M^{-1} v_j = v_{j+1} + a_j v_j - b_j v_{j-1}, which is what T_out stores.
* Two-stage (Fig. 5): each panel's MPK starts from the last pre-processed
  vector; the panel is projected against the previous big panels (Line 10),
  sketched, orthogonalised in sketch space by BCGS2-HH against the accumulated
  sketch of the big panel (Fig. 8), and the full vectors follow by forward
  substitution (Line 12).  The big panel is closed by CholQR (Line 15) and, when
  s_hat < m, by BCGS against the previous big panels plus CholQR (Line 19).
"""
from __future__ import annotations

import math

import numpy as np

from .dense import trsm_right_upper
from .orth import bcgs2_block, cholqr, sketch_bcgs2_hh
from .sketch import Sketch


def spmv(A, x: np.ndarray) -> np.ndarray:
    """y = A x for a CSR matrix (rowptr, colind, val): y_i = sum_{e in row i} val_e x_{col_e}."""
    rowptr = np.asarray(A.rowptr, dtype=np.int64)
    counts = np.diff(rowptr)
    rows = np.repeat(np.arange(A.n), counts)
    prod = A.val * x[A.colind]
    return np.bincount(rows, weights=prod, minlength=A.n)


def csr_diagonal(A) -> np.ndarray:
    rowptr = np.asarray(A.rowptr, dtype=np.int64)
    rows = np.repeat(np.arange(A.n), np.diff(rowptr))
    d = np.zeros(A.n)
    on = rows == A.colind
    d[rows[on]] = A.val[on]
    return d


def mpk(A, dinv: np.ndarray | None, q: np.ndarray, s: int) -> np.ndarray:
    """Monomial matrix-powers kernel: [q, (A M^{-1}) q, ..., (A M^{-1})^s q]."""
    V = np.empty((q.size, s + 1))
    V[:, 0] = q
    for i in range(1, s + 1):
        x = V[:, i - 1] if dinv is None else dinv * V[:, i - 1]
        V[:, i] = spmv(A, x)
    return V


def mpk_newton(A, dinv: np.ndarray | None, q: np.ndarray, s: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Newton-basis matrix-powers kernel: v_0 = q, v_{j+1} = (A M^{-1} - a_j) v_j + b_j v_{j-1}."""
    V = np.empty((q.size, s + 1))
    V[:, 0] = q
    for j in range(s):
        x = V[:, j] if dinv is None else dinv * V[:, j]
        v = spmv(A, x) - a[j] * V[:, j]
        if b[j] != 0.0:
            v = v + b[j] * V[:, j - 1]
        V[:, j + 1] = v
    return V


def leja_order(points: np.ndarray) -> np.ndarray:
    """Leja ordering of a set closed under conjugation.  Candidates are the points with
    imaginary part >= 0, sorted by (real, imaginary part); the first is the one of largest
    modulus, each next one maximises the product of distances to those chosen (sum of
    logarithms; the first maximum in the sorted order wins).  A complex point is followed by
    its conjugate."""
    pts = np.asarray(points, dtype=np.complex128)
    cand = sorted((complex(z) for z in pts if z.imag >= 0.0), key=lambda z: (z.real, z.imag))
    order = []
    while cand:
        if not order:
            best = max(range(len(cand)), key=lambda i: (abs(cand[i]), -i))
        else:
            def score(z):
                tot = 0.0
                for c in order:
                    d = abs(z - c)
                    if d == 0.0:
                        return -math.inf
                    tot += math.log(d)
                return tot
            scores = [score(z) for z in cand]
            top = max(scores)
            best = scores.index(top)
        z = cand.pop(best)
        order.append(z)
        if z.imag > 0.0:
            order.append(z.conjugate())
    return np.array(order)


def newton_coefficients(ritz: np.ndarray, s: int):
    """Recurrence coefficients (a_j, b_j), j < s, from the first s Leja-ordered Ritz values; a
    complex pair that would not fit in the last step enters by its real part."""
    z = leja_order(ritz)
    a = np.zeros(s)
    b = np.zeros(s)
    j = i = 0
    while j < s and i < len(z):
        t = z[i]
        if t.imag > 0.0:
            if j + 1 < s:
                a[j], a[j + 1], b[j + 1] = t.real, t.real, t.imag ** 2
                j += 2
            else:
                a[j] = t.real
                j += 1
            i += 2
        else:
            a[j] = t.real
            j += 1
            i += 1
    return a, b


def hessenberg_lsq(H: np.ndarray, g: np.ndarray):
    """min_y ||g - H y|| for (k+1) x k upper Hessenberg H by Givens rotations.

    Returns (y, residual norm).
    """
    H = np.array(H, dtype=np.float64, copy=True)
    g = np.array(g, dtype=np.float64, copy=True)
    k = H.shape[1]
    for i in range(k):
        a, b = H[i, i], H[i + 1, i]
        rad = math.hypot(a, b)
        if rad == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / rad, b / rad
        top = c * H[i, i:] + s * H[i + 1, i:]
        bot = -s * H[i, i:] + c * H[i + 1, i:]
        H[i, i:], H[i + 1, i:] = top, bot
        gi, gj = c * g[i] + s * g[i + 1], -s * g[i] + c * g[i + 1]
        g[i], g[i + 1] = gi, gj
    y = np.zeros(k)
    for i in reversed(range(k)):
        acc = g[i]
        for j in range(i + 1, k):
            acc -= H[i, j] * y[j]
        y[i] = acc / H[i, i]
    return y, abs(g[k])


class GmresResult:
    def __init__(self):
        self.x = None
        self.converged = False
        self.iters = 0
        self.restarts = 0
        self.relres = float("nan")
        self.relres_implicit = float("nan")
        self.breakdown_col = 0
        self.history = []           # (iters, implicit relres) at every check
        self.explicit_history = []  # (iters, explicit relres) at every restart
        self.last_Q = None
        self.last_H = None
        self.ritz = None            # Newton basis: Ritz values of the first cycle
        self.newton = None          # Newton basis: recurrence coefficients (a, b)


class _Coefs:
    """Coefficient vectors of T_in, T_out and g over the (m+1)-dimensional basis."""

    def __init__(self, m: int, beta: float):
        self.Tin = np.zeros((m + 1, m))
        self.Tout = np.zeros((m + 1, m))
        self.g = np.zeros(m + 1)
        self.g[0] = beta

    def replace_row(self, row: int, sub: np.ndarray, ncols: int):
        """Old basis vector ``row`` = sum_i sub[i] * new vector i (i <= row)."""
        for M in (self.Tin[:, :ncols], self.Tout[:, :ncols]):
            t = M[row, :].copy()
            M[:row, :] += np.outer(sub[:row], t)
            M[row, :] = t * sub[row]
        t = self.g[row]
        self.g[:row] += t * sub[:row]
        self.g[row] = t * sub[row]

    def store_block(self, kk: int, coef: np.ndarray, s: int, newton=None):
        """Inputs are coef[:, 0..s-1], outputs coef[:, 1..s] (coef is (m+1) x (s+1)); with the
        Newton recurrence (a, b) the output of step j is v_{j+1} + a_j v_j - b_j v_{j-1}."""
        self.Tin[:, kk:kk + s] = coef[:, :s]
        self.Tout[:, kk:kk + s] = coef[:, 1:]
        if newton is not None:
            a, b = newton
            for j in range(s):
                self.Tout[:, kk + j] += a[j] * coef[:, j]
                if b[j] != 0.0:
                    self.Tout[:, kk + j] -= b[j] * coef[:, j - 1]

    def lsq(self, k: int):
        H = trsm_right_upper(self.Tout[:k + 1, :k], self.Tin[:k, :k])
        y, res = hessenberg_lsq(H, self.g[:k + 1])
        return H, y, res


def _mpk(A, dinv, q, s, newton):
    return mpk(A, dinv, q, s) if newton is None else mpk_newton(A, dinv, q, s, *newton)


def _cycle_one_stage(A, dinv, r, beta, bnorm, s, m, intra, sk, tol, res, maxiter, newton=None):
    n = r.size
    Q = np.zeros((n, m + 1))
    Q[:, 0] = r / beta
    co = _Coefs(m, beta)
    k = 0
    y = np.zeros(0)
    H = None
    while k < m:
        V = _mpk(A, dinv, Q[:, k], s, newton)
        Qj, Rp, Rd, info = bcgs2_block(Q[:, :k], V, intra, sk)
        if info:
            res.breakdown_col = k + info
            return None, Q, H
        sub = np.zeros(m + 1)
        sub[:k] = Rp[:, 0]
        sub[k] = Rd[0, 0]
        co.replace_row(k, sub, k)
        Q[:, k:k + s + 1] = Qj
        coef = np.zeros((m + 1, s + 1))
        coef[:k, :] = Rp
        coef[k:k + s + 1, :] = Rd
        co.store_block(k, coef, s, newton)
        k += s
        res.iters += s
        H, y, rimp = co.lsq(k)
        res.relres_implicit = rimp / bnorm
        res.history.append((res.iters, res.relres_implicit))
        if res.relres_implicit <= tol or res.iters >= maxiter:
            break
    return Q[:, :k] @ y, Q[:, :k + 1], H


def _cycle_two_stage(A, dinv, r, beta, bnorm, s, shat, m, sk, tol, res, maxiter, newton=None):
    n = r.size
    Q = np.zeros((n, m + 1))
    Q[:, 0] = r / beta
    co = _Coefs(m, beta)
    reorth = shat < m
    y = np.zeros(0)
    H = None
    k0 = 0
    k = 0
    while k0 < m:
        W = shat + 1
        Qold = Q[:, :k0]
        Qbar = np.zeros((n, W))
        Qbar[:, 0] = Q[:, k0]
        Yacc = np.zeros((sk.k, 0))
        for i in range(shat // s):
            loc = i * s
            kk = k0 + loc
            V = _mpk(A, dinv, Qbar[:, loc], s, newton)
            if k0 > 0:
                C = Qold.T @ V
                Vh = V - Qold @ C
            else:
                C = np.zeros((0, s + 1))
                Vh = V
            yk = sk.apply(Vh)
            q, rr, rho, info = sketch_bcgs2_hh(Yacc[:, :loc], yk)
            if info:
                res.breakdown_col = kk + info
                return None, Q, H
            Yacc = np.concatenate([Yacc[:, :loc], q], axis=1)
            X = Vh - Qbar[:, :loc] @ rr if loc > 0 else Vh
            Qbar[:, loc:loc + s + 1] = trsm_right_upper(X, rho)
            coef = np.zeros((m + 1, s + 1))
            coef[:k0, :] = C
            coef[k0:kk, :] = rr
            coef[kk:kk + s + 1, :] = rho
            co.replace_row(kk, coef[:, 0], kk)
            co.store_block(kk, coef, s, newton)
            res.iters += s
        Qh, Rh, info = cholqr(Qbar)
        if info:
            res.breakdown_col = k0 + info
            return None, Q, H
        if reorth:
            if k0 > 0:
                C2 = Qold.T @ Qh
                Vb = Qh - Qold @ C2
            else:
                C2 = np.zeros((0, W))
                Vb = Qh
            QP, Rt, info = cholqr(Vb)
            if info:
                res.breakdown_col = k0 + info
                return None, Q, H
        else:
            C2 = np.zeros((k0, W))
            QP, Rt = Qh, np.eye(W)
        # rows k0..k0+W-1 of every stored vector refer to Q_bar; rewrite them in Q_old, Q_P
        kend = k0 + shat
        bc = slice(k0, k0 + W)
        for M in (co.Tin[:, :kend], co.Tout[:, :kend], co.g[:, None]):
            t = M[bc, :].copy()
            M[:k0, :] += C2 @ (Rh @ t)
            M[bc, :] = Rt @ (Rh @ t)
        Q[:, bc] = QP
        k = kend
        H, y, rimp = co.lsq(k)
        res.relres_implicit = rimp / bnorm
        res.history.append((res.iters, res.relres_implicit))
        if res.relres_implicit <= tol or res.iters >= maxiter:
            break
        k0 = k
    return Q[:, :k] @ y, Q[:, :k + 1], H


def sstep_gmres(A, b: np.ndarray, *, x0: np.ndarray | None = None, s: int = 5, m: int = 30,
                shat: int | None = None, two_stage: bool = False, intra: str = "randcholqr",
                sk: Sketch | None = None, jacobi: bool = False, tol: float = 1e-10,
                maxiter: int = 50000, max_restarts: int | None = None,
                basis: str = "monomial") -> GmresResult:
    """Restarted s-step GMRES (one- or two-stage); returns a GmresResult.  basis="newton":
    Newton basis from the second cycle on, shifts from the first cycle's Ritz values."""
    if basis not in ("monomial", "newton"):
        raise ValueError(basis)
    if m % s:
        raise ValueError("m must be a multiple of s")
    if two_stage:
        shat = m if shat is None else shat
        if shat % s or m % shat:
            raise ValueError("need s | s_hat and s_hat | m")
    res = GmresResult()
    dinv = 1.0 / csr_diagonal(A) if jacobi else None
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    while True:
        r = b - spmv(A, x)
        beta = float(np.linalg.norm(r))
        res.relres = beta / bnorm
        res.explicit_history.append((res.iters, res.relres))
        if res.relres <= tol:
            res.converged = True
            break
        if res.iters >= maxiter or (max_restarts is not None and res.restarts >= max_restarts):
            break
        if two_stage:
            dx, Qc, H = _cycle_two_stage(A, dinv, r, beta, bnorm, s, shat, m, sk, tol, res, maxiter, res.newton)
        else:
            dx, Qc, H = _cycle_one_stage(A, dinv, r, beta, bnorm, s, m, intra, sk, tol, res, maxiter, res.newton)
        res.last_Q, res.last_H = Qc, H
        if dx is None:
            break
        if basis == "newton" and res.newton is None and H is not None:
            k = H.shape[1]
            res.ritz = np.linalg.eigvals(H[:k, :k])
            res.newton = newton_coefficients(res.ritz, s)
        x += dx if dinv is None else dinv * dx
        res.restarts += 1
    res.x = x
    return res
