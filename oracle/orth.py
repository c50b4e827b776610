"""Block orthogonalisation schemes of the paper, step by step, in float64.

The algorithm figures of the paper are described in its text; each routine
follows that description in the paper's order and notation:

* CholQR (Fig. 2b): G = V^T V, R = chol(G), Q = V R^{-1}.
* CholQR2 (Section 5.1): CholQR applied twice, R = R_2 R_1.
* RandHH (Fig. 4a): sketch v = Theta^T V, R = HH(v), Q_bar = V R^{-1}.
* RandCholQR (Fig. 4b, Section 5.2): RandHH followed by CholQR, R = R_2 R_1.
* BCGS2 (Fig. 2c, Section 4): BCGS against the previous basis, the first
  intra-block step (CholQR2 or RandCholQR), BCGS again and CholQR, giving
  R_{1:p,j} = C_1 + C_2 R_hat and R_{j,j} = R_bar R_hat.
* Two-stage without MPK (Fig. 6, Sections 6-7.2): BCGS2 over big panels whose
  first intra-block step is the RandBCGS2 pre-processing (Fig. 8: each panel is
  sketched, orthogonalised in sketch space by BCGS2 with Householder, and the
  full vectors follow by forward substitution), then CholQR of the big panel.
  The deterministic alternative pre-processing is BCGS-PIP (Fig. 7, Section 7.1):
  one reduction gives P = Q_bar_prev^T V and G = V^T V, the Pythagorean rule gives
  the Gram matrix of the projected panel as G - P^T P, R = chol(G - P^T P) and
  Q_bar = (V - Q_bar_prev P) R^{-1}.
* Recursive CholQR (Fig. 3, Section 5.1): when the Cholesky factorisation of the
  Gram matrix meets a non-positive pivot at column k, the first k-1 columns are
  finished with the partial factor, the remaining columns are projected against
  them with the partial factor's off-diagonal block (no new dot products), and
  CholQR is applied recursively to the projected remainder (whose Gram matrix is
  computed afresh).

Breakdown follows Section 5.1 / Fig. 9: a Cholesky pivot that is not positive, or
an exactly zero diagonal of the Householder R, stops the computation; the
1-based global column index is returned.
"""
from __future__ import annotations

import numpy as np

from .dense import cholesky_upper, householder_qr, trsm_right_upper
from .sketch import Sketch


class OrthResult:
    def __init__(self, Q, R, info=0):
        self.Q, self.R, self.info = Q, R, int(info)

    def __iter__(self):
        return iter((self.Q, self.R, self.info))


def cholqr(X: np.ndarray):
    """Fig. 2b: (Q, R, info)."""
    G = X.T @ X
    R, info = cholesky_upper(G)
    if info:
        return None, R, info
    return trsm_right_upper(X, R), R, 0


def cholqr2(X: np.ndarray):
    """Section 5.1: CholQR twice; R = R_2 R_1."""
    Q1, R1, info = cholqr(X)
    if info:
        return None, R1, info
    Q, R2, info = cholqr(Q1)
    if info:
        return None, R2, info
    return Q, R2 @ R1, 0


def cholqr_recursive(X: np.ndarray):
    """Fig. 3: recursive CholQR.  (Q, R, info); info > 0 only when a column is numerically
    dependent on the ones before it (a failing pivot at the first column of a recursion)."""
    n, w = X.shape
    G = X.T @ X
    R, info = cholesky_upper(G)
    if info == 0:
        return trsm_right_upper(X, R), R, 0
    if info == 1:
        return None, R, 1
    m1 = info - 1
    R11, R12 = R[:m1, :m1], R[:m1, m1:]   # rows finished before the failing pivot
    Q1 = trsm_right_upper(X[:, :m1], R11)
    X2 = X[:, m1:] - Q1 @ R12
    Q2, R22, info2 = cholqr_recursive(X2)
    if info2:
        return None, R, m1 + info2
    Rfull = np.zeros((w, w))
    Rfull[:m1, :m1] = R11
    Rfull[:m1, m1:] = R12
    Rfull[m1:, m1:] = R22
    return np.hstack([Q1, Q2]), Rfull, 0


def cholqr2_recursive(X: np.ndarray):
    """CholQR2 with the recursive CholQR of Fig. 3 in both passes; R = R_2 R_1."""
    Q1, R1, info = cholqr_recursive(X)
    if info:
        return None, R1, info
    Q, R2, info = cholqr_recursive(Q1)
    if info:
        return None, R2, info
    return Q, R2 @ R1, 0


def bcgs_pip_step(Qbar_prev: np.ndarray, V: np.ndarray):
    """One BCGS-PIP step (Fig. 7): V against the columns Qbar_prev with one reduction.

    Returns (Qbar, P, R, info) with V = Qbar_prev P + Qbar R.  With no previous columns
    P is empty and the step is CholQR (Section 7.1 footnote)."""
    p = Qbar_prev.shape[1]
    P = Qbar_prev.T @ V
    G = V.T @ V
    S = G - P.T @ P if p > 0 else G
    R, info = cholesky_upper(S)
    if info:
        return None, P, R, info
    X = V - Qbar_prev @ P if p > 0 else V
    return trsm_right_upper(X, R), P, R, 0


def randhh(X: np.ndarray, sk: Sketch):
    """Fig. 4a: v = Theta^T X; R = HH(v) (diag >= 0); Q_bar = X R^{-1}."""
    v = sk.apply(X)
    _, R1, info = householder_qr(v)
    if info:
        return None, R1, info
    return trsm_right_upper(X, R1), R1, 0


def randcholqr(X: np.ndarray, sk: Sketch):
    """Fig. 4b: RandHH, then CholQR of Q_bar; R = R_2 R_1."""
    Qb, R1, info = randhh(X, sk)
    if info:
        return None, R1, info
    Q, R2, info = cholqr(Qb)
    if info:
        return None, R2, info
    return Q, R2 @ R1, 0


def first_intra(X: np.ndarray, intra: str, sk: Sketch | None):
    if intra == "cholqr2":
        return cholqr2(X)
    if intra == "cholqr2_recursive":
        return cholqr2_recursive(X)
    if intra == "randcholqr":
        return randcholqr(X, sk)
    raise ValueError(intra)


def bcgs2_block(Qp: np.ndarray, V: np.ndarray, intra: str = "randcholqr", sk: Sketch | None = None):
    """One block of BCGS2 (Fig. 2c) against the orthonormal Qp (n x p).

    Returns (Qj, R_proj (p x w), R_diag (w x w), info).  With p = 0 the two
    projections vanish and the final CholQR still runs.
    """
    n, w = V.shape
    p = Qp.shape[1]
    if p > 0:
        C1 = Qp.T @ V
        Vh = V - Qp @ C1
    else:
        C1 = np.zeros((0, w))
        Vh = V
    Qh, Rh, info = first_intra(Vh, intra, sk)
    if info:
        return None, None, Rh, info
    if p > 0:
        C2 = Qp.T @ Qh
        Vb = Qh - Qp @ C2
    else:
        C2 = np.zeros((0, w))
        Vb = Qh
    # with the recursive CholQR2 first intra step, the final CholQR is recursive too
    Qj, Rb, info = (cholqr_recursive if intra == "cholqr2_recursive" else cholqr)(Vb)
    if info:
        return None, None, Rb, info
    return Qj, C1 + C2 @ Rh, Rb @ Rh, 0


def orth_blocks_one_stage(V: np.ndarray, w: int, intra: str = "randcholqr", sk: Sketch | None = None):
    """Orthogonalise nb = N/w disjoint column blocks of V (n x N) one after another.

    Returns OrthResult(Q, R, info): V = Q R with R upper triangular (N x N).
    """
    n, N = V.shape
    if N % w:
        raise ValueError("number of columns must be a multiple of w")
    Q = np.zeros((n, N))
    R = np.zeros((N, N))
    for j in range(N // w):
        p = j * w
        cols = slice(p, p + w)
        Qj, Rp, Rd, info = bcgs2_block(Q[:, :p], V[:, cols], intra, sk)
        if info:
            return OrthResult(Q, R, p + info)
        Q[:, cols] = Qj
        R[:p, cols] = Rp
        R[cols, cols] = Rd
    return OrthResult(Q, R, 0)


def sketch_bcgs2_hh(Yacc: np.ndarray, y: np.ndarray):
    """Sketch-space step of RandBCGS2 (Fig. 8a): BCGS2 of y against the orthonormal
    columns of Yacc with Householder as the intra-block step.

    Returns (q, r, rho, info): y = Yacc r + q rho with q^T q = I, rho upper with
    non-negative diagonal, r = r_1 + r_2.
    """
    kk, w = y.shape
    if Yacc.shape[1] > 0:
        r1 = Yacc.T @ y
        z = y - Yacc @ r1
        r2 = Yacc.T @ z
        z = z - Yacc @ r2
        r = r1 + r2
    else:
        r = np.zeros((0, w))
        z = y
    q, rho, info = householder_qr(z)
    return q, r, rho, info


def orth_blocks_two_stage(V: np.ndarray, w: int, panels_per_big: int, sk: Sketch | None, reorth: bool = True,
                          preproc: str = "randbcgs2"):
    """Two-stage block orthogonalisation without MPK (Fig. 6) with RandBCGS2 pre-processing
    (or, preproc="pip", BCGS-PIP pre-processing of each panel against the big panel's
    previous pre-processed panels, Fig. 7; no sketch).

    Big panels of ``panels_per_big`` blocks of width w.  For each big panel with
    previous basis Q_old (n x p_old):
      per panel i: C_i = Q_old^T V_i, V_hat_i = V_i - Q_old C_i      (inter, first pass)
                   y = Theta^T V_hat_i; sketch-space BCGS2-HH against Y_acc -> q, r, rho
                   Q_bar_i = (V_hat_i - Q_bar_prev r) rho^{-1}          (forward substitution)
      [Q_hat, R_hat] = CholQR(Q_bar_P)                                  (first intra, Line 7)
      C_2 = Q_old^T Q_hat, V_bar = Q_hat - Q_old C_2, [Q_P, R_til] = CholQR(V_bar)
    and R_{old,P} = C + C_2 R_hat R_bar, R_{P,P} = R_til R_hat R_bar.
    ``reorth=False`` skips the second inter/intra pass (R_til = I, C_2 = 0).
    """
    n, N = V.shape
    nb = N // w
    if N % w or nb % panels_per_big:
        raise ValueError("N must be a multiple of w * panels_per_big")
    Wb = w * panels_per_big
    Q = np.zeros((n, N))
    R = np.zeros((N, N))
    for big in range(nb // panels_per_big):
        p_old = big * Wb
        Qold = Q[:, :p_old]
        Qbar = np.zeros((n, Wb))
        Yacc = np.zeros((sk.k if sk is not None else 0, 0))
        Rbar = np.zeros((Wb, Wb))
        C = np.zeros((p_old, Wb))
        for i in range(panels_per_big):
            cols = slice(p_old + i * w, p_old + (i + 1) * w)
            Vi = V[:, cols]
            if p_old > 0:
                Ci = Qold.T @ Vi
                Vh = Vi - Qold @ Ci
                C[:, i * w:(i + 1) * w] = Ci
            else:
                Vh = Vi
            if preproc == "pip":
                Qbi, r, rho, info = bcgs_pip_step(Qbar[:, :i * w], Vh)
                if info:
                    return OrthResult(Q, R, p_old + i * w + info)
                Qbar[:, i * w:(i + 1) * w] = Qbi
                Rbar[:i * w, i * w:(i + 1) * w] = r
                Rbar[i * w:(i + 1) * w, i * w:(i + 1) * w] = rho
                continue
            y = sk.apply(Vh)
            q, r, rho, info = sketch_bcgs2_hh(Yacc, y)
            if info:
                return OrthResult(Q, R, p_old + i * w + info)
            Yacc = np.concatenate([Yacc, q], axis=1)
            X = Vh - Qbar[:, :i * w] @ r if i > 0 else Vh
            Qbar[:, i * w:(i + 1) * w] = trsm_right_upper(X, rho)
            Rbar[:i * w, i * w:(i + 1) * w] = r
            Rbar[i * w:(i + 1) * w, i * w:(i + 1) * w] = rho
        Qh, Rh, info = cholqr(Qbar)
        if info:
            return OrthResult(Q, R, p_old + info)
        if reorth:
            if p_old > 0:
                C2 = Qold.T @ Qh
                Vb = Qh - Qold @ C2
            else:
                C2 = np.zeros((0, Wb))
                Vb = Qh
            QP, Rt, info = cholqr(Vb)
            if info:
                return OrthResult(Q, R, p_old + info)
        else:
            C2 = np.zeros((p_old, Wb))
            QP, Rt = Qh, np.eye(Wb)
        bc = slice(p_old, p_old + Wb)
        Q[:, bc] = QP
        RhRb = Rh @ Rbar
        R[:p_old, bc] = C + C2 @ RhRb
        R[bc, bc] = Rt @ RhRb
    return OrthResult(Q, R, 0)
