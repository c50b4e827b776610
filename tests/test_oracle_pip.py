"""Pins for the deterministic comparators: BCGS-PIP pre-processing (Fig. 7, Section 7.1) and
recursive CholQR (Fig. 3, Section 5.1)."""
import numpy as np
import pytest

from oracle import metrics, orth
from oracle.dense import cholesky_upper, trsm_right_upper
from oracle.sketch import Sketch
from paper_2503_16717_amd import workloads as wl

U = 2.0 ** -53


def lapack_R(V):
    _, R = np.linalg.qr(V)
    return np.where(np.diag(R) < 0, -1.0, 1.0)[:, None] * R


def r_tol(log10_cond):
    return max(1e-12, 10.0 * 10.0 ** log10_cond * U)


def test_pip_first_block_is_cholqr():
    """Section 7.1 footnote: with nothing before it in the big panel, BCGS-PIP is CholQR."""
    V = wl.glued_block(2500, 6, 5, 0)
    Qb, P, R, info = orth.bcgs_pip_step(np.zeros((2500, 0)), V)
    Qc, Rc, infoc = orth.cholqr(V)
    assert info == infoc == 0 and P.shape == (0, 6)
    assert np.array_equal(Qb, Qc) and np.array_equal(R, Rc)


def test_pip_pythagorean_rule():
    """For orthonormal previous columns the Gram matrix of the projected block is
    G - P^T P (the Pythagorean rule), so the PIP factor equals the Cholesky factor of
    the explicitly projected block's Gram matrix (computed with compensated sums).  The
    subtraction cancels: its rounding error is u ||V||^2, so R agrees to about
    u (||V|| / sigma_min(X))^2 relative, X the projected block."""
    n = 4000
    Qp = np.linalg.qr(np.random.default_rng(0).standard_normal((n, 12)))[0]
    for scale in (1.0, 0.01):
        V = wl.glued_block(n, 6, 3, 1) + scale * Qp @ np.random.default_rng(1).standard_normal((12, 6))
        Qb, P, R, info = orth.bcgs_pip_step(Qp, V)
        assert info == 0
        X = V - Qp @ (Qp.T @ V)
        Rx, infox = cholesky_upper(metrics.gram(X))
        assert infox == 0
        amp = (np.linalg.norm(V, 2) / np.linalg.svd(X, compute_uv=False)[-1]) ** 2
        assert metrics.rel_diff(R, Rx) <= 10.0 * U * amp
        # one projection: the loss of orthogonality to Qp is u ||V|| ||R^{-1}|| up to a modest factor
        assert np.max(np.abs(Qp.T @ Qb)) <= 10.0 * U * np.linalg.norm(V, 2) * np.linalg.norm(np.linalg.inv(R), 2)


@pytest.mark.parametrize("e", [0, 4, 6])
def test_two_stage_pip_unique_R(e):
    """Below the eps^(-1/2) threshold (condition (7.1): c kappa^2 < 1/2) the PIP two-stage
    scheme reproduces the unique R with O(eps) orthogonality (Proposition 7.2)."""
    V = wl.glued_blocks(3000, 12, 5, e)
    r = orth.orth_blocks_two_stage(V, 5, 4, None, preproc="pip")
    assert r.info == 0
    assert metrics.rel_diff(r.R, lapack_R(V)) <= r_tol(e)
    assert metrics.orth_error(r.Q)[0] <= 1e-14
    assert metrics.backward_error(V, r.Q, r.R) <= 1e-15


def test_pip_single_panel_big_panels_are_bcgs2_cholqr2():
    """With one panel per big panel, the PIP step is CholQR (footnote) and the close is
    CholQR plus BCGS + CholQR: the same operations as one-stage BCGS2 with CholQR2."""
    V = wl.glued_blocks(2000, 5, 6, 4)
    a = orth.orth_blocks_two_stage(V, 6, 1, None, preproc="pip")
    b = orth.orth_blocks_one_stage(V, 6, "cholqr2")
    assert a.info == b.info == 0
    assert np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)


def test_fig10_pip_breaks_down_randbcgs2_holds():
    """Section 9, Fig. 10, (n, m, s_hat, s) = (1e5, 180, 60, 5): on blocks far beyond
    eps^(-1/2) the Cholesky factorisation in BCGS-PIP meets a non-positive pivot inside the
    first big panel, while RandBCGS2 keeps O(eps) orthogonality and the unique R.  At
    kappa = 1e10 (150x past eps^(-1/2) = 6.7e7) PIP fails; at 1e6 it holds (near the
    threshold the outcome depends on rounding)."""
    n, w, nb, ppb = 100000, 5, 36, 12
    V = wl.glued_blocks(n, nb, w, 12)
    r = orth.orth_blocks_two_stage(V, w, ppb, None, preproc="pip")
    assert 1 <= r.info <= ppb * w
    r = orth.orth_blocks_two_stage(V, w, ppb, Sketch.sparse_sign(128, 8, 0))
    assert r.info == 0
    assert metrics.orth_error(r.Q)[0] <= 1e-14
    assert metrics.rel_diff(r.R, lapack_R(V)) <= r_tol(12)
    Vs = wl.glued_blocks(20000, 12, w, 10)
    assert orth.orth_blocks_two_stage(Vs, w, 4, None, preproc="pip").info > 0
    Vs = wl.glued_blocks(20000, 12, w, 6)
    assert orth.orth_blocks_two_stage(Vs, w, 4, None, preproc="pip").info == 0


def test_recursive_cholqr_without_breakdown_is_cholqr():
    V = wl.glued_block(3000, 6, 4, 2)
    a = orth.cholqr_recursive(V)
    b = orth.cholqr(V)
    assert a[2] == b[2] == 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_recursive_cholqr_splits_at_the_failing_pivot():
    """Fig. 3: where CholQR meets a non-positive pivot at column k, the first k-1 columns
    are finished with the rows of the partial factor (which are the Cholesky factor of the
    leading Gram block), and the remainder is projected and factorised recursively."""
    X = wl.glued_block(3000, 6, 12, 0)
    _, Rp, k = orth.cholqr(X)
    assert k > 1
    Q, R, info = orth.cholqr_recursive(X)
    assert info == 0
    m1 = k - 1
    R11, info11 = cholesky_upper(X[:, :m1].T @ X[:, :m1])
    assert info11 == 0
    assert metrics.rel_diff(R[:m1, :m1], R11) <= 1e-14
    assert metrics.rel_diff(Q[:, :m1], trsm_right_upper(X[:, :m1], R11)) <= 1e-14
    assert np.allclose(np.tril(R, -1), 0.0, atol=0) and np.all(np.diag(R) > 0)
    assert metrics.backward_error(X, Q, R) <= 1e-15


def test_recursive_cholqr_reports_a_zero_column():
    X = wl.glued_block(2000, 6, 2, 3)
    X[:, 3] = 0.0
    assert orth.cholqr(X)[2] == 4
    assert orth.cholqr_recursive(X)[2] == 4


@pytest.mark.parametrize("seed", range(3))
def test_recursive_cholqr2_past_the_threshold(seed):
    """CholQR2 breaks down at kappa = 1e12 (Fig. 9); with the recursive CholQR of Fig. 3 it
    completes.  The recursive variant alone has no orthogonality bound (Section 5.1), but
    BCGS2 with it reproduces the unique R with O(eps) orthogonality."""
    X = wl.glued_block(3000, 6, 12, seed)
    assert orth.cholqr2(X)[2] > 0
    Q, R, info = orth.cholqr2_recursive(X)
    assert info == 0
    assert metrics.rel_diff(R, lapack_R(X)) <= r_tol(12)
    assert metrics.backward_error(X, Q, R) <= 1e-15
    V = wl.glued_blocks(3000, 6, 6, 12)
    r = orth.orth_blocks_one_stage(V, 6, "cholqr2_recursive")
    assert r.info == 0
    assert metrics.rel_diff(r.R, lapack_R(V)) <= r_tol(12)
    assert metrics.orth_error(r.Q)[0] <= 1e-14
