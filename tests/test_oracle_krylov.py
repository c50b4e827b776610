"""Pins for the oracle's SpMV, matrix-powers kernel and s-step GMRES (Section 4, Fig. 1;
Section 6, Fig. 5) against scipy and closed forms."""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import krylov, metrics, orth
from oracle.sketch import Sketch
from paper_2503_16717_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(key):
    with open(os.path.join(GOLDEN, "paper_printed_values.txt")) as f:
        for line in f:
            if line.startswith(key + " |"):
                return line.split("|")[1].strip()
    raise KeyError(key)


def test_generator_sizes():
    A = wl.laplacian_2d(100)
    assert A.n == 10000 and A.nnz == 5 * 100 ** 2 - 4 * 100  # 49 600
    for N in (5, 12):
        A3 = wl.laplacian_3d(N)
        assert A3.nnz == 7 * N ** 3 - 6 * N ** 2
        C3 = wl.convdiff_3d(N, (10, 20, 30))
        assert C3.nnz == A3.nnz
    S = wl.laplacian_2d(9).to_scipy()
    assert abs(S - S.T).max() == 0
    # interior row sums vanish for the Laplacian, are h*|b|-free for convection-diffusion
    C = wl.convdiff_2d(9, 30.0, 7.0).to_scipy()
    rs = np.asarray(C.sum(axis=1)).ravel().reshape(9, 9)
    assert np.allclose(rs[1:-1, 1:-1], 0.0, atol=1e-15)


@pytest.mark.parametrize("gen", [lambda: wl.laplacian_2d(17), lambda: wl.convdiff_2d(13, 40.0, 3.0),
                                 lambda: wl.convdiff_3d(7, (10, 20, 30))])
def test_spmv_matches_scipy_and_dense(gen):
    A = gen()
    x = np.random.default_rng(0).standard_normal(A.n)
    y = krylov.spmv(A, x)
    S = A.to_scipy()
    assert np.max(np.abs(y - S @ x)) <= 1e-14 * np.abs(y).max()
    assert np.max(np.abs(y - S.toarray() @ x)) <= 1e-14 * np.abs(y).max()


def test_mpk_dense_powers_with_jacobi():
    A = wl.convdiff_2d(11, 20.0, 10.0)
    D = A.to_scipy().toarray()
    dinv = 1.0 / np.diag(D)
    q = np.random.default_rng(2).standard_normal(A.n)
    V = krylov.mpk(A, dinv, q, 5)
    ref = q.copy()
    for i in range(1, 6):
        ref = D @ (dinv * ref)
        assert np.max(np.abs(V[:, i] - ref)) <= 1e-13 * np.abs(ref).max()


def _scipy_history(S, b, m, iters):
    hist = []
    spla.gmres(S, b, rtol=1e-14, restart=m, maxiter=iters // m + 1,
               callback=lambda r: hist.append(float(r)), callback_type="pr_norm")
    return hist


@pytest.mark.parametrize("s,m,two_stage,shat", [(5, 30, False, None), (1, 10, False, None),
                                               (5, 30, True, 15), (5, 30, True, 30), (3, 12, False, None)])
def test_sstep_matches_gmres_history(s, m, two_stage, shat):
    """s-step GMRES(m) iterates equal GMRES(m) iterates at every check point (multiples of
    s, or of s_hat for two-stage) in exact arithmetic (Section 4); scipy is the reference."""
    A = wl.convdiff_2d(20, 30.0, 10.0)
    b = wl.rhs_uniform(A.n, 3)
    res = krylov.sstep_gmres(A, b, s=s, m=m, shat=shat, two_stage=two_stage,
                             sk=Sketch.sparse_sign(64, 8, 0), tol=1e-12, maxiter=90)
    ref = _scipy_history(A.to_scipy(), b, m, 90)
    assert len(res.history) >= 3
    for it, rr in res.history:
        assert it % (shat if two_stage else s) == 0
        assert abs(rr - ref[it - 1]) <= 1e-8 * ref[it - 1]


def test_sstep_jacobi_is_gmres_on_scaled_matrix():
    """Right Jacobi preconditioning: GMRES on A D^{-1} with x = D^{-1} z."""
    A = wl.convdiff_2d(18, 45.0, 5.0)
    b = wl.rhs_uniform(A.n, 4)
    S = A.to_scipy()
    dinv = 1.0 / S.diagonal()
    res = krylov.sstep_gmres(A, b, s=5, m=20, jacobi=True, sk=Sketch.sparse_sign(48, 8, 1),
                             tol=1e-12, maxiter=60)
    import scipy.sparse as sp
    ref = _scipy_history((S @ sp.diags(dinv)).tocsr(), b, 20, 60)
    for it, rr in res.history:
        assert abs(rr - ref[it - 1]) <= 1e-8 * ref[it - 1]


@pytest.mark.parametrize("two_stage", [False, True])
def test_arnoldi_relation(two_stage):
    A = wl.convdiff_2d(16, 10.0, 25.0)
    b = wl.rhs_uniform(A.n, 6)
    res = krylov.sstep_gmres(A, b, s=5, m=30, shat=15 if two_stage else None, two_stage=two_stage,
                             sk=Sketch.sparse_sign(64, 8, 0), tol=1e-30, maxiter=30)
    Q, H = res.last_Q, res.last_H
    k = H.shape[1]
    AQ = np.stack([krylov.spmv(A, Q[:, i]) for i in range(k)], 1)
    S = A.to_scipy()
    rel = np.linalg.norm(AQ - Q @ H) / math.sqrt((S.multiply(S)).sum())
    assert rel <= 1e-13
    assert metrics.orth_error(Q)[0] <= 1e-13


def test_config1_converges():
    """Config 1: 2-D Laplacian 100x100, Gaussian sketch k=24, s=5, m=30, tol 1e-10."""
    A = wl.laplacian_2d(100)
    b = wl.rhs_uniform(A.n, 1)
    res = krylov.sstep_gmres(A, b, s=5, m=30, sk=Sketch.gaussian(wl.gaussian_theta(A.n, 24, 0)), tol=1e-10)
    assert res.converged and res.relres <= 1e-10
    assert res.iters % 5 == 0
    r = b - A.to_scipy() @ res.x
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_check_granularity_matches_time_to_solution_table():
    """Table 4 reports 1660 = 5*332 iterations for s-step (s=5) and 1700 = 17*100 for
    two-stage with s_hat = m = 100: the implicit check runs every s resp. s_hat vectors."""
    assert int(golden("time_to_solution_iters_sstep")) % 5 == 0
    assert int(golden("time_to_solution_iters_two_stage")) % 100 == 0
    A = wl.convdiff_2d(24, 20.0, 20.0)
    b = wl.rhs_uniform(A.n, 8)
    r1 = krylov.sstep_gmres(A, b, s=5, m=40, sk=Sketch.sparse_sign(64, 8, 0), tol=1e-8)
    r2 = krylov.sstep_gmres(A, b, s=5, m=40, shat=40, two_stage=True, sk=Sketch.sparse_sign(128, 8, 0), tol=1e-8)
    assert r1.converged and r2.converged
    assert r1.iters % 5 == 0 and r2.iters % 40 == 0 and r2.iters >= r1.iters


def test_mpk_laplacian_fig12():
    """Fig. 12 (Section 9): monomial MPK basis V_{1:j+1} of the 2-D Laplacian 128^2, v_1 = b/||b||,
    b = A*1, v_{j+1} = A v_j.  What the prose fixes, independent of the unstated details: the
    condition number grows quickly with j; CholQR2 keeps O(eps) orthogonality while the basis is
    below eps^(-1/2) (Section 5.1) and breaks down once it is far beyond; RandCholQR keeps O(eps)
    orthogonality as long as the basis is numerically full rank.

    The printed breakdown index j = 11 is NOT reproduced (parity unpinned for that value).
    Here CholQR2 first breaks down at j = 16, where the equilibrated condition number is about
    2e10; at j = 11 it is 4.7e6 and CholQR2 is still at 6e-15.  Rescaling A does not move the
    breakdown (it scales column j of V by c^j, a diagonal scaling), so the stencil scaling
    cannot explain the difference."""
    A = wl.laplacian_2d(128)
    b = krylov.spmv(A, np.ones(A.n))
    V = krylov.mpk(A, None, b / np.linalg.norm(b), 17)
    th = Sketch.gaussian(wl.gaussian_theta(A.n, 40, 0))
    first_fail = None
    prev = 1.0
    for j in range(2, 18):
        X = V[:, :j + 1]
        keq = metrics.cond2(X / np.linalg.norm(X, axis=0))
        assert keq > 2.0 * prev     # grows quickly (by more than 2x per added vector)
        prev = keq
        Qc, _, info = orth.cholqr2(X)
        if keq < 1e7:               # below eps^(-1/2) ~ 6.7e7 with a margin
            assert info == 0 and metrics.orth_error(Qc)[0] <= 1e-13
        if info and first_fail is None:
            first_fail = j
        if keq > 1e11:              # far beyond: the Gram matrix is numerically singular
            assert info != 0
        Qr, _, info_r = orth.randcholqr(X, th)
        assert info_r == 0 and metrics.orth_error(Qr)[0] <= 1e-13
    assert first_fail is not None
