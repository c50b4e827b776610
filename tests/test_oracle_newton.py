"""Pins for the Newton basis (Section 4; Bai, Hu and Reichel 1994) and the larger step sizes
that sketching makes usable (Section 9, the discussion of Fig. 12)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import krylov
from oracle.sketch import Sketch
from paper_2503_16717_amd import workloads as wl


def _diag_csr(lam):
    n = lam.size
    return wl.CSR(n, np.arange(n + 1), np.arange(n), lam)


def test_newton_mpk_with_zero_shifts_is_monomial():
    A = wl.convdiff_2d(12, 20.0, 5.0)
    q = np.random.default_rng(0).standard_normal(A.n)
    dinv = 1.0 / krylov.csr_diagonal(A)
    V0 = krylov.mpk(A, dinv, q, 6)
    V1 = krylov.mpk_newton(A, dinv, q, 6, np.zeros(6), np.zeros(6))
    assert np.array_equal(V0, V1)


def test_newton_mpk_closed_form_real_and_complex_shifts():
    """For diagonal A, v_j = prod_l (lambda - theta_l) v_0 entrywise; a complex pair enters as
    |lambda - theta|^2 (the real two-step recurrence)."""
    lam = np.linspace(-2.0, 3.0, 41)
    A = _diag_csr(lam)
    q = np.random.default_rng(1).standard_normal(lam.size)
    theta = 0.7 + 1.3j
    a = np.array([0.5, theta.real, theta.real, -1.25])
    b = np.array([0.0, 0.0, abs(theta.imag) ** 2, 0.0])
    V = krylov.mpk_newton(A, None, q, 4, a, b)
    ref = [q, (lam - 0.5) * q]
    ref.append((lam - theta.real) * ref[1])
    ref.append(np.abs(lam - theta) ** 2 * ref[1])
    ref.append((lam + 1.25) * ref[3])
    for j in range(5):
        assert np.max(np.abs(V[:, j] - ref[j])) <= 1e-14 * np.max(np.abs(ref[j]))


def test_leja_order_hand_example():
    """{3, -1, 0.5, 2.2}: 3 has the largest modulus; -1 is farthest from it; then 0.5
    (distance product 2.5 * 1.5 = 3.75 against 0.8 * 3.2 = 2.56 for 2.2); then 2.2.  A complex
    point is followed by its conjugate."""
    z = krylov.leja_order(np.array([0.5, 2.2, -1.0, 3.0]))
    assert np.array_equal(z, np.array([3.0, -1.0, 0.5, 2.2]))
    # {1, 2i, -2i, -0.5}: 2i has the largest modulus and brings -2i; then 1 (product of
    # distances |1 - 2i|^2 = 5 against 4.25 for -0.5); then -0.5
    z = krylov.leja_order(np.array([1.0, 2j, -2j, -0.5]))
    assert list(z) == [2j, -2j, 1.0, -0.5]


def test_newton_coefficients_pair_handling():
    a, b = krylov.newton_coefficients(np.array([4.0, 1 + 2j, 1 - 2j, -3.0]), 3)
    # Leja: 4, then 1+2j (|1+2j-4| = 3.6 against 7 for -3?  -3 is farther) -> 4, -3, pair
    assert np.array_equal(a[:2], [4.0, -3.0])
    assert a[2] == 1.0 and b[2] == 0.0          # the pair does not fit: its real part
    a, b = krylov.newton_coefficients(np.array([4.0, 1 + 2j, 1 - 2j]), 3)
    assert list(a) == [4.0, 1.0, 1.0] and list(b) == [0.0, 0.0, 4.0]


def _scipy_history(S, b, m, iters):
    hist = []
    spla.gmres(S, b, rtol=1e-14, restart=m, maxiter=iters // m + 1,
               callback=lambda r: hist.append(float(r)), callback_type="pr_norm")
    return hist


@pytest.mark.parametrize("s,m,two_stage,shat,jacobi", [(5, 30, False, None, False), (10, 30, False, None, True),
                                                       (5, 30, True, 15, False)])
def test_newton_sstep_matches_gmres_history(s, m, two_stage, shat, jacobi):
    """Any basis of the same Krylov spaces gives the GMRES(m) iterates at the check points in
    exact arithmetic; the Newton cycles (from the second on) must keep scipy's history."""
    A = wl.convdiff_2d(20, 30.0, 10.0)
    b = wl.rhs_uniform(A.n, 3)
    res = krylov.sstep_gmres(A, b, s=s, m=m, shat=shat, two_stage=two_stage, jacobi=jacobi,
                             sk=Sketch.sparse_sign(64, 8, 0), tol=1e-12, maxiter=150, basis="newton")
    S = A.to_scipy()
    if jacobi:
        S = (S @ sp.diags(1.0 / S.diagonal())).tocsr()
    ref = _scipy_history(S, b, m, 150)
    assert res.newton is not None and np.any(res.newton[0] != 0.0)
    # before stagnation (relative residual >= 1e-8; below it both histories are rounding)
    late = [(it, rr) for it, rr in res.history if it > m and ref[it - 1] >= 1e-8]
    assert len(late) >= 3
    for it, rr in res.history:
        if ref[it - 1] >= 1e-8:
            assert abs(rr - ref[it - 1]) <= 1e-6 * ref[it - 1]


def test_newton_arnoldi_relation_and_ritz_values():
    """A Q_{1:k} = Q_{1:k+1} H holds in a Newton cycle; for the symmetric Laplacian the Ritz
    values are real and inside the spectrum (Cauchy interlacing)."""
    A = wl.laplacian_2d(20)
    b = wl.rhs_uniform(A.n, 6)
    res = krylov.sstep_gmres(A, b, s=5, m=30, sk=Sketch.sparse_sign(64, 8, 0), tol=1e-30, maxiter=60,
                             basis="newton")
    assert np.all(np.abs(res.ritz.imag) <= 1e-10 * np.abs(res.ritz).max())
    ev = np.linalg.eigvalsh(A.to_scipy().toarray())
    assert res.ritz.real.min() >= ev[0] - 1e-10 and res.ritz.real.max() <= ev[-1] + 1e-10
    Q, H = res.last_Q, res.last_H
    k = H.shape[1]
    AQ = np.stack([krylov.spmv(A, Q[:, i]) for i in range(k)], 1)
    assert np.linalg.norm(AQ - Q[:, :k + 1] @ H) <= 1e-10 * np.linalg.norm(AQ)


def test_larger_step_size_with_sketching_and_newton():
    """2-D Laplacian 64^2, m = 60, s = 20: CholQR2 breaks down in the first block (kappa of
    the monomial panel far beyond eps^(-1/2)); RandCholQR continues but the monomial basis
    costs iterations; with the Newton basis the s = 20 solver needs no more iterations than
    the s = 5 one (up to one check interval)."""
    A = wl.laplacian_2d(64)
    b = wl.rhs_uniform(A.n, 1)
    sk = Sketch.sparse_sign(128, 8, 0)
    kw = dict(s=20, m=60, sk=sk, tol=1e-10, maxiter=20000)
    r = krylov.sstep_gmres(A, b, intra="cholqr2", **kw)
    assert not r.converged and r.breakdown_col > 0
    mono = krylov.sstep_gmres(A, b, intra="randcholqr", **kw)
    newt = krylov.sstep_gmres(A, b, intra="randcholqr", basis="newton", **kw)
    base = krylov.sstep_gmres(A, b, s=5, m=60, intra="randcholqr", sk=sk, tol=1e-10)
    assert mono.converged and newt.converged and base.converged
    assert newt.iters <= base.iters + 20
    assert mono.iters > newt.iters + 60
