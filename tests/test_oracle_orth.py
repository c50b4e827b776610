"""Pins for the oracle's block orthogonalisation schemes (Sections 4-7, Fig. 9).

Every scheme computes, in exact arithmetic, the unique thin QR factorisation with
non-negative diag(R) of the concatenated blocks (Fig. 1 caption), so its R is
pinned to LAPACK's Householder R (sign-normalised).  Perturbation theory for the
R factor bounds the difference between two backward-stable QR factorisations by
a modest multiple of kappa(V) * u, which gives the tolerance used here.
"""
import math

import numpy as np
import pytest

from oracle import metrics, orth
from oracle.dense import householder_qr
from oracle.sketch import Sketch
from paper_2503_16717_amd import workloads as wl

U = 2.0 ** -53


def lapack_R(V):
    _, R = np.linalg.qr(V)
    return np.where(np.diag(R) < 0, -1.0, 1.0)[:, None] * R


def r_tol(log10_cond):
    return max(1e-12, 10.0 * 10.0 ** log10_cond * U)


SCHEMES = [
    ("one-stage randcholqr", lambda V, w, sk: orth.orth_blocks_one_stage(V, w, "randcholqr", sk)),
    ("one-stage cholqr2", lambda V, w, sk: orth.orth_blocks_one_stage(V, w, "cholqr2", sk)),
    ("two-stage x2", lambda V, w, sk: orth.orth_blocks_two_stage(V, w, 2, sk)),
    ("two-stage x3", lambda V, w, sk: orth.orth_blocks_two_stage(V, w, 3, sk)),
    ("two-stage x6 no-reorth", lambda V, w, sk: orth.orth_blocks_two_stage(V, w, 6, sk, reorth=False)),
]


@pytest.mark.parametrize("name,fn", SCHEMES)
@pytest.mark.parametrize("e", [0, 4])
def test_R_unique_well_conditioned(name, fn, e):
    n, nb, w = 2048, 6, 6
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, info = fn(V, w, Sketch.sparse_sign(64, 8, 0))
    assert info == 0
    assert np.allclose(np.tril(R, -1), 0.0, atol=0)
    assert np.all(np.diag(R) > 0)
    assert metrics.rel_diff(R, lapack_R(V)) <= r_tol(e)
    assert metrics.orth_error(Q)[0] <= 1e-14
    assert metrics.backward_error(V, Q, R) <= 1e-15


@pytest.mark.parametrize("name,fn", [s for s in SCHEMES if "cholqr2" not in s[0]])
@pytest.mark.parametrize("e", [8, 12])
def test_R_unique_ill_conditioned_randomized(name, fn, e):
    """Randomized schemes stay O(eps) up to kappa ~ 1/eps (Section 9, first experiment)."""
    n, nb, w = 2048, 6, 6
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, info = fn(V, w, Sketch.sparse_sign(64, 8, 0))
    assert info == 0
    assert metrics.rel_diff(R, lapack_R(V)) <= r_tol(e)
    assert metrics.orth_error(Q)[0] <= 1e-14
    assert metrics.backward_error(V, Q, R) <= 1e-15


def test_gaussian_sketch_scheme():
    n, w = 1500, 6
    V = wl.glued_blocks(n, 4, w, 10)
    th = wl.gaussian_theta(n, 24, 0)
    Q, R, info = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.gaussian(th))
    assert info == 0
    assert metrics.rel_diff(R, lapack_R(V)) <= r_tol(10)
    assert metrics.orth_error(Q)[0] <= 1e-14


@pytest.mark.parametrize("two_stage", [False, True])
def test_count_gauss_sketch_schemes(two_stage):
    """Count-Gaussian sketch (Section 5.2) in RandCholQR and in the two-stage pre-processing:
    the same unique R and O(eps) orthogonality at kappa = 1e12.  Sizes as in the paper's
    setup: Count to 2 s^2 rows per panel, Gaussian to 2 (s + 1); two-stage, 2 s_hat^2 capped
    at a 128-row Count part (one nonzero per row) and Gaussian to 2 (s_hat + 1)."""
    n, nb, w, e = 3000, 6, 6, 12
    V = wl.glued_blocks(n, nb, w, e)
    if two_stage:
        kc, k = 128, 2 * 18 + 2
        sk = Sketch.count_gauss(kc, 1, 3, wl.gaussian_theta(kc, k, 1))
        Q, R, info = orth.orth_blocks_two_stage(V, w, 3, sk)
    else:
        kc, k = 2 * 25, 2 * 6
        sk = Sketch.count_gauss(kc, 1, 3, wl.gaussian_theta(kc, k, 1))
        Q, R, info = orth.orth_blocks_one_stage(V, w, "randcholqr", sk)
    assert info == 0
    assert metrics.rel_diff(R, lapack_R(V)) <= r_tol(e)
    assert metrics.orth_error(Q)[0] <= 1e-14
    assert metrics.backward_error(V, Q, R) <= 1e-15


def test_cholqr2_regimes_fig9():
    """Fig. 9 caption: CholQR breaks down (non-positive pivot) for kappa(V) >= 1e8; below
    eps^-1/2 CholQR2 keeps O(eps) orthogonality.  Tests stay far from the threshold."""
    sk = Sketch.sparse_sign(64, 8, 0)
    for e in (2, 4, 6):
        V = wl.glued_blocks(2048, 6, 6, e)
        Q, R, info = orth.orth_blocks_one_stage(V, 6, "cholqr2", sk)
        assert info == 0 and metrics.orth_error(Q)[0] <= 1e-14
    for e in (12, 14):
        V = wl.glued_blocks(2048, 6, 6, e)
        _, _, info = orth.orth_blocks_one_stage(V, 6, "cholqr2", sk)
        assert 1 <= info <= 6 * 6
        _, _, info_r = orth.orth_blocks_one_stage(V, 6, "randcholqr", sk)
        assert info_r == 0


def test_randhh_well_conditioned_output():
    """Section 5.2: RandHH turns a numerically full-rank block into Q_bar with kappa = O(1)."""
    for e in (4, 8, 12, 14):
        V = wl.glued_block(4096, 6, e, 0)
        Qb, R1, info = orth.randhh(V, Sketch.sparse_sign(64, 8, 3))
        assert info == 0
        assert metrics.cond2(Qb) <= 10.0


def test_randhh_identity_sketch_is_householder():
    """With Theta = I, RandHH is Householder QR (Fig. 4a with the sketch removed)."""
    V = wl.glued_block(300, 6, 5, 1)
    Qb, R1, info = orth.randhh(V, Sketch.dense(np.eye(300)))
    _, Rh, _ = householder_qr(V)
    assert info == 0
    assert metrics.rel_diff(R1, Rh) <= 1e-15
    assert metrics.rel_diff(R1, lapack_R(V)) <= r_tol(5)
    assert metrics.orth_error(Qb)[0] <= 10 * 1e5 * U  # V R^{-1} is orthonormal only to O(kappa u)


def test_two_stage_single_panel_is_one_stage():
    """s_hat = s: the two-stage scheme performs exactly the one-stage operations."""
    V = wl.glued_blocks(1024, 4, 6, 9)
    sk = Sketch.sparse_sign(64, 8, 2)
    Q1, R1, i1 = orth.orth_blocks_one_stage(V, 6, "randcholqr", sk)
    Q2, R2, i2 = orth.orth_blocks_two_stage(V, 6, 1, sk)
    assert i1 == i2 == 0
    assert np.array_equal(R1, R2) and np.array_equal(Q1, Q2)


def test_bcgs2_block_against_previous():
    n, w = 3000, 6
    Qp, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((n, 18)))
    Vj = wl.glued_block(n, w, 10, 5) + Qp @ np.random.default_rng(1).standard_normal((18, w))
    Qj, Rp, Rd, info = orth.bcgs2_block(Qp, Vj, "randcholqr", Sketch.sparse_sign(64, 8, 0))
    assert info == 0
    assert np.max(np.abs(Qp.T @ Qj)) <= 1e-15 * math.sqrt(n)
    assert metrics.orth_error(Qj)[0] <= 1e-14
    resid = Vj - Qp @ Rp - Qj @ Rd
    assert np.linalg.norm(resid) <= 1e-15 * np.linalg.norm(Vj) * 10


def test_breakdown_on_duplicated_column():
    V = wl.glued_blocks(512, 2, 6, 2)
    V[:, 9] = V[:, 8]
    _, _, info = orth.orth_blocks_one_stage(V, 6, "cholqr2", Sketch.sparse_sign(64, 8, 0))
    assert info >= 7
