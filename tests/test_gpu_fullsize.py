"""Full-size checks in the benchmark's launch configuration: n = 2^24 rows, 12 blocks of 6
columns, kappa = 1e12 per block, one-stage RandCholQR-BCGS2 with the sparse-sign sketch
(k = 64, zeta = 8).

At this size the oracle recomputes what it can: the first block's R factor (a full-length
oracle run on n x 6); the whole 72 x 72 R against the sign-normalised Householder R of V
(LAPACK), which every scheme must reproduce because the QR factorisation with a positive
diagonal is unique (Fig. 1 caption); and the properties that hold at any size --
||I - Q^T Q||_2 <= 1e-13 and ||V - Q R||_F / ||V||_F <= 1e-14 measured by the oracle's
compensated metrics on the downloaded Q -- plus bitwise repeatability of the GPU result.
The full oracle run of all twelve blocks is compared at 2^21 rows, where it takes seconds
and each workgroup still walks several row strips.  Launch shapes are autotuned first, as
the benchmark does.  Every R comparison prints the difference it achieved.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import metrics, orth  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
N_ROWS, NB, W, E = 1 << 24, 12, 6, 12.0


@pytest.fixture(scope="module")
def full_input():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return wl.glued_blocks(N_ROWS, NB, W, E, threads=min(12, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def full(full_input):
    from paper_2503_16717_amd import binding as B
    V = full_input
    Vd = B.colmajor_from_numpy(V, "cuda")
    ctx = B.Context(0)
    sk = B.make_sketch("sparse_sign", 64, 8, 0)
    ctx.autotune_orth(N_ROWS, NB, W, intra="randcholqr", sketch=sk)
    outs = []
    for _ in range(3):
        Q, R, st, col = ctx.orth_blocks(Vd, W, intra="randcholqr", sketch=sk)
        torch.cuda.synchronize()
        assert st == B.SKO_OK, (st, col)
        outs.append((Q, R))
    ctx.close()
    return V, outs


def test_fullsize_repeatable(full):
    V, outs = full
    (Q0, R0) = outs[0]
    for Q, R in outs[1:]:
        assert np.array_equal(R, R0)
        assert torch.equal(Q, Q0)


def test_fullsize_properties(full):
    V, outs = full
    Q, R = outs[-1]
    assert np.allclose(np.tril(R, -1), 0.0, atol=0.0)
    assert np.all(np.diag(R) > 0)
    Qh = Q.cpu().numpy()
    oe = metrics.orth_error(Qh)[0]
    be = metrics.backward_error(V, Qh, R)
    print(f"n=2^24: ||I-Q^TQ||_2 = {oe:.3e}, backward error = {be:.3e}")
    assert oe <= 1e-13
    assert be <= 1e-14


def test_fullsize_first_block_against_oracle(full):
    V, outs = full
    _, R = outs[-1]
    ref = orth.orth_blocks_one_stage(np.asfortranarray(V[:, :W]), W, "randcholqr", Sketch.sparse_sign(64, 8, 0))
    assert ref.info == 0
    rd = metrics.rel_diff(R[:W, :W], ref.R)
    print(f"first block R rel diff {rd:.3e}")
    assert rd <= max(1e-12, 10 * 10.0 ** E * U)


@pytest.fixture(scope="module")
def householder_R(full_input):
    """Sign-normalised LAPACK Householder R of the full 2^24 x 72 input and its condition."""
    R = np.linalg.qr(full_input, mode="r")
    R = np.where(np.diag(R) < 0, -1.0, 1.0)[:, None] * R
    return R, float(np.linalg.cond(R))


def test_fullsize_R_against_householder(full, householder_R):
    """Perturbation bound for the R factor of two backward-stable QR factorisations of the
    same V: ||dR||_F / ||R||_F <= max(1e-12, 10 kappa(V) u)."""
    _, outs = full
    R = outs[-1][1]
    Rref, kappa = householder_R
    rd = metrics.rel_diff(R, Rref)
    print(f"n=2^24 one-stage: R vs Householder R rel diff {rd:.3e} (kappa(V) = {kappa:.2e}, "
          f"bound {max(1e-12, 10 * kappa * U):.2e})")
    assert rd <= max(1e-12, 10 * kappa * U)


@pytest.fixture(scope="module")
def full_two_stage(full_input):
    """The same input through the two-stage scheme as the benchmark runs it: s_hat = 30, so
    big panels of 6 blocks (36 columns), two big panels; twice."""
    from paper_2503_16717_amd import binding as B
    V = full_input
    Vd = B.colmajor_from_numpy(V, "cuda")
    ctx = B.Context(0)
    sk = B.make_sketch("sparse_sign", 64, 8, 0)
    ctx.autotune_orth(N_ROWS, NB, W, two_stage=True, panels_per_big=6, sketch=sk)
    outs = []
    for _ in range(2):
        Q, R, st, col = ctx.orth_blocks(Vd, W, two_stage=True, panels_per_big=6, sketch=sk)
        torch.cuda.synchronize()
        assert st == B.SKO_OK, (st, col)
        outs.append((Q, R))
    ctx.close()
    return V, outs


def test_fullsize_two_stage(full_two_stage):
    """Bitwise repeatable, R upper triangular with a positive diagonal, and the properties that
    hold at any size, measured by the oracle's compensated metrics."""
    V, outs = full_two_stage
    (Q0, R0), (Q, R) = outs
    assert np.array_equal(R, R0)
    assert torch.equal(Q, Q0)
    assert np.allclose(np.tril(R, -1), 0.0, atol=0.0)
    assert np.all(np.diag(R) > 0)
    Qh = Q.cpu().numpy()
    oe = metrics.orth_error(Qh)[0]
    be = metrics.backward_error(V, Qh, R)
    print(f"n=2^24 two-stage: ||I-Q^TQ||_2 = {oe:.3e}, backward error = {be:.3e}")
    assert oe <= 1e-13
    assert be <= 1e-14


def test_fullsize_two_stage_R_against_householder(full_two_stage, householder_R):
    _, outs = full_two_stage
    R = outs[-1][1]
    Rref, kappa = householder_R
    rd = metrics.rel_diff(R, Rref)
    print(f"n=2^24 two-stage: R vs Householder R rel diff {rd:.3e} (bound {max(1e-12, 10 * kappa * U):.2e})")
    assert rd <= max(1e-12, 10 * kappa * U)


@pytest.mark.parametrize("scheme", ["one-stage", "two-stage"])
def test_twelve_blocks_2p21_rows_R_against_oracle(scheme):
    """All twelve blocks through the oracle's own scheme at 2^21 rows (bench recipe, kappa =
    1e12 per block), autotuned launch shapes; the full R, orthogonality and backward error."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16717_amd import binding as B
    n = 1 << 21
    V = wl.glued_blocks(n, NB, W, E, threads=min(12, os.cpu_count() or 1))
    sk = B.make_sketch("sparse_sign", 64, 8, 0)
    kw = dict(two_stage=True, panels_per_big=6) if scheme == "two-stage" else dict(intra="randcholqr")
    ctx = B.Context(0)
    ctx.autotune_orth(n, NB, W, sketch=sk, **kw)
    Q, R, st, col = ctx.orth_blocks(B.colmajor_from_numpy(V, "cuda"), W, sketch=sk, **kw)
    torch.cuda.synchronize()
    ctx.close()
    assert st == B.SKO_OK, (st, col)
    if scheme == "two-stage":
        ref = orth.orth_blocks_two_stage(V, W, 6, Sketch.sparse_sign(64, 8, 0))
    else:
        ref = orth.orth_blocks_one_stage(V, W, "randcholqr", Sketch.sparse_sign(64, 8, 0))
    assert ref.info == 0
    kappa = float(np.linalg.cond(ref.R))
    rd = metrics.rel_diff(R, ref.R)
    Qh = Q.cpu().numpy()
    oe = metrics.orth_error(Qh)[0]
    be = metrics.backward_error(V, Qh, R)
    print(f"n=2^21 {scheme}: R vs oracle rel diff {rd:.3e} (kappa {kappa:.2e}), orth {oe:.2e}, backward {be:.2e}")
    assert rd <= max(1e-12, 10 * kappa * U)
    assert oe <= 1e-13 and be <= 1e-14


@pytest.fixture(scope="module")
def full_mixed():
    """The mixed-precision benchmark shape: n = 2^24, 12 blocks of 11 columns (kappa = 1e6 per
    block) stored in FP32, one-stage RandCholQR-BCGS2 with the sparse-sign sketch."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16717_amd import binding as B
    w = 11
    V = wl.glued_blocks(N_ROWS, NB, w, 6.0, threads=min(12, os.cpu_count() or 1))
    V = V.astype(np.float32).astype(np.float64)
    Vd = B.colmajor_from_numpy(V, "cuda", dtype=torch.float32)
    ctx = B.Context(0)
    Q, R, st, col = ctx.orth_blocks(Vd, w, precision="mixed", intra="randcholqr",
                                    sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    torch.cuda.synchronize()
    ctx.close()
    assert st == B.SKO_OK, (st, col)
    del Vd
    return V, Q, R


def test_fullsize_mixed_precision(full_mixed):
    """Errors of the FP32-storage result, measured in FP64 against its own float-rounded input,
    are of the order of single precision."""
    V, Q, R = full_mixed
    assert np.allclose(np.tril(R, -1), 0.0, atol=0.0)
    assert np.all(np.diag(R) > 0)
    Qh = Q.double().cpu().numpy()
    oe = metrics.orth_error(Qh)[0]
    be = metrics.backward_error(V, Qh, R)
    print(f"n=2^24 FP32 storage: ||I-Q^TQ||_2 = {oe:.3e}, backward error = {be:.3e}")
    assert oe <= 1e-6
    assert be <= 1e-6
