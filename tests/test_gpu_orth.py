"""HIP block orthogonalisation vs the CPU oracle (same seeded inputs), through the C ABI.

Tolerances: the R factor is compared normwise, ||R_gpu - R_oracle||_F / ||R_oracle||_F, with
the perturbation bound for the R factor of a QR factorisation: two backward-stable
factorisations of V differ by at most a modest multiple of kappa(V) u, so the bound used is
max(1e-12, 10 kappa u) (u = 2^-53); it equals 1e-12 for kappa <= 1e4.  Orthogonality
||I - Q^T Q||_2 <= 1e-13 and backward error ||V - Q R||_F / ||V||_F <= 1e-14 are properties
at any size.  Q is compared entrywise only where it is well determined (kappa <= 1e6).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from parity_log import assert_rel  # noqa: E402
from oracle import metrics, orth  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def tol_r(log10_cond):
    return max(1e-12, 10.0 * 10.0 ** log10_cond * U)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16717_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def gpu_orth(B, ctx, V, w, dtype=torch.float64, **kw):
    Vd = B.colmajor_from_numpy(V, "cuda", dtype=dtype)
    Q, R, st, col = ctx.orth_blocks(Vd, w, **kw)
    torch.cuda.synchronize()
    return Q.double().cpu().numpy(), R, st, col


def check_against_oracle(V, Q, R, ref, e, q_entrywise=True):
    assert ref.info == 0
    assert np.allclose(np.tril(R, -1), 0.0, atol=0.0)
    assert np.all(np.diag(R) > 0)
    rd = metrics.rel_diff(R, ref.R)
    oe = metrics.orth_error(Q)[0]
    be = metrics.backward_error(V, Q, R)
    print(f"n={V.shape[0]} cols={V.shape[1]} 1e{e:g}: R rel diff {rd:.3e} (bound {tol_r(e):.1e}), "
          f"orth {oe:.2e}, backward {be:.2e}")
    assert rd <= tol_r(e), rd
    assert oe <= 1e-13, oe
    assert be <= 1e-14, be
    if q_entrywise and e <= 6:
        assert np.max(np.abs(Q - ref.Q)) <= max(1e-12, 100 * 10.0 ** e * U)


@pytest.mark.parametrize("n", [256, 3000, 70001])
@pytest.mark.parametrize("w", [6, 11])
@pytest.mark.parametrize("e", [4, 10])
def test_one_stage_randcholqr_sparse(B, ctx, n, w, e):
    nb = 4
    V = wl.glued_blocks(n, nb, w, e)
    sk = B.make_sketch("sparse_sign", 64, 8, 7)
    Q, R, st, col = gpu_orth(B, ctx, V, w, intra="randcholqr", sketch=sk)
    assert st == B.SKO_OK, (st, col)
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.sparse_sign(64, 8, 7))
    check_against_oracle(V, Q, R, ref, e)


@pytest.mark.parametrize("w", [1, 2, 3, 5, 8, 12, 16])
def test_one_stage_widths(B, ctx, w):
    n, nb, e = 5000, 3, 3
    V = wl.glued_blocks(n, nb, w, e)
    k = 48 if w <= 12 else 64
    sk = B.make_sketch("sparse_sign", k, 8, 1)
    Q, R, st, col = gpu_orth(B, ctx, V, w, intra="randcholqr", sketch=sk)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.sparse_sign(k, 8, 1))
    check_against_oracle(V, Q, R, ref, e)


@pytest.mark.parametrize("n", [513, 20000])
def test_one_stage_cholqr2(B, ctx, n):
    e = 4
    V = wl.glued_blocks(n, 5, 6, e)
    Q, R, st, col = gpu_orth(B, ctx, V, 6, intra="cholqr2")
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, 6, "cholqr2")
    check_against_oracle(V, Q, R, ref, e)


def test_cholqr2_breakdown_reported(B, ctx):
    """Fig. 9: CholQR2 breaks down for kappa = 1e12 while RandCholQR succeeds."""
    V = wl.glued_blocks(4096, 3, 6, 12)
    _, _, st, col = gpu_orth(B, ctx, V, 6, intra="cholqr2")
    assert st == B.SKO_EBREAKDOWN and 1 <= col <= 18
    _, _, st2, _ = gpu_orth(B, ctx, V, 6, intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    assert st2 == B.SKO_OK


def test_gaussian_sketch_config1_shape(B, ctx):
    n, w, e = 10000, 6, 8
    V = wl.glued_blocks(n, 5, w, e)
    th = wl.gaussian_theta(n, 24, 0)
    thd = B.colmajor_from_numpy(th, "cuda")
    sk = B.make_sketch("gaussian", theta=thd)
    Q, R, st, col = gpu_orth(B, ctx, V, w, intra="randcholqr", sketch=sk)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.gaussian(th))
    check_against_oracle(V, Q, R, ref, e)


def test_orth_block_against_previous(B, ctx):
    n, p, w = 9000, 18, 6
    Qp, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((n, p)))
    Vj = wl.glued_block(n, w, 8, 5) + Qp @ np.random.default_rng(1).standard_normal((p, w))
    Qpd = B.colmajor_from_numpy(Qp, "cuda")
    Vd = B.colmajor_from_numpy(Vj, "cuda")
    Qo, Rp, Rd, st, col = ctx.orth_block(Qpd, Vd, intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 3))
    torch.cuda.synchronize()
    assert st == B.SKO_OK
    Qj, Rp_ref, Rd_ref, info = orth.bcgs2_block(Qp, Vj, "randcholqr", Sketch.sparse_sign(64, 8, 3))
    assert info == 0
    Rfull = np.vstack([Rp, Rd])
    Rref = np.vstack([Rp_ref, Rd_ref])
    assert_rel(Rfull, Rref, tol_r(8))
    Qo = Qo.cpu().numpy()
    assert np.max(np.abs(Qp.T @ Qo)) <= 1e-13
    assert metrics.orth_error(Qo)[0] <= 1e-13


def test_bitwise_reproducible(B, ctx):
    V = wl.glued_blocks(50000, 4, 6, 10)
    a = gpu_orth(B, ctx, V, 6, intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 2))
    b = gpu_orth(B, ctx, V, 6, intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 2))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_in_place(B, ctx):
    V = wl.glued_blocks(3000, 3, 6, 6)
    Vd = B.colmajor_from_numpy(V, "cuda")
    Q, R, st, _ = ctx.orth_blocks(Vd, 6, Q=Vd, intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    torch.cuda.synchronize()
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, 6, "randcholqr", Sketch.sparse_sign(64, 8, 0))
    check_against_oracle(V, Vd.cpu().numpy(), R, ref, 6)


def test_invalid_arguments(B, ctx):
    V = B.colmajor_from_numpy(np.ones((100, 12)), "cuda")
    _, _, st, _ = ctx.orth_blocks(V, 6, raise_on_error=False, sketch=B.make_sketch("sparse_sign", 4, 8, 0))
    assert st == B.SKO_EINVAL  # zeta does not divide k
    _, _, st, _ = ctx.orth_blocks(V, 6, raise_on_error=False, sketch=B.make_sketch("sparse_sign", 4, 1, 0))
    assert st == B.SKO_EINVAL  # sketch smaller than the block
    W17 = B.colmajor_from_numpy(np.ones((100, 17)), "cuda")
    _, _, st, _ = ctx.orth_blocks(W17, 17, raise_on_error=False)
    assert st == B.SKO_EINVAL


def test_mixed_precision_storage(B, ctx):
    """Float storage of the tall arrays (double arithmetic in the kernels); errors against
    the FP64 oracle on the float-rounded input are of the order of single precision."""
    n, w, e = 20000, 11, 4
    V = wl.glued_blocks(n, 3, w, e).astype(np.float32).astype(np.float64)
    Q, R, st, col = gpu_orth(B, ctx, V, w, dtype=torch.float32, precision="mixed",
                             intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.sparse_sign(64, 8, 0))
    assert metrics.orth_error(Q)[0] <= 1e-5
    assert metrics.backward_error(V, Q, R) <= 1e-6
    assert_rel(R, ref.R, 1e-5)


@pytest.mark.parametrize("w", [6, 11])
@pytest.mark.parametrize("n,pad", [(20000, 0), (20001, 0), (20000, 1)])
def test_mixed_precision_layouts(B, ctx, w, n, pad):
    """Float storage in both strip layouts: pairs of rows read as one 8-byte access (even n,
    even leading dimension), a partial last pair (odd n) and the element-wise fallback (odd
    leading dimension).  Errors against the FP64 oracle on the float-rounded input are of the
    order of single precision."""
    e = 4
    V = wl.glued_blocks(n, 3, w, e).astype(np.float32).astype(np.float64)
    buf = torch.zeros((3 * w, n + pad), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(V.T)).to("cuda", torch.float32)
    Vd = buf.t()[:n]
    Q, R, st, col = ctx.orth_blocks(Vd, w, precision="mixed", intra="randcholqr",
                                    sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    torch.cuda.synchronize()
    assert st == B.SKO_OK
    Qh = Q.double().cpu().numpy()
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.sparse_sign(64, 8, 0))
    assert metrics.orth_error(Qh)[0] <= 1e-5
    assert metrics.backward_error(V, Qh, R) <= 1e-6
    assert_rel(R, ref.R, 1e-5)


@pytest.mark.parametrize("k", [96, 128])
@pytest.mark.parametrize("w", [6, 11])
def test_sketch_beyond_four_tiles(B, ctx, k, w):
    """Sparse sketches of 96 and 128 rows run as one launch of 8 tiles of 16 sketch rows (for
    96 rows two tiles hold no live slot and are not written out)."""
    n, nb, e = 20001, 3, 6
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, st, col = gpu_orth(B, ctx, V, w, intra="randcholqr", sketch=B.make_sketch("sparse_sign", k, 8, 2))
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.sparse_sign(k, 8, 2))
    check_against_oracle(V, Q, R, ref, e)


@pytest.mark.parametrize("n,nb", [(12, 2), (13, 2), (255, 3), (257, 3)])
@pytest.mark.parametrize("intra", ["randcholqr", "cholqr2"])
def test_few_rows(B, ctx, n, nb, intra):
    """Fewer rows than one strip, down to a square matrix (n = nb w).  The R tolerance uses
    the condition number of the whole matrix, which for so few rows exceeds the blocks' own."""
    w = 6
    V = wl.glued_blocks(n, nb, w, 3)
    kw = dict(sketch=B.make_sketch("sparse_sign", 64, 8, 4)) if intra == "randcholqr" else {}
    Q, R, st, col = gpu_orth(B, ctx, V, w, intra=intra, **kw)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_one_stage(V, w, intra, Sketch.sparse_sign(64, 8, 4) if kw else None)
    assert ref.info == 0
    kappa = np.linalg.cond(V)
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0.0, atol=0.0)
    assert_rel(R, ref.R, max(1e-12, 10.0 * kappa * U))
    assert metrics.orth_error(Q)[0] <= 1e-13
    assert metrics.backward_error(V, Q, R) <= 1e-14


@pytest.mark.parametrize("intra", ["randcholqr", "cholqr2"])
def test_zero_block_reports_breakdown(B, ctx, intra):
    """An all-zero block has no QR with a positive diagonal: the call reports breakdown at a
    column of that block (1-based), as the oracle does."""
    n, w = 5000, 6
    V = wl.glued_blocks(n, 3, w, 3)
    V[:, w:2 * w] = 0.0
    kw = dict(sketch=B.make_sketch("sparse_sign", 64, 8, 0)) if intra == "randcholqr" else {}
    _, _, st, col = gpu_orth(B, ctx, V, w, intra=intra, raise_on_error=False, **kw)
    assert st == B.SKO_EBREAKDOWN
    assert w + 1 <= col <= 2 * w
    ref = orth.orth_blocks_one_stage(V, w, intra, Sketch.sparse_sign(64, 8, 0) if kw else None)
    assert ref.info != 0

