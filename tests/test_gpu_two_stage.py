"""HIP two-stage block orthogonalisation (Fig. 6 with RandBCGS2 pre-processing, Fig. 8)
vs the CPU oracle on the same seeded inputs, through the C ABI.  Tolerances as in
test_gpu_orth.py (R within max(1e-12, 10 kappa u); orthogonality 1e-13; backward 1e-14)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from parity_log import assert_rel  # noqa: E402
from oracle import metrics, orth  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def tol_r(e):
    return max(1e-12, 10.0 * 10.0 ** e * U)


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


def run(B, ctx, V, w, ppb, reorth=True, k=64, seed=0, dtype=torch.float64, **kw):
    Vd = B.colmajor_from_numpy(V, "cuda", dtype=dtype)
    Q, R, st, col = ctx.orth_blocks(Vd, w, two_stage=True, panels_per_big=ppb, reorth=reorth, raise_on_error=False,
                                    sketch=B.make_sketch("sparse_sign", k, 8, seed), **kw)
    torch.cuda.synchronize()
    return Q.double().cpu().numpy(), R, st, col


@pytest.mark.parametrize("ppb", [1, 2, 3, 6])
@pytest.mark.parametrize("e", [4, 10])
@pytest.mark.parametrize("n", [700, 40000])
def test_two_stage_matches_oracle(B, ctx, ppb, e, n):
    w, nb = 6, 6
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, st, col = run(B, ctx, V, w, ppb)
    assert st == B.SKO_OK, (st, col)
    ref = orth.orth_blocks_two_stage(V, w, ppb, Sketch.sparse_sign(64, 8, 0))
    assert ref.info == 0
    assert np.all(np.diag(R) > 0)
    assert_rel(R, ref.R, tol_r(e))
    assert metrics.orth_error(Q)[0] <= 1e-13
    assert metrics.backward_error(V, Q, R) <= 1e-14
    if e <= 6:
        assert np.max(np.abs(Q - ref.Q)) <= max(1e-12, 100 * 10.0 ** e * U)


def test_two_stage_without_reorth_single_big_panel(B, ctx):
    """One big panel spanning the basis: the second pass (Fig. 5 Line 19) is skipped."""
    n, w, nb = 30000, 5, 12
    V = wl.glued_blocks(n, nb, w, 8)
    Q, R, st, col = run(B, ctx, V, w, 12, reorth=False, k=128)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_two_stage(V, w, 12, Sketch.sparse_sign(128, 8, 0), reorth=False)
    assert_rel(R, ref.R, tol_r(8))
    assert metrics.orth_error(Q)[0] <= 1e-13


def test_two_stage_width11(B, ctx):
    n, w, nb = 20000, 11, 4
    V = wl.glued_blocks(n, nb, w, 9)
    Q, R, st, col = run(B, ctx, V, w, 2, k=64)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_two_stage(V, w, 2, Sketch.sparse_sign(64, 8, 0))
    assert_rel(R, ref.R, tol_r(9))
    assert metrics.orth_error(Q)[0] <= 1e-13


def test_two_stage_config2_shape_reduced_rows(B, ctx):
    """Config-2 shape (12 blocks of 6, s_hat = 30 -> 6 blocks per big panel, W = 36) at n = 2^17."""
    n, w, nb = 1 << 17, 6, 12
    V = wl.glued_blocks(n, nb, w, 12)
    Q, R, st, col = run(B, ctx, V, w, 6)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_two_stage(V, w, 6, Sketch.sparse_sign(64, 8, 0))
    assert_rel(R, ref.R, tol_r(12))
    assert metrics.orth_error(Q)[0] <= 1e-13
    assert metrics.backward_error(V, Q, R) <= 1e-14


def test_two_stage_equals_one_stage_single_panel(B, ctx):
    """s_hat = s: identical operations to one-stage RandCholQR-BCGS2 (oracle: bitwise equal);
    the GPU paths agree to rounding."""
    V = wl.glued_blocks(9000, 4, 6, 6)
    Q2, R2, st2, _ = run(B, ctx, V, 6, 1)
    Vd = B.colmajor_from_numpy(V, "cuda")
    Q1, R1, st1, _ = ctx.orth_blocks(Vd, 6, intra="randcholqr", sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    assert st1 == st2 == B.SKO_OK
    assert_rel(R2, R1, tol_r(6))


def test_two_stage_rejects_small_sketch(B, ctx):
    V = wl.glued_blocks(1000, 6, 6, 2)
    _, _, st, _ = run(B, ctx, V, 6, 6, k=24)
    assert st == B.SKO_EINVAL


def test_two_stage_many_big_panels(B, ctx):
    """Six big panels of 36 columns (216 columns): the last big panel is projected on 180
    previous columns, whose coefficients the wide row operation reads through the scalar
    cache (no staging buffer bounds their number)."""
    n, w, nb, ppb, e = 3000, 6, 36, 6, 4
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, st, col = run(B, ctx, V, w, ppb)
    assert st == B.SKO_OK, (st, col)
    ref = orth.orth_blocks_two_stage(V, w, ppb, Sketch.sparse_sign(64, 8, 0))
    assert ref.info == 0
    kappa = np.linalg.cond(V)
    assert_rel(R, ref.R, max(tol_r(e), 10.0 * kappa * U))
    assert metrics.orth_error(Q)[0] <= 1e-13
    assert metrics.backward_error(V, Q, R) <= 1e-14


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("n", [4099, 20000])
def test_two_stage_widest_big_panels(B, ctx, mixed, n):
    """Two big panels of 55 columns (5 blocks of 11): the row solve runs its 64-column form
    with 9 slots past the width, the packed triangular factor spans 55 columns, and the
    second big panel is projected on the first (55 coefficients per column).  n = 4099
    leaves a ragged last 16-row group in the wide Gram and projection and a partial last
    strip in the row solve.  FP32 storage is compared with the oracle on the float-rounded
    input to single-precision tolerances."""
    w, nb, ppb, e = 11, 10, 5, 4
    V = wl.glued_blocks(n, nb, w, e)
    kw = {}
    dtype = torch.float64
    if mixed:
        V = V.astype(np.float32).astype(np.float64)
        kw["precision"] = "mixed"
        dtype = torch.float32
    Q, R, st, col = run(B, ctx, V, w, ppb, k=128, dtype=dtype, **kw)
    assert st == B.SKO_OK, (st, col)
    ref = orth.orth_blocks_two_stage(V, w, ppb, Sketch.sparse_sign(128, 8, 0))
    assert ref.info == 0
    if mixed:
        assert metrics.orth_error(Q)[0] <= 1e-5
        assert metrics.backward_error(V, Q, R) <= 1e-6
        assert_rel(R, ref.R, 1e-5)
    else:
        assert_rel(R, ref.R, tol_r(e))
        assert metrics.orth_error(Q)[0] <= 1e-13
        assert metrics.backward_error(V, Q, R) <= 1e-14


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("nb,ppb", [(15, 5), (12, 3)])
def test_two_stage_fused_close_widths(B, ctx, mixed, nb, ppb):
    """Big panels of 40 columns (5 blocks of 8; three big panels) or 24 columns (3 blocks of
    8; four big panels), n = 4099: the close of the first big panel runs its row solve with
    the second Gram matrix in the same sweep, later ones their row solve with the projection
    on the previous columns while there are at most 48 of them (40; 24 and 48), and the
    separate projection beyond (80; 72).  40 columns is the widest panel the fused row solve
    accepts; the last strip is ragged.  FP32 storage is compared with the oracle on the
    float-rounded input to single-precision tolerances."""
    n, w, e = 4099, 8, 4
    V = wl.glued_blocks(n, nb, w, e)
    kw = {}
    dtype = torch.float64
    if mixed:
        V = V.astype(np.float32).astype(np.float64)
        kw["precision"] = "mixed"
        dtype = torch.float32
    Q, R, st, col = run(B, ctx, V, w, ppb, k=64, dtype=dtype, **kw)
    assert st == B.SKO_OK, (st, col)
    ref = orth.orth_blocks_two_stage(V, w, ppb, Sketch.sparse_sign(64, 8, 0))
    assert ref.info == 0
    if mixed:
        assert metrics.orth_error(Q)[0] <= 1e-5
        assert metrics.backward_error(V, Q, R) <= 1e-6
        assert_rel(R, ref.R, 1e-5)
    else:
        assert_rel(R, ref.R, tol_r(e))
        assert metrics.orth_error(Q)[0] <= 1e-13
        assert metrics.backward_error(V, Q, R) <= 1e-14
        assert np.max(np.abs(Q - ref.Q)) <= max(1e-12, 100 * 10.0 ** e * U)
