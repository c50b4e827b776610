"""Launch-shape autotuning (sko_autotune_orth) changes how many workgroups stream each pass,
never the arithmetic per row: after tuning, the factorisation still meets the oracle
tolerances of test_gpu_orth.py, and it is bitwise repeatable from call to call."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from parity_log import assert_rel  # noqa: E402
from oracle import metrics, orth  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
N_ROWS = 1 << 19   # 2048 strips of 256 rows: enough for the grid to matter on 256 CUs


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_16717_amd import binding
    return binding


def run(B, ctx, V, w, **kw):
    Vd = B.colmajor_from_numpy(V, "cuda")
    Q, R, st, col = ctx.orth_blocks(Vd, w, **kw)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), R, st


def test_autotuned_one_stage_matches_oracle_and_repeats(B):
    w, nb, e = 6, 4, 8.0
    V = wl.glued_blocks(N_ROWS, nb, w, e)
    sk = dict(sketch=B.make_sketch("sparse_sign", 64, 8, 1))
    ctx = B.Context(0)
    try:
        ctx.autotune_orth(N_ROWS, nb, w, intra="randcholqr", **sk)
        Q1, R1, st1 = run(B, ctx, V, w, intra="randcholqr", **sk)
        Q2, R2, st2 = run(B, ctx, V, w, intra="randcholqr", **sk)
    finally:
        ctx.close()
    assert st1 == B.SKO_OK and st2 == B.SKO_OK
    assert np.array_equal(R1, R2) and np.array_equal(Q1, Q2)
    ref = orth.orth_blocks_one_stage(V, w, "randcholqr", Sketch.sparse_sign(64, 8, 1))
    assert ref.info == 0
    assert_rel(R1, ref.R, max(1e-12, 10.0 * 10.0 ** e * U))
    assert metrics.orth_error(Q1)[0] <= 1e-13
    assert metrics.backward_error(V, Q1, R1) <= 1e-14


def test_autotuned_two_stage_properties(B):
    w, nb = 6, 6
    V = wl.glued_blocks(N_ROWS, nb, w, 8.0)
    kw = dict(two_stage=True, panels_per_big=3, sketch=B.make_sketch("sparse_sign", 64, 8, 2))
    ctx = B.Context(0)
    try:
        ctx.autotune_orth(N_ROWS, nb, w, **kw)
        Q, R, st = run(B, ctx, V, w, **kw)
    finally:
        ctx.close()
    assert st == B.SKO_OK
    assert metrics.orth_error(Q)[0] <= 1e-13
    assert metrics.backward_error(V, Q, R) <= 1e-14


def test_autotune_arguments(B):
    ctx = B.Context(0)
    try:
        o = B.orth_opts()
        assert ctx.sko_autotune_orth(N_ROWS, 0, 6, o) == B.SKO_EINVAL
        assert ctx.sko_autotune_orth(N_ROWS, 4, 0, o) == B.SKO_EINVAL
        assert ctx.sko_autotune_orth(1000, 4, 6, o) == B.SKO_OK   # too small to tune: nothing to do
    finally:
        ctx.close()
