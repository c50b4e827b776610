"""The deterministic comparators on the HIP path against the oracle: two-stage
orthogonalisation with BCGS-PIP pre-processing (Fig. 7, Section 7.1) and one-stage BCGS2
with the recursive CholQR of Fig. 3 in its CholQR2 and final CholQR.

Bars as for the other schemes: R within max(1e-12, 10 kappa u) of the oracle's, ||I - Q^T Q||
<= 1e-13, backward error <= 1e-14 (FP64); breakdown where the oracle breaks down."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import metrics, orth  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def r_tol(e):
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


def run(B, ctx, V, w, dtype=torch.float64, **kw):
    Q, R, st, col = ctx.orth_blocks(B.colmajor_from_numpy(V, "cuda", dtype=dtype), w, raise_on_error=False, **kw)
    torch.cuda.synchronize()
    return Q.double().cpu().numpy(), R, st, col


def check(V, Q, R, ref, e, label):
    assert ref.info == 0
    rd = metrics.rel_diff(R, ref.R)
    oe = metrics.orth_error(Q)[0]
    be = metrics.backward_error(V, Q, R)
    print(f"{label}: R rel diff {rd:.2e} (bound {r_tol(e):.1e}), orth {oe:.2e}, backward {be:.2e}")
    assert np.allclose(np.tril(R, -1), 0.0, atol=0) and np.all(np.diag(R) > 0)
    assert rd <= r_tol(e) and oe <= 1e-13 and be <= 1e-14


@pytest.mark.parametrize("n,e,ppb", [(20000, 0, 4), (20000, 4, 4), (50001, 6, 3), (7000, 4, 12)])
def test_pip_two_stage_matches_oracle(B, ctx, n, e, ppb):
    w, nb = 5, 12
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, st, col = run(B, ctx, V, w, two_stage=True, panels_per_big=ppb, preproc="pip")
    assert st == B.SKO_OK, col
    ref = orth.orth_blocks_two_stage(V, w, ppb, None, preproc="pip")
    check(V, Q, R, ref, e, f"pip n={n} e={e} ppb={ppb}")


def test_pip_two_stage_mixed_precision(B, ctx):
    n, w, nb, e = 30000, 5, 12, 3
    V = wl.glued_blocks(n, nb, w, e).astype(np.float32).astype(np.float64)
    Q, R, st, col = run(B, ctx, V, w, dtype=torch.float32, two_stage=True, panels_per_big=4, preproc="pip",
                        precision="mixed")
    assert st == B.SKO_OK
    oe = metrics.orth_error(Q)[0]
    be = metrics.backward_error(V, Q, R)
    print(f"pip mixed: orth {oe:.2e}, backward {be:.2e}")
    assert oe <= 1e-5 and be <= 1e-6


def test_pip_breaks_down_where_the_oracle_does(B, ctx):
    """Section 9: BCGS-PIP fails once a big panel's condition number passes eps^(-1/2);
    the breakdown column lies in the first big panel on both sides.  Near the threshold
    (kappa ~ 1e8) breakdown depends on rounding, so the cases sit >= 100x past it."""
    w, nb, ppb = 5, 12, 4
    for e in (10, 12):
        V = wl.glued_blocks(20000, nb, w, e)
        _, _, st, col = run(B, ctx, V, w, two_stage=True, panels_per_big=ppb, preproc="pip")
        ref = orth.orth_blocks_two_stage(V, w, ppb, None, preproc="pip")
        print(f"pip e={e}: GPU breakdown column {col}, oracle {ref.info}")
        assert st == B.SKO_EBREAKDOWN and 1 <= col <= ppb * w
        assert 1 <= ref.info <= ppb * w


def test_fig10_shape_contrast(B, ctx):
    """Fig. 10, (n, m, s_hat, s) = (1e5, 180, 60, 5), blocks of condition 1e12: PIP breaks
    down, RandBCGS2 reproduces the oracle's R with O(eps) orthogonality."""
    n, w, nb, ppb, e = 100000, 5, 36, 12, 12.0
    V = wl.glued_blocks(n, nb, w, e)
    _, _, st, col = run(B, ctx, V, w, two_stage=True, panels_per_big=ppb, preproc="pip")
    assert st == B.SKO_EBREAKDOWN and 1 <= col <= ppb * w
    sk = B.make_sketch("sparse_sign", 128, 8, 0)
    Q, R, st, col = run(B, ctx, V, w, two_stage=True, panels_per_big=ppb, sketch=sk)
    assert st == B.SKO_OK
    ref = orth.orth_blocks_two_stage(V, w, ppb, Sketch.sparse_sign(128, 8, 0))
    check(V, Q, R, ref, e, "fig10 randbcgs2")


def test_pip_one_panel_per_big_panel_is_bcgs2_cholqr2(B, ctx):
    V = wl.glued_blocks(20000, 5, 6, 4)
    Qa, Ra, sta, _ = run(B, ctx, V, 6, two_stage=True, panels_per_big=1, preproc="pip")
    Qb, Rb, stb, _ = run(B, ctx, V, 6, intra="cholqr2")
    assert sta == stb == B.SKO_OK
    print(f"pip ppb=1 vs bcgs2-cholqr2: R {metrics.rel_diff(Ra, Rb):.2e}, Q {np.max(np.abs(Qa - Qb)):.2e}")
    assert metrics.rel_diff(Ra, Rb) <= 1e-13 and np.max(np.abs(Qa - Qb)) <= 1e-11


@pytest.mark.parametrize("n,e", [(20000, 12), (50001, 10), (3001, 4)])
def test_recursive_cholqr2_matches_oracle(B, ctx, n, e):
    w, nb = 6, 6
    V = wl.glued_blocks(n, nb, w, e)
    Q, R, st, col = run(B, ctx, V, w, intra="cholqr2_recursive")
    assert st == B.SKO_OK, col
    ref = orth.orth_blocks_one_stage(V, w, "cholqr2_recursive")
    check(V, Q, R, ref, e, f"recursive cholqr2 n={n} e={e}")
    if e >= 10:  # plain CholQR2 breaks down on the same input (Fig. 9)
        _, _, st2, col2 = run(B, ctx, V, w, intra="cholqr2")
        assert st2 == B.SKO_EBREAKDOWN and col2 >= 1


def test_recursive_block_step_against_previous(B, ctx):
    n, p, w = 30000, 12, 6
    Qp = np.linalg.qr(np.random.default_rng(0).standard_normal((n, p)))[0]
    Vj = wl.glued_block(n, w, 12, 5) + Qp @ np.random.default_rng(1).standard_normal((p, w))
    Qo, Rp, Rd, st, col = ctx.orth_block(B.colmajor_from_numpy(Qp, "cuda"), B.colmajor_from_numpy(Vj, "cuda"),
                                         intra="cholqr2_recursive")
    torch.cuda.synchronize()
    assert st == B.SKO_OK
    Qj, Rp_ref, Rd_ref, info = orth.bcgs2_block(Qp, Vj, "cholqr2_recursive")
    assert info == 0
    rd = metrics.rel_diff(np.vstack([Rp, Rd]), np.vstack([Rp_ref, Rd_ref]))
    Qo = Qo.cpu().numpy()
    print(f"recursive block step: R rel diff {rd:.2e}, orth {metrics.orth_error(Qo)[0]:.2e}")
    assert rd <= r_tol(12)
    assert np.max(np.abs(Qp.T @ Qo)) <= 1e-13 and metrics.orth_error(Qo)[0] <= 1e-13


def test_recursive_reports_a_zero_column(B, ctx):
    V = wl.glued_blocks(5000, 2, 6, 2)
    V[:, 9] = 0.0
    _, _, st, col = run(B, ctx, V, 6, intra="cholqr2_recursive")
    ref = orth.orth_blocks_one_stage(V, 6, "cholqr2_recursive")
    print(f"zero column: GPU breakdown column {col}, oracle {ref.info}")
    assert st == B.SKO_EBREAKDOWN and col == 10 and ref.info == 10
