"""HIP s-step GMRES (one- and two-stage, FP64 and mixed precision, Jacobi) vs the CPU oracle.

The oracle's iterates are pinned to scipy's GMRES(m) history (test_oracle_krylov.py).  The
GPU solver uses the same check points (every s basis vectors, or every s_hat for two-stage),
so the iteration counts must agree up to one check interval (rounding can move the crossing
of the tolerance by one check), the explicit relative residual must meet tol, and the
solution must agree with the oracle's within the accuracy the tolerance implies."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import krylov  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


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


def explicit_relres(A, x, b):
    r = b - A.to_scipy() @ x
    return np.linalg.norm(r) / np.linalg.norm(b)


def check(A, b, x, info, ref, tol, step):
    assert info["converged"] == 1
    assert ref.converged
    assert explicit_relres(A, x, b) <= tol * 1.01
    assert abs(info["iters"] - ref.iters) <= step
    assert info["iters"] % step == 0
    assert np.linalg.norm(x - ref.x) <= 1e3 * tol * np.linalg.norm(ref.x)


@pytest.mark.parametrize("intra", ["randcholqr", "cholqr2"])
def test_one_stage_convdiff(B, ctx, intra):
    A = wl.convdiff_2d(24, 30.0, 10.0)
    b = wl.rhs_uniform(A.n, 3)
    x, info, st = ctx.gmres(A, b, s=5, m=30, intra=intra, tol=1e-10,
                            sketch=B.make_sketch("sparse_sign", 64, 8, 0))
    assert st == B.SKO_OK, info
    ref = krylov.sstep_gmres(A, b, s=5, m=30, intra=intra, sk=Sketch.sparse_sign(64, 8, 0), tol=1e-10)
    check(A, b, x.cpu().numpy(), info, ref, 1e-10, 5)


def test_config1_laplacian_gaussian(B, ctx):
    """Config 1: 2-D Laplacian 100 x 100, s = 5, m = 30, Gaussian sketch k = 24, tol 1e-10."""
    A = wl.laplacian_2d(100)
    b = wl.rhs_uniform(A.n, 1)
    th = wl.gaussian_theta(A.n, 24, 0)
    thd = B.colmajor_from_numpy(th, "cuda")
    x, info, st = ctx.gmres(A, b, s=5, m=30, tol=1e-10, sketch=B.make_sketch("gaussian", theta=thd))
    assert st == B.SKO_OK, info
    ref = krylov.sstep_gmres(A, b, s=5, m=30, sk=Sketch.gaussian(th), tol=1e-10)
    check(A, b, x.cpu().numpy(), info, ref, 1e-10, 5)


@pytest.mark.parametrize("shat,m", [(15, 30), (30, 30), (20, 40)])
def test_two_stage(B, ctx, shat, m):
    A = wl.convdiff_2d(22, 40.0, 15.0)
    b = wl.rhs_uniform(A.n, 5)
    k = 2 * (shat + 1) if 2 * (shat + 1) <= 128 else 128
    k = ((k + 7) // 8) * 8
    x, info, st = ctx.gmres(A, b, s=5, m=m, shat=shat, two_stage=True, tol=1e-10,
                            sketch=B.make_sketch("sparse_sign", k, 8, 2))
    assert st == B.SKO_OK, info
    ref = krylov.sstep_gmres(A, b, s=5, m=m, shat=shat, two_stage=True, sk=Sketch.sparse_sign(k, 8, 2), tol=1e-10)
    check(A, b, x.cpu().numpy(), info, ref, 1e-10, shat)


@pytest.mark.parametrize("two_stage", [False, True])
def test_large_restart_basis(B, ctx, two_stage):
    """m = 80 is past what the least squares keeps in LDS (m <= 62): the Hessenberg solve and,
    two-stage, the big-panel close run on global memory."""
    A = wl.convdiff_2d(22, 40.0, 15.0)
    b = wl.rhs_uniform(A.n, 6)
    shat, k = (40, 88) if two_stage else (5, 64)
    kw = dict(shat=shat, two_stage=True) if two_stage else {}
    x, info, st = ctx.gmres(A, b, s=5, m=80, tol=1e-10, sketch=B.make_sketch("sparse_sign", k, 8, 1), **kw)
    assert st == B.SKO_OK, info
    ref = krylov.sstep_gmres(A, b, s=5, m=80, sk=Sketch.sparse_sign(k, 8, 1), tol=1e-10, **kw)
    check(A, b, x.cpu().numpy(), info, ref, 1e-10, shat)


def test_config5_shape_small_grid_jacobi(B, ctx):
    """Config-5 shape on a 16^3 grid: 3-D convection-diffusion, wind (10, 20, 30), Jacobi,
    two-stage s = 10, s_hat = m = 60, sparse-sign k = 128."""
    A = wl.convdiff_3d(16, (10.0, 20.0, 30.0))
    b = np.ones(A.n)
    x, info, st = ctx.gmres(A, b, s=10, m=60, shat=60, two_stage=True, precond=1, tol=1e-10,
                            sketch=B.make_sketch("sparse_sign", 128, 8, 0))
    assert st == B.SKO_OK, info
    ref = krylov.sstep_gmres(A, b, s=10, m=60, shat=60, two_stage=True, jacobi=True,
                             sk=Sketch.sparse_sign(128, 8, 0), tol=1e-10)
    check(A, b, x.cpu().numpy(), info, ref, 1e-10, 60)


def test_one_stage_jacobi(B, ctx):
    A = wl.convdiff_2d(20, 45.0, 5.0)
    b = wl.rhs_uniform(A.n, 4)
    x, info, st = ctx.gmres(A, b, s=5, m=20, precond=1, tol=1e-10, sketch=B.make_sketch("sparse_sign", 48, 8, 1))
    assert st == B.SKO_OK
    ref = krylov.sstep_gmres(A, b, s=5, m=20, jacobi=True, sk=Sketch.sparse_sign(48, 8, 1), tol=1e-10)
    check(A, b, x.cpu().numpy(), info, ref, 1e-10, 5)


@pytest.mark.parametrize("two_stage", [False, True])
def test_mixed_precision_reaches_fp64_tolerance(B, ctx, two_stage):
    """Float basis and MPK; the explicit residual and x stay double, so restarts refine the
    solution to the FP64 tolerance."""
    A = wl.convdiff_2d(24, 30.0, 10.0)
    b = wl.rhs_uniform(A.n, 3)
    kw = dict(shat=30, two_stage=True) if two_stage else {}
    x, info, st = ctx.gmres(A, b, s=5, m=30, precision="mixed", tol=1e-10,
                            sketch=B.make_sketch("sparse_sign", 64, 8, 0), **kw)
    assert st == B.SKO_OK, info
    assert explicit_relres(A, x.cpu().numpy(), b) <= 1.01e-10


@pytest.mark.parametrize("s,shat,m", [(5, 20, 60), (10, 60, 60)])
def test_mixed_two_stage_tracks_fp64_iterations(B, ctx, s, shat, m):
    """Mixed precision, two-stage: the matrix-powers vectors of a panel stay in FP64 until
    the panel step writes the orthogonalised columns into the FP32 basis, so the iteration
    count follows the FP64 solve (to one check interval) instead of growing with the
    conditioning of the monomial panel.  k = 128 sketch rows take two sketch launches;
    s_hat < m projects panels on earlier big panels of the FP32 basis."""
    A = wl.convdiff_3d(16, (10.0, 20.0, 30.0))
    b = np.ones(A.n)
    kw = dict(s=s, m=m, shat=shat, two_stage=True, precond=1, tol=1e-10,
              sketch=B.make_sketch("sparse_sign", 128, 8, 0))
    x64, i64, st64 = ctx.gmres(A, b, **kw)
    x32, i32, st32 = ctx.gmres(A, b, precision="mixed", **kw)
    assert st64 == B.SKO_OK and st32 == B.SKO_OK, (i64, i32)
    assert explicit_relres(A, x32.cpu().numpy(), b) <= 1.01e-10
    assert i32["iters"] <= i64["iters"] + shat, (i32["iters"], i64["iters"])


def test_maxiter_and_resume(B, ctx):
    """ENOCONV at maxiter with a valid partial x; resuming from it converges (restart = resume)."""
    A = wl.convdiff_2d(24, 30.0, 10.0)
    b = wl.rhs_uniform(A.n, 3)
    sk = B.make_sketch("sparse_sign", 64, 8, 0)
    x1, info1, st1 = ctx.gmres(A, b, s=5, m=30, tol=1e-10, maxiter=30, sketch=sk)
    assert st1 == B.SKO_ENOCONV and info1["converged"] == 0 and info1["iters"] == 30
    r1 = explicit_relres(A, x1.cpu().numpy(), b)
    assert np.isfinite(r1) and r1 < 1.0
    assert abs(r1 - info1["relres"]) <= 1e-12 + 1e-9 * r1 or info1["restarts"] >= 1
    x2, info2, st2 = ctx.gmres(A, b, x0=x1, s=5, m=30, tol=1e-10, sketch=sk)
    assert st2 == B.SKO_OK
    assert explicit_relres(A, x2.cpu().numpy(), b) <= 1.01e-10


def test_zero_rhs(B, ctx):
    A = wl.laplacian_2d(10)
    x, info, st = ctx.gmres(A, np.zeros(A.n), s=5, m=10, tol=1e-10)
    assert st == B.SKO_OK and np.all(x.cpu().numpy() == 0)


def test_invalid_options(B, ctx):
    A = wl.laplacian_2d(10)
    b = np.ones(A.n)
    _, _, st = ctx.gmres(A, b, s=5, m=12)
    assert st == B.SKO_EINVAL
    _, _, st = ctx.gmres(A, b, s=5, m=30, shat=12, two_stage=True)
    assert st == B.SKO_EINVAL
