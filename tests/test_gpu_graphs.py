"""Launch graphs of the one-stage solver against plain launches.

Each s-step block's launches are captured once per block position and replayed in every
restart cycle, with the solver's own eager work (explicit residual, solution update, Ritz
values) and host synchronisations between the replays.  The replayed kernels take the same
arguments as the eager ones, so the solution and every reported count must agree bit for bit;
the solution is also held to the oracle's bars."""
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


def both(B, ctx, A, b, **kw):
    xg, ig, sg = ctx.gmres(A, b, **kw)
    xe, ie, se = ctx.gmres(A, b, eager=True, **kw)
    torch.cuda.synchronize()
    return (xg.cpu().numpy(), ig, sg), (xe.cpu().numpy(), ie, se)


@pytest.mark.parametrize("case", ["config1_gaussian", "sparse_cholqr2", "newton", "mixed"])
def test_graph_replays_equal_eager(B, ctx, case):
    if case == "config1_gaussian":
        A = wl.laplacian_2d(100)
        b = wl.rhs_uniform(A.n, 1)
        th = wl.gaussian_theta(A.n, 24, 0)
        thd = B.colmajor_from_numpy(th, "cuda")
        kw = dict(s=5, m=30, tol=1e-10, sketch=B.make_sketch("gaussian", theta=thd))
        ref = krylov.sstep_gmres(A, b, s=5, m=30, sk=Sketch.gaussian(th), tol=1e-10)
    elif case == "sparse_cholqr2":
        A = wl.convdiff_2d(30, 20.0, 10.0)
        b = wl.rhs_uniform(A.n, 2)
        kw = dict(s=5, m=30, intra="cholqr2", tol=1e-10, precond=1, sketch=B.make_sketch("sparse_sign", 64, 8, 1))
        ref = krylov.sstep_gmres(A, b, s=5, m=30, intra="cholqr2", jacobi=True, sk=Sketch.sparse_sign(64, 8, 1),
                                 tol=1e-10)
    elif case == "newton":
        A = wl.convdiff_2d(24, 30.0, 10.0)
        b = wl.rhs_uniform(A.n, 3)
        kw = dict(s=6, m=36, tol=1e-10, basis="newton", sketch=B.make_sketch("sparse_sign", 64, 8, 0))
        ref = krylov.sstep_gmres(A, b, s=6, m=36, sk=Sketch.sparse_sign(64, 8, 0), tol=1e-10, basis="newton")
    else:
        A = wl.laplacian_2d(60)
        b = wl.rhs_uniform(A.n, 4)
        kw = dict(s=5, m=30, tol=1e-10, precision="mixed", sketch=B.make_sketch("sparse_sign", 64, 8, 2))
        ref = None
    (xg, ig, sg), (xe, ie, se) = both(B, ctx, A, b, **kw)
    print(f"{case}: graphs {ig['iters']} iterations in {ig['t_total'] * 1e3:.2f} ms, "
          f"eager {ie['iters']} in {ie['t_total'] * 1e3:.2f} ms", flush=True)
    assert sg == se == B.SKO_OK
    assert np.array_equal(xg, xe)
    for f in ("iters", "restarts", "relres", "relres_implicit", "converged"):
        assert ig[f] == ie[f], f
    if ref is not None:
        assert ref.converged and abs(ig["iters"] - ref.iters) <= kw["s"]
        assert np.linalg.norm(xg - ref.x) <= 1e3 * 1e-10 * np.linalg.norm(ref.x)


def test_graphs_follow_a_new_right_hand_side(B, ctx):
    """Two solves in a row on one context (graphs are captured per solve): the second must
    not see anything of the first."""
    A = wl.laplacian_2d(50)
    sk = B.make_sketch("sparse_sign", 64, 8, 0)
    for seed in (5, 6):
        b = wl.rhs_uniform(A.n, seed)
        (xg, ig, _), (xe, ie, _) = both(B, ctx, A, b, s=5, m=30, tol=1e-10, sketch=sk)
        assert np.array_equal(xg, xe) and ig["iters"] == ie["iters"]
        assert np.linalg.norm(b - A.to_scipy() @ xg) / np.linalg.norm(b) <= 1.01e-10
