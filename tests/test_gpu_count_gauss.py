"""Count-Gaussian sketch (Section 5.2) on the HIP path against the oracle.

Theta = Theta_c Theta_g: the tall passes apply the hashed sparse-sign Count part Theta_c
(kc rows) and the reduction's small step applies the Gaussian factor Theta_g (kc x k, drawn
by the input generator and passed to both sides).  Checks:
* Y = Theta^T X against a reference summed in extended precision: normwise 1e-14, and
  entrywise against |Theta_g|^T |Theta_c^T| |X| (the product's error bound scale);
* one-stage RandCholQR-BCGS2 and the two-stage scheme with the composite sketch: R within
  max(1e-12, 10 kappa u) of the oracle's, orthogonality 1e-13, backward error 1e-14;
* s-step GMRES with it (one-stage, two-stage, and a batch in lock step): iteration counts
  within one check interval of the oracle's, x within 1e3 tol.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import krylov, metrics, orth  # noqa: E402
from oracle import sketch as osk  # noqa: E402
from paper_2503_16717_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


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


def _sketches(B, kc, k, zeta, seed, gseed):
    tg = wl.gaussian_theta(kc, k, gseed)
    tgd = B.colmajor_from_numpy(tg, "cuda")
    return B.make_sketch("count_gauss", zeta=zeta, seed=seed, theta=tgd), osk.Sketch.count_gauss(kc, zeta, seed, tg), tgd


@pytest.mark.parametrize("n,kc,k,zeta,precision", [(20000, 50, 12, 1, "f64"), (70001, 128, 24, 1, "f64"),
                                                   (5000, 256, 64, 8, "f64"), (30000, 72, 16, 1, "mixed")])
def test_count_gauss_sketch_apply(B, ctx, n, kc, k, zeta, precision):
    w = 6
    X = np.random.default_rng(n).standard_normal((n, w))
    if precision == "mixed":
        X = X.astype(np.float32).astype(np.float64)
    dt = torch.float32 if precision == "mixed" else torch.float64
    skd, sko, _keep = _sketches(B, kc, k, zeta, 5, 6)
    Y = ctx.sketch_apply(B.colmajor_from_numpy(X, "cuda", dtype=dt), skd, precision=precision)
    assert Y.shape == (k, w)
    tc = osk.sparse_sign_dense(n, kc, zeta, 5)
    tg = sko.theta
    # reference: Count part with exact sums (at most n terms of +-x/sqrt(zeta)), then the
    # Gaussian factor with exact sums
    Yc = np.array([[math.fsum(tc[:, h] * X[:, c]) for c in range(w)] for h in range(kc)])
    ref = np.array([[math.fsum(tg[:, i] * Yc[:, c]) for c in range(w)] for i in range(k)])
    mag = np.abs(tg).T @ (np.abs(tc).T @ np.abs(X))
    nrm = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    ent = np.max(np.abs(Y - ref) / mag)
    print(f"count-gauss n={n} kc={kc} k={k} zeta={zeta} {precision}: normwise {nrm:.2e}, entrywise {ent:.2e}")
    assert nrm <= 1e-14 and ent <= 1e-14
    Yo = sko.apply(X)
    assert np.linalg.norm(Y - Yo) / np.linalg.norm(Yo) <= 1e-14


@pytest.mark.parametrize("two_stage", [False, True])
def test_count_gauss_orthogonalisation(B, ctx, two_stage):
    n, nb, w, e = 30000, 6, 6, 12.0
    V = wl.glued_blocks(n, nb, w, e)
    if two_stage:
        kc, k = 128, 38
        skd, sko, _keep = _sketches(B, kc, k, 1, 3, 1)
        ref = orth.orth_blocks_two_stage(V, w, 3, sko)
        kw = dict(two_stage=True, panels_per_big=3)
    else:
        kc, k = 50, 12
        skd, sko, _keep = _sketches(B, kc, k, 1, 3, 1)
        ref = orth.orth_blocks_one_stage(V, w, "randcholqr", sko)
        kw = dict(intra="randcholqr")
    Q, R, st, col = ctx.orth_blocks(B.colmajor_from_numpy(V, "cuda"), w, sketch=skd, **kw)
    torch.cuda.synchronize()
    assert st == B.SKO_OK and ref.info == 0
    Qh = Q.cpu().numpy()
    rd = metrics.rel_diff(R, ref.R)
    oe = metrics.orth_error(Qh)[0]
    be = metrics.backward_error(V, Qh, R)
    print(f"count-gauss {'two' if two_stage else 'one'}-stage: R rel diff {rd:.2e} "
          f"(bound {max(1e-12, 10 * 10.0 ** e * U):.1e}), orth {oe:.2e}, backward {be:.2e}")
    assert rd <= max(1e-12, 10 * 10.0 ** e * U)
    assert oe <= 1e-13 and be <= 1e-14


def _check_gmres(A, b, x, info, ref, tol, step):
    assert info["converged"] == 1 and ref.converged
    r = b - A.to_scipy() @ x
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol * 1.01
    assert abs(info["iters"] - ref.iters) <= step
    assert np.linalg.norm(x - ref.x) <= 1e3 * tol * np.linalg.norm(ref.x)


def test_count_gauss_gmres_one_stage(B, ctx):
    A = wl.laplacian_2d(60)
    b = wl.rhs_uniform(A.n, 1)
    skd, sko, _keep = _sketches(B, 50, 12, 1, 0, 0)
    x, info, st = ctx.gmres(A, b, s=5, m=30, tol=1e-10, sketch=skd)
    assert st == B.SKO_OK, info
    ref = krylov.sstep_gmres(A, b, s=5, m=30, sk=sko, tol=1e-10)
    print(f"gmres one-stage count-gauss: iters {info['iters']} (oracle {ref.iters})")
    _check_gmres(A, b, x.cpu().numpy(), info, ref, 1e-10, 5)


def test_count_gauss_gmres_two_stage_and_batched(B, ctx):
    skd, sko, _keep = _sketches(B, 128, 42, 1, 4, 2)
    systems = [wl.convdiff_2d(N, bx, by) for N, bx, by in ((20, 30.0, 10.0), (26, 5.0, 40.0), (17, 12.0, 12.0))]
    rhs = [wl.rhs_uniform(A.n, 10 + i) for i, A in enumerate(systems)]
    kw = dict(s=5, m=40, shat=20, two_stage=True, tol=1e-10)
    for A, b in zip(systems[:1], rhs[:1]):
        x, info, st = ctx.gmres(A, b, sketch=skd, **kw)
        assert st == B.SKO_OK, info
        ref = krylov.sstep_gmres(A, b, s=5, m=40, shat=20, two_stage=True, sk=sko, tol=1e-10)
        print(f"gmres two-stage count-gauss: iters {info['iters']} (oracle {ref.iters})")
        _check_gmres(A, b, x.cpu().numpy(), info, ref, 1e-10, 20)
    # batched lock step: system i uses Count seed 4 + i and the shared Gaussian factor
    devs = [B.csr_to_device(A, "cuda") for A in systems]
    bds = [torch.from_numpy(b).cuda() for b in rhs]
    xds = [torch.zeros_like(bd) for bd in bds]
    st, infos = ctx.sko_gmres_batched([d[0] for d in devs], [bd.data_ptr() for bd in bds],
                                      [xd.data_ptr() for xd in xds], B.gmres_opts(sketch=skd, **kw))
    torch.cuda.synchronize()
    assert st == B.SKO_OK
    for i, (A, b) in enumerate(zip(systems, rhs)):
        skoi = osk.Sketch.count_gauss(128, 1, 4 + i, sko.theta)
        ref = krylov.sstep_gmres(A, b, s=5, m=40, shat=20, two_stage=True, sk=skoi, tol=1e-10)
        inf = B.info_dict(infos[i])
        print(f"batched system {i} n={A.n}: iters {inf['iters']} (oracle {ref.iters})")
        _check_gmres(A, b, xds[i].cpu().numpy(), inf, ref, 1e-10, 20)
