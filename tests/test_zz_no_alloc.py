"""sko_orth_block_noalloc (fixed device scratch, no allocation) against sko_orth_block.

Both entry points run the same kernels with the same launch shapes and the same order of
partial sums, so on one context their outputs must agree bit for bit; the test also holds
them to the parity bar against the oracle (R within max(1e-12, 10 kappa u), orthogonality
1e-13, backward error 1e-14).  Two calls in a row, the second on a smaller block, show that
what the first call leaves in the shared scratch does not leak into the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import metrics, orth  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
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


def _block_case(n, p, w, e, seed):
    """Orthonormal Q (n x p) and a block V (n x w) of condition 10^e with a component in
    range(Q)."""
    Qp = np.linalg.qr(np.random.default_rng([7, seed]).standard_normal((n, p)))[0] if p else None
    V = wl.glued_block(n, w, e, seed)
    if p:
        V = V + Qp @ np.random.default_rng([8, seed]).standard_normal((p, w))
    return Qp, np.asfortranarray(V)


@pytest.mark.parametrize("intra,precision", [("randcholqr", "f64"), ("cholqr2", "f64"),
                                             ("randcholqr", "mixed")])
def test_noalloc_matches_orth_block_two_calls(B, ctx, intra, precision):
    sk = B.make_sketch("sparse_sign", 64, 8, 3)
    dt = torch.float32 if precision == "mixed" else torch.float64
    e = 6.0 if intra == "cholqr2" else 10.0
    for n, p, w in ((40000, 12, 6), (3001, 6, 5)):
        print(f"noalloc case intra={intra} precision={precision} n={n} p={p} w={w}", flush=True)
        Qp, V = _block_case(n, p, w, e, n)
        Vd = B.colmajor_from_numpy(V, "cuda", dtype=dt)
        Qd = B.colmajor_from_numpy(Qp, "cuda", dtype=dt) if p else None
        out_ref = torch.empty((w, n), dtype=dt, device="cuda").t()
        out_na = torch.full((w, n), float("nan"), dtype=dt, device="cuda").t()
        kw = dict(intra=intra, precision=precision, sketch=sk)
        _, Rp0, Rd0, st0, _ = ctx.orth_block(Qd, Vd, out_ref, **kw)
        _, Rp1, Rd1, st1, _ = ctx.orth_block(Qd, Vd, out_na, noalloc=True, **kw)
        torch.cuda.synchronize()
        assert st0 == B.SKO_OK and st1 == B.SKO_OK
        assert torch.equal(out_ref, out_na)
        assert np.array_equal(Rd0, Rd1) and np.array_equal(Rp0, Rp1)
        if precision != "f64":
            continue
        osk = Sketch.sparse_sign(64, 8, 3) if intra == "randcholqr" else None
        Qj, Rp_ref, Rd_ref, info = orth.bcgs2_block(Qp if p else np.zeros((n, 0)), V, intra, osk)
        assert info == 0
        R = np.vstack([Rp1, Rd1])
        Rref = np.vstack([Rp_ref, Rd_ref])
        rd = metrics.rel_diff(R, Rref)
        Qh = out_na.cpu().numpy()
        oe = metrics.orth_error(Qh)[0]
        cross = float(np.max(np.abs(Qp.T @ Qh)))
        print(f"  R rel diff vs oracle {rd:.2e} (bound {max(1e-12, 10 * 10.0 ** e * U):.1e}), "
              f"orth {oe:.2e}, |Qp^T Q| {cross:.1e}", flush=True)
        assert rd <= max(1e-12, 10 * 10.0 ** e * U)
        assert oe <= 1e-13 and cross <= 1e-13


def test_noalloc_rejects_request_beyond_scratch(B, ctx):
    # 2^19 rows fill the full grid (8 workgroups per compute unit); k = 256 sketch rows of a
    # 16-column block then need 64 MiB of partial sums, twice the scratch.  The library
    # rejects the call on the host, before any launch.
    n, w = 1 << 19, 16
    V = torch.zeros((w, n), dtype=torch.float64, device="cuda").t()
    out = torch.empty((w, n), dtype=torch.float64, device="cuda").t()
    sk = B.make_sketch("sparse_sign", 256, 8, 0)
    _, _, _, st, _ = ctx.orth_block(None, V, out, noalloc=True, raise_on_error=False, intra="randcholqr",
                                    sketch=sk)
    assert st == B.SKO_ESCRATCH
    assert "scratch" in B.strerror(st)
