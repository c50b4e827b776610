"""The sketch Y = Theta^T X of the HIP path (sko_sketch_apply) against the oracle's Theta.

Section 3 applies a sketch to a block as Theta^T X; Section 5.2's Count sketch (here the
sparse-sign sketch with zeta nonzeros per row of Theta) is applied without storing Theta,
so both sides build it from the same written placement rule (include/sko.h, sko_sketch)
and the published SplitMix64 generator, independently.  The R factor, Q and the error
metrics of an orthogonalisation do not depend on Theta in exact arithmetic, so only a
direct comparison of Y can show a wrong slot, sign or hash word.

* One-hot columns: column c of X is x_c e_i, so Y[:, c] is row i of Theta times x_c, with a
  single nonzero term per entry: the GPU must reproduce it bit for bit (slot, sign and the
  1/sqrt(zeta) scale), also for rows near 2^24 (the counters of the 2^24-row workload).
* Integer-valued X at n = 2^24 (the benchmarked shape): every partial sum of +-x is an
  integer below 2^53, so sum order does not matter and Y = (integer sum) / sqrt(zeta) is
  bit exact on both sides.
* Random X: normwise within 1e-14 of a reference summed in extended precision, and
  entrywise within 1e-14 of |Theta|^T |X|.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sketch as osk  # noqa: E402
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


def _one_hot(n, rows, vals, dtype=torch.float64):
    X = torch.zeros((len(rows), n), dtype=dtype, device="cuda")
    for c, (r, v) in enumerate(zip(rows, vals)):
        X[c, r] = v
    return X.t()


def _oracle_rows(rows, vals, k, zeta, seed):
    """Y[:, c] = Theta[rows[c], :] * vals[c] from the oracle's pattern (terms formed as the
    oracle forms them: sign * (1/sqrt(zeta)) * x)."""
    slots, signs = osk.sparse_sign_pattern(np.asarray(rows), k, zeta, seed)
    scale = 1.0 / math.sqrt(zeta)
    Y = np.zeros((k, len(rows)))
    for c, v in enumerate(vals):
        for t in range(zeta):
            Y[slots[c, t], c] += signs[c, t] * scale * v
    return Y


@pytest.mark.parametrize("k", [48, 64, 96, 128])
@pytest.mark.parametrize("zeta", [1, 8])
def test_one_hot_rows_bit_exact(B, ctx, k, zeta):
    n, seed = 5003, 17
    rng = np.random.default_rng(k * 10 + zeta)
    rows = [0, 1, 255, 256, n - 2, n - 1] + list(rng.integers(0, n, 6))
    vals = list(rng.standard_normal(len(rows)))
    Y = ctx.sketch_apply(_one_hot(n, rows, vals), B.make_sketch("sparse_sign", k, zeta, seed))
    ref = _oracle_rows(rows, vals, k, zeta, seed)
    print(f"k={k} zeta={zeta}: max |dY| = {np.max(np.abs(Y - ref)):.3e}")
    assert np.array_equal(Y, ref)
    assert np.all((Y != 0).sum(axis=0) == zeta)


@pytest.mark.parametrize("k,zeta", [(64, 8), (128, 8), (48, 8)])
def test_one_hot_rows_near_2p24_bit_exact(B, ctx, k, zeta):
    n = 1 << 24
    rows = [n - 1, n - 2, n - 64, n - 257, (1 << 23) + 12345, n - 4093]
    vals = [1.0, -2.5, 0.75, 3.0, -1.0, 1.0 / 3.0]
    Y = ctx.sketch_apply(_one_hot(n, rows, vals), B.make_sketch("sparse_sign", k, zeta, 0))
    assert np.array_equal(Y, _oracle_rows(rows, vals, k, zeta, 0))


def test_integer_data_full_size_bit_exact(B, ctx):
    """n = 2^24, 6 columns, k = 64, zeta = 8 (the benchmarked sketch): every row's hash word
    takes part."""
    n, w, k, zeta, seed = 1 << 24, 6, 64, 8, 0
    g = torch.Generator(device="cuda").manual_seed(5)
    Xd = torch.randint(-3, 4, (w, n), generator=g, device="cuda", dtype=torch.int64).double()
    Y = ctx.sketch_apply(Xd.t(), B.make_sketch("sparse_sign", k, zeta, seed))
    X = Xd.t().cpu().numpy()
    slots, signs = osk.sparse_sign_pattern(np.arange(n), k, zeta, seed)
    S = np.zeros((k, w))
    for t in range(zeta):
        for c in range(w):
            S[:, c] += np.bincount(slots[:, t], weights=signs[:, t] * X[:, c], minlength=k)
    assert np.all(S == np.round(S))            # integer sums: exact in any order
    ref = S * (1.0 / math.sqrt(zeta))
    print(f"full size integer data: max |dY| = {np.max(np.abs(Y - ref)):.3e}")
    assert np.array_equal(Y, ref)


def _extended_reference(theta_rows, X):
    """Theta^T X summed in extended precision (products and sums with a 64-bit significand)."""
    T = np.asarray(theta_rows, dtype=np.longdouble)
    Xl = np.asarray(X, dtype=np.longdouble)
    return (T.T @ Xl).astype(np.float64), (np.abs(T).T @ np.abs(Xl)).astype(np.float64)


@pytest.mark.parametrize("k,zeta", [(48, 8), (64, 8), (96, 1), (128, 8), (128, 1)])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_random_block_close_to_extended_precision(B, ctx, k, zeta, precision):
    n, w, seed = 70001, 11, 3
    X = np.random.default_rng(k + zeta).standard_normal((n, w))
    if precision == "mixed":
        X = X.astype(np.float32).astype(np.float64)
    dt = torch.float32 if precision == "mixed" else torch.float64
    Xd = B.colmajor_from_numpy(X, "cuda", dtype=dt)
    Y = ctx.sketch_apply(Xd, B.make_sketch("sparse_sign", k, zeta, seed), precision=precision)
    ref, mag = _extended_reference(osk.sparse_sign_dense(n, k, zeta, seed), X)
    nrm = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    ent = np.max(np.abs(Y - ref) / mag)
    print(f"k={k} zeta={zeta} {precision}: normwise {nrm:.2e}, entrywise {ent:.2e}")
    assert nrm <= 1e-14 and ent <= 1e-14
    # and the oracle's own product agrees within its rounding
    Yo = osk.Sketch.sparse_sign(k, zeta, seed).apply(X)
    assert np.linalg.norm(Y - Yo) / np.linalg.norm(Yo) <= 1e-14


def test_gaussian_sketch_k24(B, ctx):
    n, w = 10000, 6
    th = wl.gaussian_theta(n, 24, 0)
    thd = B.colmajor_from_numpy(th, "cuda")
    X = np.random.default_rng(9).standard_normal((n, w))
    Y = ctx.sketch_apply(B.colmajor_from_numpy(X, "cuda"), B.make_sketch("gaussian", theta=thd))
    ref, mag = _extended_reference(th, X)
    nrm = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    ent = np.max(np.abs(Y - ref) / mag)
    print(f"gaussian k=24: normwise {nrm:.2e}, entrywise {ent:.2e}")
    assert nrm <= 1e-14 and ent <= 1e-14


def test_invalid_arguments_rejected(B, ctx):
    n, w = 1000, 6
    X = torch.zeros((w, n), dtype=torch.float64, device="cuda").t()
    Y = np.zeros((64, w), order="F")
    bad = [B.make_sketch("sparse_sign", 60, 8, 0),   # zeta does not divide k
           B.make_sketch("sparse_sign", 512, 8, 0),  # k too large
           B.make_sketch("sparse_sign", 64, 0, 0)]   # no nonzeros
    for sk in bad:
        assert ctx.sko_sketch_apply(n, w, X.data_ptr(), n, B.SKO_F64, sk, Y, 64) == B.SKO_EINVAL
    good = B.make_sketch("sparse_sign", 64, 8, 0)
    assert ctx.sko_sketch_apply(n, w, X.data_ptr(), n, B.SKO_F64, good, Y, 63) == B.SKO_EINVAL   # ldy < k
    assert ctx.sko_sketch_apply(n, 17, X.data_ptr(), n, B.SKO_F64, good, Y, 64) == B.SKO_EINVAL  # w > 16
    assert ctx.sko_sketch_apply(n, w, X.data_ptr(), n - 1, B.SKO_F64, good, Y, 64) == B.SKO_EINVAL
    with pytest.raises(TypeError):
        ctx.sketch_apply(X.float(), good)                                 # dtype checked
