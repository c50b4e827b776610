"""Pins for the oracle's sketches (Section 3; Section 5.2)."""
import math
import os

import numpy as np
import pytest

from oracle import sketch as osk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_splitmix_golden():
    out = []
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            c, v = line.split()
            out.append((int(c), int(v, 16)))
    return out


def test_splitmix64_published_outputs():
    for c, v in _read_splitmix_golden():
        assert osk.splitmix64_scalar(0, c) == v
        assert int(osk.splitmix64(0, np.array([c], dtype=np.uint64))[0]) == v


def test_splitmix64_vector_matches_scalar_any_seed():
    rng = np.random.default_rng(7)
    for seed in (1, 12345, (1 << 63) + 17):
        cs = rng.integers(0, 1 << 40, 50)
        vec = osk.splitmix64(seed, cs.astype(np.uint64))
        for c, v in zip(cs, vec):
            assert int(v) == osk.splitmix64_scalar(seed, int(c))


@pytest.mark.parametrize("k,zeta", [(64, 8), (48, 8), (128, 8), (24, 1), (16, 16), (40, 10)])
def test_sparse_sign_structure(k, zeta):
    n = 3000
    th = osk.sparse_sign_dense(n, k, zeta, seed=5)
    B = k // zeta
    nz = th != 0
    assert np.all(nz.sum(axis=1) == zeta)
    assert np.allclose(np.abs(th[nz]), 1.0 / math.sqrt(zeta), rtol=0, atol=0)
    for t in range(zeta):  # exactly one nonzero per slot block
        assert np.all(nz[:, t * B:(t + 1) * B].sum(axis=1) == 1)
    # both signs and every slot occur with roughly the expected frequency
    frac_neg = np.mean(th[nz] < 0)
    assert abs(frac_neg - 0.5) < 0.05
    counts = nz.sum(axis=0)
    assert counts.min() > 0.6 * n / B and counts.max() < 1.4 * n / B


@pytest.mark.parametrize("kind", ["sparse_sign", "gaussian"])
def test_apply_equals_dense_product(kind):
    n, k, w = 777, 64, 6
    X = np.random.default_rng(3).standard_normal((n, w))
    if kind == "sparse_sign":
        sk = osk.Sketch.sparse_sign(k, 8, 11)
        dense = osk.sparse_sign_dense(n, k, 8, 11)
    else:
        dense = np.random.default_rng(4).standard_normal((n, k)) / math.sqrt(k)
        sk = osk.Sketch.gaussian(dense)
    Y = sk.apply(X)
    # brute force: Y[h, c] = sum_i Theta[i, h] X[i, c] with exact-order Python sums
    Yb = np.zeros((k, w))
    for h in range(k):
        rows = np.nonzero(dense[:, h])[0]
        for c in range(w):
            Yb[h, c] = math.fsum(dense[rows, h] * X[rows, c])
    assert np.max(np.abs(Y - Yb)) <= 1e-13 * np.max(np.abs(Yb))


def test_count_gauss_is_the_composite_product():
    """Section 5.2: the Count-Gaussian sketch is Theta = Theta_c Theta_g (n x kc times kc x k),
    applied as Theta_g^T (Theta_c^T X).  Brute force from the materialised n x k product; kc != k
    and w != k, so a transposed or swapped factor cannot even be multiplied."""
    n, kc, k, w = 500, 50, 12, 6
    X = np.random.default_rng(1).standard_normal((n, w))
    tg = np.random.default_rng(2).standard_normal((kc, k)) / math.sqrt(k)
    sk = osk.Sketch.count_gauss(kc, 1, 9, tg)
    theta = osk.sparse_sign_dense(n, kc, 1, 9) @ tg
    Y = sk.apply(X)
    Yb = np.array([[math.fsum(theta[:, h] * X[:, c]) for c in range(w)] for h in range(k)])
    assert Y.shape == (k, w)
    assert np.max(np.abs(Y - Yb)) <= 1e-13 * np.max(np.abs(Yb))


def test_count_gauss_with_identity_factor_is_the_count_sketch():
    n, kc, w = 2000, 48, 5
    X = np.random.default_rng(3).standard_normal((n, w))
    Y = osk.Sketch.count_gauss(kc, 8, 4, np.eye(kc)).apply(X)
    assert np.array_equal(Y, osk.Sketch.sparse_sign(kc, 8, 4).apply(X))


@pytest.mark.parametrize("kind,k,zeta", [("sparse_sign", 64, 8), ("gaussian", 24, 0), ("sparse_sign", 48, 8),
                                         ("count_gauss", 24, 1)])
def test_subspace_embedding(kind, k, zeta):
    """Def. 3.1 / Cor. 3.2-3.3: for orthonormal Q the singular values of Theta^T Q lie in
    [sqrt(1-mu), sqrt(1+mu)].  Section 3 sizes the sketch as k ~ d / mu^2 (a rule of thumb,
    not a bound).  Every one of 20 draws must be an embedding (mu < 1, so Theta^T Q has full
    rank and Cor. 3.3 bounds kappa), with kappa(Theta^T Q) small and a typical distortion
    near the rule of thumb."""
    n, d = 4096, 6
    mus = []
    for seed in range(20):
        Q, _ = np.linalg.qr(np.random.default_rng(100 + seed).standard_normal((n, d)))
        if kind == "gaussian":
            sk = osk.Sketch.gaussian(np.random.default_rng(seed).standard_normal((n, k)) / math.sqrt(k))
        elif kind == "count_gauss":
            # Section 5.2 sizes: Count to O(d^2) rows (2 d^2 = 72), then Gaussian to O(d) rows
            tg = np.random.default_rng(seed).standard_normal((2 * d * d, k)) / math.sqrt(k)
            sk = osk.Sketch.count_gauss(2 * d * d, 1, seed, tg)
        else:
            sk = osk.Sketch.sparse_sign(k, zeta, seed)
        sv = np.linalg.svd(sk.apply(Q), compute_uv=False)
        mus.append(max(1.0 - sv[-1] ** 2, sv[0] ** 2 - 1.0))
        assert 1.0 - sv[-1] ** 2 < 1.0 and sv[0] / sv[-1] < 5.0
    # two embeddings compose: (1 +- mu_c)(1 +- mu_g), so the composite's typical distortion is
    # allowed the sum of the parts' (about 0.4 for the Count part at 72 rows)
    assert np.median(mus) < (1.0 if kind == "count_gauss" else 0.85)
