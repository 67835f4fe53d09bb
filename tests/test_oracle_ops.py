"""Pins for the oracle's event-driven CSR matvec, JIT matvec and their
reverse modes (CPU only): dense brute force over every event vector of tiny
matrices, a library sparse product, exact special cases, exact finite
differences of the (linear) operators, and distribution tests of the JIT
weights."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy import stats

import oracle as O
import synthetic as S


def _random_csr(rng, n_pre, n_post, dens, dup=True):
    indptr = [0]
    idx = []
    for _ in range(n_pre):
        m = rng.binomial(n_post, dens)
        cols = list(rng.integers(0, n_post, m)) if dup else sorted(rng.choice(n_post, m, replace=False))
        idx += cols
        indptr.append(len(idx))
    return np.array(indptr, np.int32), np.array(idx, np.int32)


def _dense(indptr, indices, data, w, n_pre, n_post):
    D = np.zeros((n_pre, n_post))
    for j in range(n_pre):
        for idx in range(indptr[j], indptr[j + 1]):
            D[j, indices[idx]] += data[idx] if data is not None else w
    return D


@pytest.mark.parametrize("hetero", [False, True])
def test_event_csr_bruteforce_all_event_vectors(hetero):
    # Appendix B defines y = M^T e over rows that fire; with duplicated and
    # unsorted columns each entry adds.  All 2^8 event vectors.
    rng = np.random.default_rng(3)
    n_pre, n_post = 8, 13
    ip, ix = _random_csr(rng, n_pre, n_post, 0.4, dup=True)
    data = rng.standard_normal(ix.size).astype(np.float32) if hetero else None
    w = 0.6
    D = _dense(ip, ix, data, w, n_pre, n_post)
    for bits in itertools.product([0, 1], repeat=n_pre):
        e = np.array(bits, np.uint8)
        y = O.event_csr_matvec(ip, ix, data, w, n_post, e)
        np.testing.assert_allclose(y, D.T @ e, rtol=0, atol=1e-12)


def test_event_csr_vs_scipy():
    rng = np.random.default_rng(4)
    n_pre, n_post = 3000, 2000
    ip, ix = _random_csr(rng, n_pre, n_post, 0.01)
    data = S.hetero_data(ix.size, 1)
    e = S.events(n_pre, 0.1, 2)
    M = sp.csr_matrix((data.astype(np.float64), ix, ip), shape=(n_pre, n_post))
    y = O.event_csr_matvec(ip, ix, data, 0.0, n_post, e)
    np.testing.assert_allclose(y, M.T @ (e != 0).astype(np.float64), rtol=1e-12, atol=1e-12)


def test_event_csr_special_cases():
    ip, ix = O.csr_build(1, 19, 500, 400, 0)
    z = O.event_csr_matvec(ip, ix, None, 0.6, 400, np.zeros(500, np.uint8))
    assert np.all(z == 0.0)
    ones = O.event_csr_matvec(ip, ix, None, 0.6, 400, np.ones(500, np.uint8))
    indeg = np.bincount(ix, minlength=400)
    np.testing.assert_allclose(ones, 0.6 * indeg, rtol=1e-13)
    e = S.events(500, 0.3, 5)
    cnt = O.event_csr_counts(ip, ix, 400, e)
    np.testing.assert_allclose(O.event_csr_matvec(ip, ix, None, 0.6, 400, e), 0.6 * cnt, rtol=1e-13)
    # event values are truthiness: any non-zero byte is one event
    e2 = e * np.uint8(7)
    np.testing.assert_array_equal(O.event_csr_counts(ip, ix, 400, e2), cnt)


def test_batched_products_bruteforce():
    # a batch of spike vectors E [batch, n_pre]: Y = E M, the dense matrix
    # product of numpy, for stored (duplicated, unsorted columns, data and
    # homogeneous) and JIT matrices; all-zero and all-one vectors included
    rng = np.random.default_rng(8)
    n_pre, n_post = 30, 41
    ip, ix = _random_csr(rng, n_pre, n_post, 0.3, dup=True)
    data = rng.standard_normal(ix.size).astype(np.float32)
    E = np.stack([S.events(n_pre, f, 20 + i) for i, f in enumerate((0.0, 0.2, 0.5, 1.0, 0.05))])
    E[2] *= np.uint8(5)  # any non-zero byte is a spike
    for d, w in ((None, 0.6), (data, 0.0)):
        D = _dense(ip, ix, d, w, n_pre, n_post)
        np.testing.assert_allclose(O.event_csr_matmat(ip, ix, d, w, n_post, E), (E != 0) @ D, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(O.event_csr_counts_batch(ip, ix, n_post, E),
                                  (E != 0).astype(np.int64) @ _dense(ip, ix, None, 1, n_pre, n_post).astype(np.int64))
    seed, K, B = 6, 5, 16
    for wkind, w0, w1 in ((O.W_HOMO, 0.7, 0.0), (O.W_NORMAL, 0.5, 0.1), (O.W_UNIFORM, -1.0, 2.0)):
        D = np.zeros((n_pre, n_post))
        for j in range(n_pre):
            for b in range(-(-n_post // B)):
                for m, k in enumerate(O.row_block(seed, K, n_post, B, j, b)):
                    D[j, k] += O.jit_weight(seed, wkind, w0, w1, j, b, m)[0]
        np.testing.assert_allclose(O.jit_matmat(seed, K, B, wkind, w0, w1, n_post, E), (E != 0) @ D,
                                   rtol=1e-12, atol=1e-12)
    ipj, ixj = O.csr_build(seed, K, n_pre, n_post, B)
    np.testing.assert_array_equal(O.jit_counts_batch(seed, K, B, n_post, E),
                                  O.event_csr_counts_batch(ipj, ixj, n_post, E))


@pytest.mark.parametrize("B", [0, 64])
def test_jit_equals_csr_of_same_seed(B):
    seed, K, n_pre, n_post = 77, 49, 700, 900
    ip, ix = O.csr_build(seed, K, n_pre, n_post, B)
    for frac in (0.0, 0.05, 1.0):
        e = S.events(n_pre, frac, 9)
        np.testing.assert_array_equal(O.jit_counts(seed, K, B, n_post, e), O.event_csr_counts(ip, ix, n_post, e))
        y = O.jit_matvec(seed, K, B, O.W_HOMO, 6.7, 0.0, n_post, e)
        np.testing.assert_allclose(y, 6.7 * O.event_csr_counts(ip, ix, n_post, e), rtol=1e-13)


@pytest.mark.parametrize("wkind", [O.W_NORMAL, O.W_UNIFORM])
def test_jit_weighted_bruteforce(wkind):
    seed, K, n_pre, n_post, B = 5, 9, 40, 60, 16
    w0, w1 = (0.5, 0.1) if wkind == O.W_NORMAL else (-1.0, 2.0)
    D = np.zeros((n_pre, n_post))
    nb = -(-n_post // B)
    for j in range(n_pre):
        for b in range(nb):
            r = O.row_block(seed, K, n_post, B, j, b)
            for m, k in enumerate(r):
                D[j, k] += O.jit_weight(seed, wkind, w0, w1, j, b, m)[0]
    e = S.events(n_pre, 0.5, 1)
    y = O.jit_matvec(seed, K, B, wkind, w0, w1, n_post, e)
    np.testing.assert_allclose(y, D.T @ e, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("wkind", [O.W_HOMO, O.W_NORMAL, O.W_UNIFORM])
def test_jit_dense_vector_bruteforce(wkind):
    # Section 5.2's JIT operator on a float vector: y = sum_j v[j] J[j, :],
    # the dense matrix assembled entry by entry and multiplied by numpy.
    seed, K, n_pre, n_post, B = 8, 7, 45, 70, 16
    w0, w1 = {O.W_HOMO: (0.3, 0.0), O.W_NORMAL: (0.5, 0.1), O.W_UNIFORM: (-1.0, 2.0)}[wkind]
    D = np.zeros((n_pre, n_post))
    for j in range(n_pre):
        for b in range(-(-n_post // B)):
            for m, k in enumerate(O.row_block(seed, K, n_post, B, j, b)):
                D[j, k] += O.jit_weight(seed, wkind, w0, w1, j, b, m)[0]
    v = S.dense_vector(n_pre, 2, zero_frac=0.3).astype(np.float64)
    y = O.jit_matvec_dense(seed, K, B, wkind, w0, w1, n_post, v)
    np.testing.assert_allclose(y, D.T @ v, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("B", [0, 64])
def test_jit_dense_vector_special_cases(B):
    # On a 0/1 vector the float product is the event product; a stored CSR of
    # the same seed gives the same homogeneous product through scipy; the
    # product is linear in v; v = 0 gives 0.
    seed, K, n_pre, n_post = 31, 23, 300, 410
    e = S.events(n_pre, 0.2, 4)
    for wk, w0, w1 in [(O.W_HOMO, 0.7, 0.0), (O.W_NORMAL, 0.5, 0.1)]:
        np.testing.assert_array_equal(O.jit_matvec_dense(seed, K, B, wk, w0, w1, n_post, e.astype(np.float64)),
                                      O.jit_matvec(seed, K, B, wk, w0, w1, n_post, e))
    ip, ix = O.csr_build(seed, K, n_pre, n_post, B)
    M = sp.csr_matrix((np.ones(ix.size), ix, ip), shape=(n_pre, n_post))
    v1 = S.dense_vector(n_pre, 5).astype(np.float64)
    v2 = S.dense_vector(n_pre, 6, zero_frac=0.5).astype(np.float64)
    y1 = O.jit_matvec_dense(seed, K, B, O.W_HOMO, 1.5, 0.0, n_post, v1)
    np.testing.assert_allclose(y1, 1.5 * (M.T @ v1), rtol=1e-12, atol=1e-12)
    y2 = O.jit_matvec_dense(seed, K, B, O.W_UNIFORM, -0.5, 1.0, n_post, v2)
    y12 = O.jit_matvec_dense(seed, K, B, O.W_UNIFORM, -0.5, 1.0, n_post, 2.0 * v1 - 3.0 * v2)
    y1u = O.jit_matvec_dense(seed, K, B, O.W_UNIFORM, -0.5, 1.0, n_post, v1)
    np.testing.assert_allclose(y12, 2.0 * y1u - 3.0 * y2, rtol=1e-11, atol=1e-11)
    assert not O.jit_matvec_dense(seed, K, B, O.W_NORMAL, 0.5, 0.1, n_post, np.zeros(n_pre)).any()


@pytest.mark.parametrize("wkind", [O.W_HOMO, O.W_NORMAL, O.W_UNIFORM])
def test_jit_dense_matrix_bruteforce(wkind):
    # m vectors at once: Y = D^T X with D assembled entry by entry (numpy
    # product), and column c of Y equal to the single-vector product of
    # column c of X (same row order, so exactly).
    seed, K, n_pre, n_post, B, m = 8, 7, 45, 70, 16, 5
    w0, w1 = {O.W_HOMO: (0.3, 0.0), O.W_NORMAL: (0.5, 0.1), O.W_UNIFORM: (-1.0, 2.0)}[wkind]
    D = np.zeros((n_pre, n_post))
    for j in range(n_pre):
        for b in range(-(-n_post // B)):
            for t, k in enumerate(O.row_block(seed, K, n_post, B, j, b)):
                D[j, k] += O.jit_weight(seed, wkind, w0, w1, j, b, t)[0]
    X = np.stack([S.dense_vector(n_pre, 40 + c, zero_frac=0.3) for c in range(m)], 1).astype(np.float64)
    X[3] = 0.0
    Y = O.jit_matmat_dense(seed, K, B, wkind, w0, w1, n_post, X)
    np.testing.assert_allclose(Y, D.T @ X, rtol=1e-12, atol=1e-12)
    for c in range(m):
        np.testing.assert_array_equal(Y[:, c], O.jit_matvec_dense(seed, K, B, wkind, w0, w1, n_post, X[:, c]))


@pytest.mark.parametrize("wkind", [O.W_HOMO, O.W_NORMAL, O.W_UNIFORM])
def test_jit_abs_terms_bruteforce(wkind):
    # the tolerance scale of the FP32 products: with each weight split into
    # the two terms of its formula, w = a + b (a = w0; b = w1 z normal,
    # (w1 - w0) u uniform, 0 homogeneous), the scale equals
    # (|A| + |B|)^T |X| for the two term matrices assembled entry by entry;
    # it is at least |D|^T |X| (D = A + B), and equals the product itself
    # when every term and every x is non-negative
    seed, K, n_pre, n_post, B, m = 9, 5, 40, 66, 16, 3
    w0, w1 = {O.W_HOMO: (-0.3, 0.0), O.W_NORMAL: (0.1, 1.0), O.W_UNIFORM: (-1.0, 2.0)}[wkind]
    D = np.zeros((n_pre, n_post))
    TA = np.zeros((n_pre, n_post))
    TB = np.zeros((n_pre, n_post))
    for j in range(n_pre):
        for b in range(-(-n_post // B)):
            for t, k in enumerate(O.row_block(seed, K, n_post, B, j, b)):
                w, unit = O.jit_weight(seed, wkind, w0, w1, j, b, t)
                D[j, k] += w
                TA[j, k] += abs(w0)
                if wkind == O.W_NORMAL:
                    TB[j, k] += abs(w1 * unit)
                elif wkind == O.W_UNIFORM:
                    TB[j, k] += abs((w1 - w0) * unit)
    assert (D < 0).any()
    np.testing.assert_allclose(D, np.where(TA > 0, D, 0.0))  # every weight sits on a connection
    X = np.stack([S.dense_vector(n_pre, 70 + c, zero_frac=0.3) for c in range(m)], 1).astype(np.float64)
    sc = O.jit_abs_terms(seed, K, B, wkind, w0, w1, n_post, X)
    np.testing.assert_allclose(sc, (TA + TB).T @ np.abs(X), rtol=1e-12, atol=1e-12)
    assert np.all(sc >= np.abs(D).T @ np.abs(X) - 1e-12)
    e = S.events(n_pre, 0.4, 3)
    np.testing.assert_allclose(O.jit_abs_terms(seed, K, B, wkind, w0, w1, n_post, e), (TA + TB).T @ e,
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(O.jit_abs_terms(seed, K, B, O.W_UNIFORM, 0.5, 2.0, n_post, np.abs(X)),
                               O.jit_matmat_dense(seed, K, B, O.W_UNIFORM, 0.5, 2.0, n_post, np.abs(X)),
                               rtol=1e-12, atol=1e-12)
    if wkind == O.W_HOMO:
        np.testing.assert_allclose(sc, np.abs(D).T @ np.abs(X), rtol=1e-12, atol=1e-12)


def test_jit_normal_weights_are_normal():
    z = np.array([O.jit_weight(3, O.W_NORMAL, 0.0, 1.0, j, 0, m)[1] for j in range(400) for m in range(50)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    w = np.array([O.jit_weight(3, O.W_NORMAL, 0.5, 0.1, j, 0, 7)[0] for j in range(2000)])
    assert abs(w.mean() - 0.5) < 5 * 0.1 / math.sqrt(w.size)


def test_jit_normal_weight_pairs():
    # connections 2q and 2q + 1 are the two halves of one Box-Muller pair:
    # uncorrelated N(0, 1) values whose squares sum to a chi-square with two
    # degrees of freedom (the shared radius), and the pair's angle is uniform
    z = np.array([[O.jit_weight(6, O.W_NORMAL, 0.0, 1.0, j, 2, m)[1] for m in (2 * q, 2 * q + 1)]
                  for j in range(300) for q in range(10)])
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5 / math.sqrt(len(z))
    assert stats.kstest(z[:, 0] ** 2 + z[:, 1] ** 2, "chi2", args=(2,)).pvalue > 1e-3
    ang = np.arctan2(z[:, 1], z[:, 0]) / (2 * math.pi) % 1.0
    assert stats.kstest(ang, "uniform").pvalue > 1e-3
    # and the pair is built from the words 2q, 2q + 1 of the weight stream
    for j, b, q in [(0, 0, 0), (7, 3, 5), (123, 1, 17)]:
        u1 = ((O.hash_word(6, O.STREAM_W, j, b, 2 * q) >> 8) + 1) / 2.0 ** 24
        u2 = (O.hash_word(6, O.STREAM_W, j, b, 2 * q + 1) >> 8) / 2.0 ** 24
        z0 = O.jit_weight(6, O.W_NORMAL, 0.0, 1.0, j, b, 2 * q)[1]
        z1 = O.jit_weight(6, O.W_NORMAL, 0.0, 1.0, j, b, 2 * q + 1)[1]
        assert z0 ** 2 + z1 ** 2 == pytest.approx(-2.0 * math.log(u1), rel=1e-12)
        assert math.atan2(z1, z0) / (2 * math.pi) % 1.0 == pytest.approx(u2, abs=1e-12)


def test_jit_uniform_weights_are_uniform():
    u = np.array([O.jit_weight(4, O.W_UNIFORM, 0.0, 1.0, j, 1, m)[0] for j in range(400) for m in range(50)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert u.min() >= 0.0 and u.max() < 1.0


# ----------------------------------------------------------------- reverse mode
def test_event_csr_vjp_exact_differences():
    # The operator is linear, so switching one row on changes L = dy . y by
    # exactly d_ev[j]; moving one weight by h changes L by h e_j dy_k; moving
    # w by h changes L by h d_w.
    rng = np.random.default_rng(12)
    n_pre, n_post = 60, 45
    ip, ix = _random_csr(rng, n_pre, n_post, 0.2)
    data = (rng.integers(-8, 8, ix.size) / 4).astype(np.float32)  # dyadic: exact sums
    dy = (rng.integers(-8, 8, n_post) / 8).astype(np.float64)
    e = S.events(n_pre, 0.4, 3)
    d_ev, d_data, _ = O.event_csr_vjp(ip, ix, data, 0.0, n_post, e, dy)

    def L(ev, dat, w=0.0):
        return float(dy @ O.event_csr_matvec(ip, ix, dat, w, n_post, ev))

    for j in range(n_pre):
        on, off = e.copy(), e.copy()
        on[j], off[j] = 1, 0
        assert L(on, data) - L(off, data) == d_ev[j]
    for idx in rng.choice(ix.size, 40, replace=False):
        d2 = data.copy()
        d2[idx] += np.float32(0.5)
        assert (L(e, d2) - L(e, data)) / 0.5 == d_data[idx]
    _, _, d_w = O.event_csr_vjp(ip, ix, None, 0.25, n_post, e, dy)
    assert (L(e, None, 0.75) - L(e, None, 0.25)) / 0.5 == pytest.approx(d_w, abs=1e-12)


@pytest.mark.parametrize("wkind,w0,w1", [(O.W_HOMO, 0.6, 0.0), (O.W_NORMAL, 0.5, 0.1), (O.W_UNIFORM, -0.5, 1.5)])
def test_jit_vjp_differences(wkind, w0, w1):
    seed, K, B, n_pre, n_post = 21, 9, 32, 50, 70
    e = S.events(n_pre, 0.4, 2)
    dy = S.cotangent(n_post, 1)
    d_ev, g0, g1 = O.jit_vjp(seed, K, B, wkind, w0, w1, n_post, e, dy)

    def L(ev, a, b):
        return float(dy @ O.jit_matvec(seed, K, B, wkind, a, b, n_post, ev))

    for j in range(n_pre):
        on, off = e.copy(), e.copy()
        on[j], off[j] = 1, 0
        assert L(on, w0, w1) - L(off, w0, w1) == pytest.approx(d_ev[j], abs=1e-10)
    h = 1e-3
    assert (L(e, w0 + h, w1) - L(e, w0 - h, w1)) / (2 * h) == pytest.approx(g0, rel=1e-7, abs=1e-9)
    if wkind != O.W_HOMO:
        assert (L(e, w0, w1 + h) - L(e, w0, w1 - h)) / (2 * h) == pytest.approx(g1, rel=1e-7, abs=1e-9)
