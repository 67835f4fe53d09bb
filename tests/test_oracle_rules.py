"""Pins for the oracle's exact-statistics connectivity rules (CPU only).

Geometric gaps (Appendix C's exact Bernoulli process: the distance to the next
connection is Geo[p], gap = 1 + floor(log U / log(1 - p))): the FP32 logarithm
against numpy's FP64 log over every one of its 2^24 inputs, the gap law, the
per-position Bernoulli law and independence, row lengths Binomial(n, p), with
and without block restarts.  Exactly fixed out-degree k: every row has k
distinct targets, the keyed permutation is a bijection, in-degrees follow
Binomial(n_pre, k/n_post), target positions are uniform.  The products over a
rule's matrix: dense brute force."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
import synthetic as S


def _chi2_pvalue(obs, exp, min_exp=5.0):
    # pool the cells whose expectation is small into one
    obs = np.asarray(obs, np.float64)
    exp = np.asarray(exp, np.float64)
    keep = exp >= min_exp
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    return stats.chisquare(o, e * o.sum() / e.sum()).pvalue


def test_ln_f32_against_fp64_log_on_every_input():
    k = np.arange(1, (1 << 24) + 1, dtype=np.uint32)
    got = O.ln_f32(k).astype(np.float64)
    ref = np.log(k.astype(np.float64) / 2.0**24)
    err = np.abs(got - ref)
    # a few units in the last place of FP32 (relative 2^-24 = 6e-8)
    assert np.all(err <= 2.5e-7 * np.abs(ref) + 1e-12)
    assert got[-1] == 0.0 and got[0] < -16.6


@pytest.mark.parametrize("p", [0.5, 0.1, 0.01, 2e-4])
def test_geometric_gap_law(p):
    inv = O.geo_inv_rate(p)
    assert abs(inv - 1.0 / -math.log1p(-p)) <= 1e-7 * inv
    rng = np.random.default_rng(11)
    w = rng.integers(0, 2**32, 1 << 20, dtype=np.uint64).astype(np.uint32)
    g = O.geo_gaps(w, inv).astype(np.int64)
    assert g.min() >= 1
    # the inverse-CDF definition in FP64 gives the same gap except where the
    # quotient is within FP32 rounding (a few units of 2^-24 relative) of an
    # integer: a fraction of the draws of order 1e-6 times the mean gap
    u = ((w >> 8).astype(np.float64) + 1.0) / 2.0**24
    g64 = 1 + np.floor(np.log(u) / np.log1p(-p)).astype(np.int64)
    assert np.all(np.abs(g - g64) <= 1) and np.mean(g != g64) <= max(1e-4, 1e-6 / p)
    # P(G = g) = (1 - p)^(g - 1) p
    n = g.size
    mean, var = 1.0 / p, (1.0 - p) / p**2
    assert abs(g.mean() - mean) < 5 * math.sqrt(var / n)
    gmax = int(min(g.max(), 30 / p))
    cells = np.arange(1, gmax + 1)
    if gmax > 2000:  # bin long gaps by quantiles of the geometric law
        edges = np.unique(np.floor(stats.geom.ppf(np.linspace(0, 1, 201)[1:-1], p)).astype(np.int64))
        obs = np.histogram(g, bins=np.concatenate([[0], edges, [np.inf]]))[0]
        cdf = stats.geom.cdf(np.concatenate([[0], edges, [np.inf]]), p)
        exp = np.diff(cdf) * n
    else:
        obs = np.bincount(g, minlength=gmax + 2)[1:gmax + 1]
        exp = stats.geom.pmf(cells, p) * n
    assert _chi2_pvalue(obs, exp) > 1e-4


def test_geometric_rows_are_bernoulli_per_position():
    # n_pre rows of 60 positions: each position connected with probability p,
    # independently of its neighbour; row lengths Binomial(60, p); the same
    # with post blocks of 16 (memoryless restarts)
    p, n_pre, n_post = 0.1, 20000, 60
    inv = O.geo_inv_rate(p)
    for B in (0, 16):
        ip, ix, _, _ = O.rule_csr(5, O.RULE_GEOMETRIC, 0, inv, 0, n_pre, n_post, B)
        M = np.zeros((n_pre, n_post), np.int8)
        M[np.repeat(np.arange(n_pre), np.diff(ip)), ix] = 1
        assert M.sum() == ix.size  # no duplicates
        col = M.sum(0)
        assert _chi2_pvalue(col, np.full(n_post, n_pre * p)) > 1e-4
        assert np.all(np.abs(col - n_pre * p) < 5 * math.sqrt(n_pre * p * (1 - p)))
        both = (M[:, :-1] & M[:, 1:]).sum()
        exp_both = n_pre * (n_post - 1) * p * p
        assert abs(both - exp_both) < 5 * math.sqrt(exp_both)
        rl = np.diff(ip)
        obs = np.bincount(rl, minlength=n_post + 1)
        assert _chi2_pvalue(obs, stats.binom.pmf(np.arange(n_post + 1), n_post, p) * n_pre) > 1e-4


def test_geometric_first_target_is_memoryless():
    # the first target of a block sits gap - 1 after the block start
    p, inv = 0.05, O.geo_inv_rate(0.05)
    first = np.array([O.rule_row_block(3, O.RULE_GEOMETRIC, 0, inv, 0, 400, 100, j, 2)[:1] for j in range(4000)],
                     dtype=object)
    f = np.array([x[0] - 200 if len(x) else 100 for x in first])
    obs = np.bincount(np.minimum(f, 100), minlength=101)
    exp = np.append(stats.geom.pmf(np.arange(1, 101), p), stats.geom.sf(100, p)) * f.size
    assert _chi2_pvalue(obs, exp) > 1e-4
    # p near 1: every position connected
    assert np.array_equal(O.rule_row_block(3, O.RULE_GEOMETRIC, 0, O.geo_inv_rate(1 - 1e-12), 0, 50, 0, 7, 0),
                          np.arange(50))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 65, 1000, 4097])
def test_fixed_degree_permutation_is_a_bijection(n):
    key = np.array([0x12345678, 0x9ABCDEF0, 0x0F1E2D3C, 0x4B5A6978], np.uint32)
    t = np.array([O.fd_target(key, n, i) for i in range(n)])
    assert np.array_equal(np.sort(t), np.arange(n))


def test_fixed_degree_rows():
    n_pre, n_post, k = 20000, 500, 20
    ip, ix, blk, idx = O.rule_csr(9, O.RULE_FIXED_DEGREE, 0, 0.0, k, n_pre, n_post, 0)
    assert np.all(np.diff(ip) == k)
    rows = ix.reshape(n_pre, k)
    assert rows.min() >= 0 and rows.max() < n_post
    assert all(np.unique(r).size == k for r in rows[:2000])
    assert np.all(idx.reshape(n_pre, k) == np.arange(k)) and np.all(blk == 0)
    # in-degrees: Binomial(n_pre, k / n_post) for uniform k-subsets
    indeg = np.bincount(ix, minlength=n_post)
    q = k / n_post
    lo, hi = int(n_pre * q - 6 * math.sqrt(n_pre * q)), int(n_pre * q + 6 * math.sqrt(n_pre * q))
    obs = np.histogram(indeg, bins=np.arange(lo, hi + 2))[0]
    exp = stats.binom.pmf(np.arange(lo, hi + 1), n_pre, q) * n_post
    assert _chi2_pvalue(obs, exp, min_exp=3.0) > 1e-4
    # the target of each index is uniform over the columns
    for i in (0, k - 1):
        assert _chi2_pvalue(np.bincount(rows[:, i], minlength=n_post), np.full(n_post, n_pre / n_post)) > 1e-4
    # co-occurrence of columns 0 and 1: k (k - 1) / (n (n - 1)) per row
    both = np.sum(np.any(rows == 0, 1) & np.any(rows == 1, 1))
    exp_both = n_pre * k * (k - 1) / (n_post * (n_post - 1))
    assert abs(both - exp_both) < 5 * math.sqrt(exp_both) + 1
    # k >= n_post: every column
    ipd, ixd, _, _ = O.rule_csr(9, O.RULE_FIXED_DEGREE, 0, 0.0, 80, 10, 30, 0)
    assert np.all(np.diff(ipd) == 30)
    assert all(np.array_equal(np.sort(ixd[ipd[j]:ipd[j + 1]]), np.arange(30)) for j in range(10))


def test_rule_zero_is_the_paper_sampler():
    for B in (0, 64):
        for j in range(50):
            np.testing.assert_array_equal(O.rule_row_block(4, 0, 19, 0.0, 0, 700, B, j, 1 if B else 0),
                                          O.row_block(4, 19, 700, B, j, 1 if B else 0))


@pytest.mark.parametrize("rule", [O.RULE_GEOMETRIC, O.RULE_FIXED_DEGREE])
def test_rule_products_bruteforce(rule):
    seed, n_pre, n_post = 12, 40, 70
    B = 16 if rule == O.RULE_GEOMETRIC else 0
    inv, deg = O.geo_inv_rate(0.15), 9
    ip, ix, blk, idx = O.rule_csr(seed, rule, 0, inv, deg, n_pre, n_post, B)
    for wkind, w0, w1 in ((O.W_HOMO, 0.6, 0.0), (O.W_NORMAL, 0.5, 0.1), (O.W_UNIFORM, -1.0, 2.0)):
        D = np.zeros((n_pre, n_post))
        nb = -(-n_post // B) if B else 1
        for j in range(n_pre):
            for b in range(nb):
                for m, k in enumerate(O.rule_row_block(seed, rule, 0, inv, deg, n_post, B, j, b)):
                    D[j, k] += O.jit_weight(seed, wkind, w0, w1, j, b, m)[0]
        w = O.rule_weights(seed, wkind, w0, w1, ip, blk, idx)
        e = S.events(n_pre, 0.4, 2)
        np.testing.assert_allclose(O.rule_matvec(ip, ix, w, n_post, e), D.T @ (e != 0), rtol=1e-12, atol=1e-12)
        v = S.dense_vector(n_pre, 5, zero_frac=0.3).astype(np.float64)
        np.testing.assert_allclose(O.rule_matvec(ip, ix, w, n_post, v), D.T @ v, rtol=1e-12, atol=1e-12)
    ips, ixs = O.rule_csr_sorted(seed, rule, 0, inv, deg, n_pre, n_post, B)
    assert all(np.all(np.diff(ixs[ips[j]:ips[j + 1]]) > 0) for j in range(n_pre))
    np.testing.assert_array_equal(O.event_csr_counts(ips, ixs, n_post, e),
                                  O.rule_matvec(ip, ix, None, n_post, e).astype(np.int64))
