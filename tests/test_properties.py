"""Property-based tests (hypothesis, CPU only) of the oracle's definitions and
of the host-side scheduler: every generated case must satisfy what the paper
and the mathematics fix, on shapes and seeds hypothesis chooses.

* Event CSR product (Appendix B): equals the dense product D^T e for random
  small matrices with duplicated, unsorted columns and random spike bytes.
* Connectivity rows (Appendix C and the exact-statistics rules): positions in
  range, strictly increasing within a row for the gap rules, each block's
  positions inside the block; exactly min(k, n) distinct targets for the
  fixed degree; the keyed permutation is a bijection for any key and size.
* The FP32 logarithm is monotone and the geometric gap never increases with
  the uniform draw; the uniform gap lies in [1, K].
* Serving admission never exceeds either budget, admits in arrival order and
  retires every request after exactly its steps."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle as O
from paper_2311_05106_amd.serving import Scheduler

SET = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@SET
@given(n_pre=st.integers(1, 12), n_post=st.integers(1, 15), seed=st.integers(0, 2**32 - 1),
       dens=st.floats(0.0, 1.0), frac=st.floats(0.0, 1.0), hetero=st.booleans())
def test_event_csr_equals_dense_product(n_pre, n_post, seed, dens, frac, hetero):
    rng = np.random.default_rng(seed)
    lens = rng.binomial(n_post, dens, n_pre)
    ip = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ix = rng.integers(0, n_post, ip[-1]).astype(np.int32)      # duplicates, any order
    data = rng.standard_normal(ip[-1]).astype(np.float32) if hetero else None
    e = (rng.random(n_pre) < frac).astype(np.uint8) * rng.integers(1, 256, n_pre).astype(np.uint8)
    D = np.zeros((n_pre, n_post))
    for j in range(n_pre):
        for k in range(ip[j], ip[j + 1]):
            D[j, ix[k]] += float(data[k]) if hetero else 0.7
    y = O.event_csr_matvec(ip, ix, data, 0.7, n_post, e)
    np.testing.assert_allclose(y, D.T @ (e != 0), rtol=0, atol=1e-12)


@SET
@given(seed=st.integers(0, 2**64 - 1), p=st.floats(1e-4, 1.0), n_post=st.integers(1, 3000),
       B=st.sampled_from([0, 1, 7, 64, 1000]), j=st.integers(0, 2**31 - 1), rule=st.sampled_from([0, 1]))
def test_gap_rule_rows_are_increasing_and_in_block(seed, p, n_post, B, j, rule):
    K = O.max_gap(p)
    inv = O.geo_inv_rate(min(p, 1 - 1e-9))
    nb = -(-n_post // B) if B else 1
    for b in range(min(nb, 4)):
        r = O.rule_row_block(seed, rule, K, inv, 0, n_post, B, j, b)
        lo, hi = (b * B, min((b + 1) * B, n_post)) if B else (0, n_post)
        assert np.all(r >= lo) and np.all(r < hi)
        assert np.all(np.diff(r) > 0)
        if rule == 0:
            np.testing.assert_array_equal(r, O.row_block(seed, K, n_post, B, j, b))


@SET
@given(seed=st.integers(0, 2**64 - 1), n_post=st.integers(1, 5000), k=st.integers(0, 300),
       j=st.integers(0, 2**31 - 1))
def test_fixed_degree_rows_have_exactly_k_distinct_targets(seed, n_post, k, j):
    r = O.rule_row_block(seed, O.RULE_FIXED_DEGREE, 0, 0.0, k, n_post, 0, j, 0)
    assert r.size == min(k, n_post)
    assert np.unique(r).size == r.size
    assert np.all((r >= 0) & (r < n_post))


@SET
@given(key=st.lists(st.integers(0, 2**32 - 1), min_size=4, max_size=4), n=st.integers(1, 3000))
def test_keyed_permutation_is_a_bijection(key, n):
    kk = np.array(key, np.uint32)
    t = np.array([O.fd_target(kk, n, i) for i in range(n)])
    assert np.array_equal(np.sort(t), np.arange(n))


@SET
@given(ks=st.lists(st.integers(1, 2**24), min_size=2, max_size=50), p=st.floats(1e-5, 0.99))
def test_logarithm_monotone_and_geometric_gap_non_increasing(ks, p):
    k = np.sort(np.array(ks, np.uint32))
    ln = O.ln_f32(k)
    assert np.all(np.diff(ln) >= 0) and np.all(ln <= 0)
    words = ((k.astype(np.uint64) - 1) << 8).astype(np.uint32)  # draws whose top 24 bits are k - 1
    g = O.geo_gaps(words, O.geo_inv_rate(p)).astype(np.int64)
    assert np.all(g >= 1) and np.all(np.diff(g) <= 0)


@SET
@given(p=st.floats(1e-6, 1.0), words=st.lists(st.integers(0, 2**32 - 1), min_size=1, max_size=20))
def test_uniform_gap_range_and_k(p, words):
    K = O.max_gap(p)
    assert K >= 1
    # first positions of rows use draw 0 below K; every gap is 1 + below(K)
    for w in words:
        g = 1 + ((w * K) >> 32)
        assert 1 <= g <= K


@SET
@given(reqs=st.lists(st.tuples(st.integers(1, 120), st.integers(1, 12), st.integers(1, 3000)), min_size=1,
                     max_size=25),
       hbm=st.integers(50, 300), wgs=st.integers(4, 24), quantum=st.integers(1, 1000))
def test_scheduler_budgets_order_and_retirement(reqs, hbm, wgs, quantum):
    s = Scheduler(hbm_budget=hbm, wg_budget=wgs, max_nets=8)
    accepted = []
    for i, (b, w, steps) in enumerate(reqs):
        r = dict(id=i, bytes=b, wgs=w, steps=steps)
        if s.submit(r):
            accepted.append(r)
        else:
            assert b > hbm or w > wgs
    admitted_order, finished = [], []
    for _ in range(10000):
        for r in s.admit():
            admitted_order.append(r["id"])
        assert s.hbm_used <= hbm and s.wg_used <= wgs and len(s.active) <= 8
        if not s.active:
            break
        plan = s.plan(quantum)
        assert all(0 < k <= quantum for _, k in plan)
        finished += s.advance(plan)
    assert admitted_order == [r["id"] for r in accepted]          # arrival order
    assert sorted(r["id"] for r in finished) == [r["id"] for r in accepted]
    assert all(r["done"] == r["steps"] for r in finished)
    assert s.hbm_used == 0 and s.wg_used == 0
