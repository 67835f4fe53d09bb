"""GPU parity of the exact-statistics connectivity rules (geometric gaps,
exactly fixed out-degree) against the oracle, through the C ABI: the seeded
CSR build and the homogeneous products bit-exact (the FP32 logarithm decides
the same integer gaps on both sides), weighted products within 1e-5 of the
sum of |terms|, the reverse mode, and network rasters bit-identical to the
oracle's FP32 recursion run on the rule's matrix (one and many workgroups,
stored and regenerated connectivity, the 400k net with exactly 80 targets
per neuron)."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

dev = "cuda"
GEO, FD = O.RULE_GEOMETRIC, O.RULE_FIXED_DEGREE


@pytest.fixture(scope="module")
def bp():
    import paper_2311_05106_amd as m
    assert torch.cuda.is_available()
    return m


def _conn(bp, n_pre, n_post, rule, p, degree, B, seed, **kw):
    return bp.JitConn(n_pre, n_post, p=p, block=B, seed=seed, rule=rule, degree=degree, **kw)


CASES = [  # rule, n_pre, n_post, p, degree, block
    (GEO, 3000, 20000, 0.01, 0, 0),
    (GEO, 3000, 20000, 0.01, 0, 1024),
    (GEO, 2000, 5000, 0.2, 0, 0),
    (GEO, 500, 40000, 2e-4, 0, 3125),
    (FD, 3000, 20000, 0.0, 200, 0),
    (FD, 2000, 5000, 0.0, 80, 0),
    (FD, 300, 700, 0.0, 700, 0),   # every column
    (FD, 100, 3, 0.0, 5, 0),       # degree above n_post
]


@pytest.mark.parametrize("rule,n_pre,n_post,p,degree,B", CASES)
def test_rule_csr_build_bitwise(bp, rule, n_pre, n_post, p, degree, B):
    inv = O.geo_inv_rate(p) if rule == GEO else 0.0
    assert rule != GEO or bp.geo_inv_rate(p) == inv
    ip_r, ix_r = O.rule_csr_sorted(7, rule, 0, inv, degree, n_pre, n_post, B)
    ip, ix = bp.csr_build(_conn(bp, n_pre, n_post, rule, p, degree, B, 7))
    np.testing.assert_array_equal(ip.cpu().numpy(), ip_r)
    np.testing.assert_array_equal(ix.cpu().numpy(), ix_r)


@pytest.mark.parametrize("rule,n_pre,n_post,p,degree,B", CASES)
def test_rule_jit_products(bp, rule, n_pre, n_post, p, degree, B):
    inv = O.geo_inv_rate(p) if rule == GEO else 0.0
    seed = 11
    ip, ix, blk, idx = O.rule_csr(seed, rule, 0, inv, degree, n_pre, n_post, B)
    e = S.events(n_pre, 0.1, 3)
    # homogeneous: exact integer counts
    cnt = O.rule_matvec(ip, ix, None, n_post, e)
    y = bp.jit_conn_matvec(_conn(bp, n_pre, n_post, rule, p, degree, B, seed, w0=0.6), torch.from_numpy(e).to(dev))
    np.testing.assert_array_equal(y.cpu().numpy(), cnt.astype(np.float32) * np.float32(0.6))
    # normal weights N(0.5, 0.1): 1e-5 of the sum of |w0| + |w1 z| over the terms
    w = O.rule_weights(seed, O.W_NORMAL, float(np.float32(0.5)), float(np.float32(0.1)), ip, blk, idx)
    z = O.rule_weights(seed, O.W_NORMAL, 0.0, 1.0, ip, blk, idx)
    terms = np.float32(0.5) + np.abs(np.float32(0.1) * z)
    cw = _conn(bp, n_pre, n_post, rule, p, degree, B, seed, wkind=O.W_NORMAL, w0=0.5, w1=0.1)
    yw = bp.jit_conn_matvec(cw, torch.from_numpy(e).to(dev)).cpu().numpy()
    ref, scale = O.rule_matvec(ip, ix, w, n_post, e), O.rule_matvec(ip, ix, terms, n_post, e)
    assert np.all(np.abs(yw - ref) <= 1e-5 * scale + 1e-30) and np.all(yw[scale == 0] == 0)
    # dense float vector
    v = S.dense_vector(n_pre, 4, zero_frac=0.5)
    yd = bp.jit_conn_matvec_dense(cw, torch.from_numpy(v).to(dev)).cpu().numpy()
    vd = v.astype(np.float64)
    ref, scale = O.rule_matvec(ip, ix, w, n_post, vd), O.rule_matvec(ip, ix, terms, n_post, np.abs(vd))
    assert np.all(np.abs(yd - ref) <= 1e-5 * scale + 1e-30)
    # a batch of five spike vectors
    E = np.stack([S.events(n_pre, f, 30 + i) for i, f in enumerate((0.05, 0.0, 0.3, 1.0, 0.01))])
    Y = bp.jit_conn_matmat(_conn(bp, n_pre, n_post, rule, p, degree, B, seed, w0=0.6),
                           torch.from_numpy(E).to(dev)).cpu().numpy()
    for b in range(E.shape[0]):
        np.testing.assert_array_equal(Y[b], O.rule_matvec(ip, ix, None, n_post, E[b]).astype(np.float32)
                                      * np.float32(0.6))
    # reverse mode: d_events[j] = sum over row j of w_jk dy[k]
    dy = S.dense_vector(n_post, 9)
    d_ev, _ = bp.jit_conn_backward(cw, torch.from_numpy(e).to(dev), torch.from_numpy(dy).to(dev), want_w=False)
    rows = np.repeat(np.arange(n_pre), np.diff(ip))
    ref = np.bincount(rows, weights=w * dy[ix].astype(np.float64), minlength=n_pre)
    sc = np.bincount(rows, weights=terms * np.abs(dy[ix].astype(np.float64)), minlength=n_pre)
    assert np.all(np.abs(d_ev.cpu().numpy() - ref) <= 1e-5 * sc + 1e-30)


def test_rule_argument_errors(bp):
    import ctypes as C
    from paper_2311_05106_amd import _abi
    L = _abi.lib()
    c = _conn(bp, 10, 10, FD, 0.0, 5, 4, 0).c  # fixed degree with post blocks
    assert L.bp_csr_count(C.byref(c), C.c_void_p(0x1000), None) == _abi.BP_EINVAL
    c = _conn(bp, 10, 10, GEO, 0.1, 0, 0, 0).c
    c.rule = 7
    assert L.bp_csr_count(C.byref(c), C.c_void_p(0x1000), None) == _abi.BP_EINVAL


COBA = dict(w_exc=0.6, w_inh=6.7, tau_m=20.0, tau_e=5.0, tau_i=10.0, tau_ref=5.0, v_rest=-60.0, v_th=-50.0,
            v_reset=-60.0, e_exc=0.0, e_inh=-80.0, r=1.0, i_ext=20.0, dt=0.1, v0_lo=-60.0, v0_hi=-50.0)


@pytest.mark.parametrize("rule,conn,n,p,degree,block,max_wgs,T", [
    (FD, O.CONN_CSR, 4000, 0.0, 80, 0, 0, 400),        # one workgroup, stored rows
    (FD, O.CONN_JIT, 4000, 0.0, 80, 0, 0, 400),        # one workgroup, regenerated
    (FD, O.CONN_JIT, 40000, 0.0, 80, 0, 10, 300),      # targets pushed by the writers
    (FD, O.CONN_JIT, 20000, 0.0, 400, 0, 8, 200),      # lines overflow: readers regenerate
    (GEO, O.CONN_JIT, 40000, 80 / 40000, 0, 0, 10, 300),
    (GEO, O.CONN_JIT, 20000, 80 / 20000, 0, 1024, 16, 300),  # spike ids, blocks regenerated
    (GEO, O.CONN_CSR, 20000, 80 / 20000, 0, 1024, 16, 300),
])
def test_rule_net_raster_bitwise(bp, rule, conn, n, p, degree, block, max_wgs, T):
    n_exc = int(0.8 * n)
    inv = O.geo_inv_rate(p) if rule == GEO else 0.0
    ip, ix = O.rule_csr_sorted(3, rule, 0, inv, degree, n, n, block)
    P = O.net_params(model=0, n=n, n_exc=n_exc, conn=O.CONN_CSR, max_gap=1, block=block, seed=3, **COBA)
    d = bp.net_desc(n, n_exc=n_exc, p=p if p > 0 else None, K=1, conn=conn, block=block, seed=3, max_wgs=max_wgs,
                    rule=rule, degree=degree, inv_rate=inv if rule == GEO else None, **COBA)
    net = bp.Net(d)
    if max_wgs:
        assert net.info().n_wg > 1
    st = O.NetState(P)
    r_ref, c_ref, ev_ref = O.net_run(P, st, T, ip, ix)
    r, c = net.run(T, raster=True)
    r, c = r.cpu().numpy(), c.cpu().numpy()
    diff = np.flatnonzero((r != r_ref).any(axis=1))
    assert diff.size == 0, f"first differing step {diff[0]}"
    np.testing.assert_array_equal(c, c_ref)
    assert int(net.events().item()) == ev_ref
    assert net.error_flag() == 0 and c_ref.sum() > 0
    net.close()


def test_fixed_degree_400k_net_first_steps(bp):
    # the 400k COBA net with exactly 80 targets per neuron (3.2e7 synapses),
    # regenerated every step and pushed by the writers: 40 steps bit-identical
    n = 400_000
    ip, ix = O.rule_csr_sorted(0, FD, 0, 0.0, 80, n, n, 0)
    assert ix.size == 80 * n
    P = O.net_params(model=0, n=n, n_exc=int(0.8 * n), conn=O.CONN_CSR, max_gap=1, block=0, seed=0, **COBA)
    d = bp.net_desc(n, n_exc=int(0.8 * n), K=1, conn=bp.CONN_JIT, block=0, seed=0, rule=FD, degree=80, **COBA)
    net = bp.Net(d)
    st = O.NetState(P)
    r_ref, c_ref, ev_ref = O.net_run(P, st, 40, ip, ix, want_raster=True)
    r, c = net.run(40, raster=True)
    np.testing.assert_array_equal(c.cpu().numpy(), c_ref)
    assert np.array_equal(r.cpu().numpy(), r_ref)
    assert int(net.events().item()) == ev_ref == 80 * int(c_ref[:-1].sum())
    net.close()
