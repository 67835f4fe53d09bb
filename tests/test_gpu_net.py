"""GPU parity of the E/I LIF network against the oracle's FP32 recursion:
spike rasters bit-identical (the threshold decision is taken in FP32 on both
sides, integer synaptic counts), for stored and regenerated connectivity,
one and many workgroups, COBA and CUBA; resume, checkpoint round trip,
external current, event counts and batched runs."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

COBA_PARAMS = dict(w_exc=0.6, w_inh=6.7, tau_m=20.0, tau_e=5.0, tau_i=10.0, tau_ref=5.0, v_rest=-60.0,
                   v_th=-50.0, v_reset=-60.0, e_exc=0.0, e_inh=-80.0, r=1.0, i_ext=20.0, dt=0.1,
                   v0_lo=-60.0, v0_hi=-50.0)
CUBA_PARAMS = dict(COBA_PARAMS, v_rest=-49.0, w_exc=1.62, w_inh=-9.0, i_ext=0.0)


@pytest.fixture(scope="module")
def bp():
    import paper_2311_05106_amd as m
    assert torch.cuda.is_available()
    return m


def make(bp, n, p, conn, block=0, seed=0, model=0, max_wgs=0, **over):
    params = dict(CUBA_PARAMS if model == 1 else COBA_PARAMS)
    params.update(over)
    n_exc = int(0.8 * n)
    K = O.max_gap(p)
    P = O.net_params(model=model, n=n, n_exc=n_exc, conn=conn, max_gap=K, block=block, seed=seed, **params)
    d = bp.net_desc(n, n_exc=n_exc, K=K, conn=conn, block=block, seed=seed, model=model, max_wgs=max_wgs, **params)
    net = bp.Net(d)
    ip = ix = None
    if conn == O.CONN_CSR:
        ip, ix = O.csr_build(seed, K, n, n, block)
    return P, net, ip, ix


def run_both(bp, P, net, ip, ix, T, state=None):
    st = state if state is not None else O.NetState(P)
    r_ref, c_ref, ev_ref = O.net_run(P, st, T, ip, ix)
    r, c = net.run(T, raster=True)
    return st, r_ref, c_ref, ev_ref, r.cpu().numpy(), c.cpu().numpy()


def first_diff(a, b):
    d = np.flatnonzero((a != b).any(axis=1))
    return int(d[0]) if d.size else None


@pytest.mark.parametrize("conn,n,p,block,max_wgs,T", [
    (O.CONN_CSR, 4000, 0.02, 0, 0, 1000),      # the 4000-neuron E/I net, one workgroup
    (O.CONN_JIT, 4000, 0.02, 0, 0, 1000),
    (O.CONN_JIT, 20000, 80 / 20000, 1024, 16, 400),   # 16 workgroups, blocked rows
    (O.CONN_JIT, 20000, 80 / 20000, 0, 8, 300),       # 8 workgroups, whole rows
    (O.CONN_CSR, 20000, 80 / 20000, 1024, 16, 400),   # stored rows, block index
    (O.CONN_CSR, 12000, 80 / 12000, 0, 6, 300),       # stored rows, searched segments
    (O.CONN_JIT, 9000, 0.01, 700, 5, 300),            # range not a multiple of the block
    (O.CONN_JIT, 100000, 80 / 100000, 0, 25, 200),    # whole rows pushed as targets, lines mostly fit
    (O.CONN_JIT, 20000, 0.02, 0, 8, 200),             # 400 targets per row: lines overflow, regenerated
    (O.CONN_JIT, 20000, 80 / 20000, 2560, 8, 300),    # ranges of 2560: three neurons on some threads
    (O.CONN_JIT, 30000, 80 / 30000, 0, 8, 200),       # whole rows, ranges of 3750
])
def test_raster_bitwise(bp, conn, n, p, block, max_wgs, T):
    P, net, ip, ix = make(bp, n, p, conn, block, seed=1, max_wgs=max_wgs)
    info = net.info()
    if max_wgs:
        assert info.n_wg > 1
    st, r_ref, c_ref, ev_ref, r, c = run_both(bp, P, net, ip, ix, T)
    assert first_diff(r, r_ref) is None, f"first differing step {first_diff(r, r_ref)}"
    np.testing.assert_array_equal(c, c_ref)
    assert int(net.events().item()) == ev_ref
    assert net.error_flag() == 0
    s = net.get_state()
    np.testing.assert_array_equal(s["V"].cpu().numpy(), st.V)
    np.testing.assert_array_equal(s["ge"].cpu().numpy(), st.ge)
    np.testing.assert_array_equal(s["gi"].cpu().numpy(), st.gi)
    np.testing.assert_array_equal(s["ref"].cpu().numpy(), st.ref)
    np.testing.assert_array_equal(s["s_prev"].cpu().numpy(), st.s_prev)
    assert c_ref.sum() > 0


def test_c0_first_200_steps_match_fp64_and_rates(bp):
    # COBA 4000 (3200/800), p = 0.02, stored CSR, 1000 steps: identical raster
    # to the FP64 recursion for the first 200 steps, E and I rates within 2 %.
    P, net, ip, ix = make(bp, 4000, 0.02, O.CONN_CSR, 0, seed=0)
    st64 = O.NetState(P, 64)
    r64, _, _ = O.net_run(P, st64, 1000, ip, ix)
    r, _ = net.run(1000, raster=True)
    r = r.cpu().numpy()
    np.testing.assert_array_equal(r[:200], r64[:200])
    for sl in (slice(0, 3200), slice(3200, 4000)):
        assert abs(r[200:, sl].mean() - r64[200:, sl].mean()) <= 0.02 * r64[200:, sl].mean()


@pytest.mark.parametrize("model", [0, 1])
def test_cuba_and_coba_multi_wg(bp, model):
    P, net, ip, ix = make(bp, 15000, 80 / 15000, O.CONN_JIT, 1024, seed=4, model=model, max_wgs=12)
    _, r_ref, c_ref, _, r, c = run_both(bp, P, net, ip, ix, 250)
    assert first_diff(r, r_ref) is None
    assert c_ref.sum() > 0


@pytest.mark.parametrize("block", [1024, 0])
def test_resume_and_checkpoint_roundtrip(bp, block):
    P, net, ip, ix = make(bp, 20000, 80 / 20000, O.CONN_JIT, block, seed=2, max_wgs=16)
    st = O.NetState(P)
    rr1, _, _ = O.net_run(P, st, 150)
    r1, _ = net.run(150, raster=True)
    snap = net.get_state()
    raw = snap["raw"].clone()
    rr2, _, _ = O.net_run(P, st, 100)
    r2, _ = net.run(100, raster=True)
    np.testing.assert_array_equal(np.concatenate([r1.cpu().numpy(), r2.cpu().numpy()]), np.concatenate([rr1, rr2]))
    # restore the snapshot into a fresh net and replay the 100 steps
    P2, net2, _, _ = make(bp, 20000, 80 / 20000, O.CONN_JIT, block, seed=2, max_wgs=16)
    net2.set_state(raw, 150)
    r2b, _ = net2.run(100, raster=True)
    np.testing.assert_array_equal(r2b.cpu().numpy(), rr2)
    # and into the same net (rewind)
    net.set_state(raw, 150)
    r2c, _ = net.run(100, raster=True)
    np.testing.assert_array_equal(r2c.cpu().numpy(), rr2)


@pytest.mark.parametrize("block", [1024, 0])
@pytest.mark.parametrize("at", [15, 16, 17, 31])
def test_resume_at_tag_wrap_steps(bp, block, at):
    """Inbox words carry the step modulo 16: restoring at steps around a wrap
    of that tag (fresh net and rewind of a net that ran further) replays the
    oracle's raster exactly."""
    P, net, _, _ = make(bp, 20000, 80 / 20000, O.CONN_JIT, block, seed=5, max_wgs=16)
    st = O.NetState(P)
    O.net_run(P, st, at)
    net.run(at)
    raw = net.get_state()["raw"].clone()
    rr, _, _ = O.net_run(P, st, 40)
    r, _ = net.run(40, raster=True)
    np.testing.assert_array_equal(r.cpu().numpy(), rr)
    P2, net2, _, _ = make(bp, 20000, 80 / 20000, O.CONN_JIT, block, seed=5, max_wgs=16)
    net2.set_state(raw, at)
    r2, _ = net2.run(40, raster=True)
    np.testing.assert_array_equal(r2.cpu().numpy(), rr)
    net.run(7)  # the lines now hold later steps' tags
    net.set_state(raw, at)
    r3, _ = net.run(40, raster=True)
    np.testing.assert_array_equal(r3.cpu().numpy(), rr)


def test_step_api_with_external_current(bp):
    P, net, ip, ix = make(bp, 3000, 0.02, O.CONN_CSR, 0, seed=6, i_ext=0.0)
    st = O.NetState(P)
    rng = np.random.default_rng(3)
    for t in range(30):
        iv = rng.uniform(0, 40, 3000).astype(np.float32)
        rr, _, _ = O.net_run(P, st, 1, ip, ix, iext_vec=iv)
        s = net.step(torch.from_numpy(iv).cuda())
        np.testing.assert_array_equal(s.cpu().numpy(), rr[0])


def test_run_batch_equals_solo_runs(bp):
    cases = [(4000, 0.02, O.CONN_CSR, 0, 0, 0), (2500, 0.03, O.CONN_JIT, 0, 1, 0),
             (20000, 0.004, O.CONN_JIT, 1024, 0, 16), (12000, 80 / 12000, O.CONN_CSR, 1024, 1, 8),
             (1000, 0.08, O.CONN_CSR, 0, 0, 0), (30000, 80 / 30000, O.CONN_JIT, 0, 0, 12)]
    steps = [300, 120, 250, 200, 0, 180]
    nets, refs = [], []
    for i, (n, p, conn, blk, model, mw) in enumerate(cases):
        P, net, ip, ix = make(bp, n, p, conn, blk, seed=10 + i, model=model, max_wgs=mw)
        _, c_ref, ev = O.net_run(P, O.NetState(P), steps[i], ip, ix)
        nets.append(net)
        refs.append((c_ref, ev))
    counts = [torch.empty(max(s, 1), dtype=torch.int32, device="cuda") for s in steps]
    bp.run_batch(nets, steps, counts)
    for i, net in enumerate(nets):
        np.testing.assert_array_equal(counts[i][:steps[i]].cpu().numpy(), refs[i][0])
        assert int(net.events().item()) == refs[i][1]
        assert net.info().step == steps[i]


def test_run_batch_of_target_exchange_nets(bp):
    # a batch whose nets all push their spikes as targets (regenerated rows of
    # one post block on several workgroups): COBA and CUBA nets side by side
    # in one launch, each against the oracle
    cases = [(20000, 80 / 20000, 0, 8), (30000, 80 / 30000, 1, 12), (12000, 0.02, 0, 6)]
    steps = [260, 150, 200]
    nets, refs = [], []
    for i, (n, p, model, mw) in enumerate(cases):
        P, net, _, _ = make(bp, n, p, O.CONN_JIT, 0, seed=40 + i, model=model, max_wgs=mw)
        assert net.info().n_wg > 1
        _, c_ref, ev = O.net_run(P, O.NetState(P), steps[i], None, None)
        nets.append(net)
        refs.append((c_ref, ev))
    counts = [torch.empty(s, dtype=torch.int32, device="cuda") for s in steps]
    bp.run_batch(nets, steps, counts)
    for i, net in enumerate(nets):
        np.testing.assert_array_equal(counts[i].cpu().numpy(), refs[i][0])
        assert int(net.events().item()) == refs[i][1]


@pytest.mark.parametrize("block", [2560, 0])
def test_large_jit_net_first_steps(bp, block):
    # 400k neurons (320k E / 80k I), p = 80/N, post blocks of 2560 (spike ids
    # exchanged) or whole rows (targets exchanged): the first 40 steps
    # bit-identical to the oracle (full-size shape of the scaled net).
    n = 400_000
    P, net, _, _ = make(bp, n, 80 / n, O.CONN_JIT, block, seed=0)
    assert net.info().n_wg >= 128
    st = O.NetState(P)
    r_ref, c_ref, ev_ref = O.net_run(P, st, 40)
    r, c = net.run(40, raster=True)
    assert first_diff(r.cpu().numpy(), r_ref) is None
    assert int(net.events().item()) == ev_ref


def _raw_state(st):
    return np.concatenate([st.V.view(np.uint8), st.ge.view(np.uint8), st.gi.view(np.uint8),
                           st.ref.astype(np.int32).view(np.uint8), st.s_prev.astype(np.uint8)])


@pytest.mark.parametrize("block", [0, 2560])
def test_large_jit_net_steady_state(bp, block):
    # 400k neurons in the regime the benchmark times (after the initial
    # transient): the oracle's FP32 run of 1000 steps from the initial state
    # equals the GPU's run bit for bit (state at step 1000), and from the
    # oracle's state at step 1000 the net (given that state with
    # bp_set_state) and the oracle step 100 more steps with identical rasters,
    # event counts and final states.
    n = 400_000
    print(f"steady-state 400k net, block {block}", flush=True)
    P, net, _, _ = make(bp, n, 80 / n, O.CONN_JIT, block, seed=0)
    st = O.NetState(P)
    _, c_ref, _ = O.net_run(P, st, 1000, want_raster=False, parallel=True)
    _, c = net.run(1000, counts=True)
    np.testing.assert_array_equal(c.cpu().numpy(), c_ref)
    g = net.get_state()
    np.testing.assert_array_equal(g["raw"].cpu().numpy(), _raw_state(st))
    # steady state: well below the transient's rates, about 2 spikes per ms per 100 neurons
    assert 200 < c_ref[-100:].mean() < 2000
    P2, net2, _, _ = make(bp, n, 80 / n, O.CONN_JIT, block, seed=0)
    net2.set_state(torch.from_numpy(_raw_state(st)).cuda(), 1000)
    ev0 = int(net2.events().item())
    r_ref, c2_ref, ev_ref = O.net_run(P, st, 100, parallel=True)
    r, c2 = net2.run(100, raster=True)
    assert first_diff(r.cpu().numpy(), r_ref) is None
    np.testing.assert_array_equal(c2.cpu().numpy(), c2_ref)
    assert int(net2.events().item()) - ev0 == ev_ref
    np.testing.assert_array_equal(net2.get_state()["raw"].cpu().numpy(), _raw_state(st))
    assert net2.info().step == 1100
    net.close()
    net2.close()


def test_destroy_twice_is_rejected(bp):
    from paper_2311_05106_amd import _abi
    _, net, _, _ = make(bp, 2000, 0.02, O.CONN_JIT, 0, seed=1)
    h = net.h
    assert _abi.lib().bp_destroy_net(h) == _abi.BP_OK
    assert _abi.lib().bp_destroy_net(h) == _abi.BP_ESTATE
    assert _abi.lib().bp_run(h, 1, None, None, None, None) == _abi.BP_ESTATE
    net.h = None


def test_net_inputs_are_validated(bp):
    _, net, _, _ = make(bp, 2000, 0.02, O.CONN_JIT, 0, seed=1)
    with pytest.raises(ValueError):
        net.run(5, i_ext=torch.zeros(1999, device="cuda"))
    with pytest.raises(TypeError):
        net.run(5, i_ext=torch.zeros(2000))
    with pytest.raises(ValueError):
        net.set_state(torch.zeros(10, dtype=torch.uint8, device="cuda"), 0)
    with pytest.raises(TypeError):
        net.set_state(torch.zeros(2000 * 17, dtype=torch.uint8), 0)
    net.close()
