"""Pins for the oracle's E/I LIF network (CPU only): the closed-form LIF
response to a constant current (Euler recurrence), the exact exponential
synapse response to one spike (Appendix E), the CUBA variant's closed form,
invariants (resume = uninterrupted run, stored CSR = regenerated JIT), and
the FP32 recursion against the FP64 one."""
import math

import numpy as np
import pytest

import oracle as O

COBA_PARAMS = dict(w_exc=0.6, w_inh=6.7, tau_m=20.0, tau_e=5.0, tau_i=10.0, tau_ref=5.0, v_rest=-60.0,
                   v_th=-50.0, v_reset=-60.0, e_exc=0.0, e_inh=-80.0, r=1.0, i_ext=20.0, dt=0.1,
                   v0_lo=-60.0, v0_hi=-50.0)


def params(n, n_exc, p, conn=O.CONN_JIT, block=0, seed=0, model=O.COBA, **over):
    kw = dict(COBA_PARAMS)
    kw.update(over)
    return O.net_params(model=model, n=n, n_exc=n_exc, conn=conn, max_gap=O.max_gap(p), block=block, seed=seed,
                        **kw)


def lif_first_spike_steps(v0, v_inf, v_th, a):
    # V_n = V_inf + (V0 - V_inf)(1 - a)^n; first n with V_n > V_th
    return math.ceil(math.log((v_inf - v_th) / (v_inf - v0)) / math.log(1 - a))


@pytest.mark.parametrize("precision", [32, 64])
def test_lif_closed_form_constant_current(precision):
    P = params(1, 1, 1.0, w_exc=0.0, w_inh=0.0, v0_lo=-60.0, v0_hi=-60.0)
    st = O.NetState(P, precision)
    assert st.V[0] == -60.0
    raster, counts, _ = O.net_run(P, st, 1000)
    a = 0.1 / 20.0
    n1 = lif_first_spike_steps(-60.0, -40.0, -50.0, a)
    assert n1 == 139  # tau ln 2 / dt = 138.6 in continuous time
    spikes = np.flatnonzero(raster[:, 0])
    ref = O.net_ref_steps(P)
    assert ref == 50
    isi = n1 + ref  # 50 held steps after each spike, then 139 steps from V_reset
    assert isi == 189
    expect = np.arange(n1 - 1, 1000, isi)
    np.testing.assert_array_equal(spikes, expect)
    assert 1000.0 / (isi * 0.1) == pytest.approx(52.91, abs=0.01)


def test_lif_trajectory_fp64():
    P = params(1, 1, 1.0, w_exc=0.0, w_inh=0.0, v0_lo=-60.0, v0_hi=-60.0)
    st = O.NetState(P, 64)
    a = float(np.float32(0.1)) / 20.0  # parameters are FP32 values; dt = float32(0.1)
    for n in range(1, 120):
        O.net_run(P, st, 1)
        assert st.V[0] == pytest.approx(-40.0 + (-20.0) * (1 - a) ** n, rel=1e-13)


def test_cuba_closed_form():
    # CUBA: I = ge + gi + I_ext; with V_rest = -49 above threshold and no drive
    P = params(1, 1, 1.0, model=O.CUBA, w_exc=0.0, w_inh=0.0, v_rest=-49.0, i_ext=0.0,
               v0_lo=-60.0, v0_hi=-60.0)
    st = O.NetState(P, 64)
    raster, _, _ = O.net_run(P, st, 2000)
    n1 = lif_first_spike_steps(-60.0, -49.0, -50.0, 0.005)
    spikes = np.flatnonzero(raster[:, 0])
    np.testing.assert_array_equal(spikes[:3], np.array([n1 - 1, n1 - 1 + n1 + 50, n1 - 1 + 2 * (n1 + 50)]))


@pytest.mark.parametrize("precision", [32, 64])
def test_exponential_synapse_single_spike(precision):
    # Neuron 0 (excitatory) is driven over threshold once; p = 1 connects it to
    # both neurons.  With one-step delay, g_e after step t >= 1 is w d^(t-1),
    # d = exp(-dt/tau_e), the sampled solution of dg/dt = -g/tau + w delta(t).
    P = params(2, 1, 1.0, i_ext=0.0, v0_lo=-60.0, v0_hi=-60.0)
    st = O.NetState(P, precision)
    r0, _, _ = O.net_run(P, st, 1, iext_vec=np.array([1e4, 0.0]))
    assert r0[0].tolist() == [1, 0]
    g = []
    for t in range(1, 45):
        r, _, _ = O.net_run(P, st, 1)
        assert r.sum() == 0
        g.append(float(st.ge[1]))
    t = np.arange(1, 45)
    w, dt = float(np.float32(0.6)), float(np.float32(0.1))  # the parameters are FP32 values
    expect = w * np.exp(-(t - 1) * dt / 5.0)
    tol = 1e-12 if precision == 64 else 5e-6
    np.testing.assert_allclose(np.array(g), expect, rtol=tol)
    assert float(st.gi[1]) == 0.0


@pytest.mark.parametrize("conn,block", [(O.CONN_CSR, 0), (O.CONN_JIT, 0), (O.CONN_JIT, 512)])
def test_resume_equals_uninterrupted(conn, block):
    P = params(1500, 1200, 80 / 1500, conn=conn, block=block, seed=3)
    ip = ix = None
    if conn == O.CONN_CSR:
        ip, ix = O.csr_build(P.seed, P.max_gap, P.n, P.n, block)
    a = O.NetState(P)
    ra, ca, ea = O.net_run(P, a, 400, ip, ix)
    b = O.NetState(P)
    rb1, _, eb1 = O.net_run(P, b, 150, ip, ix)
    rb2, _, eb2 = O.net_run(P, b, 250, ip, ix)
    np.testing.assert_array_equal(ra, np.concatenate([rb1, rb2]))
    assert ea == eb1 + eb2
    for f in ("V", "ge", "gi", "ref", "s_prev"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert ca.sum() > 0


@pytest.mark.parametrize("block", [0, 700])
def test_stored_csr_equals_regenerated(block):
    Pj = params(2000, 1600, 0.02, conn=O.CONN_JIT, block=block, seed=9)
    Pc = params(2000, 1600, 0.02, conn=O.CONN_CSR, block=block, seed=9)
    ip, ix = O.csr_build(9, Pj.max_gap, 2000, 2000, block)
    rj, _, ej = O.net_run(Pj, O.NetState(Pj), 300)
    rc, _, ec = O.net_run(Pc, O.NetState(Pc), 300, ip, ix)
    np.testing.assert_array_equal(rj, rc)
    assert ej == ec


def test_c0_network_fp32_vs_fp64():
    # COBA 4000 (3200 E / 800 I), p = 0.02, 1000 steps.  The FP32 recursion
    # stays on the FP64 trajectory for at least the first 200 steps, and the
    # E and I population rates over steps 200-999 agree within 2 %.
    P = params(4000, 3200, 0.02, conn=O.CONN_CSR, seed=0)
    ip, ix = O.csr_build(0, P.max_gap, 4000, 4000, 0)
    r32, c32, _ = O.net_run(P, O.NetState(P, 32), 1000, ip, ix)
    r64, c64, _ = O.net_run(P, O.NetState(P, 64), 1000, ip, ix)
    np.testing.assert_array_equal(r32[:200], r64[:200])
    for sl in (slice(0, 3200), slice(3200, 4000)):
        f32 = r32[200:, sl].mean()
        f64 = r64[200:, sl].mean()
        assert abs(f32 - f64) <= 0.02 * f64
    rate = r32.mean() / 1e-4
    assert 1.0 < rate < 200.0  # Hz, an active asynchronous regime


@pytest.mark.parametrize("conn,block", [(0, 0), (1, 0), (1, 256)])
def test_openmp_build_is_identical(conn, block):
    # the CPU baseline runs the OpenMP build of the network loops; it must
    # give exactly the plain build's rasters, counts, events and state
    n, K = 3000, O.max_gap(0.05)
    P = O.net_params(model=0, n=n, n_exc=2400, conn=conn, max_gap=K, block=block, seed=3, **COBA_PARAMS)
    ip, ix = O.csr_build(3, K, n, n, block) if conn == 0 else (None, None)
    a, b = O.NetState(P), O.NetState(P)
    ra, ca, ea = O.net_run(P, a, 120, ip, ix)
    assert O.set_threads(4) >= 1
    rb, cb, eb = O.net_run(P, b, 120, ip, ix, parallel=True)
    assert ca.sum() > 0
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(ca, cb)
    assert ea == eb
    for f in ("V", "ge", "gi", "ref", "s_prev"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
