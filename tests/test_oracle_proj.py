"""Pins for the oracle's synaptic projections with multi-step delays (CPU
only): the AlignPre and AlignPost forms of the exponential synapse give the
same postsynaptic input (Appendix D: neither is an approximation; the map is
linear), a single delayed spike follows the closed form w d^(t - t0 - D)
(Appendix E), the saturating presynaptic trace follows its own closed form,
delays shift the whole trajectory, and the FP32 recursion stays within
rounding of FP64."""
import math

import numpy as np
import pytest

import oracle as O
import synthetic as S


def _csr(seed=3, n_pre=300, n_post=200, p=0.05, B=0):
    return O.csr_build(seed, O.max_gap(p), n_pre, n_post, B)


def _raster(T, n, frac, seed):
    return np.stack([S.events(n, frac, seed + t) for t in range(T)])


@pytest.mark.parametrize("delay", [0, 1, 7])
@pytest.mark.parametrize("hetero", [False, True])
def test_align_pre_equals_align_post_for_exponential_synapses(delay, hetero):
    ip, ix = _csr()
    data = S.hetero_data(ix.size, 2) if hetero else None
    R = _raster(60, 300, 0.05, 10)
    d = math.exp(-0.1 / 5.0)
    g_post, _ = O.proj_run(ip, ix, data, 0.6, 200, O.ALIGN_POST, O.SYN_EXP, d, 0.0, delay, R)
    g_pre, _ = O.proj_run(ip, ix, data, 0.6, 200, O.ALIGN_PRE, O.SYN_EXP, d, 0.0, delay, R)
    assert np.abs(g_post).max() > 0
    np.testing.assert_allclose(g_pre, g_post, rtol=1e-12, atol=1e-12)
    # and it equals the delayed spikes filtered by the exponential kernel,
    # summed through the matrix (a direct convolution)
    D = np.zeros((300, 200))
    for j in range(300):
        for e in range(ip[j], ip[j + 1]):
            D[j, ix[e]] += data[e] if hetero else 0.6
    conv = np.zeros((60, 200))
    for t in range(60):
        for t0 in range(0, t - delay + 1):
            conv[t] += d ** (t - delay - t0) * (R[t0] != 0) @ D
    np.testing.assert_allclose(g_post, conv, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("delay", [0, 3, 25])
def test_single_delayed_spike_closed_form(delay):
    ip, ix = _csr()
    T, j, t0 = 80, 17, 5
    R = np.zeros((T, 300), np.uint8)
    R[t0, j] = 1
    d = math.exp(-0.1 / 10.0)
    g, _ = O.proj_run(ip, ix, None, 6.7, 200, O.ALIGN_POST, O.SYN_EXP, d, 0.0, delay, R)
    col = np.zeros(200)
    col[ix[ip[j]:ip[j + 1]]] = 1.0
    for t in range(T):
        want = 6.7 * d ** (t - t0 - delay) * col if t >= t0 + delay else np.zeros(200)
        np.testing.assert_allclose(g[t], want, rtol=1e-12, atol=1e-300)
    # a delay past the end of the raster: nothing arrives
    g, _ = O.proj_run(ip, ix, None, 6.7, 200, O.ALIGN_POST, O.SYN_EXP, d, 0.0, T, R)
    assert np.all(g == 0)


def test_saturating_trace_closed_form():
    ip, ix = _csr()
    T, u, d = 40, 0.3, 0.9
    R = np.zeros((T, 300), np.uint8)
    R[[2, 5, 6], 11] = 1
    _, x = O.proj_run(ip, ix, None, 1.0, 200, O.ALIGN_PRE, O.SYN_SAT, d, u, 0, R)
    # by hand: x = u after step 2, then d^3 decay, saturating increments
    x2 = u
    x5 = x2 * d**3
    x5 = x5 + u * (1 - x5)
    x6 = x5 * d
    x6 = x6 + u * (1 - x6)
    assert abs(x[11] - x6 * d ** (T - 1 - 6)) < 1e-15
    assert np.all(x[np.arange(300) != 11] == 0)
    # never above one; the postsynaptic input is M^T x
    R = _raster(T, 300, 0.5, 3)
    g, x = O.proj_run(ip, ix, None, 0.5, 200, O.ALIGN_PRE, O.SYN_SAT, d, u, 0, R)
    assert x.max() < 1.0
    D = np.zeros((300, 200))
    for j in range(300):
        D[j, ix[ip[j]:ip[j + 1]]] += 0.5
    np.testing.assert_allclose(g[-1], x @ D, rtol=1e-12)


@pytest.mark.parametrize("delay", [2, 9])
def test_delay_shifts_the_trajectory(delay):
    ip, ix = _csr()
    R = _raster(50, 300, 0.1, 40)
    d = 0.95
    g0, _ = O.proj_run(ip, ix, None, 1.0, 200, O.ALIGN_POST, O.SYN_EXP, d, 0.0, 0, R)
    gd, _ = O.proj_run(ip, ix, None, 1.0, 200, O.ALIGN_POST, O.SYN_EXP, d, 0.0, delay, R)
    assert np.all(gd[:delay] == 0)
    np.testing.assert_array_equal(gd[delay:], g0[:50 - delay])


@pytest.mark.parametrize("align,syn", [(0, 0), (1, 0), (1, 1)])
def test_fp32_recursion_within_rounding(align, syn):
    ip, ix = _csr()
    R = _raster(200, 300, 0.05, 70)
    d = math.exp(-0.1 / 5.0)
    g64, s64 = O.proj_run(ip, ix, None, 0.6, 200, align, syn, d, 0.2, 4, R)
    g32, s32 = O.proj_run(ip, ix, None, 0.6, 200, align, syn, np.float32(d), np.float32(0.2), 4, R, precision=32)
    # the recursion is contracting (d < 1): errors stay a few units of FP32
    # rounding relative to the values
    np.testing.assert_allclose(g32, g64, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(s32, s64, rtol=2e-6, atol=1e-6)
