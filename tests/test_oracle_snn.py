"""Pins for the oracle's BPTT of the recurrent LIF network (CPU only).

* Smooth mode (the forward spike is S, the antiderivative of the surrogate):
  the reverse pass equals central finite differences of the loss, for the
  sigmoid surrogate (slope 4) and the ReLU surrogate of Appendix I
  (alpha 0.3, width 1.0), with the reset differentiated.
* Detached reset (the default of the training workload): the reverse pass
  equals central finite differences of the smooth forward in which every
  reset factor (1 - z_{t-1}) is frozen at the free run's value, a function
  whose exact gradient is the detached gradient.
* The surrogates' shapes: each integrates to the spike's full rise (1 for the
  sigmoid, alpha width^2 for the ReLU form), is even, peaks at threshold
  (slope / 4; alpha width), vanishes outside |x| < width (ReLU) and is linear
  on each side of the peak; S' equals the surrogate by finite differences.
* Hard spikes: teacher forcing with the network's own spikes reproduces the
  free run; the readout gradient has its softmax closed form."""
import math

import numpy as np
import pytest

import oracle as O
import synthetic as S


def tiny(seed=0, T=15, B=2, Cc=6, N=12, Ocls=3, p=0.3):
    K = O.max_gap(p)
    ip, ix = O.csr_build(seed, K, N, N, 0)
    rng = np.random.default_rng(seed)
    x = S.poisson_inputs(T, B, Cc, 20.0, seed, 50.0, 400.0)  # dense enough to drive a tiny net
    lab = S.labels(B, Ocls, seed)
    W_in = rng.standard_normal((Cc, N)) * 1.5
    w_rec = rng.standard_normal(ix.size) * 0.5
    W_out = rng.standard_normal((N, Ocls))
    b_out = rng.standard_normal(Ocls) * 0.1
    return dict(x=x, labels=lab, W_in=W_in, indptr=ip, indices=ix, w_rec=w_rec, W_out=W_out, b_out=b_out)


def loss_of(P, d, **kw):
    return O.snn_grad(P, d["x"], d["labels"], d["W_in"], d["indptr"], d["indices"], d["w_rec"], d["W_out"],
                      d["b_out"], **kw)


# the two surrogates: sigmoid of slope 4 (the training workload) and the ReLU
# form of Appendix I with its stated alpha = 0.3, width = 1.0
SURR = {"sigmoid": dict(surrogate=0, slope=4.0), "relu": dict(surrogate=1, relu_a=0.3, relu_width=1.0)}


def smooth_params(kind, detach, T=15):
    return O.snn_params(2, 6, 12, 3, T, alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), theta=1.0, smooth=1,
                        detach_reset=detach, **SURR[kind])


def fd_check(P, d, g, n_per=12, seed=1, **kw):
    """Central differences (h = 1e-6) of the loss against the gradient g on
    sampled entries of every parameter; returns the largest relative error."""
    rng = np.random.default_rng(seed)
    h = 1e-6
    worst = 0.0
    for name, gname in (("W_in", "dW_in"), ("w_rec", "dw_rec"), ("W_out", "dW_out"), ("b_out", "db_out")):
        flat = d[name].reshape(-1)
        for i in rng.choice(flat.size, min(flat.size, n_per), replace=False):
            orig = flat[i]
            flat[i] = orig + h
            lp = loss_of(P, d, **kw)["loss"]
            flat[i] = orig - h
            lm = loss_of(P, d, **kw)["loss"]
            flat[i] = orig
            fd = (lp - lm) / (2 * h)
            an = g[gname].reshape(-1)[i]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, i, an, fd)
            worst = max(worst, abs(an - fd) / max(abs(fd), 1e-9))
    return worst


@pytest.mark.parametrize("kind", ["sigmoid", "relu"])
def test_smooth_bptt_equals_finite_differences(kind):
    """Reset differentiated: the full reverse pass is the exact gradient of
    the smooth forward."""
    P = smooth_params(kind, detach=0)
    d = tiny(T=15)
    g = loss_of(P, d)
    fd_check(P, d, g)


def frozen_resets(P, d):
    """The free run's reset factors: entry t is 1 - z_{t-1} (entry 0 unused)."""
    z = loss_of(P, d, want_zval=True)["zval"]
    R = np.ones_like(z)
    R[1:] = 1.0 - z[:-1]
    return R, z


@pytest.mark.parametrize("kind", ["sigmoid", "relu"])
def test_detached_reset_equals_frozen_reset_finite_differences(kind):
    """Detached reset: finite differences of the forward with every reset
    factor frozen at the free run's value equal the detached reverse pass."""
    P = smooth_params(kind, detach=1)
    d = tiny(T=15)
    R, z = frozen_resets(P, d)
    assert 0.02 < z.mean() < 0.98  # the reset factors are far from trivial
    g = loss_of(P, d)
    # freezing at the free run's values does not move the forward pass
    assert loss_of(P, d, reset_in=R)["loss"] == pytest.approx(g["loss"], rel=1e-14)
    fd_check(P, d, g, reset_in=R)


@pytest.mark.parametrize("kind", ["sigmoid", "relu"])
def test_frozen_reset_check_separates_the_two_reverse_passes(kind):
    """The frozen-reset differences are not also matched by the attached
    reverse pass (so the test above can fail on a reset term in the wrong
    place), and the attached pass is not matched by the frozen differences."""
    P1 = smooth_params(kind, detach=1)
    P0 = smooth_params(kind, detach=0)
    d = tiny(T=15)
    R, _ = frozen_resets(P1, d)
    g0 = loss_of(P0, d)
    rng = np.random.default_rng(3)
    h = 1e-6
    flat = d["W_in"].reshape(-1)
    differs = 0
    for i in rng.choice(flat.size, 12, replace=False):
        orig = flat[i]
        flat[i] = orig + h
        lp = loss_of(P1, d, reset_in=R)["loss"]
        flat[i] = orig - h
        lm = loss_of(P1, d, reset_in=R)["loss"]
        flat[i] = orig
        fd = (lp - lm) / (2 * h)
        if abs(g0["dW_in"].reshape(-1)[i] - fd) > 1e-4 * max(abs(fd), 1e-6):
            differs += 1
    assert differs >= 6


@pytest.mark.parametrize("kind", ["sigmoid", "relu"])
def test_surrogate_shapes(kind):
    from scipy import integrate
    P = O.snn_params(1, 1, 1, 1, 1, alpha=0.5, beta=0.5, theta=1.0, smooth=1, **SURR[kind])
    theta = 1.0
    sg = lambda x: float(O.snn_spike_fns(P, np.array([theta + x]))[1][0])
    if kind == "sigmoid":
        rise, peak, lim = 1.0, 4.0 / 4.0, 40.0
    else:
        a, w = 0.3, 1.0
        rise, peak, lim = a * w * w, a * w, 1.0
    # area = the spike's full rise; even; peak at threshold
    area = integrate.quad(sg, -lim, lim, points=[0.0], limit=200, epsabs=1e-13, epsrel=1e-12)[0]
    assert area == pytest.approx(rise, rel=1e-9)
    xs = np.linspace(-3, 3, 601)
    s, ds = O.snn_spike_fns(P, theta + xs)
    np.testing.assert_allclose(ds, ds[::-1], rtol=0, atol=1e-15)
    assert ds.max() == pytest.approx(peak, rel=1e-12) and ds[300] == pytest.approx(peak, rel=1e-12)
    # S rises from 0 to the full rise, and S' = the surrogate (central differences)
    s_ends = O.snn_spike_fns(P, theta + np.array([-60.0, 60.0]))[0]
    assert s_ends[0] == pytest.approx(0.0, abs=1e-12) and s_ends[1] == pytest.approx(rise, rel=1e-12)
    h = 1e-6
    sp, _ = O.snn_spike_fns(P, theta + xs + h)
    sm, _ = O.snn_spike_fns(P, theta + xs - h)
    # (at the kinks of the ReLU form, x = 0 and |x| = width, S'' jumps and the
    # central difference is off by alpha h / 4)
    np.testing.assert_allclose((sp - sm) / (2 * h), ds, rtol=1e-6, atol=1e-7)
    if kind == "relu":
        # zero outside |x| < width, positive inside, linear on each side
        assert np.all(ds[np.abs(xs) >= 1.0] == 0.0) and np.all(ds[np.abs(xs) < 1.0 - 1e-12] > 0.0)
        left = (xs > -1.0 + 1e-9) & (xs < -1e-9)
        second = np.diff(ds[left], 2)
        np.testing.assert_allclose(second, 0.0, atol=1e-13)


def test_detached_reset_drops_only_the_reset_path():
    T = 15
    kw = dict(alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), theta=1.0, slope=4.0, smooth=1)
    d = tiny(T=T)
    g0 = loss_of(O.snn_params(2, 6, 12, 3, T, detach_reset=0, **kw), d)
    g1 = loss_of(O.snn_params(2, 6, 12, 3, T, detach_reset=1, **kw), d)
    assert g0["loss"] == g1["loss"]  # forward unchanged
    np.testing.assert_array_equal(g0["dW_out"], g1["dW_out"])  # readout path has no reset term
    assert not np.allclose(g0["dW_in"], g1["dW_in"])


def test_hard_spikes_teacher_forced_with_own_raster():
    T = 30
    P = O.snn_params(2, 6, 12, 3, T, alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), theta=1.0, slope=4.0)
    d = tiny(T=T)
    a = loss_of(P, d, want_z=True)
    assert 0 < a["z"].mean() < 1
    b = loss_of(P, d, z_force=a["z"])
    assert a["loss"] == b["loss"]
    for k in ("dW_in", "dw_rec", "dW_out", "db_out"):
        np.testing.assert_array_equal(a[k], b[k])


def test_readout_gradient_closed_form():
    # dL/db_out = mean over the batch of softmax(logits) - onehot(label)
    T = 10
    P = O.snn_params(2, 6, 12, 3, T, alpha=0.8, beta=0.9)
    d = tiny(T=T)
    g = loss_of(P, d)
    lg = g["logits"]
    sm = np.exp(lg - lg.max(1, keepdims=True))
    sm /= sm.sum(1, keepdims=True)
    oh = np.eye(3)[d["labels"]]
    np.testing.assert_allclose(g["db_out"], (sm - oh).mean(0), rtol=1e-12, atol=1e-15)
    lse = np.log(np.exp(lg).sum(1))
    assert g["loss"] == pytest.approx(float((lse - lg[np.arange(2), d["labels"]]).mean()), rel=1e-12)


@pytest.mark.parametrize("detach,kind", [(1, "sigmoid"), (0, "sigmoid"), (1, "relu")])
def test_gradient_magnitude_companion(detach, kind):
    # the per-entry tolerance scale of the GPU's reverse pass: the same
    # recursion on absolute values bounds every gradient entry (triangle
    # inequality) and vanishes exactly where no term reaches an entry; with
    # one sample the readout gradients have a single term per entry, so
    # there it equals |gradient|
    T = 25
    P = O.snn_params(2, 6, 12, 3, T, alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), theta=1.0,
                     detach_reset=detach, **SURR[kind])
    d = tiny(T=T)
    g = loss_of(P, d, want_z=True)
    a = O.snn_grad_abs(P, d["x"], d["labels"], d["W_in"], d["indptr"], d["indices"], d["w_rec"], d["W_out"],
                       d["b_out"], g["z"])
    for k in ("dW_in", "dw_rec", "dW_out", "db_out"):
        assert np.all(a[k] >= np.abs(g[k]) * (1 - 1e-12) - 1e-300), k
        assert np.all(np.isfinite(a[k]))
        assert np.all(g[k][a[k] == 0] == 0), k
    assert (a["dW_in"] > np.abs(g["dW_in"]) * 1.0001).any()  # cancellation happens in the recursion
    P1 = O.snn_params(1, 6, 12, 3, T, alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), theta=1.0,
                      detach_reset=detach, **SURR[kind])
    d1 = dict(d, x=d["x"][:, :1], labels=d["labels"][:1])
    g1 = loss_of(P1, d1, want_z=True)
    a1 = O.snn_grad_abs(P1, d1["x"], d1["labels"], d1["W_in"], d1["indptr"], d1["indices"], d1["w_rec"],
                        d1["W_out"], d1["b_out"], g1["z"])
    np.testing.assert_allclose(a1["db_out"], np.abs(g1["db_out"]), rtol=1e-12)
    np.testing.assert_allclose(a1["dW_out"], np.abs(g1["dW_out"]), rtol=1e-12)
