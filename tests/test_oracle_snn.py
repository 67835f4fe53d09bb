"""Pins for the oracle's BPTT of the recurrent LIF network (CPU only): in the
smooth mode (sigmoid spikes, reset differentiated) the reverse pass must equal
central finite differences of the loss; with hard spikes, teacher forcing with
the network's own spikes reproduces the free run; the surrogates' closed
forms."""
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


def loss_of(P, d):
    return O.snn_grad(P, d["x"], d["labels"], d["W_in"], d["indptr"], d["indices"], d["w_rec"], d["W_out"],
                      d["b_out"])


@pytest.mark.parametrize("detach", [0])
def test_smooth_bptt_equals_finite_differences(detach):
    T = 15
    P = O.snn_params(2, 6, 12, 3, T, alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), theta=1.0, slope=4.0,
                     smooth=1, detach_reset=detach)
    d = tiny(T=T)
    g = loss_of(P, d)
    rng = np.random.default_rng(1)
    h = 1e-6
    for name, gname in (("W_in", "dW_in"), ("w_rec", "dw_rec"), ("W_out", "dW_out"), ("b_out", "db_out")):
        arr = d[name]
        flat = arr.reshape(-1)
        for i in rng.choice(flat.size, min(flat.size, 12), replace=False):
            orig = flat[i]
            flat[i] = orig + h
            lp = loss_of(P, d)["loss"]
            flat[i] = orig - h
            lm = loss_of(P, d)["loss"]
            flat[i] = orig
            fd = (lp - lm) / (2 * h)
            an = g[gname].reshape(-1)[i]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, i, an, fd)


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
    a = O.snn_grad(P, d["x"], d["labels"], d["W_in"], d["indptr"], d["indices"], d["w_rec"], d["W_out"],
                   d["b_out"], want_z=True)
    assert 0 < a["z"].mean() < 1
    b = O.snn_grad(P, d["x"], d["labels"], d["W_in"], d["indptr"], d["indices"], d["w_rec"], d["W_out"],
                   d["b_out"], z_force=a["z"])
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
