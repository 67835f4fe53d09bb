"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds none of the method's arithmetic: only numpy draws of the
workloads' inputs (spike vectors, heterogeneous weights, Poisson input spikes,
labels, initial weights, request streams).

Workload shapes follow the paper's experiments: firing fractions 0.1 %, 1 %,
10 % (10, 100, 1000 Hz at dt = 0.1 ms, Section 5.1), heterogeneous weights
N(0.5, 0.1), COBA E/I networks with 80/20 excitatory/inhibitory split
(Appendix N).
"""
import math

import numpy as np


def events(n, frac, seed, count=1):
    """Bernoulli(frac) spike vectors, uint8 [count, n] (or [n] if count == 1)."""
    rng = np.random.default_rng([seed, 5])
    ev = (rng.random((count, n)) < frac).astype(np.uint8)
    return ev[0] if count == 1 else ev


def hetero_data(nnz, seed, mean=0.5, std=0.1):
    """Heterogeneous CSR weights ~ N(mean, std) in FP32 (drawn in FP64)."""
    rng = np.random.default_rng([seed, 9])
    return rng.normal(mean, std, nnz).astype(np.float32)


def signed_data(nnz, seed, scale=1.0):
    rng = np.random.default_rng([seed, 10])
    return (rng.standard_normal(nnz) * scale).astype(np.float32)


def cotangent(n, seed):
    """A dense upstream gradient dy for reverse-mode checks."""
    rng = np.random.default_rng([seed, 11])
    return rng.standard_normal(n)


def dense_vector(n, seed, zero_frac=0.0):
    """A dense FP32 input vector ~ N(0, 1) with a fraction of exact zeros."""
    rng = np.random.default_rng([seed, 12])
    v = rng.standard_normal(n).astype(np.float32)
    v[rng.random(n) < zero_frac] = 0.0
    return v


def poisson_inputs(T, B, C, dt_ms, seed, lo_hz=5.0, hi_hz=50.0):
    """x[t, b, c] ~ Bernoulli(r_bc dt), r_bc ~ U(lo, hi) Hz.  uint8 [T, B, C]."""
    rng = np.random.default_rng([seed, 4])
    rates = rng.uniform(lo_hz, hi_hz, (B, C))
    p = rates * dt_ms * 1e-3
    return (rng.random((T, B, C)) < p[None]).astype(np.uint8)


def labels(B, n_classes, seed):
    rng = np.random.default_rng([seed, 6])
    return rng.integers(0, n_classes, B).astype(np.int32)


def snn_weights(C, N, O, nnz, seed, rec_std):
    """W_in ~ N(0, 1/sqrt(C)), recurrent CSR data ~ N(0, rec_std), W_out ~ N(0, 1/sqrt(N)), b_out = 0."""
    rng = np.random.default_rng([seed, 8])
    W_in = (rng.standard_normal((C, N)) / math.sqrt(C)).astype(np.float32)
    w_rec = (rng.standard_normal(nnz) * rec_std).astype(np.float32)
    W_out = (rng.standard_normal((N, O)) / math.sqrt(N)).astype(np.float32)
    b_out = np.zeros(O, np.float32)
    return W_in, w_rec, W_out, b_out


def request_stream(n_requests, rate_hz, seed, n_lo=1000, n_hi=200000, dur_lo_ms=100.0, dur_hi_ms=2000.0,
                   dt_ms=0.1):
    """Serving workload: Poisson arrivals at rate_hz; per request a network size
    N ~ log-uniform[n_lo, n_hi], duration ~ U(dur_lo, dur_hi) ms, COBA or CUBA
    with probability 1/2, and a per-request seed."""
    rng = np.random.default_rng([seed, 7])
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        dur = rng.uniform(dur_lo_ms, dur_hi_ms)
        steps = int(math.ceil(dur / dt_ms))
        model = int(rng.integers(0, 2))
        out.append(dict(id=i, arrival=float(t[i]), n=n, steps=steps, model=model, seed=1000 + i))
    return out
