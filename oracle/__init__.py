"""CPU oracle for the event-driven / JIT-connectivity synaptic propagation path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the GPU library or its
Python binding.  All arithmetic lives in ``oracle.c`` / ``snn.c`` (plain C
loops, FP64 unless stated); this module only marshals numpy arrays.

The Philox-4x32-10 source is pinned by the generator's published
known-answer vectors (tests/golden/philox4x32_10_kat.txt).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

STREAM_CONN, STREAM_W, STREAM_V0 = 1, 2, 3
W_HOMO, W_NORMAL, W_UNIFORM = 0, 1, 2
COBA, CUBA = 0, 1
CONN_CSR, CONN_JIT = 0, 1

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C")


class NetParams(C.Structure):
    _fields_ = [("model", C.c_int32), ("n", C.c_int32), ("n_exc", C.c_int32),
                ("conn", C.c_int32), ("max_gap", C.c_int32), ("block", C.c_int32),
                ("seed", C.c_uint64),
                ("w_exc", C.c_float), ("w_inh", C.c_float),
                ("tau_m", C.c_float), ("tau_e", C.c_float), ("tau_i", C.c_float), ("tau_ref", C.c_float),
                ("v_rest", C.c_float), ("v_th", C.c_float), ("v_reset", C.c_float),
                ("e_exc", C.c_float), ("e_inh", C.c_float), ("r", C.c_float), ("i_ext", C.c_float),
                ("dt", C.c_float), ("v0_lo", C.c_float), ("v0_hi", C.c_float)]


class SnnParams(C.Structure):
    _fields_ = [("B", C.c_int32), ("C", C.c_int32), ("N", C.c_int32), ("O", C.c_int32), ("T", C.c_int32),
                ("surrogate", C.c_int32), ("smooth", C.c_int32), ("detach_reset", C.c_int32),
                ("alpha", C.c_double), ("beta", C.c_double), ("theta", C.c_double),
                ("slope", C.c_double), ("relu_a", C.c_double), ("relu_width", C.c_double)]


def lib():
    """The oracle built as plain C (loops run as written, one thread)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = _load(_build.LIB)
    return _lib


_lib_omp = None


def lib_omp():
    """The same oracle built with its OpenMP pragmas: the network loops spread
    over the host cores (the CPU baseline).  Results are identical."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_build.LIB_OMP):
            _build.build()
        _lib_omp = _load(_build.LIB_OMP)
    return _lib_omp


def _load(path):
    L = C.CDLL(path)
    L.or_set_threads.restype = C.c_int32
    L.or_set_threads.argtypes = [C.c_int32]
    L.or_hash.restype = C.c_uint32
    L.or_hash.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
    L.or_hash_many.argtypes = [C.c_uint64, C.c_uint32, _u32p, _u32p, _u32p, _u32p, C.c_int64]
    L.or_philox.argtypes = [_u32p, C.c_uint32, C.c_uint32, _u32p]
    L.or_philox_many.argtypes = [_u32p, _u32p, _u32p, C.c_int64]
    L.or_max_gap.restype = C.c_int32
    L.or_max_gap.argtypes = [C.c_double]
    L.or_row_block.restype = C.c_int64
    L.or_row_block.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]
    L.or_row.restype = C.c_int64
    L.or_row.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]
    L.or_csr_count.restype = C.c_int64
    L.or_csr_count.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]
    L.or_csr_build.restype = C.c_int64
    L.or_csr_build.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _i32p, _i32p, C.c_int64]
    L.or_compact.restype = C.c_int32
    L.or_compact.argtypes = [_u8p, C.c_int32, _i32p]
    L.or_event_csr_matvec.argtypes = [_i32p, _i32p, C.c_void_p, C.c_double, C.c_int32, C.c_int32, _u8p, _f64p]
    L.or_event_csr_counts.argtypes = [_i32p, _i32p, C.c_int32, C.c_int32, _u8p, _i64p]
    L.or_event_csr_vjp.argtypes = [_i32p, _i32p, C.c_void_p, C.c_double, C.c_int32, C.c_int32, _u8p, _f64p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
    L.or_jit_weight.restype = C.c_double
    L.or_jit_weight.argtypes = [C.c_uint64, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                C.c_int64, C.c_void_p]
    L.or_jit_matvec.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                C.c_int32, C.c_int32, _u8p, _f64p]
    L.or_jit_counts.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _u8p, _i64p]
    L.or_jit_matmat_dense.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                      C.c_int32, C.c_int32, C.c_int32, _f64p, _f64p]
    L.or_jit_abs_terms.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                   C.c_int32, C.c_int32, C.c_int32, _f64p, _f64p]
    L.or_jit_matvec_dense.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                      C.c_int32, C.c_int32, _f64p, _f64p]
    L.or_jit_vjp.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                             C.c_int32, C.c_int32, _u8p, _f64p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.or_ln_f32.restype = C.c_float
    L.or_ln_f32.argtypes = [C.c_uint32]
    L.or_ln_f32_many.argtypes = [_u32p, _f32p, C.c_int64]
    L.or_geo_inv_rate.restype = C.c_float
    L.or_geo_inv_rate.argtypes = [C.c_double]
    L.or_geo_gap.restype = C.c_uint32
    L.or_geo_gap.argtypes = [C.c_uint32, C.c_float]
    L.or_geo_gap_many.argtypes = [_u32p, C.c_float, _u32p, C.c_int64]
    L.or_fd_target.restype = C.c_uint32
    L.or_fd_target.argtypes = [_u32p, C.c_int32, C.c_uint32]
    L.or_rule_row_block.restype = C.c_int64
    L.or_rule_row_block.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_float, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int32, C.c_int32, C.c_void_p]
    L.or_rule_csr.restype = C.c_int64
    L.or_rule_csr.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_float, C.c_int32, C.c_int32, C.c_int32,
                              C.c_int32, _i32p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
    L.or_rule_weights.argtypes = [C.c_uint64, C.c_int32, C.c_double, C.c_double, C.c_int32, _i32p, _i32p, _i32p,
                                  _f64p]
    L.or_proj_run_f64.argtypes = [_i32p, _i32p, C.c_void_p, C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_double, C.c_double, C.c_int32, C.c_int32, _u8p, _f64p, _f64p]
    L.or_proj_run_f32.argtypes = [_i32p, _i32p, C.c_void_p, C.c_float, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_float, C.c_float, C.c_int32, C.c_int32, _u8p, _f32p, _f64p]
    L.or_net_v0.argtypes = [C.POINTER(NetParams), _f32p]
    L.or_net_ref_steps.restype = C.c_int32
    L.or_net_ref_steps.argtypes = [C.POINTER(NetParams)]
    L.or_net_run_f32.argtypes = [C.POINTER(NetParams), C.c_void_p, C.c_void_p, C.c_int32,
                                 _f32p, _f32p, _f32p, _i32p, _u8p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]
    L.or_net_run_f64.argtypes = [C.POINTER(NetParams), C.c_void_p, C.c_void_p, C.c_int32,
                                 _f64p, _f64p, _f64p, _i32p, _u8p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]
    L.or_snn_grad.restype = C.c_int
    L.or_snn_grad.argtypes = [C.POINTER(SnnParams), _u8p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p,
                              C.c_void_p, C.c_void_p, C.POINTER(C.c_double), _f64p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.or_snn_grad_abs.restype = C.c_int
    L.or_snn_grad_abs.argtypes = [C.POINTER(SnnParams), _u8p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p, _u8p,
                                  _f64p, _f64p, _f64p, _f64p]
    L.or_snn_spike_fns.argtypes = [C.POINTER(SnnParams), _f64p, C.c_int64, C.c_void_p, C.c_void_p]
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- hash / K
def hash_word(seed, stream, a, b, k):
    return int(lib().or_hash(seed, stream, a, b, k))


def hash_many(seed, stream, a, b, k):
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    k = np.ascontiguousarray(k, np.uint32)
    out = np.empty(a.shape[0], np.uint32)
    lib().or_hash_many(seed, stream, a, b, k, out, a.shape[0])
    return out


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    out = np.empty(4, np.uint32)
    lib().or_philox(c, int(key[0]), int(key[1]), out)
    return out


def philox_many(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32).reshape(-1, 2)
    out = np.empty_like(c)
    lib().or_philox_many(c, k, out, c.shape[0])
    return out


def max_gap(p):
    return int(lib().or_max_gap(float(p)))


# ---------------------------------------------------------------- rows / CSR
def row_block(seed, K, n_post, B, j, b):
    n = lib().or_row_block(seed, K, n_post, B, j, b, None)
    out = np.empty(max(n, 1), np.int32)
    lib().or_row_block(seed, K, n_post, B, j, b, _ptr(out))
    return out[:n]


def row(seed, K, n_post, B, j):
    n = lib().or_row(seed, K, n_post, B, j, None)
    out = np.empty(max(n, 1), np.int32)
    lib().or_row(seed, K, n_post, B, j, _ptr(out))
    return out[:n]


def csr_build(seed, K, n_pre, n_post, B):
    rowlen = np.empty(max(n_pre, 1), np.int32)
    nnz = lib().or_csr_count(seed, K, n_pre, n_post, B, _ptr(rowlen))
    indptr = np.empty(n_pre + 1, np.int32)
    indices = np.empty(max(nnz, 1), np.int32)
    got = lib().or_csr_build(seed, K, n_pre, n_post, B, indptr, indices, nnz)
    assert got == nnz
    return indptr, indices[:nnz]


# ---------------------------------------------------------------- connectivity rules
RULE_UNIFORM, RULE_GEOMETRIC, RULE_FIXED_DEGREE = 0, 1, 2


def ln_f32(k):
    """ln(k 2^-24) by the fixed FP32 operation sequence (k in [1, 2^24])."""
    kk = np.ascontiguousarray(k, np.uint32)
    out = np.empty(kk.shape, np.float32)
    lib().or_ln_f32_many(kk.reshape(-1), out.reshape(-1), kk.size)
    return out


def geo_inv_rate(p):
    """1 / (-ln(1 - p)) computed in FP64, rounded once to FP32."""
    return float(lib().or_geo_inv_rate(float(p)))


def geo_gaps(words, inv_rate):
    w = np.ascontiguousarray(words, np.uint32)
    out = np.empty(w.shape, np.uint32)
    lib().or_geo_gap_many(w.reshape(-1), C.c_float(inv_rate), out.reshape(-1), w.size)
    return out


def fd_target(key, n, i):
    """Target i of a fixed-degree row with Feistel round keys `key` (4 words)."""
    kk = np.ascontiguousarray(key, np.uint32)
    return int(lib().or_fd_target(kk, int(n), int(i)))


def rule_row_block(seed, rule, K, inv_rate, degree, n_post, B, j, b):
    """Targets of (row j, block b) under a connectivity rule, generation order."""
    buf = np.empty(max(n_post, 1), np.int32)
    c = lib().or_rule_row_block(seed, rule, K, C.c_float(inv_rate), degree, n_post, B, j, b, _ptr(buf))
    return buf[:c].copy()


def rule_csr(seed, rule, K, inv_rate, degree, n_pre, n_post, B):
    """(indptr, indices, blk, idx) of a rule's matrix in generation order."""
    indptr = np.empty(n_pre + 1, np.int32)
    nnz = lib().or_rule_csr(seed, rule, K, C.c_float(inv_rate), degree, n_pre, n_post, B, indptr, None, None,
                            None, 1 << 62)
    indices = np.empty(max(nnz, 1), np.int32)
    blk = np.empty(max(nnz, 1), np.int32)
    idx = np.empty(max(nnz, 1), np.int32)
    lib().or_rule_csr(seed, rule, K, C.c_float(inv_rate), degree, n_pre, n_post, B, indptr, _ptr(indices),
                      _ptr(blk), _ptr(idx), nnz)
    return indptr, indices[:nnz], blk[:nnz], idx[:nnz]


def rule_csr_sorted(seed, rule, K, inv_rate, degree, n_pre, n_post, B):
    """(indptr, indices) of the rule's matrix with every row ascending (the
    stored CSR form)."""
    ip, ix, _, _ = rule_csr(seed, rule, K, inv_rate, degree, n_pre, n_post, B)
    ix = ix.copy()
    for j in range(n_pre):
        ix[ip[j]:ip[j + 1]].sort()
    return ip, ix


def rule_weights(seed, wkind, w0, w1, indptr, blk, idx):
    w = np.empty(max(int(indptr[-1]), 1), np.float64)
    lib().or_rule_weights(seed, wkind, float(w0), float(w1), indptr.size - 1, indptr, blk, idx, w)
    return w[:int(indptr[-1])]


def rule_matvec(indptr, indices, weights, n_post, X):
    """y = M^T x for a rule CSR in generation order with per-entry weights
    (None: count each entry once), FP64: x a spike vector (truthy bytes) or
    a float vector; the sum over rows of weight times x[row]."""
    x = np.asarray(X)
    xv = (x != 0).astype(np.float64) if x.dtype == np.uint8 else x.astype(np.float64)
    rows = np.repeat(np.arange(indptr.size - 1), np.diff(indptr))
    terms = xv[rows] * (1.0 if weights is None else weights)
    return np.bincount(indices, weights=terms, minlength=n_post).astype(np.float64)


def compact(s):
    s = np.ascontiguousarray(s, np.uint8)
    ids = np.empty(max(s.shape[0], 1), np.int32)
    c = lib().or_compact(s, s.shape[0], ids)
    return ids[:c]


# ---------------------------------------------------------------- matvecs
def event_csr_matvec(indptr, indices, data, w, n_post, events):
    ev = np.ascontiguousarray(events, np.uint8)
    y = np.empty(n_post, np.float64)
    d = None if data is None else np.ascontiguousarray(data, np.float32)
    lib().or_event_csr_matvec(np.ascontiguousarray(indptr, np.int32), np.ascontiguousarray(indices, np.int32),
                              _ptr(d), float(w), ev.shape[0], n_post, ev, y)
    return y


def event_csr_counts(indptr, indices, n_post, events):
    ev = np.ascontiguousarray(events, np.uint8)
    cnt = np.empty(n_post, np.int64)
    lib().or_event_csr_counts(np.ascontiguousarray(indptr, np.int32), np.ascontiguousarray(indices, np.int32),
                              ev.shape[0], n_post, ev, cnt)
    return cnt


def event_csr_matmat(indptr, indices, data, w, n_post, E):
    """Y[b] = M^T E[b] for a batch of spike vectors E [batch, n_pre]: the
    single-vector product of Appendix B applied to each vector; FP64."""
    E = np.asarray(E)
    Y = np.empty((E.shape[0], n_post), np.float64)
    for b in range(E.shape[0]):
        Y[b] = event_csr_matvec(indptr, indices, data, w, n_post, E[b])
    return Y


def event_csr_counts_batch(indptr, indices, n_post, E):
    """Integer counts of event_csr_matmat with homogeneous weight 1."""
    E = np.asarray(E)
    Y = np.empty((E.shape[0], n_post), np.int64)
    for b in range(E.shape[0]):
        Y[b] = event_csr_counts(indptr, indices, n_post, E[b])
    return Y


def event_csr_vjp(indptr, indices, data, w, n_post, events, dy):
    ev = np.ascontiguousarray(events, np.uint8)
    n_pre = ev.shape[0]
    nnz = int(indptr[-1])
    d = None if data is None else np.ascontiguousarray(data, np.float32)
    d_ev = np.empty(n_pre, np.float64)
    d_data = np.empty(max(nnz, 1), np.float64)
    d_w = np.zeros(1, np.float64)
    lib().or_event_csr_vjp(np.ascontiguousarray(indptr, np.int32), np.ascontiguousarray(indices, np.int32),
                           _ptr(d), float(w), n_pre, n_post, ev, np.ascontiguousarray(dy, np.float64),
                           _ptr(d_ev), _ptr(d_data), _ptr(d_w))
    return d_ev, d_data[:nnz], float(d_w[0])


def jit_weight(seed, wkind, w0, w1, j, b, m):
    u = C.c_double(0.0)
    w = lib().or_jit_weight(seed, wkind, w0, w1, j, b, m, C.byref(u))
    return w, u.value


def jit_matvec(seed, K, B, wkind, w0, w1, n_post, events):
    ev = np.ascontiguousarray(events, np.uint8)
    y = np.empty(n_post, np.float64)
    lib().or_jit_matvec(seed, K, B, wkind, float(w0), float(w1), ev.shape[0], n_post, ev, y)
    return y


def jit_matvec_dense(seed, K, B, wkind, w0, w1, n_post, v):
    """y = J v for a float vector v (Section 5.2's JIT operator on a dense
    vector); FP64."""
    vv = np.ascontiguousarray(v, np.float64)
    y = np.empty(n_post, np.float64)
    lib().or_jit_matvec_dense(seed, K, B, wkind, float(w0), float(w1), vv.shape[0], n_post, vv, y)
    return y


def jit_matmat_dense(seed, K, B, wkind, w0, w1, n_post, X):
    """Y = J^T X for X [n_pre, m] (m float vectors at once); FP64."""
    XX = np.ascontiguousarray(X, np.float64)
    Y = np.empty((n_post, XX.shape[1]), np.float64)
    lib().or_jit_matmat_dense(seed, K, B, wkind, float(w0), float(w1), XX.shape[0], n_post, XX.shape[1],
                              XX.reshape(-1), Y.reshape(-1))
    return Y


def jit_abs_terms(seed, K, B, wkind, w0, w1, n_post, X):
    """Sum of (|a_jk| + |b_jk|) |X[j, c]| over rows j, with w_jk = a_jk + b_jk
    the two terms of the weight formula (a = w0; b = w1 z normal, (w1 - w0) u
    uniform, 0 homogeneous): the magnitude of the terms of J^T X, the
    tolerance scale of FP32 weights and sums.  X: a vector (spike bytes as 0/1,
    or floats) or a [n_pre, m] matrix; the result has the same rank."""
    XX = np.asarray(X)
    vec = XX.ndim == 1
    XX = np.ascontiguousarray(XX.reshape(XX.shape[0], -1), np.float64)
    Sm = np.empty((n_post, XX.shape[1]), np.float64)
    lib().or_jit_abs_terms(seed, K, B, wkind, float(w0), float(w1), XX.shape[0], n_post, XX.shape[1],
                           XX.reshape(-1), Sm.reshape(-1))
    return Sm[:, 0] if vec else Sm


def jit_counts(seed, K, B, n_post, events):
    ev = np.ascontiguousarray(events, np.uint8)
    cnt = np.empty(n_post, np.int64)
    lib().or_jit_counts(seed, K, B, ev.shape[0], n_post, ev, cnt)
    return cnt


def jit_matmat(seed, K, B, wkind, w0, w1, n_post, E):
    """Y[b] = M^T E[b] with the JIT matrix of (seed, K, B, weights), for a
    batch of spike vectors E [batch, n_pre]; FP64."""
    E = np.asarray(E)
    Y = np.empty((E.shape[0], n_post), np.float64)
    for b in range(E.shape[0]):
        Y[b] = jit_matvec(seed, K, B, wkind, w0, w1, n_post, E[b])
    return Y


def jit_counts_batch(seed, K, B, n_post, E):
    E = np.asarray(E)
    Y = np.empty((E.shape[0], n_post), np.int64)
    for b in range(E.shape[0]):
        Y[b] = jit_counts(seed, K, B, n_post, E[b])
    return Y


def jit_vjp(seed, K, B, wkind, w0, w1, n_post, events, dy):
    ev = np.ascontiguousarray(events, np.uint8)
    d_ev = np.empty(ev.shape[0], np.float64)
    g0 = np.zeros(1, np.float64)
    g1 = np.zeros(1, np.float64)
    lib().or_jit_vjp(seed, K, B, wkind, float(w0), float(w1), ev.shape[0], n_post, ev,
                     np.ascontiguousarray(dy, np.float64), _ptr(d_ev), _ptr(g0), _ptr(g1))
    return d_ev, float(g0[0]), float(g1[0])


# ---------------------------------------------------------------- network
def net_params(**kw):
    """NetParams from keyword arguments (names as in the struct)."""
    p = NetParams()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def net_v0(P):
    V = np.empty(P.n, np.float32)
    lib().or_net_v0(C.byref(P), V)
    return V


def net_ref_steps(P):
    return int(lib().or_net_ref_steps(C.byref(P)))


class NetState:
    """FP32 (default) or FP64 network state in host arrays."""

    def __init__(self, P, precision=32):
        self.precision = precision
        dt = np.float32 if precision == 32 else np.float64
        self.V = net_v0(P).astype(dt)
        self.ge = np.zeros(P.n, dt)
        self.gi = np.zeros(P.n, dt)
        self.ref = np.zeros(P.n, np.int32)
        self.s_prev = np.zeros(P.n, np.uint8)
        self.t = 0


def set_threads(threads=0):
    """Threads of the OpenMP build's network loops (0: the runtime default);
    returns how many it will use."""
    return int(lib_omp().or_set_threads(int(threads)))


def net_run(P, state, T, indptr=None, indices=None, iext_vec=None, want_raster=True, parallel=False):
    """T steps of the network from `state` (updated in place).  parallel: run
    the OpenMP build of the same loops (identical results)."""
    L = lib_omp() if parallel else lib()
    raster = np.empty((T, P.n), np.uint8) if want_raster else None
    counts = np.empty(T, np.int32)
    events = np.zeros(1, np.int64)
    ip = None if indptr is None else np.ascontiguousarray(indptr, np.int32)
    ix = None if indices is None else np.ascontiguousarray(indices, np.int32)
    if state.precision == 32:
        iv = None if iext_vec is None else np.ascontiguousarray(iext_vec, np.float32)
        fn = L.or_net_run_f32
    else:
        iv = None if iext_vec is None else np.ascontiguousarray(iext_vec, np.float64)
        fn = L.or_net_run_f64
    fn(C.byref(P), _ptr(ip), _ptr(ix), T, state.V, state.ge, state.gi, state.ref, state.s_prev,
       _ptr(iv), _ptr(raster), _ptr(counts), _ptr(events))
    state.t += T
    return raster, counts, int(events[0])


# ---------------------------------------------------------------- projections
ALIGN_POST, ALIGN_PRE = 0, 1
SYN_EXP, SYN_SAT = 0, 1


def proj_run(indptr, indices, data, w, n_post, align, syn, decay, u, delay, raster, state=None, precision=64):
    """T steps of a projection with a `delay`-step spike delay driven by the
    presynaptic raster [T, n_pre] (Section 4.3, Appendix D).  Returns
    (g [T, n_post] FP64, final state).  precision 32: the FP32 recursion of
    the state in the library's order of operations."""
    R = np.ascontiguousarray(raster, np.uint8)
    T, n_pre = R.shape
    ip = np.ascontiguousarray(indptr, np.int32)
    ix = np.ascontiguousarray(indices, np.int32)
    d = None if data is None else np.ascontiguousarray(data, np.float32)
    g = np.empty((T, n_post), np.float64)
    n_state = n_post if align == ALIGN_POST else n_pre
    if precision == 64:
        st = np.zeros(n_state, np.float64) if state is None else np.array(state, np.float64)
        lib().or_proj_run_f64(ip, ix, _ptr(d), float(w), n_pre, n_post, align, syn, float(decay), float(u), delay, T,
                              R.reshape(-1), st, g.reshape(-1))
    else:
        st = np.zeros(n_state, np.float32) if state is None else np.array(state, np.float32)
        lib().or_proj_run_f32(ip, ix, _ptr(d), C.c_float(w), n_pre, n_post, align, syn, C.c_float(decay),
                              C.c_float(u), delay, T, R.reshape(-1), st, g.reshape(-1))
    return g, st


# ---------------------------------------------------------------- SNN
def snn_params(B, C_, N, O, T, alpha, beta, theta=1.0, slope=4.0, surrogate=0, smooth=0, detach_reset=1,
               relu_a=0.3, relu_width=1.0):
    return SnnParams(B, C_, N, O, T, surrogate, smooth, detach_reset, alpha, beta, theta, slope, relu_a,
                     relu_width)


def snn_spike_fns(P, v):
    """(S(v), S'(v)): the smooth spike function of smooth mode and the
    surrogate derivative used by the reverse pass, at membrane values v."""
    vv = np.ascontiguousarray(v, np.float64).reshape(-1)
    s = np.empty_like(vv)
    ds = np.empty_like(vv)
    lib().or_snn_spike_fns(C.byref(P), vv, vv.size, _ptr(s), _ptr(ds))
    return s, ds


def snn_grad_abs(P, x, labels, W_in, indptr, indices, w_rec, W_out, b_out, z_force):
    """Per-entry sum of |terms| reaching each gradient entry through the
    reverse pass (spikes z_force [T, B, N]): the scale of the parity
    tolerance of an FP32 reverse pass."""
    Cc, N, O = P.C, P.N, P.O
    nnz = int(indptr[-1])
    a = dict(dW_in=np.empty((Cc, N), np.float64), dw_rec=np.empty(max(nnz, 1), np.float64),
             dW_out=np.empty((N, O), np.float64), db_out=np.empty(O, np.float64))
    rc = lib().or_snn_grad_abs(C.byref(P), np.ascontiguousarray(x, np.uint8), np.ascontiguousarray(labels, np.int32),
                               np.ascontiguousarray(W_in, np.float64), np.ascontiguousarray(indptr, np.int32),
                               np.ascontiguousarray(indices, np.int32), np.ascontiguousarray(w_rec, np.float64),
                               np.ascontiguousarray(W_out, np.float64), np.ascontiguousarray(b_out, np.float64),
                               np.ascontiguousarray(z_force, np.uint8), a["dW_in"], a["dw_rec"], a["dW_out"],
                               a["db_out"])
    assert rc == 0
    a["dw_rec"] = a["dw_rec"][:nnz]
    return a


def snn_grad(P, x, labels, W_in, indptr, indices, w_rec, W_out, b_out, z_force=None, want_z=False,
             want_margin=False, reset_in=None, want_zval=False):
    """Loss, logits and BPTT gradients of the recurrent LIF network (FP64).
    z_force: spikes [T, B, N] to use instead of the threshold; reset_in:
    frozen reset factors [T, B, N] (entry t multiplies V_{t-1} at step t);
    want_zval: also return the spike values z_t (fractional in smooth mode)."""
    B, N, O, T, Cc = P.B, P.N, P.O, P.T, P.C
    loss = C.c_double(0.0)
    logits = np.empty((B, O), np.float64)
    z_out = np.empty((T, B, N), np.uint8) if want_z else None
    vm = np.empty((T, B, N), np.float64) if want_margin else None
    dW_in = np.empty((Cc, N), np.float64)
    nnz = int(indptr[-1])
    dw_rec = np.empty(max(nnz, 1), np.float64)
    dW_out = np.empty((N, O), np.float64)
    db_out = np.empty(O, np.float64)
    zf = None if z_force is None else np.ascontiguousarray(z_force, np.uint8)
    rf = None if reset_in is None else np.ascontiguousarray(reset_in, np.float64)
    zv = np.empty((T, B, N), np.float64) if want_zval else None
    rc = lib().or_snn_grad(C.byref(P), np.ascontiguousarray(x, np.uint8), np.ascontiguousarray(labels, np.int32),
                           np.ascontiguousarray(W_in, np.float64), np.ascontiguousarray(indptr, np.int32),
                           np.ascontiguousarray(indices, np.int32), np.ascontiguousarray(w_rec, np.float64),
                           np.ascontiguousarray(W_out, np.float64), np.ascontiguousarray(b_out, np.float64),
                           _ptr(zf), _ptr(rf), C.byref(loss), logits, _ptr(z_out), _ptr(vm), _ptr(zv), _ptr(dW_in),
                           _ptr(dw_rec), _ptr(dW_out), _ptr(db_out))
    assert rc == 0
    return dict(loss=loss.value, logits=logits, z=z_out, vmargin=vm, zval=zv, dW_in=dW_in, dw_rec=dw_rec[:nnz],
                dW_out=dW_out, db_out=db_out)
