"""MI355X (gfx950) event-driven spiking-network path: Python binding.

Thin marshalling over the C ABI of ``libbpmi.so`` (include/bp.h).  Every
step of the path runs in the HIP kernels; PyTorch only provides device
memory and the current stream.  Importing this module does not touch the
GPU; the first call loads the library and fails loudly if it is missing.
"""
import ctypes as C
import math

import torch

from . import _abi
from ._abi import (ALIGN_POST, ALIGN_PRE, COBA, CONN_CSR, CONN_JIT, CUBA, RULE_FIXED_DEGREE, RULE_GEOMETRIC,
                   RULE_UNIFORM, STREAM_CONN, STREAM_V0, STREAM_W, SYN_EXP, SYN_SAT, W_HOMO, W_NORMAL, W_UNIFORM,
                   BpError, check, lib)

__all__ = [
    "lib", "BpError", "max_gap", "hash_words", "csr_build", "csr_tile_index", "compact", "event_csr_matvec",
    "event_csr_matvec_noalloc", "event_csr_matmat", "jit_conn_matmat",
    "jit_conn_matvec", "jit_conn_matvec_dense", "jit_conn_matmat_dense", "event_csr_backward", "jit_conn_backward", "Net", "run_batch", "JitConn",
    "COBA", "CUBA", "CONN_CSR", "CONN_JIT", "W_HOMO", "W_NORMAL", "W_UNIFORM", "RULE_UNIFORM", "RULE_GEOMETRIC",
    "RULE_FIXED_DEGREE", "geo_inv_rate", "csr_matvec_dense", "Projection", "ALIGN_POST", "ALIGN_PRE", "SYN_EXP",
    "SYN_SAT",
]


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def _events(t, n, name="events"):
    """A spike vector for the kernels: a contiguous CUDA uint8 (or bool, read
    as its bytes) tensor of exactly n entries; raises before any launch."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype == torch.bool:
        t = t.view(torch.uint8)
    if t.dtype != torch.uint8:
        raise TypeError(f"{name} must be uint8 or bool (one byte per neuron), got {t.dtype}")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t.contiguous()


def _vec(t, n, dtype, name):
    """A contiguous CUDA tensor of `dtype` with exactly n entries."""
    t = _dev(t, dtype, name)
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t


def _out(t, n, dtype, device, name="out"):
    """The caller's output buffer, or a new one."""
    if t is None:
        return torch.empty(n, dtype=dtype, device=device)
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous() \
            or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of {n} entries")
    return t


def _csr_args(indptr, indices, data, n_post):
    indptr = _dev(indptr, torch.int32, "indptr")
    indices = _dev(indices, torch.int32, "indices")
    if indptr.dim() != 1 or indptr.numel() < 1:
        raise ValueError("indptr must be a vector of n_pre + 1 entries")
    if data is not None:
        data = _vec(data, indices.numel(), torch.float32, "data")
    if n_post < 0:
        raise ValueError("n_post must be >= 0")
    return indptr, indices, data


def max_gap(p):
    """K of the connectivity sampler (Appendix C), -1 for p outside (0, 1]."""
    return int(lib().bp_max_gap(float(p)))


def geo_inv_rate(p):
    """1 / -ln(1 - p) in FP64 rounded to FP32: the geometric rule's rate."""
    return float(lib().bp_geo_inv_rate(float(p)))


def hash_words(seed, rng_stream, a, b, k):
    a = _dev(a, torch.int32, "a")
    b = _dev(b, torch.int32, "b")
    k = _dev(k, torch.int32, "k")
    out = torch.empty_like(a)
    check(lib().bp_hash(seed, rng_stream, _p(a), _p(b), _p(k), _p(out), a.numel(), _stream()))
    return out


class JitConn:
    """Fixed-probability connectivity regenerated from a seed.  rule:
    RULE_UNIFORM (the paper's gaps uniform on [1, K]), RULE_GEOMETRIC (exact
    Bernoulli(p): pass p or inv_rate), RULE_FIXED_DEGREE (exactly `degree`
    targets per row, block 0)."""

    def __init__(self, n_pre, n_post, p=None, K=None, block=0, seed=0, wkind=W_HOMO, w0=1.0, w1=0.0,
                 rule=RULE_UNIFORM, inv_rate=None, degree=0):
        if rule == RULE_UNIFORM:
            if K is None:
                K = max_gap(p)
            if K < 1:
                raise ValueError(f"invalid connection probability {p}")
        else:
            K = 1 if K is None else K
        if rule == RULE_GEOMETRIC and inv_rate is None:
            inv_rate = geo_inv_rate(p)
        self.c = _abi.JitConn(n_pre, n_post, K, block, seed, wkind, w0, w1, rule,
                              0.0 if inv_rate is None else inv_rate, degree)

    def __getattr__(self, name):
        return getattr(self.__dict__["c"], name)


def csr_build(conn: JitConn, device="cuda"):
    """(indptr, indices) int32 device tensors of the seeded matrix."""
    c = conn.c
    indptr = torch.empty(c.n_pre + 1, dtype=torch.int32, device=device)
    check(lib().bp_csr_count(C.byref(c), _p(indptr), _stream()))
    nnz = int(indptr[-1].item())
    if nnz < 0:
        raise BpError(_abi.BP_EUNSUPPORTED, "more than 2^31-1 synapses")
    indices = torch.empty(max(nnz, 1), dtype=torch.int32, device=device)
    check(lib().bp_csr_fill(C.byref(c), _p(indptr), _p(indices), _stream()))
    return indptr, indices[:nnz]


def csr_tile_index(indptr, indices, n_post, tile_width):
    n_pre = indptr.numel() - 1
    n_tiles = max(1, -(-n_post // tile_width))
    tp = torch.empty(max(n_pre, 1) * (n_tiles + 1), dtype=torch.int32, device=indptr.device)
    check(lib().bp_csr_tile_index(_p(indptr), _p(indices), n_pre, n_post, tile_width, _p(tp), _stream()))
    return tp


def compact(s):
    s = _dev(s, torch.uint8, "s")
    n = s.numel()
    ids = torch.empty(max(n, 1), dtype=torch.int32, device=s.device)
    count = torch.empty(1, dtype=torch.int32, device=s.device)
    wsb = int(lib().bp_compact_ws_bytes(n))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=s.device)
    check(lib().bp_compact(_p(s), n, _p(ids), _p(count), _p(ws), wsb, _stream()))
    return ids, count


def _csr_struct(indptr, indices, data, w, n_post, tile_ptr=None, tile_width=0, sorted_rows=True):
    n_pre = indptr.numel() - 1
    return _abi.Csr(indptr.data_ptr(), indices.data_ptr() if indices.numel() else None,
                    None if data is None else data.data_ptr(), float(w), n_pre, n_post, int(bool(sorted_rows)),
                    None if tile_ptr is None else tile_ptr.data_ptr(), int(tile_width))


def event_csr_matvec(indptr, indices, data, w, n_post, events, tile_ptr=None, tile_width=0, sorted_rows=True,
                     out=None, ws=None):
    """y = M^T e over the firing rows (Appendix B).  data None: homogeneous w."""
    indptr, indices, data = _csr_args(indptr, indices, data, n_post)
    events = _events(events, indptr.numel() - 1)
    if tile_ptr is not None:
        tile_ptr = _dev(tile_ptr, torch.int32, "tile_ptr")
    m = _csr_struct(indptr, indices, data, w, n_post, tile_ptr, tile_width, sorted_rows)
    y = _out(out, n_post, torch.float32, events.device)
    wsb = int(lib().bp_event_csr_ws_bytes(C.byref(m)))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=events.device)
    check(lib().bp_event_csr_matvec(C.byref(m), _p(events), _p(y), _p(ws), wsb, _stream()))
    return y


def event_csr_matvec_noalloc(indptr, indices, data, w, n_post, events, out, tile_ptr=None, tile_width=0,
                             sorted_rows=True):
    """event_csr_matvec into the caller's `out` with the library's static
    scratch in place of a workspace: allocates nothing (for graph capture and
    callers that cannot allocate).  Calls that overlap on one GPU race."""
    indptr, indices, data = _csr_args(indptr, indices, data, n_post)
    events = _events(events, indptr.numel() - 1)
    if tile_ptr is not None:
        tile_ptr = _dev(tile_ptr, torch.int32, "tile_ptr")
    m = _csr_struct(indptr, indices, data, w, n_post, tile_ptr, tile_width, sorted_rows)
    if out is None:
        raise ValueError("out is required (the call allocates nothing)")
    y = _out(out, n_post, torch.float32, events.device)
    check(lib().bp_event_csr_matvec_noalloc(C.byref(m), _p(events), _p(y), _stream()))
    return y


def csr_matvec_dense(indptr, indices, data, w, n_post, v, tile_ptr=None, tile_width=0, sorted_rows=True, out=None,
                     ws=None):
    """y = M^T v for a dense FP32 vector v and a stored CSR (rows with
    v[j] == 0 skipped)."""
    indptr, indices, data = _csr_args(indptr, indices, data, n_post)
    v = _vec(v, indptr.numel() - 1, torch.float32, "v")
    if tile_ptr is not None:
        tile_ptr = _dev(tile_ptr, torch.int32, "tile_ptr")
    m = _csr_struct(indptr, indices, data, w, n_post, tile_ptr, tile_width, sorted_rows)
    y = _out(out, n_post, torch.float32, v.device)
    wsb = int(lib().bp_csr_matvec_dense_ws_bytes(C.byref(m)))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=v.device)
    check(lib().bp_csr_matvec_dense(C.byref(m), _p(v), _p(y), _p(ws), wsb, _stream()))
    return y


class Projection:
    """A synaptic projection with a `delay`-step spike delay (Section 4.3,
    Appendix D): align ALIGN_POST (state g per postsynaptic neuron) or
    ALIGN_PRE (one trace per presynaptic neuron, g = M^T x); syn SYN_EXP or
    SYN_SAT (AlignPre only).  Connectivity: a stored CSR (indptr, indices,
    data or w) or a JitConn.  Holds the delay line, the state and the
    scratch in device memory."""

    def __init__(self, align, decay, delay=0, depth=None, syn=SYN_EXP, u=0.0, csr=None, jit=None, device="cuda"):
        self._keep = []
        if csr is not None:
            indptr, indices, data, w, n_post = csr
            indptr, indices, data = _csr_args(indptr, indices, data, n_post)
            self._keep += [indptr, indices, data]
            self._csr = _csr_struct(indptr, indices, data, w, n_post)
            self.n_pre, self.n_post, conn = indptr.numel() - 1, n_post, CONN_CSR
            cp, jp = C.pointer(self._csr), None
        else:
            self._jit = jit.c
            self.n_pre, self.n_post, conn = jit.n_pre, jit.n_post, CONN_JIT
            cp, jp = None, C.pointer(self._jit)
        self.depth = int(depth if depth is not None else delay + 1)
        self.p = _abi.Proj(align, syn, conn, cp, jp, int(delay), float(decay), float(u))
        self.ring = torch.zeros(max(self.depth * self.n_pre, 1), dtype=torch.uint8, device=device)
        self.state = torch.zeros(max(self.n_post if align == ALIGN_POST else self.n_pre, 1), dtype=torch.float32,
                                 device=device)
        wsb = int(lib().bp_proj_ws_bytes(C.byref(self.p)))
        self.ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=device)
        self.wsb = wsb
        self.t = 0

    def run(self, raster, g_out=None):
        """Steps driven by a presynaptic raster [T, n_pre] (CUDA uint8);
        returns g [T, n_post]."""
        raster = _dev(raster, torch.uint8, "raster")
        if raster.dim() != 2 or raster.shape[1] != self.n_pre:
            raise ValueError(f"raster must be [T, {self.n_pre}]")
        T = int(raster.shape[0])
        g = g_out if g_out is not None else torch.empty((T, self.n_post), dtype=torch.float32, device=raster.device)
        check(lib().bp_proj_run(C.byref(self.p), _p(raster), T, _p(self.ring), self.depth, self.t, _p(self.state),
                                _p(g), _p(self.ws), self.wsb, _stream()))
        self.t += T
        return g


def event_csr_ws(indptr, indices, data, w, n_post, tile_ptr=None, tile_width=0, sorted_rows=True):
    m = _csr_struct(indptr, indices, data, w, n_post, tile_ptr, tile_width, sorted_rows)
    return int(lib().bp_event_csr_ws_bytes(C.byref(m)))


def _spike_matrix(E, n, name="events"):
    """A batch of spike vectors for the kernels: a CUDA uint8 (or bool) matrix
    [batch, n] whose rows are contiguous (any row stride >= n); returns the
    byte view and its row stride."""
    if not isinstance(E, torch.Tensor) or not E.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if E.dtype == torch.bool:
        E = E.view(torch.uint8)
    if E.dtype != torch.uint8:
        raise TypeError(f"{name} must be uint8 or bool (one byte per neuron), got {E.dtype}")
    if E.dim() != 2 or E.shape[1] != n:
        raise ValueError(f"{name} must be [batch, {n}], got {tuple(E.shape)}")
    if E.shape[0] > 0 and (E.stride(1) != 1 or E.stride(0) < n):
        E = E.contiguous()
    return E, (E.stride(0) if E.shape[0] > 0 else n)


def _out_matrix(out, batch, n, device):
    if out is None:
        Y = torch.empty((batch, n), dtype=torch.float32, device=device)
    else:
        Y = out
        if not isinstance(Y, torch.Tensor) or not Y.is_cuda or Y.dtype != torch.float32 or Y.dim() != 2 \
                or tuple(Y.shape) != (batch, n) or (batch > 0 and (Y.stride(1) != 1 or Y.stride(0) < n)):
            raise ValueError(f"out must be a CUDA float32 [batch, {n}] matrix with contiguous rows")
    return Y, (Y.stride(0) if batch > 0 else n)


def event_csr_matmat(indptr, indices, data, w, n_post, E, tile_ptr=None, tile_width=0, out=None, ws=None):
    """Y[b] = M^T E[b] for a batch of spike vectors E [batch, n_pre] (rows may
    be strided); each firing row is streamed once per group of up to eight
    vectors (sorted rows)."""
    indptr, indices, data = _csr_args(indptr, indices, data, n_post)
    E, ev_stride = _spike_matrix(E, indptr.numel() - 1)
    if tile_ptr is not None:
        tile_ptr = _dev(tile_ptr, torch.int32, "tile_ptr")
    m = _csr_struct(indptr, indices, data, w, n_post, tile_ptr, tile_width, True)
    batch = int(E.shape[0])
    Y, y_stride = _out_matrix(out, batch, n_post, E.device)
    wsb = int(lib().bp_event_csr_matmat_ws_bytes(C.byref(m), batch))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=E.device)
    check(lib().bp_event_csr_matmat(C.byref(m), _p(E), batch, ev_stride, _p(Y), y_stride, _p(ws), wsb, _stream()))
    return Y


def jit_conn_matmat(conn: JitConn, E, out=None, ws=None):
    """Y[b] = M^T E[b] for a batch of spike vectors with M regenerated from
    the seed; each firing (row, block) is generated once per group of up to
    eight vectors."""
    c = conn.c
    E, ev_stride = _spike_matrix(E, c.n_pre)
    batch = int(E.shape[0])
    Y, y_stride = _out_matrix(out, batch, c.n_post, E.device)
    wsb = int(lib().bp_jit_conn_matmat_ws_bytes(C.byref(c), batch))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=E.device)
    check(lib().bp_jit_conn_matmat(C.byref(c), _p(E), batch, ev_stride, _p(Y), y_stride, _p(ws), wsb, _stream()))
    return Y


def event_csr_matmat_ws(indptr, indices, data, w, n_post, batch, tile_ptr=None, tile_width=0):
    m = _csr_struct(indptr, indices, data, w, n_post, tile_ptr, tile_width, True)
    return int(lib().bp_event_csr_matmat_ws_bytes(C.byref(m), batch))


def jit_conn_matmat_ws(conn: JitConn, batch):
    return int(lib().bp_jit_conn_matmat_ws_bytes(C.byref(conn.c), batch))


def jit_conn_matvec(conn: JitConn, events, out=None, ws=None):
    """y = M^T e with M regenerated from the seed (Appendix C)."""
    c = conn.c
    events = _events(events, c.n_pre)
    y = _out(out, c.n_post, torch.float32, events.device)
    wsb = int(lib().bp_jit_ws_bytes(C.byref(c)))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=events.device)
    check(lib().bp_jit_conn_matvec(C.byref(c), _p(events), _p(y), _p(ws), wsb, _stream()))
    return y


def jit_conn_matvec_dense(conn: JitConn, v, out=None, ws=None):
    """y = J^T v for a dense FP32 vector v with J regenerated from the seed
    (Section 5.2's JIT operator; rows with v[j] == 0 are skipped)."""
    c = conn.c
    _dev(v, torch.float32, "v")
    if v.numel() != c.n_pre or not v.is_contiguous():
        raise ValueError(f"v must be a contiguous float32 vector of {c.n_pre} entries")
    y = _out(out, c.n_post, torch.float32, v.device)
    wsb = int(lib().bp_jit_dense_ws_bytes(C.byref(c)))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=v.device)
    check(lib().bp_jit_conn_matvec_dense(C.byref(c), _p(v), _p(y), _p(ws), wsb, _stream()))
    return y


def jit_conn_matmat_dense(conn: JitConn, X, out=None, ws=None):
    """Y = J^T X for a contiguous FP32 matrix X [n_pre, m] (m float vectors
    at once); Y is [n_post, m]."""
    c = conn.c
    _dev(X, torch.float32, "X")
    if X.dim() != 2 or X.shape[0] != c.n_pre or not X.is_contiguous():
        raise ValueError(f"X must be a contiguous float32 matrix with {c.n_pre} rows")
    m = int(X.shape[1])
    Y = out if out is not None else torch.empty((c.n_post, m), dtype=torch.float32, device=X.device)
    wsb = int(lib().bp_jit_matmat_ws_bytes(C.byref(c), m))
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=X.device)
    check(lib().bp_jit_conn_matmat_dense(C.byref(c), _p(X), m, _p(Y), _p(ws), wsb, _stream()))
    return Y


def jit_matmat_ws(conn: JitConn, m):
    return int(lib().bp_jit_matmat_ws_bytes(C.byref(conn.c), m))


def jit_dense_ws(conn: JitConn):
    return int(lib().bp_jit_dense_ws_bytes(C.byref(conn.c)))


def jit_ws(conn: JitConn):
    return int(lib().bp_jit_ws_bytes(C.byref(conn.c)))


def event_csr_backward(indptr, indices, data, w, n_post, events, dy, want_events=True, want_data=True,
                       want_w=True):
    indptr, indices, data = _csr_args(indptr, indices, data, n_post)
    events = _events(events, indptr.numel() - 1)
    dy = _vec(dy, n_post, torch.float32, "dy")
    m = _csr_struct(indptr, indices, data, w, n_post)
    dev = events.device
    d_ev = torch.empty(indptr.numel() - 1, dtype=torch.float32, device=dev) if want_events else None
    d_data = torch.empty(max(indices.numel(), 1), dtype=torch.float32, device=dev) if want_data else None
    d_w = torch.empty(1, dtype=torch.float32, device=dev) if want_w else None
    check(lib().bp_event_csr_backward(C.byref(m), _p(events), _p(dy), _p(d_ev), _p(d_data), _p(d_w), _stream()))
    if d_data is not None:
        d_data = d_data[:indices.numel()]
    return d_ev, d_data, d_w


def jit_conn_backward(conn: JitConn, events, dy, want_events=True, want_w=True):
    c = conn.c
    events = _events(events, c.n_pre)
    dy = _vec(dy, c.n_post, torch.float32, "dy")
    dev = events.device
    d_ev = torch.empty(c.n_pre, dtype=torch.float32, device=dev) if want_events else None
    d_w = torch.empty(2, dtype=torch.float32, device=dev) if want_w else None
    check(lib().bp_jit_conn_backward(C.byref(c), _p(events), _p(dy), _p(d_ev), _p(d_w), _stream()))
    return d_ev, d_w


# ------------------------------------------------------------------ network
COBA_DEFAULTS = dict(w_exc=0.6, w_inh=6.7, tau_m=20.0, tau_e=5.0, tau_i=10.0, tau_ref=5.0, v_rest=-60.0,
                     v_th=-50.0, v_reset=-60.0, e_exc=0.0, e_inh=-80.0, r=1.0, i_ext=20.0, dt=0.1,
                     v0_lo=-60.0, v0_hi=-50.0)


def net_desc(n, n_exc=None, p=None, K=None, conn=CONN_JIT, block=0, seed=0, model=COBA, max_wgs=0,
             rule=RULE_UNIFORM, degree=0, inv_rate=None, **params):
    kw = dict(COBA_DEFAULTS)
    kw.update(params)
    if n_exc is None:
        n_exc = int(math.floor(0.8 * n))
    pp = p if p is not None else 80.0 / n
    if K is None:
        K = max_gap(pp)
    if rule == RULE_GEOMETRIC and inv_rate is None:
        inv_rate = geo_inv_rate(pp)
    return _abi.NetDesc(model=model, n=n, n_exc=n_exc, conn=conn, max_gap=K, block=block, seed=seed,
                        max_wgs=max_wgs, rule=rule, geo_inv_rate=0.0 if inv_rate is None else inv_rate,
                        degree=degree, **kw)


def net_bytes(desc):
    b = C.c_size_t(0)
    check(lib().bp_net_bytes(C.byref(desc), C.byref(b)))
    return int(b.value)


def net_workgroups(desc):
    w = C.c_int32(0)
    check(lib().bp_net_workgroups(C.byref(desc), C.byref(w)))
    return int(w.value)


class Net:
    """An E/I LIF network resident in a caller-owned device workspace."""

    def __init__(self, desc, device="cuda", workspace=None):
        self.desc = desc
        nbytes = net_bytes(desc)
        self.ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8, device=device)
        if self.ws.numel() < nbytes:
            raise BpError(_abi.BP_ENOMEM, f"workspace {self.ws.numel()} < {nbytes} bytes")
        h = C.c_void_p()
        check(lib().bp_create_net(C.byref(desc), _p(self.ws), self.ws.numel(), _stream(), C.byref(h)))
        self.h = h
        self.device = self.ws.device

    @property
    def n(self):
        return self.desc.n

    def info(self):
        i = _abi.NetInfo()
        check(lib().bp_net_get_info(self.h, C.byref(i)))
        return i

    def run(self, n_steps, raster=False, counts=True, i_ext=None, counts_out=None):
        """n_steps steps in one launch; returns (raster or None, counts or
        None).  counts_out: a caller-allocated int32 buffer of >= n_steps
        entries to write the per-step spike counts into (nothing allocated)."""
        if i_ext is not None:
            i_ext = _vec(i_ext, self.n, torch.float32, "i_ext")
        r = torch.empty((n_steps, self.n), dtype=torch.uint8, device=self.device) if raster else None
        if counts_out is not None:
            c = _dev(counts_out, torch.int32, "counts_out")
            if c.numel() < n_steps or c.data_ptr() != counts_out.data_ptr():
                raise ValueError(f"counts_out must be a contiguous int32 buffer of >= {n_steps} entries")
        else:
            c = torch.empty(max(n_steps, 1), dtype=torch.int32, device=self.device) if counts else None
        check(lib().bp_run(self.h, n_steps, _p(i_ext), _p(r), _p(c), _stream()))
        return r, (c[:n_steps] if c is not None else None)

    def step(self, i_ext=None):
        if i_ext is not None:
            i_ext = _vec(i_ext, self.n, torch.float32, "i_ext")
        s = torch.empty(self.n, dtype=torch.uint8, device=self.device)
        check(lib().bp_step(self.h, _p(i_ext), _p(s), _stream()))
        return s

    def events(self, out=None):
        """Synaptic events delivered since creation (device int64[1])."""
        out = _out(out, 1, torch.int64, self.device)
        check(lib().bp_net_events(self.h, _p(out), _stream()))
        return out

    def error_flag(self):
        """Device error word of the net (non-zero: a run gave up waiting)."""
        off = self.info().error_dev - self.ws.data_ptr()
        return int(self.ws[off:off + 4].view(torch.int32).item())

    def get_state(self):
        nb = int(lib().bp_state_bytes(self.h))
        buf = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(lib().bp_get_state(self.h, _p(buf), nb, _stream()))
        n = self.n
        return dict(V=buf[0:4 * n].view(torch.float32), ge=buf[4 * n:8 * n].view(torch.float32),
                    gi=buf[8 * n:12 * n].view(torch.float32), ref=buf[12 * n:16 * n].view(torch.int32),
                    s_prev=buf[16 * n:17 * n], raw=buf, step=self.info().step)

    def set_state(self, raw, step):
        raw = _dev(raw, torch.uint8, "raw")
        nb = int(lib().bp_state_bytes(self.h))
        if raw.numel() < nb:
            raise ValueError(f"raw state has {raw.numel()} bytes, expected {nb}")
        check(lib().bp_set_state(self.h, _p(raw), raw.numel(), int(step), _stream()))

    def close(self):
        if getattr(self, "h", None):
            lib().bp_destroy_net(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batch(nets, n_steps, counts=None):
    """Advance several nets concurrently in one launch (continuous batching)."""
    k = len(nets)
    arr = (C.c_void_p * k)(*[n.h.value for n in nets])
    st = (C.c_int64 * k)(*[int(s) for s in n_steps])
    cp = None
    if counts is not None:
        cp = (C.c_void_p * k)(*[None if c is None else c.data_ptr() for c in counts])
    check(lib().bp_run_batch(arr, k, st, cp, _stream()))
