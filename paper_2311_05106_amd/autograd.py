"""torch.autograd.Function wrappers over the C ABI (Section 4.1: every
dedicated operator has a reverse mode).  Forward and backward both run in the
library's kernels; torch provides tensors and the autograd tape."""
import ctypes as C

import torch

from . import _abi
from . import JitConn, _p, _stream, check, event_csr_backward, event_csr_matvec, jit_conn_backward, \
    jit_conn_matvec, jit_conn_matvec_dense, lib


class EventCSRMatvec(torch.autograd.Function):
    """y = M^T e over firing rows; gradients for the event values (as reals)
    and the CSR data."""

    @staticmethod
    def forward(ctx, events, data, indptr, indices, n_post, w=1.0):
        ev = events
        y = event_csr_matvec(indptr, indices, data, w, n_post, ev)
        ctx.save_for_backward(ev, data, indptr, indices)
        ctx.n_post, ctx.w = n_post, w
        return y

    @staticmethod
    def backward(ctx, dy):
        ev, data, indptr, indices = ctx.saved_tensors
        d_ev, d_data, _ = event_csr_backward(indptr, indices, data, ctx.w, ctx.n_post, ev, dy.contiguous(),
                                             want_events=True, want_data=data is not None, want_w=False)
        return d_ev, d_data, None, None, None, None


class JitConnMatvec(torch.autograd.Function):
    """y = M^T e with M regenerated from the seed; gradients for the event
    values and the two weight parameters w01 = (w0, w1).

    The kernels take the weight parameters by value, so they are read on the
    host: pass w01 as a CPU tensor to keep the call free of device syncs
    (a device tensor costs one device-to-host copy per call).  The caller's
    JitConn is not modified; its w0 and w1 are ignored."""

    @staticmethod
    def forward(ctx, events, w01, conn: JitConn):
        w = w01.detach().to("cpu", torch.float64)
        c = conn.c
        local = JitConn(c.n_pre, c.n_post, K=c.max_gap, block=c.block, seed=c.seed, wkind=c.wkind,
                        w0=float(w[0]), w1=float(w[1]))
        y = jit_conn_matvec(local, events)
        ctx.save_for_backward(events)
        ctx.conn = local
        ctx.w_device = w01.device
        return y

    @staticmethod
    def backward(ctx, dy):
        (ev,) = ctx.saved_tensors
        d_ev, d_w = jit_conn_backward(ctx.conn, ev, dy.contiguous())
        return d_ev, d_w.to(ctx.w_device), None


class JitConnMatvecDense(torch.autograd.Function):
    """y = J^T v for a dense float vector v (Section 5.2's JIT operator);
    gradient for v: dv[j] = sum over row j of w_jk dy[k], the row-wise
    product of the reverse mode, for every row.  The weights' parameters
    get no gradient here."""

    @staticmethod
    def forward(ctx, v, conn: JitConn):
        ctx.conn = conn
        return jit_conn_matvec_dense(conn, v.contiguous())

    @staticmethod
    def backward(ctx, dy):
        c = ctx.conn.c
        # the row-wise products do not depend on the spike vector; an all-zero
        # one also skips the (w0, w1) sums
        ev = torch.zeros(max(c.n_pre, 1), dtype=torch.uint8, device=dy.device)
        d_v, _ = jit_conn_backward(ctx.conn, ev, dy.contiguous(), want_w=False)
        return d_v, None


class SNN:
    """Recurrent LIF network of the BPTT workload: B samples, C input
    channels, N neurons with a sparse recurrent CSR, O readout classes."""

    def __init__(self, B, C_, N, O, T, indptr, indices, alpha, beta, theta=1.0, slope=4.0, surrogate=0,
                 detach_reset=1, ckpt_every=50, relu_a=0.3, relu_width=1.0):
        self.B, self.C, self.N, self.O, self.T = B, C_, N, O, T
        self.indptr, self.indices = indptr, indices
        self.nnz = int(indices.numel())
        self.cfg = dict(surrogate=surrogate, detach_reset=detach_reset, ckpt_every=ckpt_every, alpha=alpha,
                        beta=beta, theta=theta, slope=slope, relu_a=relu_a, relu_width=relu_width)

    def _desc(self, x, labels, W_in, w_rec, W_out, b_out):
        c = self.cfg
        return _abi.Snn(self.B, self.C, self.N, self.O, self.T, self.nnz, c["surrogate"], c["detach_reset"],
                        c["ckpt_every"], c["alpha"], c["beta"], c["theta"], c["slope"], c["relu_a"],
                        c["relu_width"], x.data_ptr(), labels.data_ptr(), W_in.data_ptr(), self.indptr.data_ptr(),
                        self.indices.data_ptr() if self.nnz else None, w_rec.data_ptr() if self.nnz else None,
                        W_out.data_ptr(), b_out.data_ptr())

    def forward(self, x, labels, W_in, w_rec, W_out, b_out, want_raster=False):
        d = self._desc(x, labels, W_in, w_rec, W_out, b_out)
        dev = x.device
        ck = torch.empty(max(int(lib().bp_snn_ckpt_bytes(C.byref(d))), 1), dtype=torch.uint8, device=dev)
        logits = torch.empty((self.B, self.O), dtype=torch.float32, device=dev)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        raster = torch.empty((self.T, self.B, self.N), dtype=torch.uint8, device=dev) if want_raster else None
        check(lib().bp_snn_forward(C.byref(d), _p(ck), _p(logits), _p(loss), _p(raster), _stream()))
        return dict(ckpt=ck, logits=logits, loss=loss, raster=raster)

    def backward(self, fwd, x, labels, W_in, w_rec, W_out, b_out, ws=None):
        d = self._desc(x, labels, W_in, w_rec, W_out, b_out)
        dev = x.device
        wsb = int(lib().bp_snn_ws_bytes(C.byref(d)))
        if ws is None or ws.numel() < wsb:
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        g = dict(dW_in=torch.empty_like(W_in), dw_rec=torch.empty_like(w_rec), dW_out=torch.empty_like(W_out),
                 db_out=torch.empty_like(b_out))
        check(lib().bp_snn_backward(C.byref(d), _p(fwd["ckpt"]), _p(fwd["logits"]), _p(g["dW_in"]),
                                    _p(g["dw_rec"]) if self.nnz else None, _p(g["dW_out"]), _p(g["db_out"]),
                                    _p(ws), wsb, _stream()))
        return g


class SnnLoss(torch.autograd.Function):
    """Mean cross-entropy of the recurrent LIF network; differentiable in
    (W_in, w_rec, W_out, b_out) through the checkpointed BPTT kernels."""

    @staticmethod
    def forward(ctx, W_in, w_rec, W_out, b_out, model: SNN, x, labels):
        fwd = model.forward(x, labels, W_in, w_rec, W_out, b_out)
        ctx.model, ctx.fwd = model, fwd
        ctx.save_for_backward(x, labels, W_in, w_rec, W_out, b_out)
        return fwd["loss"][0].clone()

    @staticmethod
    def backward(ctx, gloss):
        x, labels, W_in, w_rec, W_out, b_out = ctx.saved_tensors
        g = ctx.model.backward(ctx.fwd, x, labels, W_in, w_rec, W_out, b_out)
        s = gloss
        return g["dW_in"] * s, g["dw_rec"] * s, g["dW_out"] * s, g["db_out"] * s, None, None, None
