"""ctypes view of the C ABI declared in include/bp.h (libbpmi.so)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpmi.so")

BP_OK, BP_EINVAL, BP_ENOMEM, BP_EDEVICE, BP_ESTATE, BP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATIC_SCRATCH_BYTES = 16 << 20  # BP_STATIC_SCRATCH_BYTES
W_HOMO, W_NORMAL, W_UNIFORM = 0, 1, 2
STREAM_CONN, STREAM_W, STREAM_V0 = 1, 2, 3
COBA, CUBA = 0, 1
CONN_CSR, CONN_JIT = 0, 1
RULE_UNIFORM, RULE_GEOMETRIC, RULE_FIXED_DEGREE = 0, 1, 2
ALIGN_POST, ALIGN_PRE = 0, 1
SYN_EXP, SYN_SAT = 0, 1


class JitConn(C.Structure):
    _fields_ = [("n_pre", C.c_int32), ("n_post", C.c_int32), ("max_gap", C.c_int32), ("block", C.c_int32),
                ("seed", C.c_uint64), ("wkind", C.c_int32), ("w0", C.c_float), ("w1", C.c_float),
                ("rule", C.c_int32), ("geo_inv_rate", C.c_float), ("degree", C.c_int32)]


class Csr(C.Structure):
    _fields_ = [("indptr", C.c_void_p), ("indices", C.c_void_p), ("data", C.c_void_p), ("w", C.c_float),
                ("n_pre", C.c_int32), ("n_post", C.c_int32), ("sorted", C.c_int32), ("tile_ptr", C.c_void_p),
                ("tile_width", C.c_int32)]


class Proj(C.Structure):
    _fields_ = [("align", C.c_int32), ("syn", C.c_int32), ("conn", C.c_int32), ("csr", C.POINTER(Csr)),
                ("jit", C.POINTER(JitConn)), ("delay", C.c_int32), ("decay", C.c_float), ("u", C.c_float)]


class NetDesc(C.Structure):
    _fields_ = [("model", C.c_int32), ("n", C.c_int32), ("n_exc", C.c_int32), ("conn", C.c_int32),
                ("max_gap", C.c_int32), ("block", C.c_int32), ("seed", C.c_uint64),
                ("w_exc", C.c_float), ("w_inh", C.c_float), ("tau_m", C.c_float), ("tau_e", C.c_float),
                ("tau_i", C.c_float), ("tau_ref", C.c_float), ("v_rest", C.c_float), ("v_th", C.c_float),
                ("v_reset", C.c_float), ("e_exc", C.c_float), ("e_inh", C.c_float), ("r", C.c_float),
                ("i_ext", C.c_float), ("dt", C.c_float), ("v0_lo", C.c_float), ("v0_hi", C.c_float),
                ("max_wgs", C.c_int32), ("rule", C.c_int32), ("geo_inv_rate", C.c_float), ("degree", C.c_int32)]


class NetInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_wg", C.c_int32), ("wg_range", C.c_int32), ("nnz", C.c_int64),
                ("step", C.c_int64), ("bytes_used", C.c_size_t), ("events_dev", C.c_void_p),
                ("error_dev", C.c_void_p)]


class Snn(C.Structure):
    _fields_ = [("B", C.c_int32), ("C", C.c_int32), ("N", C.c_int32), ("O", C.c_int32), ("T", C.c_int32),
                ("nnz", C.c_int32), ("surrogate", C.c_int32), ("detach_reset", C.c_int32), ("ckpt_every", C.c_int32),
                ("alpha", C.c_float), ("beta", C.c_float), ("theta", C.c_float), ("slope", C.c_float),
                ("relu_a", C.c_float), ("relu_width", C.c_float),
                ("x", C.c_void_p), ("labels", C.c_void_p), ("W_in", C.c_void_p), ("indptr", C.c_void_p),
                ("indices", C.c_void_p), ("w_rec", C.c_void_p), ("W_out", C.c_void_p), ("b_out", C.c_void_p)]


_vp, _i32, _i64, _u32, _u64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_size_t

# name -> (restype, argtypes); every function declared in include/bp.h
SIGNATURES = {
    "bp_last_error": (C.c_char_p, []),
    "bp_version": (C.c_char_p, []),
    "bp_max_gap": (_i32, [C.c_double]),
    "bp_geo_inv_rate": (C.c_float, [C.c_double]),
    "bp_hash": (_i32, [_u64, _u32, _vp, _vp, _vp, _vp, _i64, _vp]),
    "bp_csr_count": (_i32, [C.POINTER(JitConn), _vp, _vp]),
    "bp_csr_fill": (_i32, [C.POINTER(JitConn), _vp, _vp, _vp]),
    "bp_compact_ws_bytes": (_sz, [_i32]),
    "bp_compact": (_i32, [_vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "bp_csr_tile_index": (_i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "bp_event_csr_ws_bytes": (_sz, [C.POINTER(Csr)]),
    "bp_event_csr_matvec": (_i32, [C.POINTER(Csr), _vp, _vp, _vp, _sz, _vp]),
    "bp_event_csr_matvec_noalloc": (_i32, [C.POINTER(Csr), _vp, _vp, _vp]),
    "bp_event_csr_backward": (_i32, [C.POINTER(Csr), _vp, _vp, _vp, _vp, _vp, _vp]),
    "bp_event_csr_matmat_ws_bytes": (_sz, [C.POINTER(Csr), _i32]),
    "bp_event_csr_matmat": (_i32, [C.POINTER(Csr), _vp, _i32, _i64, _vp, _i64, _vp, _sz, _vp]),
    "bp_jit_conn_matmat_ws_bytes": (_sz, [C.POINTER(JitConn), _i32]),
    "bp_jit_conn_matmat": (_i32, [C.POINTER(JitConn), _vp, _i32, _i64, _vp, _i64, _vp, _sz, _vp]),
    "bp_csr_matvec_dense_ws_bytes": (_sz, [C.POINTER(Csr)]),
    "bp_csr_matvec_dense": (_i32, [C.POINTER(Csr), _vp, _vp, _vp, _sz, _vp]),
    "bp_delay_push": (_i32, [_vp, _i32, _i32, _i64, _vp, _vp]),
    "bp_proj_ws_bytes": (_sz, [C.POINTER(Proj)]),
    "bp_proj_step": (_i32, [C.POINTER(Proj), _vp, _i32, _i64, _vp, _vp, _vp, _sz, _vp]),
    "bp_proj_run": (_i32, [C.POINTER(Proj), _vp, _i32, _vp, _i32, _i64, _vp, _vp, _vp, _sz, _vp]),
    "bp_jit_ws_bytes": (_sz, [C.POINTER(JitConn)]),
    "bp_jit_conn_matvec": (_i32, [C.POINTER(JitConn), _vp, _vp, _vp, _sz, _vp]),
    "bp_jit_dense_ws_bytes": (_sz, [C.POINTER(JitConn)]),
    "bp_jit_conn_matvec_dense": (_i32, [C.POINTER(JitConn), _vp, _vp, _vp, _sz, _vp]),
    "bp_jit_matmat_ws_bytes": (_sz, [C.POINTER(JitConn), _i32]),
    "bp_jit_conn_matmat_dense": (_i32, [C.POINTER(JitConn), _vp, _i32, _vp, _vp, _sz, _vp]),
    "bp_jit_conn_backward": (_i32, [C.POINTER(JitConn), _vp, _vp, _vp, _vp, _vp]),
    "bp_backward": (_i32, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bp_net_bytes": (_i32, [C.POINTER(NetDesc), C.POINTER(_sz)]),
    "bp_net_workgroups": (_i32, [C.POINTER(NetDesc), C.POINTER(_i32)]),
    "bp_create_net": (_i32, [C.POINTER(NetDesc), _vp, _sz, _vp, C.POINTER(_vp)]),
    "bp_run": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "bp_step": (_i32, [_vp, _vp, _vp, _vp]),
    "bp_run_batch": (_i32, [C.POINTER(_vp), _i32, C.POINTER(_i64), C.POINTER(_vp), _vp]),
    "bp_net_get_info": (_i32, [_vp, C.POINTER(NetInfo)]),
    "bp_net_events": (_i32, [_vp, _vp, _vp]),
    "bp_state_bytes": (_sz, [_vp]),
    "bp_get_state": (_i32, [_vp, _vp, _sz, _vp]),
    "bp_set_state": (_i32, [_vp, _vp, _sz, _i64, _vp]),
    "bp_destroy_net": (_i32, [_vp]),
    "bp_snn_ckpt_bytes": (_sz, [C.POINTER(Snn)]),
    "bp_snn_ws_bytes": (_sz, [C.POINTER(Snn)]),
    "bp_snn_forward": (_i32, [C.POINTER(Snn), _vp, _vp, _vp, _vp, _vp]),
    "bp_snn_backward": (_i32, [C.POINTER(Snn), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
}

_lib = None


class BpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bp error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2311_05106_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != BP_OK:
        raise BpError(code, lib().bp_last_error().decode())
    return code
