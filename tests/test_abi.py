"""The C-ABI library loads and exports every function include/bp.h declares
(CPU only: no compute call)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(bp_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_named_entry_points():
    names = declared_functions()
    for required in ("bp_create_net", "bp_step", "bp_run", "bp_event_csr_matvec", "bp_jit_conn_matvec",
                     "bp_backward", "bp_run_batch", "bp_compact", "bp_csr_count", "bp_csr_fill", "bp_hash"):
        assert required in names


def test_library_exports_every_declared_function():
    from paper_2311_05106_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libbpmi.so is not built (run __graft_entry__.build())")
    lib = _abi.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, f"binding lacks a signature for {name}"


def test_host_only_entry_points():
    import paper_2311_05106_amd as bp
    import oracle as O
    for p in (0.02, 0.01, 2e-4, 0.1, 1.0, 80 / 12345, 0.3, 1e-6):
        assert bp.max_gap(p) == O.max_gap(p)
    assert bp.max_gap(0.0) == -1 and bp.max_gap(2.0) == -1


def test_argument_errors_are_reported_before_launch():
    import ctypes as C
    import paper_2311_05106_amd as bp
    from paper_2311_05106_amd import _abi
    L = _abi.lib()
    d = bp.net_desc(1000, p=0.02)
    d.n = 0
    b = C.c_size_t(0)
    assert L.bp_net_bytes(C.byref(d), C.byref(b)) == _abi.BP_EINVAL
    assert b"n must be" in L.bp_last_error()
    d = bp.net_desc(1000, p=0.02)
    d.n_exc = 2000
    assert L.bp_net_bytes(C.byref(d), C.byref(b)) == _abi.BP_EINVAL
    d = bp.net_desc(1000, p=0.02)
    assert L.bp_net_bytes(C.byref(d), C.byref(b)) == _abi.BP_OK and b.value > 0
    h = C.c_void_p()
    # workspace smaller than bp_net_bytes -> BP_ENOMEM without touching the device
    assert L.bp_create_net(C.byref(d), C.c_void_p(0x1000), b.value - 1, None, C.byref(h)) == _abi.BP_ENOMEM
    c = _abi.JitConn(10, 10, 0, 0, 1, 0, 1.0, 0.0)
    assert L.bp_csr_count(C.byref(c), C.c_void_p(0x1000), None) == _abi.BP_EINVAL
    assert L.bp_run(None, 1, None, None, None, None) == _abi.BP_ESTATE


def test_dense_vector_products_check_arguments_before_launch():
    import ctypes as C
    from paper_2311_05106_amd import _abi
    L = _abi.lib()
    bad = _abi.JitConn(10, 10, 0, 0, 1, 0, 1.0, 0.0)  # K = 0
    ok = _abi.JitConn(10, 20, 5, 0, 1, 0, 1.0, 0.0)
    p = C.c_void_p(0x1000)
    assert L.bp_jit_conn_matvec_dense(C.byref(bad), p, p, None, 0, None) == _abi.BP_EINVAL
    assert L.bp_jit_conn_matvec_dense(C.byref(ok), p, None, None, 0, None) == _abi.BP_EINVAL
    assert L.bp_jit_conn_matvec_dense(C.byref(ok), None, p, None, 0, None) == _abi.BP_EINVAL
    assert L.bp_jit_conn_matmat_dense(C.byref(bad), p, 4, p, None, 0, None) == _abi.BP_EINVAL
    assert L.bp_jit_conn_matmat_dense(C.byref(ok), p, -1, p, None, 0, None) == _abi.BP_EINVAL
    assert L.bp_jit_conn_matmat_dense(C.byref(ok), p, 4, None, None, 0, None) == _abi.BP_EINVAL
    assert L.bp_jit_conn_matmat_dense(C.byref(ok), None, 4, p, None, 0, None) == _abi.BP_EINVAL
    big = _abi.JitConn(10, 1 << 20, 5, 0, 1, 0, 1.0, 0.0)
    assert L.bp_jit_conn_matmat_dense(C.byref(big), p, 1 << 12, p, None, 0, None) == _abi.BP_EINVAL
    assert b"2^31" in L.bp_last_error()
    # nothing to compute: success without a launch
    assert L.bp_jit_conn_matmat_dense(C.byref(ok), p, 0, p, None, 0, None) == _abi.BP_OK
    assert L.bp_jit_matmat_ws_bytes(C.byref(ok), 0) == 0


def test_net_bytes_scales_linearly_for_jit():
    # JIT connectivity stores no synapses (Section 5.2): at a fixed workgroup
    # count (fixed exchange buffers) each extra neuron costs only its state
    # and spike-record slots, not its p*N = 80 synapses (320 B if stored).
    import paper_2311_05106_amd as bp
    from paper_2311_05106_amd import _abi
    desc = {n: bp.net_desc(n, p=80.0 / n, conn=_abi.CONN_JIT, block=1024, max_wgs=256)
            for n in (400_000, 800_000)}
    assert bp.net_workgroups(desc[400_000]) == bp.net_workgroups(desc[800_000])
    size = {n: bp.net_bytes(d) for n, d in desc.items()}
    marginal = (size[800_000] - size[400_000]) / 400_000
    assert marginal < 40
    assert size[800_000] / 800_000 < 50


def test_binding_rejects_bad_tensors_before_launch():
    # host tensors, wrong dtypes and wrong lengths are refused by the binding
    # before any pointer reaches a kernel (a host pointer in a kernel would
    # fault the GPU; a float spike vector would be read as bytes)
    import torch
    import paper_2311_05106_amd as bp
    ip = torch.zeros(11, dtype=torch.int32)
    ix = torch.zeros(0, dtype=torch.int32)
    ev = torch.zeros(10, dtype=torch.uint8)
    with pytest.raises(TypeError):
        bp.event_csr_matvec(ip, ix, None, 1.0, 5, ev)
    c = bp.JitConn(10, 20, K=5, seed=1)
    with pytest.raises(TypeError):
        bp.jit_conn_matvec(c, ev)
    with pytest.raises(TypeError):
        bp.jit_conn_backward(c, ev, torch.zeros(20))
    with pytest.raises(TypeError):
        bp.event_csr_backward(ip, ix, None, 1.0, 5, ev, torch.zeros(5))
    with pytest.raises(TypeError):
        bp.jit_conn_matvec_dense(c, torch.zeros(10))


def test_destroyed_net_handle_is_rejected():
    # a handle that was never created (or was destroyed) is refused without
    # being read
    import ctypes as C
    from paper_2311_05106_amd import _abi
    L = _abi.lib()
    fake = C.c_void_p(0x10)
    assert L.bp_destroy_net(fake) == _abi.BP_ESTATE
    assert L.bp_destroy_net(None) == _abi.BP_ESTATE
    assert L.bp_run(fake, 1, None, None, None, None) == _abi.BP_ESTATE
    assert b"destroyed" in L.bp_last_error()


def test_noalloc_product_rejects_scratch_beyond_its_static_array():
    # the allocation-free event product checks the scratch it needs against
    # the static array before any device work: an unsorted CSR wider than one
    # LDS tile needs n_post x 4 bytes of device-atomic accumulators
    import ctypes as C
    from paper_2311_05106_amd import _abi
    L = _abi.lib()
    fake = C.c_void_p(0x1000)
    n_post = 5_000_000
    m = _abi.Csr(0x1000, 0x1000, 0x1000, 0.0, 10, n_post, 0, None, 0)
    assert L.bp_event_csr_ws_bytes(C.byref(m)) == 4 * n_post > _abi.STATIC_SCRATCH_BYTES
    assert L.bp_event_csr_matvec_noalloc(C.byref(m), fake, fake, None) == _abi.BP_EINVAL
    assert b"static array" in L.bp_last_error()
    assert L.bp_event_csr_matvec_noalloc(None, fake, fake, None) == _abi.BP_EINVAL
    m = _abi.Csr(0x1000, 0x1000, None, 0.5, 10, 100, 1, None, 0)
    assert L.bp_event_csr_matvec_noalloc(C.byref(m), fake, None, None) == _abi.BP_EINVAL
