"""Benchmark of the event-driven spiking-network path on one MI355X.

Headline workload: the COBA E/I LIF network scaled to 400,000 neurons
(320,000 excitatory / 80,000 inhibitory), fixed-probability connectivity
p = 80/N regenerated every step from the seed (JIT; one block per row, the
paper's per-row gap sequence), w_e = 0.6, w_i = 6.7, tau_e = 5 ms,
tau_i = 10 ms, V_rest = -60 mV, V_th = -50 mV, refractory 5 ms,
V0 ~ U(-60, -50) mV, I_ext = 20, dt = 0.1 ms, FP32 state.  One bench step =
one persistent-kernel launch of 1000 simulation steps (0.1 s simulated) on
the same net, after W >= 1 warm-up launches (the initial transient); the
default K = 10 timed launches are one simulated second.

value = synaptic events delivered per wall second (sum over simulation steps
of the row lengths of the rows that fired the step before).  Also printed:
simulated seconds per wall second, the state-streaming roofline of the
network kernel, the oracle timed on the host cores on the same window
(started from the GPU's state, its spike counts checked against the GPU's),
and extras: the same net with blocked connectivity, the 4000-neuron net, the
operator sweep (event CSR / JIT matvec at 0.1 %, 1 %, 10 % firing,
n = 1e5, p = 0.01), the dense-vector JIT products, the SNN training step and
serving.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "synaptic events/s & sim-s per wall-s, COBA E/I net; p50/p99 serving latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


C2_BLOCK = 0  # the headline net: one block per row, the paper's per-row sequence
C2_BLOCKED = 2560  # the extra: rows restarted in post blocks of 2560 columns (one per workgroup)


def c2_desc(bp, n=400_000, seed=0, block=None):
    return bp.net_desc(n, n_exc=int(0.8 * n), p=80.0 / n, conn=bp.CONN_JIT, block=C2_BLOCK if block is None else block,
                       seed=seed)


def kernel_source_hash(name):
    with open(os.path.join(ROOT, "paper_2311_05106_amd", "csrc", name), "rb") as f:
        h = hashlib.sha256(f.read())
    with open(os.path.join(ROOT, "paper_2311_05106_amd", "csrc", "bp_device.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def counters_traffic(kernel_file, key, per_launch_units, block=None):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if the
    kernel source and the block width still match the ones they were taken on."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(key)
        if not ent or ent.get("source_hash") != kernel_source_hash(kernel_file):
            return None
        if block is not None and ent.get("block") != block:
            return None
        return ent["bytes_per_unit"] * per_launch_units
    except Exception:
        return None


LAUNCH_STEPS = 1000  # simulation steps per bench step: one persistent-kernel launch (0.1 s simulated)


def bench_network(bp, torch, steps, warmup, block=None, desc=None):
    """max(W, 1) warm-up launches of LAUNCH_STEPS steps (the initial transient
    is over after the first), then K timed launches of the same net, one per
    bench step; the state stays on the device throughout.  Every buffer is
    allocated before the first event; each launch is bracketed by HIP events
    on the stream it runs on."""
    d = desc if desc is not None else c2_desc(bp, block=block)
    net = bp.Net(d)
    warm = max(warmup, 1)
    for _ in range(warm):
        net.run(LAUNCH_STEPS, counts=False)
    stream = torch.cuda.current_stream()
    counts = torch.empty((steps, LAUNCH_STEPS), dtype=torch.int32, device="cuda")
    ev_before = torch.empty(1, dtype=torch.int64, device="cuda")
    ev_after = torch.empty(1, dtype=torch.int64, device="cuda")
    marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    net.events(out=ev_before)
    state0 = net.get_state()  # the state at the start of the timed window (CPU baseline)
    step0 = int(state0["step"])
    raw0 = state0["raw"].cpu()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        a, b = marks[i]
        a.record(stream)
        net.run(LAUNCH_STEPS, counts_out=counts[i])
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    net.events(out=ev_after)
    launch_ms = [a.elapsed_time(b) for a, b in marks]
    events = int(ev_after.item()) - int(ev_before.item())
    counts_h = counts.cpu().numpy()
    err = net.error_flag()
    info = net.info()
    net.close()
    assert err == 0, "network kernel gave up waiting"
    return dict(wall=wall, launch_ms=launch_ms, events=events, spikes=int(counts_h.sum()), counts=counts_h,
                n=d.n, n_wg=info.n_wg, range=info.wg_range, dt_ms=d.dt, block=d.block, warmup_launches=warm,
                step0=step0, raw0=raw0)


def oracle_window(r, min_seconds=10.0, single_steps=200):
    """The oracle on the benchmark's own window: started from the GPU's state
    at the first timed step, the OpenMP build of the FP32 network loops on
    every host core runs until about min_seconds of CPU work are done; the
    plain build (one thread) runs the first single_steps steps.  Both must
    reproduce the GPU's spike counts of those steps exactly."""
    import numpy as np
    import oracle as O
    n = r["n"]
    P = O.net_params(model=0, n=n, n_exc=int(0.8 * n), conn=1, max_gap=O.max_gap(80.0 / n), block=r["block"],
                     seed=0, w_exc=0.6, w_inh=6.7, tau_m=20.0, tau_e=5.0, tau_i=10.0, tau_ref=5.0, v_rest=-60.0,
                     v_th=-50.0, v_reset=-60.0, e_exc=0.0, e_inh=-80.0, r=1.0, i_ext=20.0, dt=0.1, v0_lo=-60.0,
                     v0_hi=-50.0)
    raw = r["raw0"].numpy()

    def state():
        st = O.NetState(P)
        st.V = raw[0:4 * n].view(np.float32).copy()
        st.ge = raw[4 * n:8 * n].view(np.float32).copy()
        st.gi = raw[8 * n:12 * n].view(np.float32).copy()
        st.ref = raw[12 * n:16 * n].view(np.int32).copy()
        st.s_prev = raw[16 * n:17 * n].copy()
        st.t = r["step0"]
        return st

    gpu_counts = r["counts"].reshape(-1)
    threads = O.set_threads(0)
    st = state()
    done, ev, sec, match = 0, 0, 0.0, True
    while sec < min_seconds and done + 100 <= gpu_counts.size:
        t0 = time.perf_counter()
        _, c, e = O.net_run(P, st, 100, want_raster=False, parallel=True)
        sec += time.perf_counter() - t0
        match = match and bool(np.array_equal(c, gpu_counts[done:done + 100]))
        done += 100
        ev += e
    st1 = state()
    k = min(single_steps, gpu_counts.size)
    t0 = time.perf_counter()
    _, c1, e1 = O.net_run(P, st1, k, want_raster=False)
    sec1 = time.perf_counter() - t0
    match1 = bool(np.array_equal(c1, gpu_counts[:k]))
    return dict(value=ev / sec, threads=threads, steps=done, seconds=sec, events=ev, counts_match=match,
                single_value=e1 / sec1, single_steps=k, single_seconds=sec1, single_counts_match=match1)


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), model=model)


def bench_c0(bp, torch, reps=5):
    d = bp.net_desc(4000, n_exc=3200, p=0.02, conn=bp.CONN_CSR, block=0, seed=0)
    times, ev = [], 0
    for r in range(reps + 1):
        net = bp.Net(d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.run(1000, counts=False)
        torch.cuda.synchronize()
        if r:
            times.append(time.perf_counter() - t0)
        ev = int(net.events().item())
        del net
    t = sorted(times)[len(times) // 2]
    return dict(workload="COBA E/I 4000 (3200/800), stored CSR p=0.02, 1000 steps", ms_per_run=t * 1e3,
                us_per_step=t * 1e3, sim_s_per_wall_s=0.1 / t, synaptic_events_per_s=ev / t)


# JIT operator blocks of 3125 columns: 32 column tiles x 8 row chunks make 256
# workgroups, one per compute unit.  Measured sweep (us, homogeneous / normal
# weights at 0.1 %, 1 %, 10 % firing): 782 (128 tiles x 2 chunks): 9.8/11.3,
# 11.7/17.4, 25.5/54.3; 1564: 8.6/11.1, 10.8/18.1, 19.6/42.7; 3125: 7.9/11.6,
# 8.8/13.5, 17.6/43.3; 6250: 8.7/14.8, 9.3/16.5, 19.2/48.2.  Longer blocks
# mean longer walks per (row, block): fewer start-up draws per target and
# less spread between the walks of a wave.
JIT_OP_BLOCK = 3125
# Dense-vector products list every row, so each workgroup walks many more
# (row, block) pairs: longer blocks cut the per-pair start-up draws and even
# out the walks of a wave.  Measured sweep (us, homogeneous / U / N, one
# vector): 782: 288 / 359 / 424; 1564: 229 / 291 / 348; 3125: 197 / 254 / 306;
# 6250: 179 / 231 / 282; 12500: 215 / 281 / 342.  The 8-vector product keeps
# 8 columns in the LDS tile only up to 2048 columns: 1564: 903 / 933 us
# (U / N), 782: 1062 / 1107, 4096 (5 columns per group): 1008 / 1078.
DENSE_OP_BLOCK = 6250  # 16 column tiles x 16 row chunks
DENSE_MAT_BLOCK = 1564  # 64 column tiles x 4 row chunks


def bench_ops(bp, torch, calls=10000, fracs=(0.001, 0.01, 0.1)):
    """Operator sweep: n_pre = n_post = 1e5, p = 0.01; each point runs `calls`
    products cycling 64 event vectors, replayed from a HIP graph."""
    import numpy as np
    import synthetic as S
    n, K = 100_000, bp.max_gap(0.01)
    dev = "cuda"
    ip, ix = bp.csr_build(bp.JitConn(n, n, K=K, seed=0))
    nnz = ix.numel()
    tw = -(-n // 8)  # eight column tiles (one per XCD-sized share of the columns)
    tp = bp.csr_tile_index(ip, ix, n, tw)
    data = torch.from_numpy(S.hetero_data(nnz, 1)).to(dev)
    rowlen = (ip[1:] - ip[:-1]).to(torch.int64)
    out = []
    for frac in fracs:
        ev = torch.from_numpy(S.events(n, frac, 5, count=64)).to(dev)
        ev_f = ev.to(torch.int64)
        nnz_a = float((ev_f * rowlen[None, :]).sum(1).double().mean().item())
        act = float(ev_f.sum(1).double().mean().item())
        jc = bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, w0=0.5)
        jn = bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, wkind=bp.W_NORMAL, w0=0.5, w1=0.1)
        y = torch.empty(n, dtype=torch.float32, device=dev)
        cases = [
            ("event_csr_homo", lambda e: bp.event_csr_matvec(ip, ix, None, 0.5, n, e, tp, tw, out=y, ws=ws_c),
             bp.event_csr_ws(ip, ix, None, 0.5, n, tp, tw), n + 8 * act + 8 * act + 4 * nnz_a + 4 * n),
            ("event_csr_hetero", lambda e: bp.event_csr_matvec(ip, ix, data, 0.0, n, e, tp, tw, out=y, ws=ws_c),
             bp.event_csr_ws(ip, ix, data, 0.0, n, tp, tw), n + 8 * act + 8 * act + 8 * nnz_a + 4 * n),
            ("jit_homo", lambda e: bp.jit_conn_matvec(jc, e, out=y, ws=ws_c), bp.jit_ws(jc), 4 * nnz_a),
            ("jit_normal", lambda e: bp.jit_conn_matvec(jn, e, out=y, ws=ws_c), bp.jit_ws(jn), 8 * nnz_a),
        ]
        for name, fn, wsb, alg_bytes in cases:
            ws_c = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
            for i in range(64):
                fn(ev[i])
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                with torch.cuda.graph(g, stream=s):
                    for i in range(64):
                        fn(ev[i])
            torch.cuda.synchronize()
            reps = max(1, calls // 64)
            g.replay()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                g.replay()
            b.record()
            torch.cuda.synchronize()
            us = a.elapsed_time(b) * 1e3 / (reps * 64)
            row = dict(op=name, firing=frac, us_per_call=us, synaptic_events_per_s=nnz_a / (us * 1e-6))
            if name.startswith("event_csr"):
                gbs = alg_bytes / (us * 1e-6) / 1e9
                row.update(alg_bytes=alg_bytes, alg_GBps=gbs, hbm_frac=gbs / HBM_PEAK_GBS)
            else:
                gbs = alg_bytes / (us * 1e-6) / 1e9  # CSR-equivalent bytes (indices [+ data])
                row.update(csr_equiv_GBps=gbs, csr_equiv_frac=gbs / HBM_PEAK_GBS)
            out.append(row)
            del g
    return out


def _graph_time_us(torch, fn, items, calls):
    """Mean us per call of fn over `items`, replayed from a HIP graph of one
    pass over the items (eager warm-up first)."""
    for it in items:
        fn(it)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for it in items:
                fn(it)
    torch.cuda.synchronize()
    reps = max(1, calls // len(items))
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    us = a.elapsed_time(b) * 1e3 / (reps * len(items))
    del g
    return us


def bench_ops_batch(bp, torch, calls=1280, fracs=(0.001, 0.01, 0.1), m=8):
    """Batched spike products on the operator sweep's matrix (1e5 x 1e5,
    p = 0.01): m spike vectors per call (E [m, 1e5]), 8 distinct batches
    cycled from the same 64 vectors per firing fraction as the single-vector
    sweep.  Stored CSR with a tile index of 4096 columns (counts: 8 vectors per
    group) or 2048 (sums); JIT with the sweep's blocks of 3125."""
    import synthetic as S
    n, K = 100_000, bp.max_gap(0.01)
    dev = "cuda"
    ip, ix = bp.csr_build(bp.JitConn(n, n, K=K, seed=0))
    data = torch.from_numpy(S.hetero_data(ix.numel(), 1)).to(dev)
    rowlen = (ip[1:] - ip[:-1]).to(torch.int64)
    tp4, tp2 = bp.csr_tile_index(ip, ix, n, 4096), bp.csr_tile_index(ip, ix, n, 2048)
    out = []
    for frac in fracs:
        ev = torch.from_numpy(S.events(n, frac, 5, count=64)).to(dev)
        Es = [ev[i * m:(i + 1) * m] for i in range(64 // m)]
        nnz_a = float((ev.to(torch.int64) * rowlen[None, :]).sum(1).double().mean().item())
        jc = bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, w0=0.5)
        jn = bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, wkind=bp.W_NORMAL, w0=0.5, w1=0.1)
        Y = torch.empty((m, n), dtype=torch.float32, device=dev)
        cases = [
            ("event_csr_homo", lambda E: bp.event_csr_matmat(ip, ix, None, 0.5, n, E, tp4, 4096, out=Y, ws=ws),
             bp.event_csr_matmat_ws(ip, ix, None, 0.5, n, m, tp4, 4096)),
            ("event_csr_hetero", lambda E: bp.event_csr_matmat(ip, ix, data, 0.0, n, E, tp2, 2048, out=Y, ws=ws),
             bp.event_csr_matmat_ws(ip, ix, data, 0.0, n, m, tp2, 2048)),
            ("jit_homo", lambda E: bp.jit_conn_matmat(jc, E, out=Y, ws=ws), bp.jit_conn_matmat_ws(jc, m)),
            ("jit_normal", lambda E: bp.jit_conn_matmat(jn, E, out=Y, ws=ws), bp.jit_conn_matmat_ws(jn, m)),
        ]
        for name, fn, wsb in cases:
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
            us = _graph_time_us(torch, fn, Es, calls // m)
            out.append(dict(op=f"{name}_batch{m}", firing=frac, vectors=m, us_per_call=us, us_per_vector=us / m,
                            synaptic_events_per_s=m * nnz_a / (us * 1e-6)))
    return out


def bench_rules(bp, torch, calls=1280, fracs=(0.01, 0.1)):
    """The JIT spike product on 1e5 x 1e5 under each connectivity rule:
    uniform gaps on [1, K] (the paper's sampler, blocks of 3125), geometric
    gaps (exact Bernoulli(0.01), same blocks) and exactly 1000 targets per row
    (one block per row), homogeneous weights; Appendix C compares the first
    two samplers' cost."""
    import synthetic as S
    n, K = 100_000, bp.max_gap(0.01)
    dev = "cuda"
    conns = [("uniform_gaps", bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, w0=0.5)),
             ("geometric_gaps", bp.JitConn(n, n, p=0.01, block=JIT_OP_BLOCK, seed=0, w0=0.5,
                                           rule=bp.RULE_GEOMETRIC)),
             ("fixed_degree_1000", bp.JitConn(n, n, block=0, seed=0, w0=0.5, rule=bp.RULE_FIXED_DEGREE,
                                              degree=1000))]
    y = torch.empty(n, dtype=torch.float32, device=dev)
    out = []
    for frac in fracs:
        ev = torch.from_numpy(S.events(n, frac, 5, count=64)).to(dev)
        for name, c in conns:
            ip, _ = bp.csr_build(c)
            rowlen = (ip[1:] - ip[:-1]).to(torch.int64)
            nnz_a = float((ev.to(torch.int64) * rowlen[None, :]).sum(1).double().mean().item())
            ws = torch.empty(max(bp.jit_ws(c), 1), dtype=torch.uint8, device=dev)
            us = _graph_time_us(torch, lambda e: bp.jit_conn_matvec(c, e, out=y, ws=ws), list(ev), calls)
            out.append(dict(op=f"jit_homo_{name}", firing=frac, block=int(c.block), us_per_call=us,
                            synapses_per_s=nnz_a / (us * 1e-6)))
    return out


def bench_backward(bp, torch, calls=64):
    """Reverse mode of the operators on the sweep's matrix (1e5 x 1e5,
    p = 0.01, 10 % firing): the event-CSR VJP (d_events over every row, d_data
    over the firing rows' entries, d_w) and the JIT VJP (d_events, d_w)."""
    import synthetic as S
    n, K = 100_000, bp.max_gap(0.01)
    dev = "cuda"
    ip, ix = bp.csr_build(bp.JitConn(n, n, K=K, seed=0))
    nnz = int(ix.numel())
    data = torch.from_numpy(S.hetero_data(nnz, 1)).to(dev)
    e = torch.from_numpy(S.events(n, 0.1, 5)).to(dev)
    dy = torch.from_numpy(S.dense_vector(n, 3)).to(dev)
    out = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, fn, alg in [
        ("event_csr_vjp_hetero", lambda: bp.event_csr_backward(ip, ix, data, 0.0, n, e, dy),
         # indptr, indices, data, gathered dy and d_data per entry; d_events
         8.0 * (n + 1) + 16.0 * nnz + 4.0 * n),
        ("jit_vjp_homo", lambda: bp.jit_conn_backward(bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, w0=0.5),
                                                      e, dy), None),
        ("jit_vjp_normal", lambda: bp.jit_conn_backward(
            bp.JitConn(n, n, K=K, block=JIT_OP_BLOCK, seed=0, wkind=bp.W_NORMAL, w0=0.5, w1=0.1), e, dy), None),
    ]:
        fn()
        torch.cuda.synchronize()
        a.record()
        for _ in range(calls):
            fn()
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / calls
        row = dict(op=name, us_per_call=us, synapses=nnz, synapses_per_s=nnz / (us * 1e-6))
        if alg is not None:
            row.update(alg_bytes=alg, alg_GBps=alg / (us * 1e-6) / 1e9, hbm_frac=alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS)
        out.append(row)
    return out


def bench_proj(bp, torch, T=200):
    """Projections with a 10-step spike delay (Section 4.3, Appendix D):
    AlignPost (event product, then g <- g d + y) against AlignPre (trace
    update, then the float-vector product of the traces), on the 4000-neuron
    net's stored matrix (p = 0.02) and on a regenerated 1e5 x 1e5 matrix
    (p = 0.01, blocks of 3125), driven by T steps of 2 % firing; us per step
    (one delay push and one projection step), the T steps issued back to back."""
    import math
    import synthetic as S
    out = []
    d = float(math.exp(-0.1 / 5.0))
    for name, n, kw in [
        ("csr_4000_p0.02", 4000, None),
        ("jit_1e5_p0.01", 100_000, dict(jit=bp.JitConn(100_000, 100_000, K=bp.max_gap(0.01), block=JIT_OP_BLOCK,
                                                     seed=0, w0=0.6))),
    ]:
        if kw is None:
            ip, ix = bp.csr_build(bp.JitConn(n, n, K=bp.max_gap(0.02), seed=0))
            kw = dict(csr=(ip, ix, None, 0.6, n))
        R = torch.from_numpy(S.events(n, 0.02, 9, count=T)).to("cuda")
        for align in (bp.ALIGN_POST, bp.ALIGN_PRE):
            pr = bp.Projection(align, d, delay=10, depth=11, **kw)
            g = torch.empty((T, n), dtype=torch.float32, device="cuda")
            pr.run(R, g_out=g)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            pr.run(R, g_out=g)
            b.record()
            torch.cuda.synchronize()
            out.append(dict(projection=name, align="post" if align == bp.ALIGN_POST else "pre", delay=10,
                            us_per_step=a.elapsed_time(b) * 1e3 / T))
    return out


def bench_dense(bp, torch, calls=640):
    """JIT product on dense float vectors (Section 5.2's operator y = J^T v):
    n_pre = n_post = 1e5, p = 0.01, blocks of DENSE_OP_BLOCK columns, v ~ N(0, 1)
    with no zeros (every row contributes); `calls` products cycling 8
    vectors, replayed from a HIP graph; then the batched product on 8 vectors
    at once (blocks of DENSE_MAT_BLOCK, 4 distinct X, calls / 8 products)."""
    import numpy as np
    import synthetic as S
    n, K = 100_000, bp.max_gap(0.01)
    dev = "cuda"
    vs = [torch.from_numpy(S.dense_vector(n, 30 + i)).to(dev) for i in range(8)]
    y = torch.empty(n, dtype=torch.float32, device=dev)
    out = []
    for name, wk, w0, w1 in [("homo", bp.W_HOMO, 0.5, 0.0), ("uniform", bp.W_UNIFORM, -1.0, 1.0),
                             ("normal", bp.W_NORMAL, 0.5, 0.1)]:
        conn = bp.JitConn(n, n, K=K, block=DENSE_OP_BLOCK, seed=0, wkind=wk, w0=w0, w1=w1)
        ws = torch.empty(max(bp.jit_dense_ws(conn), 1), dtype=torch.uint8, device=dev)
        # synapses per product: the row lengths of the same seed (every row is listed)
        ip, _ = bp.csr_build(conn)
        nnz = float(ip[-1].item())
        fn = lambda v: bp.jit_conn_matvec_dense(conn, v, out=y, ws=ws)
        for v in vs:
            fn(v)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for v in vs:
                    fn(v)
        torch.cuda.synchronize()
        reps = max(1, calls // 8)
        g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / (reps * 8)
        # CSR-equivalent bytes: what a stored matrix would stream per synapse
        # (4 B index, plus 4 B weight unless the weights are homogeneous)
        gbs = (4.0 if wk == bp.W_HOMO else 8.0) * nnz / (us * 1e-6) / 1e9
        out.append(dict(op=f"jit_dense_{name}", block=DENSE_OP_BLOCK, us_per_call=us, synapses=nnz,
                        synapses_per_s=nnz / (us * 1e-6),
                        csr_equiv_GBps=gbs, csr_equiv_frac=gbs / HBM_PEAK_GBS))
        del g
    # batched: 8 vectors per product (X [n, 8] row-major), each row generated once per column group
    m = 8
    Xs = [torch.from_numpy(np.ascontiguousarray(np.stack([S.dense_vector(n, 60 + 8 * i + c) for c in range(m)], 1)))
          .to(dev) for i in range(4)]
    Y = torch.empty((n, m), dtype=torch.float32, device=dev)
    for name, wk, w0, w1 in [("uniform", bp.W_UNIFORM, -1.0, 1.0), ("normal", bp.W_NORMAL, 0.5, 0.1)]:
        conn = bp.JitConn(n, n, K=K, block=DENSE_MAT_BLOCK, seed=0, wkind=wk, w0=w0, w1=w1)
        ws = torch.empty(max(bp.jit_matmat_ws(conn, m), 1), dtype=torch.uint8, device=dev)
        ip, _ = bp.csr_build(conn)
        nnz = float(ip[-1].item())
        fn = lambda X: bp.jit_conn_matmat_dense(conn, X, out=Y, ws=ws)
        for X in Xs:
            fn(X)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for X in Xs:
                    fn(X)
        torch.cuda.synchronize()
        reps = max(1, calls // 32)
        g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / (reps * 4)
        out.append(dict(op=f"jit_dense_matmat{m}_{name}", block=DENSE_MAT_BLOCK, us_per_call=us, synapses=nnz,
                        columns=m,
                        synapse_columns_per_s=nnz * m / (us * 1e-6)))
        del g
    return out


def bench_snn(bp, torch, reps=5):
    """Differentiable recurrent LIF network: batch 256, 128 Poisson inputs
    (5-50 Hz), 512 neurons with p = 0.1 recurrent CSR, 10 classes, 250 steps
    of 1 ms; one training step = forward + checkpointed BPTT (every 50)."""
    import math
    import numpy as np
    import synthetic as S
    import paper_2311_05106_amd.autograd as A
    B, Cc, N, Ocls, T, p = 256, 128, 512, 10, 250, 0.1
    dev = "cuda"
    ip, ix = bp.csr_build(bp.JitConn(N, N, K=bp.max_gap(p), seed=0))
    x = S.poisson_inputs(T, B, Cc, 1.0, 0, 5.0, 50.0)
    lab = S.labels(B, Ocls, 0)
    W_in, w_rec, W_out, b_out = S.snn_weights(Cc, N, Ocls, int(ix.numel()), 0, rec_std=1.0 / math.sqrt(p * N))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    args = [t(x), t(lab), t(W_in * 4.0), t(w_rec), t(W_out), t(b_out)]
    model = A.SNN(B, Cc, N, Ocls, T, ip, ix, alpha=math.exp(-1 / 5), beta=math.exp(-1 / 20), ckpt_every=50)
    times = []
    spikes = 0.0
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fwd = model.forward(*args, want_raster=(r == 0))
        model.backward(fwd, *args)
        torch.cuda.synchronize()
        if r:
            times.append(time.perf_counter() - t0)
        else:
            spikes = float(fwd["raster"].float().sum().item())
    ms = sorted(times)[len(times) // 2] * 1e3
    return dict(workload="recurrent LIF SNN, B=256, 128 in, 512 hidden (CSR p=0.1), 10 out, T=250, "
                         "BPTT checkpoint every 50", ms_per_train_step=ms, hidden_spikes_per_step=spikes,
                hidden_spikes_per_s=spikes / (ms * 1e-3))


def bench_serving(bp, torch, n_requests=600, n_warm=50, rate_hz=100.0, budget_gib=4.0, quantum=500, max_wgs=64):
    """Serving workload: Poisson arrivals at rate_hz, N ~ log-uniform[1e3,
    2e5], p = 80/N, duration ~ U(100, 2000) ms at dt = 0.1 ms, COBA or CUBA
    with probability 1/2, per-request seed; continuous batching under an HBM
    budget against the plain one-net-at-a-time path on the same GPU.  The
    stream has n_warm + n_requests requests; statistics cover the last
    n_requests.  The arrival rate is above what the plain path serves (about
    20 requests per second), so it saturates and its queue grows."""
    import synthetic as S
    from paper_2311_05106_amd import serving as sv
    reqs = S.request_stream(n_warm + n_requests, rate_hz, 0)
    budget = int(budget_gib * 2**30)
    a = sv.summarize(sv.serve_batched(reqs, hbm_budget=budget, quantum=quantum, max_wgs=max_wgs), skip=n_warm)
    b = sv.summarize(sv.serve_plain(reqs), skip=n_warm)
    return dict(workload=f"{n_warm} warm-up + {n_requests} requests, Poisson {rate_hz:g} req/s, N ~ logU[1e3, 2e5], "
                         f"p=80/N, duration U(100, 2000) ms, COBA/CUBA", hbm_budget_gib=budget_gib,
                quantum_steps=quantum, max_wgs_per_net=max_wgs, batched=a, plain=b,
                throughput_ratio=a["synaptic_events_per_s"] / b["synaptic_events_per_s"])


def bench_copy(bp, torch, mib=1024, reps=2):
    """A plain device-to-device copy of `mib` MiB (torch copy_): the known
    byte count that calibrates the HBM traffic counters (FETCH_SIZE and
    WRITE_SIZE per dispatch) and the copy bandwidth this GPU reaches."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return dict(bytes_read=4 * n, bytes_written=4 * n, dispatches=reps + 1, ms_per_copy=ms,
                read_plus_write_GBps=8.0 * n / (ms * 1e-3) / 1e9)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help=f"timed bench steps, each one launch of {LAUNCH_STEPS} simulation steps")
    ap.add_argument("--warmup", type=int, default=2, help="warm-up launches (at least one is run)")
    ap.add_argument("--oracle-seconds", type=float, default=10.0,
                    help="CPU seconds of the OpenMP oracle on the timed window")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--block", type=int, default=C2_BLOCK, help="post-block width of the headline net's connectivity")
    ap.add_argument("--calls", type=int, default=10000, help="products per point of the operator sweep")
    ap.add_argument("--ops-frac", type=float, default=None,
                    help="run the operator sweep at this firing fraction only (for profiling)")
    ap.add_argument("--section", choices=["c0", "ops", "ops_batch", "rules", "backward", "proj", "dense", "snn",
                                          "serving", "copy"],
                    help="run only this secondary workload and print its JSON (for profiling)")
    args = ap.parse_args()
    globals()["C2_BLOCK"] = args.block
    if args.gpus != 1:
        print(f"bench.py: the implementation runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2311_05106_amd as bp
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.section:
        if args.section == "ops":
            res = bench_ops(bp, torch, calls=args.calls,
                            **({} if args.ops_frac is None else {"fracs": (args.ops_frac,)}))
        else:
            res = dict(c0=bench_c0, dense=bench_dense, snn=bench_snn, serving=bench_serving, copy=bench_copy,
                       ops_batch=bench_ops_batch, rules=bench_rules, backward=bench_backward,
                       proj=bench_proj)[args.section](bp, torch)
        print(json.dumps({args.section: res}), flush=True)
        return

    r = bench_network(bp, torch, args.steps, args.warmup)
    steps = args.steps
    sim_steps = steps * LAUNCH_STEPS
    value = r["events"] / r["wall"]
    ms_per_step = r["wall"] * 1e3 / steps
    # state-streaming roofline of the network kernel: per neuron and
    # simulation step the state V, g_e, g_i (3 x 4 B) and the refractory
    # counter (1 B) read and written once (26 B) plus the spike flag written
    # and read once (2 B) = 28 B, plus 8 B per spike (compacted id stored,
    # then loaded by the owners of its targets).  One launch = LAUNCH_STEPS
    # steps of all n neurons.
    alg_bytes = (28.0 * r["n"] * sim_steps + 8.0 * r["spikes"]) / steps  # per launch
    launch_s = sum(r["launch_ms"]) / steps * 1e-3  # average launch duration
    achieved = alg_bytes / launch_s / 1e9
    traffic = counters_traffic("net.hip", f"net_run_k_coba400k_jit_b{r['block']}", LAUNCH_STEPS, block=r["block"])
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel="net_run_k", alg_bytes_per_launch=alg_bytes,
                    launch_ms=launch_s * 1e3, launches=steps, steps_per_launch=LAUNCH_STEPS,
                    us_per_sim_step=launch_s * 1e6 / LAUNCH_STEPS)
    orc = oracle_window(r, min_seconds=args.oracle_seconds)
    cpu = dict(value=orc["value"], unit="synaptic events/s", cores=orc["threads"], kind="oracle",
               sample=f"simulation steps {r['step0']}..{r['step0'] + orc['steps'] - 1} of the timed window "
                      f"(started from the GPU's state at its first step), FP32 oracle network loops built with "
                      f"OpenMP on {orc['threads']} threads, {orc['seconds']:.1f} s; spike counts equal to the "
                      f"GPU's: {orc['counts_match']}",
               single_thread=dict(value=orc["single_value"], steps=orc["single_steps"],
                                  seconds=orc["single_seconds"], counts_match=orc["single_counts_match"]),
               host=host_cpu())
    line = dict(metric=METRIC, value=value, unit="synaptic events/s", n_gpus=1, steps=steps, warmup=args.warmup,
                ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic",
                config=dict(workload=f"COBA E/I LIF 400k (320k E / 80k I), JIT connectivity p=80/N regenerated "
                                     f"every step, one block per row (the paper's per-row gap sequence), dt=0.1 ms; "
                                     f"one bench step = one persistent launch of {LAUNCH_STEPS} simulation steps; "
                                     f"{r['warmup_launches']} warm-up launches, then {steps} timed launches = "
                                     f"{sim_steps} simulation steps ({sim_steps * r['dt_ms'] * 1e-3:g} s simulated) "
                                     f"starting at step {r['step0']}",
                            n=r["n"], block=r["block"], workgroups=r["n_wg"], neurons_per_workgroup=r["range"],
                            parallelism="1 GPU"),
                sim_steps=sim_steps, sim_s_per_wall_s=sim_steps * r["dt_ms"] * 1e-3 / r["wall"],
                us_per_sim_step=r["wall"] * 1e6 / sim_steps,
                spikes_per_sim_step=r["spikes"] / sim_steps,
                mean_rate_hz=r["spikes"] / sim_steps / r["n"] / (r["dt_ms"] * 1e-3),
                events_per_sim_step=r["events"] / sim_steps, roofline=roofline, cpu_baseline=cpu)
    if not args.no_extra:
        w = bench_network(bp, torch, 4, 1, block=C2_BLOCKED)
        line["c2_blocked"] = dict(
            workload=f"the same 400k net with connectivity restarted in post blocks of {C2_BLOCKED} columns "
                     "(a different random graph of the same statistics), spike ids exchanged; 1 warm-up + 4 "
                     f"timed launches of {LAUNCH_STEPS} steps",
            workgroups=w["n_wg"], us_per_sim_step=w["wall"] * 1e6 / (4 * LAUNCH_STEPS),
            launch_ms=sum(w["launch_ms"]) / 4, synaptic_events_per_s=w["events"] / w["wall"],
            sim_s_per_wall_s=4 * LAUNCH_STEPS * w["dt_ms"] * 1e-3 / w["wall"])
        f = bench_network(bp, torch, 4, 1, desc=bp.net_desc(400_000, n_exc=320_000, K=1, conn=bp.CONN_JIT, block=0,
                                                            seed=0, rule=bp.RULE_FIXED_DEGREE, degree=80))
        line["c2_fixed_degree"] = dict(
            workload="the 400k net with exactly 80 targets per neuron (3.2e7 synapses, the fixed out-degree of "
                     "the configuration read literally), regenerated every step and pushed by the writers; 1 warm-up "
                     f"+ 4 timed launches of {LAUNCH_STEPS} steps",
            workgroups=f["n_wg"], us_per_sim_step=f["wall"] * 1e6 / (4 * LAUNCH_STEPS),
            launch_ms=sum(f["launch_ms"]) / 4, synaptic_events_per_s=f["events"] / f["wall"],
            sim_s_per_wall_s=4 * LAUNCH_STEPS * f["dt_ms"] * 1e-3 / f["wall"],
            mean_rate_hz=f["spikes"] / (4 * LAUNCH_STEPS) / f["n"] / (f["dt_ms"] * 1e-3))
        line["c0"] = bench_c0(bp, torch)
        line["operator_sweep"] = bench_ops(bp, torch, calls=args.calls)
        line["operator_sweep_batch8"] = bench_ops_batch(bp, torch)
        line["connectivity_rules"] = bench_rules(bp, torch)
        line["reverse_mode"] = bench_backward(bp, torch)
        line["projections"] = bench_proj(bp, torch)
        line["jit_dense_vector"] = bench_dense(bp, torch)
        line["snn_training"] = bench_snn(bp, torch)
        line["serving"] = bench_serving(bp, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
