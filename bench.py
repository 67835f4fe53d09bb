"""Benchmark of the event-driven spiking-network path on one MI355X.

Headline workload: the COBA E/I LIF network scaled to 400,000 neurons
(320,000 excitatory / 80,000 inhibitory), fixed-probability connectivity
p = 80/N regenerated every step from the seed (JIT, post blocks of 1024),
w_e = 0.6, w_i = 6.7, tau_e = 5 ms, tau_i = 10 ms, V_rest = -60 mV,
V_th = -50 mV, refractory 5 ms, V0 ~ U(-60, -50) mV, I_ext = 20, dt = 0.1 ms,
FP32 state.  One bench step = one simulation time step; the default K =
10,000 steps is one simulated second, run as one persistent launch.

value = synaptic events delivered per wall second (sum over steps of the row
lengths of the rows that fired the step before).  Also printed: simulated
seconds per wall second, the state-streaming roofline of the network kernel,
the oracle timed on the host cores on a bounded sample, and the operator
sweep (event CSR / JIT matvec at 0.1 %, 1 %, 10 % firing, n = 1e5, p = 0.01).
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


C2_BLOCK = 1024


def c2_desc(bp, n=400_000, seed=0):
    return bp.net_desc(n, n_exc=int(0.8 * n), p=80.0 / n, conn=bp.CONN_JIT, block=C2_BLOCK, seed=seed)


def kernel_source_hash(name):
    with open(os.path.join(ROOT, "paper_2311_05106_amd", "csrc", name), "rb") as f:
        h = hashlib.sha256(f.read())
    with open(os.path.join(ROOT, "paper_2311_05106_amd", "csrc", "bp_device.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def counters_traffic(kernel_file, key, per_launch_units):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if the
    kernel source still matches the one they were taken on."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(key)
        if not ent or ent.get("source_hash") != kernel_source_hash(kernel_file):
            return None
        return ent["bytes_per_unit"] * per_launch_units
    except Exception:
        return None


def bench_network(bp, torch, steps, warmup):
    d = c2_desc(bp)
    # warm-up on a throw-away instance of the same net
    w = bp.Net(d)
    w.run(warmup, counts=False)
    torch.cuda.synchronize()
    del w
    net = bp.Net(d)
    ev0 = int(net.events().item())
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e_start.record(stream)
    _, counts = net.run(steps, counts=True)
    e_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = e_start.elapsed_time(e_end)
    events = int(net.events().item()) - ev0
    spikes = int(counts.sum().item())
    assert net.error_flag() == 0, "network kernel gave up waiting"
    info = net.info()
    return dict(wall=wall, kern_ms=kern_ms, events=events, spikes=spikes, n=d.n, n_wg=info.n_wg,
                range=info.wg_range, dt_ms=d.dt)


def oracle_sample(steps):
    import oracle as O
    n = 400_000
    P = O.net_params(model=0, n=n, n_exc=int(0.8 * n), conn=1, max_gap=O.max_gap(80.0 / n), block=C2_BLOCK, seed=0,
                     w_exc=0.6, w_inh=6.7, tau_m=20.0, tau_e=5.0, tau_i=10.0, tau_ref=5.0, v_rest=-60.0,
                     v_th=-50.0, v_reset=-60.0, e_exc=0.0, e_inh=-80.0, r=1.0, i_ext=20.0, dt=0.1, v0_lo=-60.0,
                     v0_hi=-50.0)
    st = O.NetState(P)
    t0 = time.perf_counter()
    _, counts, events = O.net_run(P, st, steps, want_raster=False)
    dt = time.perf_counter() - t0
    return dict(value=events / dt, events=events, seconds=dt, spikes=int(counts.sum()))


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


def bench_ops(bp, torch, calls=10000):
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
    for frac in (0.001, 0.01, 0.1):
        ev = torch.from_numpy(S.events(n, frac, 5, count=64)).to(dev)
        ev_f = ev.to(torch.int64)
        nnz_a = float((ev_f * rowlen[None, :]).sum(1).double().mean().item())
        act = float(ev_f.sum(1).double().mean().item())
        jc = bp.JitConn(n, n, K=K, block=1024, seed=0, w0=0.5)
        jn = bp.JitConn(n, n, K=K, block=1024, seed=0, wkind=bp.W_NORMAL, w0=0.5, w1=0.1)
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


def bench_serving(bp, torch, n_requests=100, rate_hz=20.0, budget_gib=1.0, quantum=500, max_wgs=64):
    """Serving workload: Poisson arrivals at rate_hz, N ~ log-uniform[1e3,
    2e5], p = 80/N, duration ~ U(100, 2000) ms at dt = 0.1 ms, COBA or CUBA
    with probability 1/2, per-request seed; continuous batching under an HBM
    budget against the plain one-net-at-a-time path on the same GPU."""
    import synthetic as S
    from paper_2311_05106_amd import serving as sv
    reqs = S.request_stream(n_requests, rate_hz, 0)
    warm = S.request_stream(4, rate_hz, 1)
    sv.serve_batched(warm, hbm_budget=int(budget_gib * 2**30), quantum=quantum, max_wgs=max_wgs)
    a = sv.summarize(sv.serve_batched(reqs, hbm_budget=int(budget_gib * 2**30), quantum=quantum, max_wgs=max_wgs))
    b = sv.summarize(sv.serve_plain(reqs))
    return dict(workload=f"{n_requests} requests, Poisson {rate_hz:g} req/s, N ~ logU[1e3, 2e5], p=80/N, "
                         f"duration U(100, 2000) ms, COBA/CUBA", hbm_budget_gib=budget_gib, quantum_steps=quantum,
                max_wgs_per_net=max_wgs, batched=a, plain=b)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--oracle-steps", type=int, default=300)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--block", type=int, default=C2_BLOCK, help="post-block width of the JIT connectivity")
    args = ap.parse_args()
    globals()["C2_BLOCK"] = args.block
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2311_05106_amd as bp
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    r = bench_network(bp, torch, args.steps, args.warmup)
    steps = args.steps
    value = r["events"] / r["wall"]
    ms_per_step = r["wall"] * 1e3 / steps
    sim_s = steps * r["dt_ms"] * 1e-3
    # state-streaming roofline of the network kernel: per neuron and step the
    # state V, ge, gi, ref (4 x 4 B) read and written once = 32 B, plus 8 B per
    # spike (list store + list load by the owner of the targets).
    alg_bytes = 32.0 * r["n"] * steps + 8.0 * r["spikes"]
    kern_s = r["kern_ms"] * 1e-3
    achieved = alg_bytes / kern_s / 1e9
    traffic = counters_traffic("net.hip", "net_run_k_c2", steps)
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel="net_run_k", alg_bytes_per_launch=alg_bytes,
                    launch_ms=r["kern_ms"])
    orc = oracle_sample(args.oracle_steps)
    cpu = dict(value=orc["value"], unit="synaptic events/s", cores=1, kind="oracle",
               sample=f"first {args.oracle_steps} of the {steps} steps of the same 400k-neuron net, "
                      f"FP32 C oracle, single thread ({orc['seconds']:.1f} s)")
    line = dict(metric=METRIC, value=value, unit="synaptic events/s", n_gpus=1, steps=steps, warmup=args.warmup,
                ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic",
                config=dict(workload="COBA E/I LIF 400k (320k E / 80k I), JIT connectivity p=80/N blocks of "
                                     f"{C2_BLOCK}, 10,000 steps dt=0.1 ms", n=r["n"], workgroups=r["n_wg"],
                            neurons_per_workgroup=r["range"], parallelism="1 GPU"),
                sim_s_per_wall_s=sim_s / r["wall"], us_per_step=r["wall"] * 1e6 / steps,
                spikes_per_step=r["spikes"] / steps, mean_rate_hz=r["spikes"] / steps / r["n"] / (r["dt_ms"] * 1e-3),
                events_per_step=r["events"] / steps, roofline=roofline, cpu_baseline=cpu)
    if not args.no_extra:
        line["c0"] = bench_c0(bp, torch)
        line["operator_sweep"] = bench_ops(bp, torch)
        line["serving"] = bench_serving(bp, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
