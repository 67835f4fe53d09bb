"""Continuous batching of network simulations on one GPU.

Requests (an E/I LIF network and a number of steps) arrive over time.  The
scheduler admits them in arrival order while the HBM budget (the sum of the
admitted nets' workspace bytes) and the workgroup budget (the nets' resident
workgroups, all co-resident in one launch) allow; every quantum the executor
advances every resident net by min(quantum, remaining) steps in one
persistent-kernel launch (bp_run_batch), retires the nets that finished and
admits new arrivals before the next launch.  The plain path runs the same
requests one at a time, first come first served.

Time: arrivals are in seconds of a virtual clock that follows the wall clock
while work is pending and jumps over idle gaps (so an idle server does not
sleep); latency = completion time - arrival time on that clock.
"""
import math
import time
from collections import deque

from . import COBA, CONN_CSR, CONN_JIT, CUBA, Net, net_bytes, net_desc, net_workgroups, run_batch

CUBA_PARAMS = dict(v_rest=-49.0, w_exc=1.62, w_inh=-9.0, i_ext=0.0)


def request_desc(req, block=1024, max_wgs=0, jit_from=50_000):
    """Network of a serving request: COBA or CUBA E/I net with N neurons,
    p = 80/N, stored CSR below `jit_from` neurons, JIT connectivity above."""
    n = int(req["n"])
    conn = CONN_JIT if n >= jit_from else CONN_CSR
    params = dict(CUBA_PARAMS) if req["model"] == CUBA else {}
    return net_desc(n, n_exc=int(0.8 * n), p=min(1.0, 80.0 / n), conn=conn, block=block, seed=int(req["seed"]),
                    model=req["model"], max_wgs=max_wgs, **params)


class Scheduler:
    """Host-side admission and quantum planning (no GPU access)."""

    def __init__(self, hbm_budget, wg_budget, max_nets=48):
        self.hbm_budget = int(hbm_budget)
        self.wg_budget = int(wg_budget)
        self.max_nets = int(max_nets)
        self.waiting = deque()
        self.active = []
        self.rejected = []
        self.hbm_used = 0
        self.wg_used = 0

    def submit(self, req):
        """req: dict with id, bytes, wgs, steps (and anything else)."""
        if req["bytes"] > self.hbm_budget or req["wgs"] > self.wg_budget:
            self.rejected.append(req)
            return False
        self.waiting.append(req)
        return True

    def admit(self):
        """Admit waiting requests in arrival order while they fit."""
        out = []
        while self.waiting and len(self.active) < self.max_nets:
            r = self.waiting[0]
            if self.hbm_used + r["bytes"] > self.hbm_budget or self.wg_used + r["wgs"] > self.wg_budget:
                break
            self.waiting.popleft()
            r["done"] = 0
            self.active.append(r)
            self.hbm_used += r["bytes"]
            self.wg_used += r["wgs"]
            out.append(r)
        return out

    def plan(self, quantum):
        return [(r, min(quantum, r["steps"] - r["done"])) for r in self.active]

    def advance(self, plan):
        """Account one executed quantum; returns the requests that finished."""
        finished = []
        for r, k in plan:
            r["done"] += k
        for r in list(self.active):
            if r["done"] >= r["steps"]:
                self.active.remove(r)
                self.hbm_used -= r["bytes"]
                self.wg_used -= r["wgs"]
                finished.append(r)
        return finished


class VirtualClock:
    def __init__(self):
        self.t0 = time.perf_counter()
        self.skipped = 0.0

    def now(self):
        return time.perf_counter() - self.t0 + self.skipped

    def skip_to(self, t):
        n = self.now()
        if t > n:
            self.skipped += t - n


def _net_info(req, max_wgs, block):
    d = request_desc(req, block=block, max_wgs=max_wgs)
    return d, net_bytes(d)


def serve_batched(requests, hbm_budget, quantum=500, max_wgs=64, wg_budget=256, block=1024, record_counts=False,
                  torch=None):
    """Continuous batching; returns per-request records and totals."""
    import torch as _torch
    torch = torch or _torch
    reqs = [dict(r) for r in sorted(requests, key=lambda r: r["arrival"])]
    for r in reqs:
        d, b = _net_info(r, max_wgs, block)
        r["desc"], r["bytes"] = d, b
        r["wgs"] = net_workgroups(d)
    sched = Scheduler(hbm_budget, wg_budget)
    clock = VirtualClock()
    pending = deque(reqs)
    done = []
    launches = 0
    while pending or sched.waiting or sched.active:
        now = clock.now()
        while pending and pending[0]["arrival"] <= now:
            sched.submit(pending.popleft())
        for r in sched.admit():
            r["net"] = Net(r["desc"])
            r["admitted"] = clock.now()
            if record_counts:
                r["counts"] = []
        if not sched.active:
            if pending:
                clock.skip_to(pending[0]["arrival"])
                continue
            break
        plan = sched.plan(quantum)
        counts = None
        if record_counts:
            counts = [torch.empty(max(k, 1), dtype=torch.int32, device="cuda") for _, k in plan]
        run_batch([r["net"] for r, _ in plan], [k for _, k in plan], counts)
        launches += 1
        torch.cuda.synchronize()
        if record_counts:
            for (r, k), c in zip(plan, counts):
                r["counts"].append(c[:k].cpu())
        t_done = clock.now()
        for r in sched.advance(plan):
            r["finished"] = t_done
            r["latency"] = t_done - r["arrival"]
            r["events"] = int(r["net"].events().item())
            r["error"] = r["net"].error_flag()
            if record_counts:
                r["counts"] = torch.cat(r["counts"]).numpy()
            r["net"].close()
            del r["net"]
            done.append(r)
    return dict(records=done, rejected=sched.rejected, launches=launches, wall=clock.now())


def serve_plain(requests, max_wgs=0, block=1024, torch=None):
    """One net at a time, first come first served, bp_run per request."""
    import torch as _torch
    torch = torch or _torch
    reqs = [dict(r) for r in sorted(requests, key=lambda r: r["arrival"])]
    clock = VirtualClock()
    done = []
    for r in reqs:
        clock.skip_to(r["arrival"])
        d, _ = _net_info(r, max_wgs, block)
        net = Net(d)
        net.run(int(r["steps"]), counts=False)
        torch.cuda.synchronize()
        r["finished"] = clock.now()
        r["latency"] = r["finished"] - r["arrival"]
        r["events"] = int(net.events().item())
        net.close()
        done.append(r)
    return dict(records=done, rejected=[], launches=len(done), wall=clock.now())


def summarize(result, skip=0):
    """p50/p99 latency and throughput of the requests with id >= skip (the
    first `skip` of the stream warm the server up); throughput is their
    synaptic events over the time from the first one's arrival to the last
    one's completion."""
    recs = [r for r in result["records"] if r["id"] >= skip]
    lat = sorted(r["latency"] for r in recs)
    ev = sum(r["events"] for r in recs)
    if skip and recs:
        wall = max(r["finished"] for r in recs) - min(r["arrival"] for r in recs)
        result = dict(result, wall=wall)

    def pct(q):
        if not lat:
            return float("nan")
        i = min(len(lat) - 1, max(0, int(math.ceil(q * len(lat))) - 1))
        return lat[i]

    return dict(requests=len(lat), rejected=len(result["rejected"]), p50_s=pct(0.5), p99_s=pct(0.99),
                mean_s=sum(lat) / max(len(lat), 1), wall_s=result["wall"], synaptic_events=ev,
                synaptic_events_per_s=ev / result["wall"] if result["wall"] > 0 else float("nan"),
                launches=result["launches"])
