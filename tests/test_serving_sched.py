"""Serving scheduler logic on the CPU: arrival-order admission under the HBM
and workgroup budgets, rejection of requests that can never fit, quantum
accounting and retirement."""
from paper_2311_05106_amd.serving import Scheduler


def req(i, b, w, steps):
    return dict(id=i, bytes=b, wgs=w, steps=steps)


def test_fifo_admission_and_budget():
    s = Scheduler(hbm_budget=100, wg_budget=10)
    for r in [req(0, 40, 2, 1000), req(1, 40, 2, 300), req(2, 40, 2, 500), req(3, 10, 1, 100)]:
        assert s.submit(r)
    adm = s.admit()
    assert [r["id"] for r in adm] == [0, 1]      # request 2 does not fit; 3 waits behind it (FIFO)
    assert s.hbm_used == 80 and s.wg_used == 4
    plan = s.plan(500)
    assert [(r["id"], k) for r, k in plan] == [(0, 500), (1, 300)]
    fin = s.advance(plan)
    assert [r["id"] for r in fin] == [1] and s.hbm_used == 40
    adm = s.admit()
    assert [r["id"] for r in adm] == [2, 3]
    plan = s.plan(500)
    assert sorted((r["id"], k) for r, k in plan) == [(0, 500), (2, 500), (3, 100)]
    fin = s.advance(plan)
    assert sorted(r["id"] for r in fin) == [0, 2, 3]
    assert s.hbm_used == 0 and s.wg_used == 0 and not s.active


def test_never_fitting_requests_are_rejected():
    s = Scheduler(hbm_budget=100, wg_budget=8)
    assert not s.submit(req(0, 101, 1, 10))
    assert not s.submit(req(1, 10, 9, 10))
    assert s.submit(req(2, 100, 8, 10))
    assert [r["id"] for r in s.rejected] == [0, 1]
    assert [r["id"] for r in s.admit()] == [2]


def test_workgroup_budget_binds():
    s = Scheduler(hbm_budget=10**12, wg_budget=64)
    for i in range(5):
        s.submit(req(i, 1, 32, 100))
    assert len(s.admit()) == 2
    s.advance(s.plan(100))
    assert len(s.admit()) == 2


def test_net_cap():
    s = Scheduler(hbm_budget=10**12, wg_budget=10**6, max_nets=3)
    for i in range(5):
        s.submit(req(i, 1, 1, 10))
    assert len(s.admit()) == 3
