"""Serving loop against the CPU executor: admission by memory footprint,
residency and eviction order, waiting instead of over-allocating, overlap of
requests in flight, validation, injected failures, deadlines and cancellation.
A virtual clock makes every schedule deterministic."""
import math

import numpy as np
import pytest

from paper_2311_15038_amd import serve as S


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def setup(edges, budget, slots=4, resident=True, **kw):
    clk = Clock()
    ex = S.FakeExecutor(np.asarray(edges), clock=clk, **kw)
    srv = S.Server(ex, budget, slots=slots, resident=resident, clock=clk, sleep=clk.sleep)
    return clk, ex, srv


def req(rid, vid, views=4, res=256, deadline=math.inf):
    return S.Request(rid, vid, views, res, deadline)


def vbytes(n):
    return n ** 3 * 2


WORK = 4 * 256 * 256 * 16          # bytes of a 4-view 256^2 request


def test_all_complete_and_slots_bound():
    clk, ex, srv = setup([64] * 8, 1 << 40, slots=3)
    trace = [(0.001 * k, req(k, k % 8)) for k in range(40)]
    st = srv.run(trace)
    assert st.done == 40 and st.failed == 0
    assert st.max_inflight == 3
    assert st.loads == 8 and st.hits == 32          # every volume loaded once, then resident
    assert all(r.status == "done" and r.result == ("frames", r.rid) for _, r in trace)
    assert all(r.t_done >= r.t_admit >= r.t_arrival for _, r in trace)
    assert len(st.latencies) == 40 and min(st.latencies) > 0


def test_requests_overlap_in_flight():
    # 8 requests of 10 ms each at t=0: 4 slots finish in two waves, one slot in eight
    for slots, waves in [(4, 2), (1, 8)]:
        clk, ex, srv = setup([64] * 8, 1 << 40, slots=slots, s_per_view=2.5e-3)
        st = srv.run([(0.0, req(k, k)) for k in range(8)])
        assert st.done == 8
        assert waves * 0.010 <= st.wall < waves * 0.010 + 1e-3


def test_late_arrival_admitted_while_others_run():
    clk, ex, srv = setup([64] * 4, 1 << 40, slots=2, s_per_view=2.5e-3)
    a, b = req(0, 0, views=40), req(1, 1)            # a runs 100 ms; b arrives at 5 ms
    srv.run([(0.0, a), (0.005, b)])
    assert b.t_admit < a.t_done                       # b did not wait for a
    assert b.t_done < a.t_done


def test_admission_by_footprint_and_lru_eviction():
    budget = 2 * vbytes(100) + WORK                  # room for two volumes + one request's frames
    clk, ex, srv = setup([100, 100, 100], budget, slots=1)
    order = [0, 1, 0, 2, 1, 0]
    st = srv.run([(0.01 * k, req(k, v)) for k, v in enumerate(order)])
    assert st.done == len(order)
    assert st.peak_bytes <= budget
    # 0,1 load; 0 hits; 2 evicts 1 (least recent); 1 reloads, evicting 0; 0 reloads, evicting 2
    assert ex.loaded == [0, 1, 2, 1, 0]
    assert ex.evicted == [1, 0, 2]
    assert st.hits == 1 and st.loads == 5


def test_memory_full_means_waiting_not_failing():
    budget = vbytes(100) + WORK                      # one volume at a time
    clk, ex, srv = setup([100, 100], budget, slots=4)
    a, b = req(0, 0), req(1, 1)
    st = srv.run([(0.0, a), (0.0, b)])
    assert st.done == 2 and st.failed == 0
    assert b.t_admit >= a.t_done                      # b waited for a's memory
    assert st.max_inflight == 1 and st.peak_bytes <= budget


def test_requests_on_a_resident_volume_share_it():
    budget = vbytes(100) + 4 * WORK
    clk, ex, srv = setup([100, 100], budget, slots=4)
    rs = [req(k, 0) for k in range(4)]
    st = srv.run([(0.0, r) for r in rs])
    assert st.loads == 1 and st.hits == 3 and st.max_inflight == 4


def test_pinned_volume_is_not_evicted():
    budget = vbytes(200) + 2 * WORK
    clk, ex, srv = setup([200, 200], budget, slots=4, s_per_view=5e-3)
    a, b, c = req(0, 0, views=8), req(1, 1), req(2, 0)
    st = srv.run([(0.0, a), (0.001, b), (0.002, c)])
    assert st.done == 3
    assert b.t_admit >= a.t_done                      # volume 0 stays while a uses it
    assert ex.evicted == [0, 1] and st.peak_bytes <= budget


def test_too_large_and_invalid_requests_fail_and_loop_continues():
    clk, ex, srv = setup([100, 2000, 50], vbytes(1000), slots=2, bad_ids=[2])
    rs = [req(0, 1), req(1, 0), req(2, 7), req(3, 0, views=0), req(4, 0, res=300), req(5, 2),
          req(6, 0)]
    st = srv.run([(0.001 * k, r) for k, r in enumerate(rs)])
    assert [r.status for r in rs] == ["failed", "done", "failed", "failed", "failed", "failed", "done"]
    assert "budget" in rs[0].error
    assert all(r.error.startswith("VR_ERR_RANGE") for r in rs[2:6])
    assert st.done == 2 and st.failed == 5


def test_executor_errors_fail_only_their_request():
    clk, ex, srv = setup([64] * 4, 1 << 40, slots=2, fail_start=[1], fail_done=[2])
    rs = [req(k, k % 4) for k in range(6)]
    st = srv.run([(0.001 * k, r) for k, r in enumerate(rs)])
    assert rs[1].status == "failed" and "injected failure" in rs[1].error
    assert rs[2].status == "failed" and "injected device error" in rs[2].error
    assert all(rs[k].status == "done" for k in (0, 3, 4, 5))
    assert st.failed == 2 and st.done == 4
    assert srv.free_slots == [0, 1] and srv.reserved == 0 and sum(srv.pins.values()) == 0


def test_failed_start_of_new_volume_drops_it():
    clk, ex, srv = setup([64] * 2, 1 << 40, slots=1, fail_start=[0])
    a, b = req(0, 0), req(1, 0)
    srv.run([(0.0, a), (0.001, b)])
    assert a.status == "failed" and b.status == "done"
    assert ex.loaded == [0] and 0 in srv.resident      # b loaded it again


def test_deadlines():
    clk, ex, srv = setup([64] * 4, 1 << 40, slots=1, s_per_view=5e-3)
    a = req(0, 0, views=4)                             # runs 20 ms, deadline 10 ms
    a.deadline = 0.010
    b = req(1, 1, views=1, deadline=0.005)             # queued behind a past its deadline
    c = req(2, 2, views=1)
    st = srv.run([(0.0, a), (0.0, b), (0.0, c)])
    assert a.status == "expired" and "running" in a.error
    assert a.t_done == pytest.approx(0.010, abs=1e-4)  # reported at the deadline
    assert b.status == "expired" and "queued" in b.error
    assert c.status == "done" and c.t_admit >= 0.020   # a's slot was held until its work ended
    assert st.expired == 2 and st.done == 1


def test_cancel():
    clk, ex, srv = setup([64] * 4, 1 << 40, slots=1, s_per_view=5e-3)
    a, b, c = req(0, 0), req(1, 1), req(2, 2)
    for r in (a, b, c):
        srv.submit(r)
    srv.pump()
    assert a.status == "running" and b.status == "queued"
    srv.cancel(b)
    srv.cancel(a)
    srv.drain()
    assert a.status == "cancelled" and a.result is None
    assert b.status == "cancelled" and b.t_admit < 0
    assert c.status == "done"
    assert srv.stats.cancelled == 2


def test_plain_mode_reloads_every_request():
    clk, ex, srv = setup([64] * 2, 1 << 40, slots=1, resident=False)
    st = srv.run([(0.001 * k, req(k, 0)) for k in range(5)])
    assert st.done == 5 and st.loads == 5 and st.hits == 0
    assert ex.loaded == [0] * 5 and ex.evicted == [0] * 5 and not srv.resident


def test_warmup_excluded_from_statistics():
    clk, ex, srv = setup([64] * 4, 1 << 40, slots=2)
    trace = [(0.01 * k, req(k, k % 4)) for k in range(20)]
    st = srv.run(trace, warmup=0.1)
    assert st.done == 20
    assert len(st.latencies) == 10                      # arrivals at 0.10 .. 0.19
    assert st.views == 40
    last = max(r.t_done for _, r in trace)
    assert st.wall == pytest.approx(last - 0.10)


def test_trace_recipe():
    trace, edges = S.make_trace(rate=50.0, duration=60.0, pool=64, seed=11)
    n = len(trace)
    assert abs(n - 3000) < 5 * math.sqrt(3000)         # Poisson count
    gaps = np.diff([0.0] + [t for t, _ in trace])
    assert abs(gaps.mean() - 0.02) < 0.002 and abs(gaps.std() / gaps.mean() - 1) < 0.1
    assert edges.min() >= 128 and edges.max() <= 1024 and len(edges) == 64
    # log-uniform: log-edges are spread evenly over [ln 128, ln 1024]
    q = (np.log(edges) - math.log(128)) / math.log(8)
    assert 0.3 < np.median(q) < 0.7
    views = np.array([r.n_views for _, r in trace])
    assert views.min() >= 1 and views.max() <= 36 and abs(views.mean() - 18.5) < 1.0
    res = np.array([r.res for _, r in trace])
    assert set(res.tolist()) == {256, 512} and abs((res == 512).mean() - 0.5) < 0.05
    t2, e2 = S.make_trace(rate=50.0, duration=60.0, pool=64, seed=11)
    assert [(t, r.vol_id, r.n_views, r.res) for t, r in t2] == [(t, r.vol_id, r.n_views, r.res) for t, r in trace]
    burst = S.copy_trace(trace[:5], burst=True)
    assert all(t == 0.0 and b.status == "new" for t, b in burst)
