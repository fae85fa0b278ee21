"""The serving scheduler on the CPU, driven by a simulated executor (virtual
clock, simulated durations and footprints): completion, admission under a
memory budget, plan cache and eviction, continuous batching, failure
isolation, arrival order."""
import numpy as np
import pytest

from paper_2202_04894_amd.serving import Request, Scheduler


class FakeExecutor:
    def __init__(self, plan_bpp=10, ws_bpp=20, us_per_point=1.0, fail_on=()):
        self.t = 0.0
        self.plan_bpp, self.ws_bpp, self.us = plan_bpp, ws_bpp, us_per_point
        self.fail_on = set(fail_on)
        self.live_plans = {}
        self.in_use = {}
        self.admit_log = []

    def now(self):
        return self.t

    def idle(self, dt):
        self.t += max(dt, 1e-4)

    def estimate(self, req):
        return self.plan_bpp * req.n_points, self.ws_bpp * req.n_points

    def build(self, req):
        if req.rid in self.fail_on:
            raise RuntimeError("plan creation failed")
        self.t += 1e-3
        key = object()
        self.live_plans[id(key)] = req.geometry
        return key, self.plan_bpp * req.n_points, self.ws_bpp * req.n_points

    def start(self, req, plan):
        self.in_use[id(plan)] = self.in_use.get(id(plan), 0) + 1
        self.admit_log.append((req.rid, self.t))
        dur = req.n_points * req.n_matvecs * self.us * 1e-6
        return dict(rid=req.rid, plan=plan, end=self.t + dur, n=req.n_matvecs, dur=dur)

    def done(self, h):
        return self.t >= h["end"]

    def finish(self, h):
        self.in_use[id(h["plan"])] -= 1
        res = [np.full(3, h["rid"] * 10 + k, dtype=np.complex64) for k in range(h["n"])]
        return h["end"], [h["dur"] * 1e3 / h["n"]] * h["n"], res

    def release_plan(self, plan):
        assert self.in_use.get(id(plan), 0) == 0, "released a plan in use"
        del self.live_plans[id(plan)]


def reqs(specs):
    out = []
    for i, (geom, n, arrival) in enumerate(specs):
        out.append(Request(rid=i, geometry=geom, make_points=lambda: None, n_points=n, kappa=1.0,
                           n_matvecs=4, arrival=arrival))
    return out


def test_all_complete_in_arrival_order_with_results():
    ex = FakeExecutor()
    rs = reqs([(f"g{i}", 1000 + 10 * i, 0.001 * i) for i in range(10)])
    out = Scheduler(ex, budget_bytes=10 ** 9, max_slots=4, keep_results=True).run(rs)
    assert [o.rid for o in out] == list(range(10)) and all(o.ok for o in out)
    assert [r for r, _ in ex.admit_log] == list(range(10))  # FIFO admission
    for o in out:
        assert o.done >= o.admitted >= o.arrival and len(o.matvec_ms) == 4
        assert o.results[2][0] == o.rid * 10 + 2
    assert not ex.live_plans  # every plan released at the end


def test_budget_forces_queueing_and_is_never_exceeded():
    ex = FakeExecutor()
    rs = reqs([(f"g{i}", 1000, 0.0) for i in range(6)])
    sch = Scheduler(ex, budget_bytes=45_000, max_slots=8)  # one (plan + workspace) of 30 kB fits
    out = sch.run(rs)
    assert all(o.ok for o in out)
    assert sch.stats["max_running"] == 1 and sch.stats["peak_bytes"] <= 45_000
    ends = sorted(o.done for o in out)
    starts = sorted(o.admitted for o in out)
    assert all(starts[i + 1] >= ends[i] - 1e-12 for i in range(5))  # strictly one after another


def test_plan_cache_hits_and_lru_eviction():
    ex = FakeExecutor()
    specs = [("a", 1000, 0.0), ("b", 1000, 0.0), ("a", 1000, 0.01), ("a", 1000, 0.02), ("c", 1000, 0.03),
             ("b", 1000, 0.04)]
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_slots=2)
    out = sch.run(reqs(specs))
    assert all(o.ok for o in out)
    assert sch.stats["builds"] == 3 and sch.stats["cache_hits"] == 3
    assert [o.plan_cached for o in out] == [False, False, True, True, False, True]
    # a budget for two plans and one workspace: plans are evicted, never while in use
    ex2 = FakeExecutor()
    sch2 = Scheduler(ex2, budget_bytes=40_000, max_slots=1)
    out2 = sch2.run(reqs(specs))
    assert all(o.ok for o in out2) and sch2.stats["evictions"] > 0


def test_continuous_batching_admits_while_others_run():
    ex = FakeExecutor(us_per_point=10.0)
    rs = reqs([("g0", 5000, 0.0), ("g1", 5000, 0.0), ("g2", 1000, 0.05), ("g3", 1000, 0.06), ("g4", 1000, 0.3)])
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_slots=3)
    out = sch.run(rs)
    assert sch.stats["max_running"] == 3
    # the late arrivals started before the first two finished
    assert out[2].admitted < out[0].done and out[3].admitted < out[1].done
    # latency includes the queueing behind the slot limit
    assert out[3].admitted >= out[2].done - 1e-12 or out[3].admitted >= out[3].arrival


def test_failures_are_isolated():
    ex = FakeExecutor(fail_on={2})
    rs = reqs([(f"g{i}", 1000, 0.0) for i in range(5)] + [("huge", 10 ** 7, 0.0)])
    sch = Scheduler(ex, budget_bytes=10 ** 6, max_slots=2)
    out = sch.run(rs)
    assert not out[2].ok and "plan creation failed" in out[2].error
    assert not out[5].ok and "budget" in out[5].error
    assert all(out[i].ok for i in (0, 1, 3, 4))
    assert sch.stats["failed"] == 2


def test_low_estimates_keep_the_budget():
    class LowEstimate(FakeExecutor):
        def estimate(self, req):
            return 1, 1  # far below what build() reports

    ex = LowEstimate()
    rs = reqs([(f"g{i}", 1000, 0.0) for i in range(5)] + [("big", 2000, 0.0)])
    sch = Scheduler(ex, budget_bytes=50_000, max_slots=4)
    out = sch.run(rs)
    assert all(o.ok for o in out[:5]) and sch.stats["peak_bytes"] <= 50_000
    assert not out[5].ok and "budget" in out[5].error  # 60 kB can never fit


def test_workspaces_are_pooled_per_plan():
    ex = FakeExecutor()
    rs = reqs([("a", 1000, 0.0), ("a", 1000, 0.1), ("a", 1000, 0.2), ("b", 1000, 0.3)])
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_slots=1)
    out = sch.run(rs)
    assert all(o.ok for o in out)
    # plan a + one workspace kept and reused, then plan b + its workspace
    assert sch.stats["peak_bytes"] == 2 * (10 + 20) * 1000


def test_graph_replay_in_the_executor_is_closed():
    """Graph replay inside the serving executor stays disabled until the cause
    of the host fault seen with it is known: asking for it raises at once."""
    from paper_2202_04894_amd import serving as S
    with pytest.raises(NotImplementedError):
        S.DeviceExecutor(graphs=True)


def test_requests_carry_the_setting_of_their_order_and_kappa():
    """Each serving request carries the knob setting measured within 1e-4 of
    the direct sum for its order and kappa*D band (the finer setting for L = 4
    at high kappa*D); the paper-literal mode gives every request (1, 2, 0)."""
    from paper_2202_04894_amd import serving as S
    reqs = S.config_requests(n_requests=64, n_geometries=16, seed=7)
    seen = set()
    for r in reqs:
        kd = 2.0 * r.kappa
        want = (S.ACCURATE_KNOBS_HIGH_KD if kd >= S.HIGH_KD else S.ACCURATE_KNOBS)[r.order_L]
        assert r.knobs == want, (r.order_L, kd, r.knobs)
        seen.add((r.order_L, kd >= S.HIGH_KD))
    assert len(seen) >= 3  # both orders and both bands appear in the mix
    assert S.accurate_knobs(4, 250.0) == (0.1, 0.75, 2) and S.accurate_knobs(4, 32.0) == (0.15, 0.75, 2)
    lit = S.config_requests(n_requests=8, n_geometries=4, seed=7, accurate=False)
    assert all(r.knobs == S.LITERAL_KNOBS for r in lit)
