"""Admission and scheduling logic of the serving loop, on the CPU with fake backends (mock
footprints and durations; a virtual clock for one lane, short real sleeps for two lanes)."""

import time
from types import SimpleNamespace

import pytest

from paper_2511_06824_amd.serve import AdmissionController, GapServer, LaneServer, Request, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class FakeBackend:
    """Every step costs step_time of virtual time and advances all active requests."""

    def __init__(self, clock, step_time=1.0):
        self.clock, self.step_time = clock, step_time
        self.live = []
        self.max_active = 0
        self.started = []

    def footprint(self, case):
        return case.fake_bytes

    def start(self, req):
        self.live.append([req, req.case.fake_steps])
        self.started.append(req.rid)
        self.max_active = max(self.max_active, len(self.live))

    def step(self):
        self.clock.t += self.step_time
        out = []
        sel = getattr(self, "selected", None)
        for item in self.live:
            if sel is None or item[0].rid in sel:
                item[1] -= 1
        for item in [x for x in self.live if x[1] <= 0]:
            self.live.remove(item)
            out.append(item[0])
        return out

    def idle(self):
        return not self.live

    @staticmethod
    def work(case):
        return case.fake_work

    def active(self):
        return [x[0] for x in self.live]

    def select(self, chosen):
        self.selected = {r.rid for r in chosen}


def req(rid, arrival, nbytes, steps, nt=64, nz=32, work=1):
    return Request(rid=rid, case=SimpleNamespace(fake_bytes=nbytes, fake_steps=steps, n_theta=nt, n_axial=nz,
                                                 fake_work=work), arrival=arrival)


def test_admission_controller_budget_and_slots():
    a = AdmissionController(100, max_active=2)
    assert a.admit(60) and not a.fits(50) and a.admit(40) and not a.admit(0)
    a.release(60)
    assert a.fits(50) and a.used == 40
    with pytest.raises(AssertionError):
        a.release(1000)


def test_requests_overlap_and_respect_the_budget():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = GapServer(be, budget_bytes=100, clock=clock)
    rs = [req(0, 0.0, 50, 5), req(1, 0.5, 50, 2), req(2, 0.6, 50, 1), req(3, 10.0, 30, 1)]
    done = srv.run(rs)
    assert sorted(r.rid for r in done) == [0, 1, 2, 3]
    assert be.max_active == 2                       # never more than the budget allows
    assert be.started == [0, 1, 2, 3]              # admitted in arrival order
    r2 = next(r for r in done if r.rid == 2)
    r1 = next(r for r in done if r.rid == 1)
    assert r2.admitted >= r1.finished              # waited for memory to free up
    r3 = next(r for r in done if r.rid == 3)
    assert r3.admitted == 10.0                     # idle server sleeps until the arrival
    assert all(r.latency > 0 for r in done)
    stats = latency_stats(done)
    assert stats["requests"] == 4 and stats["p99_s"] >= stats["p50_s"] > 0


def test_no_overtaking_in_the_queue():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = GapServer(be, budget_bytes=100, clock=clock)
    # a big request at the head blocks smaller ones behind it until it fits
    rs = [req(0, 0.0, 80, 3), req(1, 0.1, 90, 1), req(2, 0.2, 10, 1)]
    srv.run(rs)
    assert be.started == [0, 1, 2]


def test_request_larger_than_budget_is_rejected():
    clock = FakeClock()
    srv = GapServer(FakeBackend(clock), budget_bytes=10, clock=clock)
    with pytest.raises(ValueError):
        srv.run([req(0, 0.0, 11, 1)])


def test_work_cap_runs_large_requests_in_order_and_small_ones_beside_them():
    """Cap 5: two large requests (work 4) run one after the other; small ones (work 1)
    advance beside whichever large one runs."""
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = GapServer(be, budget_bytes=1000, clock=clock, work_cap=5, order="oldest")
    rs = [req(0, 0.0, 10, 4, work=4), req(1, 0.0, 10, 4, work=4), req(2, 0.5, 10, 2, work=1)]
    done = {r.rid: r for r in srv.run(rs)}
    assert done[0].finished == 4.0                 # the oldest large request is never held
    assert done[2].finished == 3.0                 # the small one advanced beside it
    assert done[1].finished == 8.0                 # the second large one waited, then ran alone


def test_without_a_cap_all_admitted_requests_share_each_step():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = GapServer(be, budget_bytes=1000, clock=clock)
    rs = [req(0, 0.0, 10, 4, work=4), req(1, 0.0, 10, 4, work=4)]
    done = {r.rid: r for r in srv.run(rs)}
    assert done[0].finished == done[1].finished == 4.0


def test_smallest_first_lets_small_requests_pass_a_large_one():
    """Cap 4 (one large request): the large request yields while small ones are present;
    small ones advance together."""
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = GapServer(be, budget_bytes=1000, clock=clock, work_cap=4)
    rs = [req(0, 0.0, 10, 5, work=4), req(1, 1.5, 10, 2, work=1), req(2, 1.5, 10, 2, work=1)]
    done = {r.rid: r for r in srv.run(rs)}
    # t=0..2: the large one alone (3 steps left); t=2..4: the two small ones together; then it resumes
    assert done[1].finished == done[2].finished == 4.0
    assert done[0].finished == 7.0
    with pytest.raises(ValueError):
        GapServer(be, budget_bytes=1, clock=clock, order="random")


class SleepBackend:
    """Real-time fake for the lane tests: every step sleeps step_s of wall time and advances
    every active request (or the selected ones) by one step."""

    def __init__(self, step_s):
        self.step_s = step_s
        self.live = []
        self.started = []
        self.selected = None
        self.max_work = 0

    def footprint(self, case):
        return case.fake_bytes

    @staticmethod
    def work(case):
        return case.fake_work

    def start(self, req):
        self.live.append([req, req.case.fake_steps])
        self.started.append(req.rid)

    def active(self):
        return [x[0] for x in self.live]

    def select(self, chosen):
        self.selected = {r.rid for r in chosen}

    def step(self):
        time.sleep(self.step_s)
        moving = [x for x in self.live if self.selected is None or x[0].rid in self.selected]
        self.max_work = max(self.max_work, sum(self.work(x[0].case) for x in moving))
        for x in moving:
            x[1] -= 1
        out = [x[0] for x in self.live if x[1] <= 0]
        self.live = [x for x in self.live if x[1] > 0]
        return out

    def idle(self):
        return not self.live


def test_lanes_split_by_work_and_small_requests_do_not_wait_for_bulk_ones():
    bulk, fast = SleepBackend(0.004), SleepBackend(0.001)
    srv = LaneServer(bulk, fast, budget_bytes=1000, bulk_work=4)
    rs = [req(0, 0.0, 100, 40, work=4), req(1, 0.0, 100, 40, work=4),
          req(2, 0.02, 10, 3, work=1), req(3, 0.03, 10, 3, work=2), req(4, 0.05, 10, 2, work=1)]
    done = {r.rid: r for r in srv.run(rs)}
    assert sorted(done) == [0, 1, 2, 3, 4]
    assert {r.meta["lane"] for r in rs if r.rid < 2} == {"bulk"}
    assert {r.meta["lane"] for r in rs if r.rid >= 2} == {"fast"}
    assert bulk.started == [0, 1] and fast.started == [2, 3, 4]
    assert bulk.max_work == 4                      # bulk requests never advance together
    assert done[1].finished > done[0].finished     # arrival order within the bulk lane
    for k in (2, 3, 4):                            # the small ones finish while bulk work runs
        assert done[k].finished < done[0].finished
    assert srv.admission.used == 0 and srv.admission.active == 0


def test_lanes_share_one_budget_and_wait_for_each_other():
    bulk, fast = SleepBackend(0.002), SleepBackend(0.001)
    srv = LaneServer(bulk, fast, budget_bytes=100, bulk_work=4)
    # each request needs 60 of the 100 bytes: at most one is on the device at any time
    rs = [req(0, 0.0, 60, 10, work=4), req(1, 0.001, 60, 5, work=1), req(2, 0.002, 60, 5, work=1)]
    done = {r.rid: r for r in srv.run(rs)}
    assert sorted(done) == [0, 1, 2]
    assert srv.admission.peak <= 100
    spans = sorted((r.admitted, r.finished) for r in done.values())
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0                            # never two on the device together


def test_large_fast_requests_yield_to_bulk_work_within_a_bound():
    bulk, fast = SleepBackend(0.003), SleepBackend(0.001)
    srv = LaneServer(bulk, fast, budget_bytes=1000, bulk_work=4, fast_cap=10, yield_work=1)
    # bulk request 0 runs about 0.09 s; fast request 1 (work 2) yields while it runs, the
    # small request 2 (work 1) does not
    rs = [req(0, 0.0, 100, 30, work=4), req(1, 0.005, 10, 3, work=2), req(2, 0.005, 10, 3, work=1)]
    done = {r.rid: r for r in srv.run(rs)}
    assert done[2].finished < done[0].finished
    assert done[1].finished >= done[0].finished
    # with a bound on the wait, the large request moves before the bulk work ends
    bulk, fast = SleepBackend(0.003), SleepBackend(0.001)
    srv = LaneServer(bulk, fast, budget_bytes=1000, bulk_work=4, fast_cap=10, yield_work=1, max_yield_s=0.02)
    rs = [req(0, 0.0, 100, 30, work=4), req(1, 0.005, 10, 3, work=2)]
    done = {r.rid: r for r in srv.run(rs)}
    assert done[1].finished < done[0].finished
    assert srv.admission.used == 0 and srv.admission.active == 0


def test_a_failing_lane_raises_in_the_caller():
    bulk, fast = SleepBackend(0.001), SleepBackend(0.001)
    srv = LaneServer(bulk, fast, budget_bytes=50, bulk_work=4)
    with pytest.raises(ValueError):
        srv.run([req(0, 0.0, 60, 2, work=4), req(1, 0.0, 10, 2, work=1)])


class FakeSolver:
    """Stands in for JointGapSolver in the handle-pool test (no device)."""
    made = 0

    def __init__(self, case):
        FakeSolver.made += 1
        self.case, self.textures, self.closed = case, [case.fake_tex], False

    @staticmethod
    def geometry_key(case):
        return (case.n_theta, case.n_axial)

    @staticmethod
    def case_dimples(case):
        return case.fake_tex

    @classmethod
    def from_case(cls, case, max_cond=9, device=None):
        return cls(case)

    def set_dimples(self, dimples):
        self.textures.append(dimples)

    def close(self):
        self.closed = True


def test_handle_pool_reuses_handles_of_the_same_grid_and_bounds_the_idle_ones():
    from paper_2511_06824_amd.serve import HandlePool
    pool = HandlePool(device=None, per_key=2)
    pool.Solver = FakeSolver
    FakeSolver.made = 0

    def case(nt, nz, tex):
        return SimpleNamespace(n_theta=nt, n_axial=nz, fake_tex=tex)

    a = pool.get(case(64, 32, "A"))
    b = pool.get(case(64, 32, "B"))
    c = pool.get(case(128, 64, "C"))
    assert FakeSolver.made == 3 and pool.created == 3 and pool.reused == 0
    pool.put(a)
    d = pool.get(case(64, 32, "D"))               # the idle 64x32 handle, re-textured
    assert d is a and a.textures == ["A", "D"] and pool.reused == 1
    e = pool.get(case(128, 64, "E"))              # no idle 128x64 handle: a new one
    assert e is not c and FakeSolver.made == 4
    extra = [pool.get(case(64, 32, "F")) for _ in range(2)]
    for s in [a, b] + extra:                      # 4 idle 64x32 handles offered, 2 kept
        pool.put(s)
    assert sum(s.closed for s in [a, b] + extra) == 2
    pool.close()
    assert all(s.closed for s in [a, b] + extra)
