"""Continuous-batching service for joint piston-gap solves.

Requests (one joint 9-condition solve each, any grid size) arrive over time.  A request is
admitted as soon as its device footprint fits the HBM budget and a batch slot is free; it is
then given a handle (a finished request's handle of the same grid and geometry, re-textured
by set_gap_dimples, or a new one), assembled and joins the running batch, whose every step advances all active requests
by a block of PCG iterations with one launch per kernel per iteration (gap_batch_* in the
HIP library).  Finished requests are integrated (forces, FD Jacobian), their budget is
released (their handle waits for the next request of its grid) and the next queued requests
are admitted.  Reusing handles keeps device allocation, and the device-wide synchronization
that freeing memory implies, out of the serving loop.  Latency = completion - arrival.

Scheduling inside the batch: without a work cap every admitted request advances in every
step (processor sharing).  With ``work_cap`` (condition-DOFs per step), each step advances
admitted requests in the order of ``order`` while their summed size fits the cap (the first
one always advances) and holds the rest on the device (``gap_batch_hold``):
  * "smallest" (default): smallest request first, then arrival.  Small requests, which
    cannot fill the GPU alone, advance together; a request as large as the cap runs alone at
    full bandwidth and yields to small requests while they are present.
  * "oldest": arrival order; large requests run one after another and small ones fill what
    the cap leaves beside them.

Two lanes (``LaneServer``): bulk requests, those whose own launches fill the GPU, run in a
batch of their own, one after another in arrival order; the others share the steps of a
second batch.  Each lane has its own stream and host thread, so the small requests iterate at
the pace of their own short launches, concurrently with the bulk launches (which are chunked
to leave room on every CU for them, ``gap_batch_set_target``), and never wait for a bulk
request to finish.  Both lanes draw on one HBM budget.

The admission and scheduling logic (``AdmissionController``, ``GapServer``, ``LaneServer``)
is independent of the device: ``BatchBackend`` drives the HIP library, tests may substitute
a fake backend with its own clock.
"""

import threading
import time
from dataclasses import dataclass, field
from typing import Any, List, Optional

import numpy as np


class AdmissionController:
    """Admits requests while their summed device footprint stays within a byte budget (safe
    to share between the lanes' threads)."""

    def __init__(self, budget_bytes, max_active=128):
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.used = 0
        self.active = 0
        self.peak = 0
        self._lock = threading.Lock()

    def fits(self, nbytes):
        with self._lock:
            return self.active < self.max_active and self.used + nbytes <= self.budget

    def admit(self, nbytes):
        with self._lock:
            if not (self.active < self.max_active and self.used + nbytes <= self.budget):
                return False
            self.used += nbytes
            self.active += 1
            self.peak = max(self.peak, self.used)
            return True

    def release(self, nbytes):
        with self._lock:
            self.used -= nbytes
            self.active -= 1
            assert self.used >= 0 and self.active >= 0


@dataclass
class Request:
    rid: int
    case: Any
    arrival: float
    nbytes: int = 0
    admitted: Optional[float] = None
    finished: Optional[float] = None
    iterations: int = 0
    status: int = 0
    F: Optional[np.ndarray] = None
    J: Optional[np.ndarray] = None
    p: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def size_class(self):
        return f"{self.case.n_theta}x{self.case.n_axial}"

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


class HandlePool:
    """Idle JointGapSolver handles by grid and geometry, reused for later requests of the same
    grid (re-textured with set_gap_dimples); at most `per_key` idle handles are kept per key."""

    def __init__(self, device, per_key=4):
        from .solver import JointGapSolver
        self.Solver, self.device, self.per_key = JointGapSolver, device, int(per_key)
        self.idle = {}
        self.created = 0
        self.reused = 0

    def get(self, case):
        key = self.Solver.geometry_key(case)
        free = self.idle.get(key)
        if free:
            s = free.pop()
            s.set_dimples(self.Solver.case_dimples(case))
            self.reused += 1
        else:
            s = self.Solver.from_case(case, max_cond=9, device=self.device)
            self.created += 1
        s.pool_key = key
        return s

    def put(self, s):
        free = self.idle.setdefault(s.pool_key, [])
        if len(free) < self.per_key:
            free.append(s)
        else:
            s.close()

    def close(self):
        for free in self.idle.values():
            for s in free:
                s.close()
        self.idle.clear()


class BatchBackend:
    """Drives the HIP library: one JointGapSolver handle per request (from a HandlePool), one
    gap_batch.

    ``stream``: the stream every call of this backend runs on (default: the current stream of
    the thread that creates it); ``wg_per_cu``: the strip kernel's chunking target for the
    requests of this batch (0: the kernel's occupancy); ``iteration``: the launch scheme of its
    requests (default: the library's, strips)."""

    def __init__(self, device="cuda:0", iterations_per_step=32, use_graph=True, keep_pressure=False,
                 stream=None, wg_per_cu=0, iteration=None):
        import torch
        from . import gapsolve as G
        from .solver import JointGapSolver
        self.torch, self.G, self.Solver = torch, G, JointGapSolver
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.iters = int(iterations_per_step)
        self.use_graph = use_graph
        self.keep_pressure = keep_pressure
        self.kind = {} if iteration is None else {"iteration": int(iteration)}
        self.pool = HandlePool(self.device)
        self.batch = G.gap_batch_create()
        G.gap_batch_set_target(self.batch, wg_per_cu)
        self.live = {}

    def footprint(self, case):
        return self.Solver.device_bytes(case.n_theta, case.n_axial, 9)

    @staticmethod
    def work(case):
        """Per-iteration size of a request: condition-DOFs."""
        return 9 * case.n_theta * case.n_axial

    def active(self):
        return [req for _, req, _ in self.live.values()]

    def select(self, chosen):
        """Advance only the requests in `chosen` in the next steps; hold the others."""
        keep = {id(r) for r in chosen}
        for bid, (s, req, _) in self.live.items():
            held = id(req) not in keep
            if held != req.meta.get("held", False):
                self.G.gap_batch_hold(self.batch, bid, held)
                req.meta["held"] = held

    def start(self, req):
        case = req.case
        with self.torch.cuda.stream(self.stream):
            s = self.pool.get(case)
            s.assemble(case.e, case.edot, case.delta, 9)
            opts = s.options(omega=case.omega, eps=case.eps, **self.kind)
            bid = self.G.gap_batch_add(self.batch, s.handle, opts, s.p.data_ptr(), self.stream.cuda_stream)
        self.live[bid] = (s, req, opts)

    def step(self):
        """Advance every active request; return the requests finished in this step."""
        stream = self.stream.cuda_stream
        self.G.gap_batch_step(self.batch, self.iters, self.use_graph, stream)
        out = []
        with self.torch.cuda.stream(self.stream):
            for bid in self.G.gap_batch_poll(self.batch):
                s, req, _ = self.live.pop(bid)
                st, info = self.G.gap_batch_remove(self.batch, bid, stream, raise_on_error=False)
                req.status, req.iterations = st, info.iterations
                req.F = s.integrate().cpu().numpy().copy()
                req.J = s.jacobian_fd().cpu().numpy().copy()
                if self.keep_pressure:
                    req.p = s.pressure().cpu().numpy().copy()
                self.pool.put(s)
                out.append(req)
        return out

    def idle(self):
        return not self.live

    def close(self):
        self.G.gap_batch_destroy(self.batch)       # releases the grids still in the batch
        self.batch = None
        for s, _, _ in self.live.values():
            s.close()
        self.live.clear()
        self.pool.close()


class GapServer:
    """Event loop: admit by arrival order and budget, step the batch, retire finished work."""

    def __init__(self, backend, budget_bytes, clock=None, work_cap=None, order="smallest", admission=None,
                 poll_s=5e-4, hold_if=None, max_hold_s=float("inf")):
        if order not in ("smallest", "oldest"):
            raise ValueError(f"unknown order {order!r}")
        self.backend = backend
        self.admission = admission if admission is not None else AdmissionController(budget_bytes)
        self.poll_s = poll_s                   # wait while another lane holds the memory a request needs
        self.clock = clock or WallClock()
        self.work_cap = work_cap
        self.order = order
        # hold_if(request): the request yields for now (it does not advance), but never for
        # more than max_hold_s after its admission
        self.hold_if = hold_if
        self.max_hold_s = max_hold_s

    def _schedule(self):
        """Requests in scheduling order while the summed work fits the cap (no cap: all); the
        first always advances, except those that yield.  Returns whether any request advances."""
        if self.order == "smallest":
            key = lambda q: (self.backend.work(q.case), q.arrival, q.rid)
        else:
            key = lambda q: (q.arrival, q.rid)
        now = self.clock.now()
        chosen, total = [], 0
        for r in sorted(self.backend.active(), key=key):
            if self.hold_if is not None and now - r.admitted < self.max_hold_s and self.hold_if(r):
                continue
            w = self.backend.work(r.case)
            if not chosen or self.work_cap is None or total + w <= self.work_cap:
                chosen.append(r)
                total += w
        self.backend.select(chosen)
        return bool(chosen)

    def run(self, requests: List[Request]):
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            r.nbytes = self.backend.footprint(r.case)
            if r.nbytes > self.admission.budget:
                raise ValueError(f"request {r.rid} needs {r.nbytes} bytes, more than the whole budget")
        done = []
        queue = []
        while pending or queue or not self.backend.idle():
            now = self.clock.now()
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            # admit in arrival order while memory and slots allow (no overtaking)
            while queue and self.admission.admit(queue[0].nbytes):
                r = queue.pop(0)
                r.admitted = self.clock.now()
                self.backend.start(r)
            if self.backend.idle():
                if queue:                      # only with a shared budget: another lane holds it
                    self.clock.sleep_until(self.clock.now() + self.poll_s)
                elif pending:
                    self.clock.sleep_until(pending[0].arrival)
                continue
            if (self.work_cap is not None or self.hold_if is not None) and not self._schedule():
                self.clock.sleep_until(self.clock.now() + self.poll_s)   # every active request yields
                continue
            for r in self.backend.step():
                r.finished = self.clock.now()
                self.admission.release(r.nbytes)
                done.append(r)
        return done


class LaneServer:
    """Two lanes over one HBM budget and one clock, each a GapServer with its own backend
    (batch, stream) driven by its own thread.  Requests of work >= ``bulk_work`` (condition-
    DOFs per iteration) go to the bulk lane, which runs them in arrival order, advancing
    together only those that fit ``bulk_cap`` (default: bulk_work); the others go to the fast
    lane, where every admitted request advances in every step, or, with ``fast_cap``, the
    smallest ones first while their work fits the cap.  With ``yield_work``, a fast-lane
    request of more work than that does not advance while the bulk lane has work, for at most
    ``max_yield_s`` after its admission: the bulk requests, which set the tail, then keep the
    device's bandwidth to themselves, and the small requests still run beside them."""

    def __init__(self, bulk, fast, budget_bytes, bulk_work, clock=None, bulk_cap=None, fast_cap=None,
                 yield_work=None, max_yield_s=float("inf")):
        self.admission = AdmissionController(budget_bytes)
        self.clock = clock or WallClock()
        self.bulk_work = int(bulk_work)
        hold_if = None
        if yield_work is not None:
            hold_if = lambda r: (not bulk.idle()) and fast.work(r.case) > yield_work
        self.lanes = {
            "bulk": GapServer(bulk, budget_bytes, clock=self.clock, work_cap=bulk_cap or self.bulk_work,
                              order="oldest", admission=self.admission),
            "fast": GapServer(fast, budget_bytes, clock=self.clock, work_cap=fast_cap, order="smallest",
                              admission=self.admission, hold_if=hold_if, max_hold_s=max_yield_s),
        }

    def lane_of(self, req):
        return "bulk" if self.lanes["bulk"].backend.work(req.case) >= self.bulk_work else "fast"

    def run(self, requests: List[Request]):
        parts = {"bulk": [], "fast": []}
        for r in requests:
            r.meta["lane"] = self.lane_of(r)
            parts[r.meta["lane"]].append(r)
        done, errors = {}, []

        def drive(name):
            try:
                done[name] = self.lanes[name].run(parts[name])
            except BaseException as exc:           # re-raised in the caller's thread
                errors.append(exc)

        threads = [threading.Thread(target=drive, args=(name,), name=f"lane-{name}") for name in parts if parts[name]]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
        return sorted((r for lane in done.values() for r in lane), key=lambda r: r.finished)


def latency_stats(done):
    """p50 / p99 latency overall and per size class, and throughput."""
    lat = np.array([r.latency for r in done])
    t_first = min(r.arrival for r in done)
    t_last = max(r.finished for r in done)
    out = {"requests": len(done), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "mean_s": float(lat.mean()), "solves_per_s": len(done) / (t_last - t_first), "per_class": {}}
    for cls in sorted({r.size_class for r in done}, key=lambda c: int(c.split("x")[0])):
        lc = np.array([r.latency for r in done if r.size_class == cls])
        out["per_class"][cls] = {"n": int(lc.size), "p50_s": float(np.percentile(lc, 50)),
                                 "p99_s": float(np.percentile(lc, 99))}
    return out


def run_fifo(requests, device="cuda:0", clock=None, pool=None):
    """Baseline: the same requests solved one at a time in arrival order, each a joint solve
    of its own (no batching), on handles reused through a HandlePool as the batched server
    reuses them (pass one to keep it across calls)."""
    import torch
    clock = clock or WallClock()
    own = pool is None
    pool = pool or HandlePool(torch.device(device))
    done = []
    for r in sorted(requests, key=lambda q: q.arrival):
        clock.sleep_until(r.arrival)
        r.admitted = clock.now()
        s = pool.get(r.case)
        s.assemble(r.case.e, r.case.edot, r.case.delta, 9)
        _, info = s.solve(omega=r.case.omega, eps=r.case.eps)
        r.iterations = info.iterations
        r.F = s.integrate().cpu().numpy().copy()
        r.J = s.jacobian_fd().cpu().numpy().copy()
        pool.put(s)
        r.finished = clock.now()
        done.append(r)
    if own:
        pool.close()
    return done
