"""GPU tests of batched execution and the serving loop: each request's result is bitwise
the same alone and in a mix of grid sizes, matches the oracle, and a Poisson stream drains."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of, texture_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_06824_amd import gapsolve as G  # noqa: E402
from paper_2511_06824_amd.serve import BatchBackend, GapServer, LaneServer, Request, latency_stats  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402


def log(msg):
    print(msg, flush=True)


CASES = [synth.smooth_case(64, 32, 0), synth.textured_case(128, 64, 1), synth.smooth_case(200, 37, 2),
         synth.textured_case(256, 128, 3), synth.smooth_case(96, 48, 4, eps=1e-12)]


ITERATIONS = pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                                      G.GAP_ITERATION_STRIPS],
                                     ids=["two_launch", "one_launch", "strips"])


def batch_solve(cases, eps_override=None, iters=8, use_graph=True, iteration=G.GAP_ITERATION_ONE_LAUNCH,
                join_every=0, neumann=1, target=0):
    """Solve the cases together in one batch; returns pressures, infos by case index.
    join_every > 0: the cases join one at a time, one step of `iters` iterations apart.
    target > 0: the strip chunking aims at that many workgroups per CU."""
    b = G.gap_batch_create()
    if target:
        G.gap_batch_set_target(b, target)
    stream = torch.cuda.current_stream().cuda_stream
    solvers, ids = [], []
    pending = list(cases)
    out = {}

    def add(c):
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        opts = s.options(omega=c.omega, eps=eps_override or c.eps, iteration=iteration, neumann=neumann)
        ids.append(G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream))
        solvers.append((s, opts))

    while pending and (not join_every or not ids):
        add(pending.pop(0))
    while len(out) < len(cases):
        if pending and join_every:
            add(pending.pop(0))
        G.gap_batch_step(b, iters, use_graph, stream)
        for bid in G.gap_batch_poll(b):
            k = ids.index(bid)
            st, info = G.gap_batch_remove(b, bid, stream)
            s = solvers[k][0]
            out[k] = (s.pressure().cpu().numpy().copy(), info.iterations, s.integrate().cpu().numpy().copy())
    for s, _ in solvers:
        s.close()
    G.gap_batch_destroy(b)
    return out


@ITERATIONS
def test_results_alone_and_in_the_mix_are_bitwise_equal(iteration):
    log(f"case: batch mix of 5 grids vs each alone, iteration kind {iteration}")
    mix = batch_solve(CASES, iteration=iteration)
    staggered = batch_solve(CASES, iteration=iteration, iters=7, join_every=1)   # joins at odd launch counts
    for k, c in enumerate(CASES):
        alone = batch_solve([c], iteration=iteration)[0]
        for other in (mix[k], staggered[k]):
            assert alone[1] == other[1]
            assert np.array_equal(alone[0], other[0]), c.label
            assert np.array_equal(alone[2], other[2]), c.label


def test_strip_march_with_and_without_barriers_is_bitwise_equal():
    """At order 1 a strip request that streams more than 512 MiB per iteration runs the march
    with a workgroup barrier per period when it is alone; in a batch with a small request the
    launch runs the march without barriers for both.  The two forms compute the same values
    in the same order, so the large request's results are bitwise equal.  2100 x 640 with 9
    conditions on 5 operators streams 1344000 x (9 x 40 + 5 x 16) B = 591 MB; its rings are
    cut into 41 strips, so the last workgroup of each row chunk has three wavefronts without
    a strip, which meet the barriers all the same."""
    big = synth.textured_case(2100, 640, 11)
    log(f"case: {big.label} alone (barriers) and with {CASES[0].label} (no barriers), strips")
    alone = batch_solve([big], iteration=G.GAP_ITERATION_STRIPS)[0]
    mixed = batch_solve([big, CASES[0]], iteration=G.GAP_ITERATION_STRIPS)[0]
    assert alone[1] == mixed[1]
    assert np.array_equal(alone[0], mixed[0])
    assert np.array_equal(alone[2], mixed[2])


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_ONE_LAUNCH, G.GAP_ITERATION_STRIPS],
                         ids=["one_launch", "strips"])
def test_one_launch_batch_matches_a_solve_of_its_own(iteration):
    """A request in a one-launch batch, joining at an odd launch count, takes the iterations
    of the same grid solved by solve_joint_pcg (its chunking follows the batch shape, so the
    iterates agree up to the summation order)."""
    c = synth.textured_case(192, 64, 10)
    log(f"case: {c.label}, batch vs own solve, iteration kind {iteration}")
    got = batch_solve([CASES[0], c], iters=5, join_every=1, eps_override=1e-12, iteration=iteration)[1]
    s = JointGapSolver.from_case(c, max_cond=9)
    s.assemble(c.e, c.edot, c.delta, 9)
    p, info = s.solve(omega=c.omega, eps=1e-12, iteration=iteration)
    p = p.cpu().numpy()
    s.close()
    assert abs(info.iterations - got[1]) <= 1
    for k in range(9):
        assert np.linalg.norm(got[0][k] - p[k]) <= 1e-10 * np.linalg.norm(p[k])


def test_neumann_order_batch_matches_own_solves_and_refuses_another_order():
    """Requests at Neumann order 2 in one strip batch, joining at odd launch counts, take the
    iterations of their own solves at that order; a request at another order is refused."""
    cases = [synth.textured_case(192, 64, 10), synth.smooth_case(130, 77, 11)]
    log("case: strip batch at Neumann order 2")
    got = batch_solve(cases, iters=5, join_every=1, eps_override=1e-12, iteration=G.GAP_ITERATION_STRIPS,
                      neumann=2)
    for k, c in enumerate(cases):
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        p, info = s.solve(omega=c.omega, eps=1e-12, neumann=2, iteration=G.GAP_ITERATION_STRIPS)
        p = p.cpu().numpy()
        s.close()
        log(f"  {c.label}: batch {got[k][1]} iterations, own solve {info.iterations}")
        assert abs(info.iterations - got[k][1]) <= 1
        for j in range(9):
            assert np.linalg.norm(got[k][0][j] - p[j]) <= 1e-10 * np.linalg.norm(p[j])
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    made = []
    for k, m in enumerate((2, 1)):
        c = synth.smooth_case(64, 32, 40 + k)
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        made.append(s)
        opts = s.options(omega=c.omega, eps=c.eps, iteration=G.GAP_ITERATION_STRIPS, neumann=m)
        if k == 0:
            bid = G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream)
        else:
            with pytest.raises(G.GapError) as ei:
                G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream)
            assert ei.value.status == G.GAP_EINVAL
    while not G.gap_batch_poll(b):
        G.gap_batch_step(b, 16, True, stream)
    G.gap_batch_remove(b, bid, stream)
    for s in made:
        s.close()
    G.gap_batch_destroy(b)


def test_batch_refuses_a_second_iteration_kind():
    log("case: batch with mixed iteration kinds")
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    made = []
    for k, it in enumerate((G.GAP_ITERATION_ONE_LAUNCH, G.GAP_ITERATION_TWO_LAUNCH)):
        c = synth.smooth_case(64, 32, 30 + k)
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        made.append(s)
        opts = s.options(omega=c.omega, eps=c.eps, iteration=it)
        if k == 0:
            bid = G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream)
        else:
            with pytest.raises(G.GapError) as ei:
                G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream)
            assert ei.value.status == G.GAP_EINVAL
    while not G.gap_batch_poll(b):
        G.gap_batch_step(b, 16, True, stream)
    G.gap_batch_remove(b, bid, stream)
    # empty again: the next request sets the kind
    s = made[1]
    opts = s.options(omega=1.6, eps=1e-10, iteration=G.GAP_ITERATION_TWO_LAUNCH)
    bid = G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream)
    while not G.gap_batch_poll(b):
        G.gap_batch_step(b, 16, True, stream)
    _, info = G.gap_batch_remove(b, bid, stream)
    assert info.status == G.GAP_OK
    for s in made:
        s.close()
    G.gap_batch_destroy(b)


@ITERATIONS
def test_batched_results_match_the_oracle(iteration):
    log(f"case: batch mix vs oracle, iteration kind {iteration}")
    cases = [synth.smooth_case(64, 32, 5), synth.textured_case(96, 48, 6)]
    got = batch_solve(cases, eps_override=1e-13, use_graph=False, iteration=iteration)
    for k, c in enumerate(cases):
        gap, tex = gap_of(c), texture_of(c)
        for j, (ek, edk) in enumerate(oracle.conditions(c.e, c.edot, c.delta)):
            F, p = oracle.condition_forces(gap, ek, edk, tex)
            pg = got[k][0][j].ravel()
            assert np.linalg.norm(pg - p) <= 1e-9 * np.linalg.norm(p)
            Fg = got[k][2][j]
            assert np.linalg.norm(Fg[:2] - F[:2]) <= 1e-8 * np.linalg.norm(F[:2])


@ITERATIONS
def test_graph_and_plain_batch_steps_agree_bitwise(iteration):
    log(f"case: batch graph vs plain steps, iteration kind {iteration}")
    a = batch_solve(CASES[:3], use_graph=True, iters=7, iteration=iteration)
    b = batch_solve(CASES[:3], use_graph=False, iters=7, iteration=iteration)
    for k in range(3):
        assert np.array_equal(a[k][0], b[k][0]) and a[k][1] == b[k][1]


def test_server_drains_a_poisson_stream():
    log("case: served Poisson stream of small grids")
    rng = np.random.default_rng(0)
    sizes = [(64, 32), (128, 64), (256, 128)]
    reqs = []
    t = 0.0
    for k in range(12):
        t += rng.exponential(0.02)
        nt, nz = sizes[k % 3]
        c = synth.textured_case(nt, nz, k) if k % 2 else synth.smooth_case(nt, nz, k)
        reqs.append(Request(rid=k, case=c, arrival=t))
    be = BatchBackend(iterations_per_step=16)
    budget = 3 * max(be.footprint(r.case) for r in reqs)      # at most a few at once
    done = GapServer(be, budget).run(reqs)
    be.close()
    assert len(done) == 12 and all(r.status == G.GAP_OK for r in done)
    stats = latency_stats(done)
    log(f"  p50 {stats['p50_s'] * 1e3:.1f} ms, p99 {stats['p99_s'] * 1e3:.1f} ms")
    assert all(np.all(np.isfinite(r.F)) and np.all(np.isfinite(r.J)) for r in done)


@ITERATIONS
def test_held_request_keeps_its_state_and_result(iteration):
    """A held request does not advance; released, it finishes bitwise as when run alone.  It
    is held after an odd number of its own iterations, while the batch steps by 7."""
    log(f"case: batch hold and release, iteration kind {iteration}")
    cases = [synth.smooth_case(128, 64, 7), synth.textured_case(96, 48, 8)]
    alone = batch_solve([cases[1]], iteration=iteration)[0]
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    solvers, ids = [], []
    for c in cases:
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        opts = s.options(omega=c.omega, eps=c.eps, iteration=iteration)
        ids.append(G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream))
        solvers.append(s)
    G.gap_batch_step(b, 7, True, stream)
    G.gap_batch_hold(b, ids[1], 1)
    for _ in range(3):
        G.gap_batch_step(b, 8, True, stream)
    p_held = solvers[1].pressure().clone()
    G.gap_batch_step(b, 7, True, stream)
    assert torch.equal(p_held, solvers[1].pressure())        # no launch touched it
    G.gap_batch_hold(b, ids[1], 0)
    result = None
    while result is None:
        G.gap_batch_step(b, 8, True, stream)
        for bid in G.gap_batch_poll(b):
            st, info = G.gap_batch_remove(b, bid, stream)
            if bid == ids[1]:
                result = (solvers[1].pressure().cpu().numpy().copy(), info.iterations)
    assert result[1] == alone[1] and np.array_equal(result[0], alone[0])
    with pytest.raises(G.GapError):
        G.gap_batch_hold(b, 12345, 1)
    for s in solvers:
        s.close()
    G.gap_batch_destroy(b)


def test_server_with_work_cap_drains_a_mixed_stream():
    log("case: served stream with a work cap")
    reqs = []
    sizes = [(256, 128), (64, 32), (256, 128), (128, 64), (64, 32)]
    for k, (nt, nz) in enumerate(sizes):
        reqs.append(Request(rid=k, case=synth.smooth_case(nt, nz, 20 + k), arrival=0.001 * k))
    be = BatchBackend(iterations_per_step=16)
    cap = be.work(reqs[0].case) + be.work(reqs[1].case)        # one 256x128 plus a small one
    done = GapServer(be, budget_bytes=10 * be.footprint(reqs[0].case), work_cap=cap).run(reqs)
    be.close()
    assert sorted(r.rid for r in done) == list(range(5)) and all(r.status == G.GAP_OK for r in done)
    by = {r.rid: r for r in done}
    assert by[0].finished <= by[2].finished                    # the two large ones in order


def test_two_lanes_give_each_request_its_result_alone():
    """Two lanes on two streams and threads (bulk: 256x128 and larger, chunked for 2
    workgroups per CU; fast: the rest, 1 per CU), over a staggered stream: every request's
    pressure, forces and FD Jacobian are bitwise those of the same request alone in a batch of
    its lane's chunking target, and match a solve of its own to 1e-9."""
    log("case: two-lane server, 7 requests 64x32 ... 512x256, targets 2 and 1")
    sizes = [(512, 256), (64, 32), (128, 64), (256, 128), (96, 48), (512, 128), (200, 37)]
    reqs = []
    for k, (nt, nz) in enumerate(sizes):
        c = (synth.textured_case(nt, nz, 20 + k, eps=1e-12) if k % 2
             else synth.smooth_case(nt, nz, 20 + k, eps=1e-12))
        reqs.append(Request(rid=k, case=c, arrival=0.004 * k))
    bulk_work = 9 * 256 * 128
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    bulk = BatchBackend(iterations_per_step=16, stream=streams[0], wg_per_cu=2, keep_pressure=True)
    fast = BatchBackend(iterations_per_step=16, stream=streams[1], wg_per_cu=1, keep_pressure=True)
    budget = 4 * max(bulk.footprint(r.case) for r in reqs)
    srv = LaneServer(bulk, fast, budget_bytes=budget, bulk_work=bulk_work)
    done = {r.rid: r for r in srv.run(reqs)}
    bulk.close()
    fast.close()
    assert sorted(done) == list(range(len(sizes))) and all(r.status == G.GAP_OK for r in done.values())
    assert {k for k, r in done.items() if r.meta["lane"] == "bulk"} == {0, 3, 5}
    for k, r in done.items():
        c = r.case
        target = 2 if r.meta["lane"] == "bulk" else 1
        be = BatchBackend(iterations_per_step=16, wg_per_cu=target, keep_pressure=True)
        alone = GapServer(be, budget).run([Request(rid=k, case=c, arrival=0.0)])[0]
        be.close()
        assert alone.iterations == r.iterations, c.label
        for a, b in ((alone.p, r.p), (alone.F, r.F), (alone.J, r.J)):
            assert np.array_equal(a, b), c.label
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        p_own, _ = s.solve(omega=c.omega, eps=c.eps)
        p_own = p_own.cpu().numpy()
        s.close()
        for m in range(9):
            assert np.linalg.norm(r.p[m] - p_own[m]) <= 1e-9 * np.linalg.norm(p_own[m]), c.label


def test_a_grid_in_a_batch_is_lent_to_it():
    """While a grid is in a batch, using it elsewhere is refused (its Krylov buffers and
    device record belong to the batch); after removal it works again."""
    log("case: grid lent to a batch")
    c = synth.smooth_case(64, 32, 9)
    b = G.gap_batch_create()
    b2 = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    s = JointGapSolver.from_case(c, max_cond=9)
    s.assemble(c.e, c.edot, c.delta, 9)
    opts = s.options(omega=c.omega, eps=c.eps)
    bid = G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream)
    for call in (lambda: s.solve(opts), lambda: s.assemble(c.e, c.edot, c.delta, 9), lambda: s.tune(opts),
                 lambda: s.set_pcg_config(), lambda: G.destroy_gap_grid(s.handle), lambda: s.set_dimples(None)):
        with pytest.raises(G.GapError) as ei:
            call()
        assert ei.value.status == G.GAP_ESTATE
    with pytest.raises(G.GapError) as ei:
        G.gap_batch_add(b2, s.handle, opts, s.p.data_ptr(), stream)
    assert ei.value.status == G.GAP_EINVAL
    while not G.gap_batch_poll(b):
        G.gap_batch_step(b, 16, True, stream)
    G.gap_batch_remove(b, bid, stream)
    _, info = s.solve(opts)                                   # free again
    assert info.status == G.GAP_OK
    s.close()
    G.gap_batch_destroy(b)
    G.gap_batch_destroy(b2)


def test_a_re_textured_handle_solves_as_a_new_one():
    """set_gap_dimples: a handle re-textured to another dimple list (and back to smooth) gives
    bitwise the pressure, forces and Jacobian of a handle created for that texture; bad
    dimples are refused and leave the handle usable."""
    dimpled = [synth.textured_case(192, 64, 31), synth.textured_case(192, 64, 32)]
    smooth = synth.smooth_case(192, 64, 33)
    log("case: 192x64 handle re-textured: dimples seed 31 -> 32 -> smooth -> 31")

    def solve(s, c):
        s.assemble(c.e, c.edot, c.delta, 9)
        p, info = s.solve(omega=c.omega, eps=1e-12)
        return p.cpu().numpy().copy(), s.integrate().cpu().numpy().copy(), s.jacobian_fd().cpu().numpy().copy()

    def fresh(c):
        s = JointGapSolver.from_case(c, max_cond=9)
        out = solve(s, c)
        s.close()
        return out

    s = JointGapSolver.from_case(dimpled[0], max_cond=9)
    solve(s, dimpled[0])
    for c in (dimpled[1], smooth, dimpled[0]):
        s.set_dimples(JointGapSolver.case_dimples(c))
        for a, b in zip(solve(s, c), fresh(c)):
            assert np.array_equal(a, b), c.label
    bad = (np.array([0.1]), np.array([0.02]), np.array([1e-3]), np.array([2e-3]))     # depth > radius
    with pytest.raises(G.GapError) as ei:
        s.set_dimples(bad)
    assert ei.value.status == G.GAP_EINVAL
    for a, b in zip(solve(s, dimpled[0]), fresh(dimpled[0])):
        assert np.array_equal(a, b)
    s.close()


@ITERATIONS
def test_random_joins_and_holds_keep_results_bitwise(iteration):
    """A seeded random schedule: requests join between steps of 3-9 iterations, and are held
    and released at random; each finishes bitwise as when solved alone.  This exercises the
    one-launch kernel's per-request parity offsets under arbitrary launch counts."""
    log(f"case: random batch schedule, iteration kind {iteration}")
    rng = np.random.default_rng(2024)
    cases = [synth.smooth_case(64, 32, 40 + k) if k % 2 else synth.textured_case(96, 24, 40 + k) for k in range(6)]
    alone = [batch_solve([c], iteration=iteration)[0] for c in cases]
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    solvers, ids, held, results = [], [], set(), {}
    pending = list(range(len(cases)))
    while len(results) < len(cases):
        if pending and (not ids or rng.random() < 0.5):
            k = pending.pop(0)
            c = cases[k]
            s = JointGapSolver.from_case(c, max_cond=9)
            s.assemble(c.e, c.edot, c.delta, 9)
            opts = s.options(omega=c.omega, eps=c.eps, iteration=iteration)
            ids.append(G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream))
            solvers.append(s)
        live = [i for i in ids if i not in results]
        for bid in live:
            if bid in held and rng.random() < 0.5:
                G.gap_batch_hold(b, bid, 0)
                held.discard(bid)
            elif bid not in held and rng.random() < 0.25 and len(held) + 1 < len(live):
                G.gap_batch_hold(b, bid, 1)
                held.add(bid)
        G.gap_batch_step(b, int(rng.integers(3, 10)), bool(rng.random() < 0.5), stream)
        for bid in G.gap_batch_poll(b):
            k = ids.index(bid)
            _, info = G.gap_batch_remove(b, bid, stream)
            results[bid] = (solvers[k].pressure().cpu().numpy().copy(), info.iterations)
            held.discard(bid)
        if not [i for i in ids if i not in results and i not in held] and held:
            bid = held.pop()                       # keep something running
            G.gap_batch_hold(b, bid, 0)
    for k, bid in enumerate(ids):
        p, it = results[bid]
        assert it == alone[k][1], (k, it, alone[k][1])
        assert np.array_equal(p, alone[k][0]), k
    for s in solvers:
        s.close()
    G.gap_batch_destroy(b)
