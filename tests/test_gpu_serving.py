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
from paper_2511_06824_amd.serve import BatchBackend, GapServer, Request, latency_stats  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402


def log(msg):
    print(msg, flush=True)


CASES = [synth.smooth_case(64, 32, 0), synth.textured_case(128, 64, 1), synth.smooth_case(200, 37, 2),
         synth.textured_case(256, 128, 3), synth.smooth_case(96, 48, 4, eps=1e-12)]


def batch_solve(cases, eps_override=None, iters=8, use_graph=True):
    """Solve the cases together in one batch; returns pressures, infos by case index."""
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    solvers, ids = [], []
    for c in cases:
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        opts = s.options(omega=c.omega, eps=eps_override or c.eps)
        ids.append(G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream))
        solvers.append((s, opts))
    out = {}
    while len(out) < len(cases):
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


def test_results_alone_and_in_the_mix_are_bitwise_equal():
    log("case: batch mix of 5 grids vs each alone")
    mix = batch_solve(CASES)
    for k, c in enumerate(CASES):
        alone = batch_solve([c])[0]
        assert alone[1] == mix[k][1]
        assert np.array_equal(alone[0], mix[k][0]), c.label
        assert np.array_equal(alone[2], mix[k][2]), c.label


def test_batched_results_match_the_oracle():
    log("case: batch mix vs oracle")
    cases = [synth.smooth_case(64, 32, 5), synth.textured_case(96, 48, 6)]
    got = batch_solve(cases, eps_override=1e-13, use_graph=False)
    for k, c in enumerate(cases):
        gap, tex = gap_of(c), texture_of(c)
        for j, (ek, edk) in enumerate(oracle.conditions(c.e, c.edot, c.delta)):
            F, p = oracle.condition_forces(gap, ek, edk, tex)
            pg = got[k][0][j].ravel()
            assert np.linalg.norm(pg - p) <= 1e-9 * np.linalg.norm(p)
            Fg = got[k][2][j]
            assert np.linalg.norm(Fg[:2] - F[:2]) <= 1e-8 * np.linalg.norm(F[:2])


def test_graph_and_plain_batch_steps_agree_bitwise():
    log("case: batch graph vs plain steps")
    a = batch_solve(CASES[:3], use_graph=True)
    b = batch_solve(CASES[:3], use_graph=False)
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


def test_held_request_keeps_its_state_and_result():
    """A held request does not advance; released, it finishes bitwise as when run alone."""
    log("case: batch hold and release")
    cases = [synth.smooth_case(128, 64, 7), synth.textured_case(96, 48, 8)]
    alone = batch_solve([cases[1]])[0]
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    solvers, ids = [], []
    for c in cases:
        s = JointGapSolver.from_case(c, max_cond=9)
        s.assemble(c.e, c.edot, c.delta, 9)
        opts = s.options(omega=c.omega, eps=c.eps)
        ids.append(G.gap_batch_add(b, s.handle, opts, s.p.data_ptr(), stream))
        solvers.append(s)
    G.gap_batch_hold(b, ids[1], 1)
    for _ in range(3):
        G.gap_batch_step(b, 8, True, stream)
    p_held = solvers[1].pressure().clone()
    G.gap_batch_step(b, 8, True, stream)
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
                 lambda: s.set_pcg_config(), lambda: G.destroy_gap_grid(s.handle)):
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
