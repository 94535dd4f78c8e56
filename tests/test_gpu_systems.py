"""GPU systems tests: graph-captured vs eager iteration blocks, determinism, timing hooks."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_06824_amd import gapsolve as G  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402


def log(msg):
    print(msg, flush=True)


def solve_copy(s, **opt):
    p, info = s.solve(**opt)
    torch.cuda.synchronize()
    return p.clone().cpu().numpy(), info.iterations, info.rel_residual


ITERATIONS = pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                                      G.GAP_ITERATION_STRIPS],
                                     ids=["two_launch", "one_launch", "strips"])


@ITERATIONS
@pytest.mark.parametrize("shape", [(256, 128), (2048, 64), (100, 37)])
def test_graph_replays_match_eager_bitwise(shape, iteration):
    """Cached graphs replayed between eager work; an odd block size (7) makes the one-launch
    kernel's graphs start at both launch parities."""
    case = synth.textured_case(*shape, 2)
    log(f"case: {case.label}, graph vs eager, iteration kind {iteration}")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    kw = dict(eps=1e-10, omega=1.6, iteration=iteration)
    pe, ie, re = solve_copy(s, graph=False, **kw)
    pg1, ig1, rg1 = solve_copy(s, graph=True, **kw)                      # captures
    F = s.integrate().clone()                                              # eager work between replays
    torch.cuda.synchronize()
    pg2, ig2, rg2 = solve_copy(s, graph=True, **kw)                      # replays the cached graph
    pg3, ig3, rg3 = solve_copy(s, graph=True, check_every=7, **kw)       # new block size
    for p, i, r in [(pg1, ig1, rg1), (pg2, ig2, rg2), (pg3, ig3, rg3)]:
        assert i == ie and r == re
        assert np.array_equal(p, pe)
    assert torch.isfinite(F).all()
    s.close()


@ITERATIONS
def test_timing_hooks_do_not_change_results(iteration):
    case = synth.smooth_case(512, 128, 1)
    log(f"case: {case.label}, timing on/off, iteration kind {iteration}")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    kw = dict(eps=1e-10, omega=1.8, iteration=iteration)
    p0, i0, _ = solve_copy(s, **kw)
    G.gap_kernel_timing(s.handle, 1)
    p1, i1, _ = solve_copy(s, **kw)
    p2, i2, _ = solve_copy(s, graph=False, **kw)
    G.gap_kernel_timing(s.handle, 0)
    n = [G.gap_kernel_stats(s.handle, k) for k in range(G.GAP_KERNEL_COUNT)]
    assert np.array_equal(p0, p1) and np.array_equal(p0, p2) and i0 == i1 == i2
    timed = {G.GAP_ITERATION_TWO_LAUNCH: [G.GAP_KERNEL_PCG_A, G.GAP_KERNEL_PCG_B],
             G.GAP_ITERATION_ONE_LAUNCH: [G.GAP_KERNEL_PCG_ONE],
             G.GAP_ITERATION_STRIPS: [G.GAP_KERNEL_PCG_STRIPS]}[iteration]
    for k in range(G.GAP_KERNEL_COUNT):
        if k in timed:
            assert n[k][0] >= 2 * i0 and n[k][1] > 0
        else:
            assert n[k][0] == 0
    # one launch in three: the same launches, a third of them timed, at the same average
    per_solve = sum(n[k][0] for k in timed) // 2
    G.gap_kernel_timing(s.handle, 3)
    p3, i3, _ = solve_copy(s, **kw)
    G.gap_kernel_timing(s.handle, 0)
    n3 = [G.gap_kernel_stats(s.handle, k) for k in range(G.GAP_KERNEL_COUNT)]
    assert np.array_equal(p0, p3) and i3 == i0
    assert sum(n3[k][0] for k in timed) == (per_solve + 2) // 3
    avg1 = sum(n[k][1] for k in timed) / sum(n[k][0] for k in timed)
    avg3 = sum(n3[k][1] for k in timed) / sum(n3[k][0] for k in timed)
    log(f"  timed launches {per_solve} per solve, {sum(n3[k][0] for k in timed)} at one in three; "
        f"average {1e3 * avg1:.1f} us against {1e3 * avg3:.1f} us")
    assert 0.5 < avg3 / avg1 < 2.0
    with pytest.raises(G.GapError) as ei:
        G.gap_kernel_timing(s.handle, -1)
    assert ei.value.status == G.GAP_EINVAL
    s.close()


def test_one_launch_agrees_with_table1_iteration():
    """Both one-launch iterations (whole rings; strips with z recomputed) take Table 1's steps
    with alpha's denominator expanded: the same iteration count (within one) and the same
    iterate up to rounding, on every preconditioner and scalar / strategy variant."""
    case = synth.textured_case(300, 96, 5)
    log(f"case: {case.label}, one-launch against two-launch")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    for v in [dict(), dict(precond=G.GAP_PRECOND_JACOBI), dict(precond=G.GAP_PRECOND_ASSOR1),
              dict(scalars=G.GAP_SCALARS_PER_COND), dict(strategy=G.GAP_STRATEGY_ASYNC),
              dict(scalars=G.GAP_SCALARS_PER_COND, strategy=G.GAP_STRATEGY_ASYNC)]:
        out = []
        for it in (G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH, G.GAP_ITERATION_STRIPS):
            p, info = s.solve(eps=1e-12, omega=1.6, iteration=it, **v)
            out.append((p.clone().cpu().numpy().reshape(9, -1), info.iterations, info.rel_residual))
        p2, i2, r2 = out[0]
        for name, (p1, i1, r1) in zip(("one launch", "strips"), out[1:]):
            d = max(np.linalg.norm(p1[k] - p2[k]) / np.linalg.norm(p2[k]) for k in range(9))
            log(f"  {v}, {name}: iterations {i2} / {i1}, residual {r2:.2e} / {r1:.2e}, difference {d:.1e}")
            assert abs(i1 - i2) <= 1 and r1 <= 1e-12 and d <= 1e-10
    s.close()


def test_repeated_solves_are_deterministic():
    case = synth.textured_case(384, 96, 4)
    log(f"case: {case.label}, determinism")
    outs = []
    for _ in range(2):
        s = JointGapSolver.from_case(case, max_cond=9)
        s.assemble(case.e, case.edot, case.delta, 9)
        p, it, rel = solve_copy(s, eps=1e-11, omega=1.6)
        F = s.integrate().cpu().numpy()
        J = s.jacobian_fd().cpu().numpy()
        outs.append((p, it, rel, F, J))
        s.close()
    a, b = outs
    assert a[1] == b[1] and a[2] == b[2]
    for x, y in zip(a[0:1] + a[3:], b[0:1] + b[3:]):
        assert np.array_equal(x, y)
