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


@pytest.mark.parametrize("shape", [(256, 128), (2048, 64), (100, 37)])
def test_graph_replays_match_eager_bitwise(shape):
    case = synth.textured_case(*shape, 2)
    log(f"case: {case.label}, graph vs eager")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    pe, ie, re = solve_copy(s, eps=1e-10, omega=1.6, graph=False)
    pg1, ig1, rg1 = solve_copy(s, eps=1e-10, omega=1.6, graph=True)      # captures
    F = s.integrate().clone()                                              # eager work between replays
    torch.cuda.synchronize()
    pg2, ig2, rg2 = solve_copy(s, eps=1e-10, omega=1.6, graph=True)      # replays the cached graph
    pg3, ig3, rg3 = solve_copy(s, eps=1e-10, omega=1.6, graph=True, check_every=7)   # new block size
    for p, i, r in [(pg1, ig1, rg1), (pg2, ig2, rg2), (pg3, ig3, rg3)]:
        assert i == ie and r == re
        assert np.array_equal(p, pe)
    assert torch.isfinite(F).all()
    s.close()


def test_timing_hooks_do_not_change_results():
    case = synth.smooth_case(512, 128, 1)
    log(f"case: {case.label}, timing on/off")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    p0, i0, _ = solve_copy(s, eps=1e-10, omega=1.8)
    G.gap_kernel_timing(s.handle, 1)
    p1, i1, _ = solve_copy(s, eps=1e-10, omega=1.8)
    p2, i2, _ = solve_copy(s, eps=1e-10, omega=1.8, graph=False)
    G.gap_kernel_timing(s.handle, 0)
    na, ta = G.gap_kernel_stats(s.handle, G.GAP_KERNEL_PCG_A)
    nb, tb = G.gap_kernel_stats(s.handle, G.GAP_KERNEL_PCG_B)
    assert np.array_equal(p0, p1) and np.array_equal(p0, p2) and i0 == i1 == i2
    assert na >= 2 * i0 and nb >= 2 * i0 and ta > 0 and tb > 0
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
