"""GPU parity of every PCG kernel configuration (workgroup shape x row chunking) and of the
autotuner's choice, through the C ABI, against the CPU oracle; configuration validation; and
the launch count of a solve that stops at max_iter."""

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
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402

P_TOL, F_TOL = 1e-9, 1e-8
EPS = 1e-13

# ring sizes and the candidate shapes (threads, columns per thread) the library lists for them
SHAPES = {300: [(512, 1), (256, 2)], 1000: [(512, 2), (1024, 1), (256, 4)], 2048: [(1024, 2), (512, 4)]}
CASES = [(300, 23, 9), (1000, 9, 9), (2048, 5, 1)]

_ref = {}


def log(msg):
    print(msg, flush=True)


def reference(nt, nz, n_cond):
    key = (nt, nz, n_cond)
    if key not in _ref:
        case = synth.textured_case(nt, nz, 11)
        gap, tex = gap_of(case), texture_of(case)
        ps, Fs = [], []
        for ek, edk in oracle.conditions(case.e, case.edot, case.delta)[:n_cond]:
            F, p = oracle.condition_forces(gap, ek, edk, tex)
            ps.append(p)
            Fs.append(F)
        _ref[key] = (case, np.array(ps), np.array(Fs))
    return _ref[key]


ITERATIONS = pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                                      G.GAP_ITERATION_STRIPS],
                                     ids=["two_launch", "one_launch", "strips"])


def check(s, case, n_cond, p_ref, F_ref, iteration=G.GAP_ITERATION_ONE_LAUNCH):
    p, info = s.solve(omega=case.omega, eps=EPS, iteration=iteration)
    F = s.integrate().cpu().numpy()
    p = p.reshape(n_cond, -1).cpu().numpy()
    perr = max(np.linalg.norm(p[k] - p_ref[k]) / np.linalg.norm(p_ref[k]) for k in range(n_cond))
    ferr = max(max(np.linalg.norm(F[k, :2] - F_ref[k, :2]) / np.linalg.norm(F_ref[k, :2]),
                   np.linalg.norm(F[k, 2:] - F_ref[k, 2:]) / np.linalg.norm(F_ref[k, 2:])) for k in range(n_cond))
    return perr, ferr, info


@ITERATIONS
@pytest.mark.parametrize("nt,nz,n_cond", CASES, ids=[f"{a}x{b}x{c}" for a, b, c in CASES])
def test_every_configuration_matches_oracle(nt, nz, n_cond, iteration):
    case, p_ref, F_ref = reference(nt, nz, n_cond)
    s = JointGapSolver.from_case(case, max_cond=9 if n_cond == 9 else 1)
    s.assemble(case.e, case.edot, case.delta, n_cond)
    cfg0 = s.pcg_config
    for k in "abf":
        assert (cfg0[f"threads_{k}"], cfg0[f"cols_per_thread_{k}"]) == SHAPES[nt][0]
    configs = []
    if iteration == G.GAP_ITERATION_STRIPS:
        assert cfg0["cols_per_lane_w"] == 1
        for Q in (1,):
            occ = s.set_strip_config(Q, 1)
            for w in sorted({1, occ["occupancy_w"]}):
                cfg = s.set_strip_config(Q, w)
                log(f"case: {case.label} x{n_cond}, strips, config {cfg}")
                perr, ferr, info = check(s, case, n_cond, p_ref, F_ref, iteration)
                log(f"  iterations {info.iterations}, pressure {perr:.2e}, forces {ferr:.2e}")
                assert perr <= P_TOL and ferr <= F_TOL
    elif iteration == G.GAP_ITERATION_TWO_LAUNCH:
        for NT, Q in SHAPES[nt]:
            occ = s.set_pcg_config(NT, Q, 1, 1)
            for wa, wb in sorted({(1, 1), (occ["occupancy_a"], occ["occupancy_b"]), (1, occ["occupancy_b"])}):
                configs.append(dict(threads=NT, cols_per_thread=Q, wg_per_cu_a=wa, wg_per_cu_b=wb))
        NA, QA = SHAPES[nt][-1]
        NB, QB = SHAPES[nt][0]                                        # A and B with different shapes
        configs.append(dict(threads=NA, cols_per_thread=QA, wg_per_cu_a=1, wg_per_cu_b=1, threads_b=NB,
                            cols_per_thread_b=QB))
    else:
        d = SHAPES[nt][0]
        for NT, Q in SHAPES[nt]:
            occ = s.set_pcg_config(d[0], d[1], 1, 1, threads_f=NT, cols_per_thread_f=Q, wg_per_cu_f=1)
            for wf in sorted({1, occ["occupancy_f"]}):
                configs.append(dict(threads=d[0], cols_per_thread=d[1], wg_per_cu_a=1, wg_per_cu_b=1, threads_f=NT,
                                    cols_per_thread_f=Q, wg_per_cu_f=wf))
    for kw in configs:
        cfg = s.set_pcg_config(**kw)
        log(f"case: {case.label} x{n_cond}, iteration kind {iteration}, config {cfg}")
        perr, ferr, info = check(s, case, n_cond, p_ref, F_ref, iteration)
        log(f"  iterations {info.iterations}, pressure {perr:.2e}, forces {ferr:.2e}")
        assert perr <= P_TOL and ferr <= F_TOL
    s.close()


@ITERATIONS
def test_autotuner_choice_is_valid_and_matches_oracle(iteration):
    case, p_ref, F_ref = reference(300, 23, 9)
    log(f"case: {case.label}, autotuner, iteration kind {iteration}")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    cfg, us = s.tune(iterations=10, omega=case.omega, iteration=iteration)
    log(f"  tuned {cfg}, {us:.1f} us per iteration")
    for k in "abf":
        assert (cfg[f"threads_{k}"], cfg[f"cols_per_thread_{k}"]) in SHAPES[300]
        assert 1 <= cfg[f"wg_per_cu_{k}"] <= cfg[f"occupancy_{k}"]
    assert cfg["cols_per_lane_w"] == 1 and 1 <= cfg["wg_per_cu_w"] <= cfg["occupancy_w"]
    assert us > 0.0 and s.pcg_config == cfg
    perr, ferr, _ = check(s, case, 9, p_ref, F_ref, iteration)   # the system survives tuning unchanged
    assert perr <= P_TOL and ferr <= F_TOL
    d = s.set_pcg_config()
    for k in "abf":
        assert (d[f"threads_{k}"], d[f"cols_per_thread_{k}"]) == SHAPES[300][0]
    s.close()


def test_configuration_validation():
    case = synth.smooth_case(300, 8, 0)
    log(f"case: {case.label}, configuration validation")
    s = JointGapSolver.from_case(case, max_cond=1)
    for NT, Q, wa, wb in [(64, 1, 1, 1), (1024, 2, 1, 1), (512, 3, 1, 1), (384, 1, 1, 1), (512, 1, 0, 1),
                          (512, 1, 1, 9)]:
        with pytest.raises(G.GapError) as ei:
            s.set_pcg_config(NT, Q, wa, wb)
        assert ei.value.status == G.GAP_EINVAL
    with pytest.raises(G.GapError) as ei:
        s.set_pcg_config(512, 1, 1, 1, threads_b=64, cols_per_thread_b=1)     # B shape too small
    assert ei.value.status == G.GAP_EINVAL
    with pytest.raises(G.GapError) as ei:
        s.set_pcg_config(512, 1, 1, 1, threads_f=64, cols_per_thread_f=1)     # F shape too small
    assert ei.value.status == G.GAP_EINVAL
    with pytest.raises(G.GapError) as ei:
        s.set_pcg_config(512, 1, 1, 1, wg_per_cu_f=9)
    assert ei.value.status == G.GAP_EINVAL
    with pytest.raises(G.GapError) as ei:                                     # unknown iteration kind
        s.solve(eps=1e-10, iteration=3)
    assert ei.value.status == G.GAP_EINVAL
    for q, w in [(0, 1), (2, 1), (1, 0), (1, 9)]:                             # strip kernel
        with pytest.raises(G.GapError) as ei:
            s.set_strip_config(q, w)
        assert ei.value.status == G.GAP_EINVAL
    # Neumann orders above 1: ASSOR II on the strip iteration only, at most 3
    for kw in [dict(neumann=2, iteration=G.GAP_ITERATION_ONE_LAUNCH),
               dict(neumann=2, iteration=G.GAP_ITERATION_TWO_LAUNCH),
               dict(neumann=2, precond=G.GAP_PRECOND_JACOBI), dict(neumann=4), dict(neumann=0)]:
        with pytest.raises(G.GapError) as ei:
            s.solve(eps=1e-10, **kw)
        assert ei.value.status == G.GAP_EINVAL
    s.assemble(case.e, case.edot, None, 1)
    with pytest.raises(G.GapError) as ei:
        G.gap_tune_pcg(s.handle, s.options(), s.p.data_ptr(), 1)
    assert ei.value.status == G.GAP_EINVAL
    s.close()


@ITERATIONS
def test_iteration_limited_solve_launches_no_idle_block(iteration):
    """max_iter = 40 with blocks of 16: 16 + 16 iterations, then the 8 remaining and the
    closing launch (A, or the one-launch kernel); no block of idle launches."""
    case = synth.smooth_case(128, 64, 2)
    log(f"case: {case.label}, max_iter 40, check_every 16, iteration kind {iteration}")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    G.gap_kernel_timing(s.handle, 1)
    kw = dict(omega=1.8, eps=1e-300, max_iter=40, raise_on_error=False, iteration=iteration)
    _, info = s.solve(check_every=16, **kw)
    n = [G.gap_kernel_stats(s.handle, k)[0] for k in range(G.GAP_KERNEL_COUNT)]
    G.gap_kernel_timing(s.handle, 0)
    assert info.iterations == 40 and info.status == G.GAP_ENOCONV
    assert n == {G.GAP_ITERATION_TWO_LAUNCH: [41, 40, 0, 0], G.GAP_ITERATION_ONE_LAUNCH: [0, 0, 41, 0],
                 G.GAP_ITERATION_STRIPS: [0, 0, 0, 41]}[iteration]
    # the same iterate as an uninterrupted run of 40 iterations in one block (graph replay)
    p1 = s.p.clone()
    s.solve(check_every=40, **kw)
    assert torch.equal(p1, s.p)
    s.close()


def test_neumann_tuner_picks_the_fastest_order_and_matches_oracle():
    """gap_tune_neumann times a complete solve at each Neumann order 1 .. 3 (each with its own
    tuned strip configuration) and keeps the fastest; the solve at that order matches the
    exact solution."""
    case = synth.textured_case(256, 128, 6)
    log(f"case: {case.label}, Neumann-order tuner")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    best, secs = s.tune_neumann(s.options(omega=1.6, eps=1e-10), max_order=3)
    log(f"  seconds per solve by order {secs}, best {best}")
    assert best == int(np.argmin(secs)) + 1 and all(x > 0 for x in secs)
    p, info = s.solve(omega=1.6, eps=1e-13, neumann=best)
    p = p.reshape(9, -1).cpu().numpy()
    for bad in (dict(iteration=G.GAP_ITERATION_ONE_LAUNCH), dict(precond=G.GAP_PRECOND_JACOBI)):
        with pytest.raises(G.GapError) as ei:
            G.gap_tune_neumann(s.handle, s.options(**bad), s.p.data_ptr(), 3)
        assert ei.value.status == G.GAP_EINVAL
    with pytest.raises(G.GapError) as ei:
        G.gap_tune_neumann(s.handle, s.options(), s.p.data_ptr(), 4)
    assert ei.value.status == G.GAP_EINVAL
    s.close()
    F_ref, p_ref = oracle.condition_forces(gap_of(case), case.e, case.edot, texture_of(case))
    assert np.linalg.norm(p[0] - p_ref) <= P_TOL * np.linalg.norm(p_ref)
