"""GPU parity at full size against the oracle's exact solution, stored by
``tests/golden/make_golden.py`` (banded Cholesky; the factorizations need about 34 GB and two
minutes each, so they are not repeated in a test run).

Joint textured 2048 x 1024 x 9 (seed 0), conditions 0, 1 and 5 of Eq 2.17-2.19:
  * pressure: relative L2 error on the stored strided sample <= 1e-9; the whole field through
    |(||p|| - ||p*||)| <= 1e-9 ||p*|| (a lower bound of ||p - p*||) and four random
    projections w . p, whose differences have the size of ||p - p*||;
  * forces: <= 1e-8 relative per (Fx, Fy) and (Mx, My) pair;
at eps 1e-12 and 1e-13, in the launch configuration the benchmark uses.  The errors at the
timed eps 1e-10 and at 1e-11 are logged, not gated: the recurrence stop of Eq 3.9 bounds the
residual, and with a preconditioned condition number near 3e5 the error is about a hundred
times larger (1.5e-8 in pressure, 2.3e-8 in the forces of condition 0 at eps 1e-10).

Textured 1024 x 512 (seed 0): the adjoint Jacobian against the oracle's complex-step
derivative and central differences, the FD Jacobian against the oracle's Eq 2.13-2.14.
"""

import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_06824_amd import gapsolve as G  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
P_TOL = 1e-9
F_TOL = 1e-8
GATE_EPS = 1e-12     # the largest eps of the sweep gated here (see the module docstring)


def log(msg):
    print(msg, flush=True)


def golden(name):
    path = os.path.join(HERE, "golden", f"{name}_seed0.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def pair_err(F, ref):
    F, ref = np.asarray(F), np.asarray(ref)
    return max(np.linalg.norm(F[:2] - ref[:2]) / np.linalg.norm(ref[:2]),
               np.linalg.norm(F[2:4] - ref[2:4]) / np.linalg.norm(ref[2:4]))


def pressure_errors(p, gold_k, rows, cols, W):
    """(sampled relative L2 error, norm gap, projection-based estimate of ||p - p*|| / ||p*||)."""
    ref = np.asarray(gold_k["sample"])
    smp = p[np.ix_(rows, cols)]
    e_s = np.linalg.norm(smp - ref) / np.linalg.norm(ref)
    nrm = gold_k["norm"]
    e_n = abs(np.linalg.norm(p) - nrm) / nrm
    d = W @ p.ravel() - np.asarray(gold_k["projections"])
    e_w = np.sqrt(np.mean(d * d)) / nrm
    return e_s, e_n, e_w


@pytest.fixture(scope="module")
def c3():
    gold = golden("joint_textured_2048x1024")
    case = synth.make_case("joint_textured_2048x1024", 0)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    W = synth.projection_weights(case.n)
    rows, cols = np.asarray(gold["sample_rows"]), np.asarray(gold["sample_cols"])
    yield gold, case, s, W, rows, cols
    s.close()


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_STRIPS, G.GAP_ITERATION_ONE_LAUNCH, G.GAP_ITERATION_TWO_LAUNCH],
                         ids=["strips", "one_launch", "two_launch"])
def test_joint_textured_2048x1024_against_exact_solution(c3, iteration):
    gold, case, s, W, rows, cols = c3
    log(f"case: {case.label}, 9 conditions, against the stored exact solution, iteration kind {iteration}")
    opts = s.options(omega=case.omega, eps=1e-13, iteration=iteration)
    cfg, _ = s.tune(opts, iterations=20)
    log(f"  launch configuration {cfg}")
    sweep = (1e-10, 1e-11, 1e-12, 1e-13) if iteration == G.GAP_ITERATION_STRIPS else (1e-13,)
    for eps in sweep:
        opts = s.options(omega=case.omega, eps=eps, iteration=iteration)
        p, info = s.solve(opts)
        F = s.integrate().cpu().numpy()
        p = p.cpu().numpy()
        log(f"  eps {eps:.0e}: {info.iterations} iterations, recurrence residual {info.rel_residual:.2e}")
        for k, gk in gold["conditions"].items():
            k = int(k)
            e_s, e_n, e_w = pressure_errors(p[k], gk, rows, cols, W)
            e_f = pair_err(F[k], gk["forces"])
            log(f"    condition {k}: pressure sample {e_s:.2e}, norm gap {e_n:.2e}, projections {e_w:.2e}; "
                f"forces {e_f:.2e}")
            if eps <= GATE_EPS:
                assert e_s <= P_TOL and e_n <= P_TOL and e_w <= 3 * P_TOL
                assert e_f <= F_TOL


def blocks(J):
    J = np.asarray(J)
    return [J[0:2, 0:4], J[0:2, 4:8], J[2:4, 0:4], J[2:4, 4:8]]


def block_errs(J, ref):
    return [np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(blocks(J), blocks(ref))]


def test_adjoint_textured_1024x512_against_oracle_jacobians():
    gold = golden("adjoint_textured_1024x512")
    case = synth.make_case("adjoint_textured_1024x512", 0)
    log(f"case: {case.label}, adjoint and FD Jacobians against the stored oracle Jacobians")
    J_cs = np.asarray(gold["jacobian_complex_step"])
    J_cen = np.asarray(gold["jacobian_central"])
    J_fwd = np.asarray(gold["jacobian_forward"])
    F9 = np.asarray(gold["forces_9"])
    s = JointGapSolver.from_case(case, max_cond=9)
    opts = s.options(omega=case.omega, eps=1e-13)
    s.assemble(case.e, case.edot, case.delta, 9)
    s.solve(opts)
    F = s.integrate().cpu().numpy()
    J_fd = s.jacobian_fd().cpu().numpy()
    J_adj, info = s.jacobian_adjoint(opts)
    J_adj = J_adj.cpu().numpy()
    s.assemble(case.e, case.edot, None, 1)
    _, J_joint, _ = s.solve_with_adjoint(opts)
    J_joint = J_joint.cpu().numpy()
    # as timed against FD: the base system at the workload's eps, the adjoint systems at 1e-7
    s.assemble(case.e, case.edot, None, 1)
    _, J_loose, info_loose = s.solve_with_adjoint(s.options(omega=case.omega, eps=case.eps, eps_adjoint=1e-7))
    J_loose = J_loose.cpu().numpy()
    s.close()
    e_force = max(pair_err(F[k], F9[k]) for k in range(9))
    e_cs = block_errs(J_adj, J_cs)
    e_joint = block_errs(J_joint, J_cs)
    e_cen = block_errs(J_adj, J_cen)
    e_fd = block_errs(J_fd, J_fwd)
    log(f"  forces of the 9 conditions {e_force:.2e}; adjoint iterations {info.iterations}")
    log(f"  adjoint vs complex step per block {np.array(e_cs)}, joint base + adjoint {np.array(e_joint)}")
    log(f"  adjoint vs central FD {np.array(e_cen)}; GPU FD vs oracle FD {np.array(e_fd)}")
    assert e_force <= F_TOL
    # the exact derivative: only the solves' tolerance separates the two
    assert max(e_cs) <= 1e-6 and max(e_joint) <= 1e-6
    e_loose = block_errs(J_loose, J_cs)
    log(f"  base at eps {case.eps:g}, adjoint at 1e-7: {info_loose.iterations} iterations, vs complex step "
        f"{np.array(e_loose)}")
    assert max(e_loose) <= 1e-6
    # the gate against finite differences: central FD (e columns, O(delta^2)), and the rate
    # columns, where forward FD is exact because F is affine in the rates
    assert max(e_cen) <= 1e-4
    assert max(block_errs(J_adj, J_fwd)[k] for k in (1, 3)) <= 1e-4
    # the FD Jacobian of Eq 2.13-2.14: force round-off amplified by 1 / delta
    assert max(e_fd) <= 1e-5
