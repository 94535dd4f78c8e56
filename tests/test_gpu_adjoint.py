"""GPU parity of the adjoint Jacobian (through the C ABI) against the oracle's exact
complex-step derivative, the finite-difference Jacobians and autograd; and of the
per-condition / asynchronized PCG variants against the oracle's block PCG."""

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
from paper_2511_06824_amd.autograd import gap_force  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402

ADJ_TOL = 1e-7       # adjoint vs exact derivative, per 2 x 4 block (solves to eps 1e-13)


def log(msg):
    print(msg, flush=True)


def blocks(J):
    return [J[0:2, 0:4], J[0:2, 4:8], J[2:4, 0:4], J[2:4, 4:8]]


def block_err(J, ref):
    return max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(blocks(J), blocks(ref)))


def adjoint_J(case, eps=1e-13, cavitation=G.GAP_CAVITATION_NONE, n_cond=9):
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, n_cond)
    opts = s.options(omega=case.omega, eps=eps)
    s.solve(opts)
    J, info = s.jacobian_adjoint(opts, cavitation=cavitation)
    out = J.cpu().numpy()
    s.close()
    return out, info


@pytest.mark.parametrize("case", [synth.textured_case(32, 16, 0), synth.smooth_case(64, 32, 1),
                                  synth.textured_case(128, 64, 2), synth.textured_case(67, 33, 3)],
                         ids=["tex32x16", "smooth64x32", "tex128x64", "tex67x33"])
def test_adjoint_matches_complex_step(case):
    log(f"case: {case.label}, adjoint vs complex step")
    J, info = adjoint_J(case)
    ref = oracle.jacobian_complex_step(gap_of(case), case.e, case.edot, texture_of(case))
    err = block_err(J, ref)
    log(f"  adjoint iterations {info.iterations}, block error {err:.2e}")
    assert err <= ADJ_TOL


@pytest.mark.parametrize("case", [synth.textured_case(32, 16, 0), synth.textured_case(67, 33, 3)],
                         ids=["tex32x16", "tex67x33"])
def test_joint_base_and_adjoint_solve(case):
    """solve_with_adjoint: the base pressure and the 4 adjoint fields in one joint solve."""
    log(f"case: {case.label}, joint base + adjoint solve")
    gap, tex = gap_of(case), texture_of(case)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, None, 1)
    opts = s.options(omega=case.omega, eps=1e-13)
    p0, J, info = s.solve_with_adjoint(opts)
    J = J.cpu().numpy()
    ref = oracle.jacobian_complex_step(gap, case.e, case.edot, tex)
    err = block_err(J, ref)
    F_ref, p_ref = oracle.condition_forces(gap, case.e, case.edot, tex)
    perr = np.linalg.norm(p0.cpu().numpy().ravel() - p_ref) / np.linalg.norm(p_ref)
    log(f"  iterations {info.iterations}, Jacobian {err:.2e}, pressure {perr:.2e}")
    assert err <= ADJ_TOL and perr <= 1e-9
    assert info.n_cond == 5 and all(info.rel_residual_cond[k] <= 1e-13 for k in range(5))
    F = s.integrate().cpu().numpy()[0]
    assert np.linalg.norm(F - F_ref) <= 1e-8 * np.linalg.norm(F_ref)
    w = [0.7, 2.0, -40.0, 15.0]
    _, v, info2 = s.solve_with_adjoint(opts, w=w)
    assert info2.n_cond == 2
    assert np.linalg.norm(v.cpu().numpy() - np.asarray(w) @ J) <= 1e-9 * np.linalg.norm(np.asarray(w) @ J)
    s.close()
    s1 = JointGapSolver.from_case(case, max_cond=1)
    s1.assemble(case.e, case.edot, None, 1)
    with pytest.raises(G.GapError) as ei:
        s1.solve_with_adjoint(opts, w=w)
    assert ei.value.status == G.GAP_EINVAL
    s1.close()


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_ONE_LAUNCH, G.GAP_ITERATION_STRIPS],
                         ids=["one_launch", "strips"])
def test_adjoint_tolerance_applies_to_the_adjoint_systems_only(iteration):
    """eps_adjoint stops the adjoint systems at their own tolerance: the base system of the
    joint solve keeps its recurrence bitwise (per-condition scalars), its residual meets eps,
    every adjoint residual meets eps_adjoint, and the Jacobian stays within 1e-6 per block of
    the exact complex-step derivative; jacobian_adjoint likewise."""
    case = synth.textured_case(128, 64, 2)
    log(f"case: {case.label}, adjoint tolerance 1e-7 against 1e-13, iteration kind {iteration}")
    gap, tex = gap_of(case), texture_of(case)
    ref = oracle.jacobian_complex_step(gap, case.e, case.edot, tex)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, None, 1)
    with pytest.raises(G.GapError) as ei:
        s.solve_with_adjoint(s.options(omega=case.omega, eps=1e-13, eps_adjoint=-1.0, iteration=iteration))
    assert ei.value.status == G.GAP_EINVAL
    tight = s.options(omega=case.omega, eps=1e-13, iteration=iteration)
    loose = s.options(omega=case.omega, eps=1e-13, eps_adjoint=1e-7, iteration=iteration)
    p_t, J_t, info_t = s.solve_with_adjoint(tight)
    p_t = p_t.clone()
    p_l, J_l, info_l = s.solve_with_adjoint(loose)
    log(f"  iterations {info_t.iterations} -> {info_l.iterations}; adjoint residuals "
        f"{[round(info_l.rel_residual_cond[k], 12) for k in range(1, 5)]}")
    assert torch.equal(p_t, p_l)
    assert info_l.rel_residual_cond[0] <= 1e-13
    assert all(info_l.rel_residual_cond[k] <= 1e-7 for k in range(1, 5))
    assert info_l.iterations <= info_t.iterations
    assert block_err(J_l.cpu().numpy(), ref) <= 1e-6
    s.assemble(case.e, case.edot, None, 1)
    s.solve(tight)
    J_a, info_a = s.jacobian_adjoint(loose)
    _, info_at = s.jacobian_adjoint(tight)
    assert all(info_a.rel_residual_cond[k] <= 1e-7 for k in range(4))
    assert info_a.iterations < info_at.iterations
    assert block_err(J_a.cpu().numpy(), ref) <= 1e-6
    s.close()


def test_vjp_equals_weighted_full_jacobian():
    case = synth.textured_case(96, 48, 4)
    log(f"case: {case.label}, vjp")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, None, 1)
    opts = s.options(omega=1.6, eps=1e-13)
    s.solve(opts)
    J, _ = s.jacobian_adjoint(opts)
    w = [0.3, -1.2, 250.0, -75.0]
    v, _ = s.jacobian_adjoint(opts, w=w)
    ref = np.asarray(w) @ J.cpu().numpy()
    assert np.linalg.norm(v.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    s.close()


def test_single_condition_handle_supports_vjp_only():
    case = synth.smooth_case(48, 24, 2)
    log(f"case: {case.label}, single-condition handle")
    s = JointGapSolver.from_case(case, max_cond=1)
    s.assemble(case.e, case.edot, None, 1)
    opts = s.options(omega=1.8, eps=1e-12)
    s.solve(opts)
    with pytest.raises(G.GapError) as ei:
        s.jacobian_adjoint(opts)
    assert ei.value.status == G.GAP_EINVAL
    v, _ = s.jacobian_adjoint(opts, w=[1.0, 0.0, 0.0, 0.0])
    ref = oracle.jacobian_complex_step(gap_of(case), case.e, case.edot)[0]
    assert np.linalg.norm(v.cpu().numpy() - ref) <= 1e-7 * np.linalg.norm(ref)
    s.close()


def test_autograd_backward_is_the_adjoint_vjp():
    case = synth.textured_case(64, 32, 5)
    log(f"case: {case.label}, autograd")
    s = JointGapSolver.from_case(case, max_cond=1)
    opts = s.options(omega=1.6, eps=1e-13)
    e = torch.tensor(case.e, dtype=torch.float64, requires_grad=True)
    ed = torch.tensor(case.edot, dtype=torch.float64, requires_grad=True)
    F = gap_force(e, ed, s, opts)
    w = torch.tensor([1.0, -0.5, 100.0, 30.0], dtype=torch.float64)
    (F.cpu() * w).sum().backward()
    ref = w.numpy() @ oracle.jacobian_complex_step(gap_of(case), case.e, case.edot, texture_of(case))
    got = np.concatenate([e.grad.numpy(), ed.grad.numpy()])
    assert np.linalg.norm(got - ref) <= 1e-7 * np.linalg.norm(ref)
    F_ref, _ = oracle.condition_forces(gap_of(case), case.e, case.edot, texture_of(case))
    assert np.linalg.norm(F.detach().cpu().numpy() - F_ref) <= 1e-8 * np.linalg.norm(F_ref)
    s.close()


def test_adjoint_against_fd_jacobians_1024x512_textured():
    """Rate columns: forward FD is exact (F is affine in the rates).  Eccentricity columns:
    forward FD carries an O(delta) error, central FD an O(delta^2) one; the adjoint must
    match central FD within 1e-4 and the forward-FD gap must halve with delta."""
    case = synth.make_case("adjoint_textured_1024x512", 0)
    log(f"case: {case.label}, adjoint vs FD")
    s = JointGapSolver.from_case(case, max_cond=9)
    opts = s.options(omega=1.6, eps=1e-12)

    def fd(delta):
        s.assemble(case.e, case.edot, delta, 9)
        s.solve(opts)
        s.integrate()
        return s.jacobian_fd().cpu().numpy(), s.F[:36].view(9, 4).cpu().numpy().copy()

    J_fwd, F_plus = fd(case.delta)
    J_fwd2, _ = fd(case.delta / 2)
    _, F_minus = fd(-case.delta)
    J_cen = (F_plus[1:] - F_minus[1:]).T / (2 * case.delta[None, :])
    s.assemble(case.e, case.edot, case.delta, 9)
    s.solve(opts)
    J_adj, info = s.jacobian_adjoint(opts)
    J_adj = J_adj.cpu().numpy()
    b_adj, b_fwd, b_cen = blocks(J_adj), blocks(J_fwd), blocks(J_cen)
    for k in (1, 3):            # rate blocks vs forward FD
        assert np.linalg.norm(b_adj[k] - b_fwd[k]) <= 1e-4 * np.linalg.norm(b_fwd[k])
    for k in (0, 2):            # eccentricity blocks vs central FD
        assert np.linalg.norm(b_adj[k] - b_cen[k]) <= 1e-4 * np.linalg.norm(b_cen[k])
    gap1 = max(np.linalg.norm(blocks(J_fwd)[k] - b_adj[k]) / np.linalg.norm(b_adj[k]) for k in (0, 2))
    gap2 = max(np.linalg.norm(blocks(J_fwd2)[k] - b_adj[k]) / np.linalg.norm(b_adj[k]) for k in (0, 2))
    log(f"  forward-FD gap {gap1:.2e}, at delta/2 {gap2:.2e}; adjoint iterations {info.iterations}")
    assert 1.6 < gap1 / gap2 < 2.4
    # the joint base + adjoint solve gives the same Jacobian
    s.assemble(case.e, case.edot, None, 1)
    _, J_joint, _ = s.solve_with_adjoint(opts)
    assert block_err(J_joint.cpu().numpy(), J_adj) <= 1e-6
    s.close()


def test_adjoint_clamp_mode_is_finite_and_close_to_fd():
    case = synth.smooth_case(64, 32, 0)
    log(f"case: {case.label}, adjoint in clamp mode")
    J, _ = adjoint_J(case, cavitation=G.GAP_CAVITATION_CLAMP)
    assert np.all(np.isfinite(J))
    Jc = oracle.jacobian_central(gap_of(case), case.e, case.edot, case.delta / 10, cavitation="clamp")
    # piecewise-smooth map: reported, loosely compared
    assert block_err(J, Jc) < 5e-2


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                          G.GAP_ITERATION_STRIPS],
                         ids=["two_launch", "one_launch", "strips"])
@pytest.mark.parametrize("scalars,strategy", [("per_cond", "sync"), ("per_cond", "async"), ("global", "async")])
def test_scalar_and_strategy_variants_follow_oracle(scalars, strategy, iteration):
    case = synth.textured_case(96, 48, 3)
    log(f"case: {case.label}, {scalars} scalars, {strategy}, iteration kind {iteration}")
    gap = gap_of(case)
    tex = texture_of(case)
    blocks_, rhs = [], []
    for ek, edk in oracle.conditions(case.e, case.edot, case.delta):
        A, S = oracle.assemble(gap, ek, edk, tex)
        blocks_.append(A)
        rhs.append(S)
    M = [oracle.assor2_precond(A, 1.6) for A in blocks_]
    p_ref, it_ref, _ = oracle.pcg_blocks(blocks_, rhs, M, 1e-10, 100000, scalars, strategy)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    p, info = s.solve(omega=1.6, eps=1e-10,
                      scalars=G.GAP_SCALARS_PER_COND if scalars == "per_cond" else G.GAP_SCALARS_GLOBAL,
                      strategy=G.GAP_STRATEGY_ASYNC if strategy == "async" else G.GAP_STRATEGY_SYNC,
                      iteration=iteration)
    p = p.reshape(9, -1).cpu().numpy()
    assert abs(info.iterations - it_ref) <= 2, (info.iterations, it_ref)
    for k in range(9):
        assert np.linalg.norm(p[k] - p_ref[k]) <= 1e-8 * np.linalg.norm(p_ref[k])
        if strategy == "async":
            assert info.rel_residual_cond[k] <= 1e-10
    s.close()
