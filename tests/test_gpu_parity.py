"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Tolerances (stated in the parity plan of the build, FP64 on both sides):
  pressure  max_k ||p_k - p*_k|| / ||p*_k|| <= 1e-9   (PCG run to eps = 1e-13)
  forces    ||dF_xy|| / ||F_xy|| and ||dM_xy|| / ||M_xy|| <= 1e-8 per condition
  FD Jacobian (same formula on both sides, amplified force round-off) <= 1e-5 per 2x4 block
"""

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

P_TOL, F_TOL, J_TOL = 1e-9, 1e-8, 1e-5
EPS_PARITY = 1e-13
# both iteration kinds: Table 1 as printed (two launches) and the one-launch default
ITERATIONS = pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                                      G.GAP_ITERATION_STRIPS],
                                     ids=["two_launch", "one_launch", "strips"])


def log(msg):
    print(msg, flush=True)


def oracle_case(case, n_cond, method="band"):
    gap = gap_of(case)
    tex = texture_of(case)
    conds = oracle.conditions(case.e, case.edot, case.delta)[:n_cond]
    ps, Fs = [], []
    for ek, edk in conds:
        F, p = oracle.condition_forces(gap, ek, edk, tex, method=method)
        ps.append(p)
        Fs.append(F)
    return np.array(ps), np.array(Fs)


def gpu_case(case, n_cond, eps=EPS_PARITY, **opt):
    s = JointGapSolver.from_case(case, max_cond=9 if n_cond == 9 else 1)
    s.assemble(case.e, case.edot, case.delta, n_cond)
    opt.setdefault("omega", case.omega)
    p, info = s.solve(eps=eps, **opt)
    F = s.integrate()
    J = s.jacobian_fd().cpu().numpy() if n_cond == 9 else None
    out = (p.reshape(n_cond, -1).cpu().numpy(), F.cpu().numpy(), J, info)
    s.close()
    return out


def pressure_err(p, p_ref):
    return max(np.linalg.norm(p[k] - p_ref[k]) / np.linalg.norm(p_ref[k]) for k in range(len(p_ref)))


def force_err(F, F_ref):
    worst = 0.0
    for k in range(len(F_ref)):
        worst = max(worst, np.linalg.norm(F[k, :2] - F_ref[k, :2]) / np.linalg.norm(F_ref[k, :2]),
                    np.linalg.norm(F[k, 2:] - F_ref[k, 2:]) / np.linalg.norm(F_ref[k, 2:]))
    return worst


def jac_err(J, J_ref):
    blocks = [(slice(0, 2), slice(0, 4)), (slice(0, 2), slice(4, 8)), (slice(2, 4), slice(0, 4)),
              (slice(2, 4), slice(4, 8))]
    return max(np.linalg.norm(J[b] - J_ref[b]) / np.linalg.norm(J_ref[b]) for b in blocks)


@pytest.mark.parametrize("seed", range(10))
def test_smooth_64x32_single_condition(seed):
    case = synth.smooth_case(64, 32, seed)
    log(f"case: {case.label}, 1 condition")
    p_ref, F_ref = oracle_case(case, 1)
    p, F, _, info = gpu_case(case, 1)
    assert info.rel_residual <= EPS_PARITY
    assert pressure_err(p, p_ref) <= P_TOL
    assert force_err(F, F_ref) <= F_TOL


@ITERATIONS
@pytest.mark.parametrize("seed", [0, 7])
def test_smooth_64x32_joint_nine_conditions(seed, iteration):
    case = synth.smooth_case(64, 32, seed)
    log(f"case: {case.label}, 9 conditions, iteration kind {iteration}")
    p_ref, F_ref = oracle_case(case, 9)
    p, F, J, info = gpu_case(case, 9, iteration=iteration)
    assert pressure_err(p, p_ref) <= P_TOL
    assert force_err(F, F_ref) <= F_TOL
    assert jac_err(J, oracle.jacobian_fd(F_ref, case.delta)) <= J_TOL


@ITERATIONS
@pytest.mark.parametrize("shape", [(3, 2), (5, 7), (67, 33), (300, 41), (1000, 3), (257, 9)])
def test_ragged_grids_textured(shape, iteration):
    case = synth.textured_case(*shape, 3)
    log(f"case: {case.label}, 9 conditions, iteration kind {iteration}")
    p_ref, F_ref = oracle_case(case, 9, method="dense" if shape[0] * shape[1] <= 64 else "band")
    p, F, J, info = gpu_case(case, 9, iteration=iteration)
    assert pressure_err(p, p_ref) <= P_TOL
    assert force_err(F, F_ref) <= F_TOL


def test_textured_256x128_joint():
    case = synth.textured_case(256, 128, 1)
    log(f"case: {case.label}, 9 conditions")
    p_ref, F_ref = oracle_case(case, 9)
    p, F, J, info = gpu_case(case, 9)
    assert pressure_err(p, p_ref) <= P_TOL
    assert force_err(F, F_ref) <= F_TOL
    assert jac_err(J, oracle.jacobian_fd(F_ref, case.delta)) <= J_TOL


def test_joint_smooth_512x256():
    case = synth.make_case("joint_smooth_512x256", 0)
    log(f"case: {case.label}, 9 conditions")
    p_ref, F_ref = oracle_case(case, 9)
    p, F, J, info = gpu_case(case, 9)
    log(f"  iterations {info.iterations}")
    assert pressure_err(p, p_ref) <= P_TOL
    assert force_err(F, F_ref) <= F_TOL
    assert jac_err(J, oracle.jacobian_fd(F_ref, case.delta)) <= J_TOL


@ITERATIONS
@pytest.mark.parametrize("precond,name", [(G.GAP_PRECOND_ASSOR2, "assor2"), (G.GAP_PRECOND_ASSOR1, "assor1"),
                                          (G.GAP_PRECOND_JACOBI, "jacobi")])
def test_iteration_counts_follow_oracle_pcg(precond, name, iteration):
    """Same recurrence as the oracle's Table 1 PCG on the joint matrix (global scalars); the
    one-launch iteration forms alpha's denominator from other sums and agrees up to rounding."""
    case = synth.textured_case(96, 48, 2)
    log(f"case: {case.label}, 9 conditions, {name}, iteration kind {iteration}")
    gap = gap_of(case)
    AG, SG = oracle.assemble_joint(gap, case.e, case.edot, case.delta, texture_of(case))
    M = {"assor2": oracle.assor2_precond(AG, 1.6), "assor1": oracle.assor1_precond(AG, 1.6),
         "jacobi": oracle.jacobi_precond(AG)}[name]
    pG, it_ref, hist = oracle.pcg(AG, SG, M, 1e-10, 100000)
    p, F, J, info = gpu_case(case, 9, eps=1e-10, precond=precond, omega=1.6, iteration=iteration)
    assert abs(info.iterations - it_ref) <= 2, (info.iterations, it_ref)
    assert np.linalg.norm(p.ravel() - pG) / np.linalg.norm(pG) < 1e-8


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("shape", [(96, 48), (300, 41)], ids=["96x48", "300x41"])
def test_neumann_order_follows_oracle(shape, m):
    """ASSOR II with the series of Eq 3.4 kept to order m in both factors (strip iteration):
    the iteration count within 2 of the oracle's Table 1 PCG with assor2_precond(neumann=m) on
    the same joint matrix, fewer iterations than order 1, and at eps 1e-13 the pressure and
    forces of conditions 0, 1 and 5 against the exact (banded-Cholesky) solution."""
    case = synth.textured_case(*shape, 3)
    log(f"case: {case.label}, 9 conditions, Neumann order {m}")
    gap, tex = gap_of(case), texture_of(case)
    blocks, rhs = [], []
    for ek, edk in oracle.conditions(case.e, case.edot, case.delta):
        A, S = oracle.assemble(gap, ek, edk, tex)
        blocks.append(A)
        rhs.append(S)
    Ms = [oracle.assor2_precond(A, 1.6, neumann=m) for A in blocks]
    _, it_ref, _ = oracle.pcg_blocks(blocks, rhs, Ms, 1e-10, 100000, "global", "sync")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    _, info1 = s.solve(omega=1.6, eps=1e-10, iteration=G.GAP_ITERATION_STRIPS)
    _, info = s.solve(omega=1.6, eps=1e-10, neumann=m, iteration=G.GAP_ITERATION_STRIPS)
    log(f"  iterations {info.iterations} (oracle {it_ref}; order 1: {info1.iterations})")
    assert abs(info.iterations - it_ref) <= 2 and info.iterations < info1.iterations
    p, info13 = s.solve(omega=1.6, eps=1e-13, neumann=m, iteration=G.GAP_ITERATION_STRIPS)
    F = s.integrate().cpu().numpy()
    p = p.reshape(9, -1).cpu().numpy()
    s.close()
    conds = oracle.conditions(case.e, case.edot, case.delta)
    for k in (0, 1, 5):
        F_ref, p_ref = oracle.condition_forces(gap, *conds[k], tex)
        assert pressure_err(p[k:k + 1], p_ref[None]) <= P_TOL
        assert force_err(F[k:k + 1], F_ref[None]) <= F_TOL


@ITERATIONS
@pytest.mark.parametrize("name,precond", [("assor2", G.GAP_PRECOND_ASSOR2), ("assor1", G.GAP_PRECOND_ASSOR1)])
@pytest.mark.parametrize("omega", [0.1, 0.46, 1.0, 1.54, 1.9])
def test_omega_sweep_iteration_counts_follow_oracle(name, precond, omega, iteration):
    """The relaxation-factor study (omega = 0.1 + 0.18 i): the GPU recurrence follows the
    oracle's Table 1 PCG with the same preconditioner at every omega."""
    case = synth.smooth_case(64, 32, 3)
    log(f"case: {case.label}, 9 conditions, {name}, omega {omega}")
    AG, SG = oracle.assemble_joint(gap_of(case), case.e, case.edot, case.delta)
    M = (oracle.assor2_precond if name == "assor2" else oracle.assor1_precond)(AG, omega)
    pG, it_ref, _ = oracle.pcg(AG, SG, M, 1e-10, 100000)
    p, F, J, info = gpu_case(case, 9, eps=1e-10, precond=precond, omega=omega, iteration=iteration)
    assert abs(info.iterations - it_ref) <= 2, (info.iterations, it_ref)
    assert np.linalg.norm(p.ravel() - pG) / np.linalg.norm(pG) < 1e-8


@ITERATIONS
def test_per_condition_scalars_reach_same_solution(iteration):
    case = synth.smooth_case(128, 64, 4)
    log(f"case: {case.label}, 9 conditions, per-condition scalars, iteration kind {iteration}")
    p_ref, F_ref = oracle_case(case, 9)
    p, F, J, info = gpu_case(case, 9, scalars=G.GAP_SCALARS_PER_COND, iteration=iteration)
    assert pressure_err(p, p_ref) <= P_TOL
    assert force_err(F, F_ref) <= F_TOL


@ITERATIONS
def test_warm_start_from_solution_takes_no_iterations(iteration):
    case = synth.smooth_case(64, 32, 2)
    log(f"case: {case.label}, warm start, iteration kind {iteration}")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    s.solve(eps=1e-12, omega=case.omega, iteration=iteration)
    _, info = s.solve(eps=1e-10, omega=case.omega, warm_start=True, iteration=iteration)
    assert info.iterations == 0
    s.close()


def test_cavitation_clamp_forces():
    case = synth.smooth_case(64, 32, 0)
    log(f"case: {case.label}, clamp")
    gap = gap_of(case)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    p, _ = s.solve(eps=EPS_PARITY, omega=case.omega)
    F = s.integrate(G.GAP_CAVITATION_CLAMP, 0.0).cpu().numpy()
    pn = p.reshape(9, -1).cpu().numpy()
    F_ref = np.array([oracle.forces_for_condition(gap, ek, pn[k], cavitation="clamp", p_cav=0.0)
                      for k, (ek, edk) in enumerate(oracle.conditions(case.e, case.edot, case.delta))])
    assert np.max(np.abs(F - F_ref) / np.abs(F_ref).max(axis=0)) <= 1e-12
    s.close()


def test_assembly_matches_oracle_elementwise():
    case = synth.textured_case(200, 90, 5)
    log(f"case: {case.label}, assembly")
    gap = gap_of(case)
    tex = texture_of(case)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    for k, (ek, edk) in enumerate(oracle.conditions(case.e, case.edot, case.delta)):
        kx, kz, S = [t.cpu().numpy() for t in s.read_system(k)]
        kx_r, kz_r = oracle.face_conductances(gap, ek, tex)
        S_r = oracle.source(gap, ek, edk, tex)
        # The oracle forms R_c^2 - R^2 literally (cancellation ~3e-14 of q, up to ~10x larger
        # relative to q where the film is thinnest, x3 through h^3); the kernel uses c (2R + c).
        assert np.max(np.abs(kx - kx_r) / np.abs(kx_r)) < 1e-12
        assert np.max(np.abs(kz - kz_r) / np.abs(kz_r)) < 1e-12
        assert np.max(np.abs(S - S_r)) < 1e-11 * np.max(np.abs(S_r))
    s.close()


def test_error_paths():
    case = synth.smooth_case(64, 32, 0)
    log("case: error paths")
    s = JointGapSolver.from_case(case, max_cond=9)
    with pytest.raises(G.GapError) as ei:
        s.solve(eps=1e-10)
    assert ei.value.status == G.GAP_ESTATE
    with pytest.raises(G.GapError) as ei:
        s.assemble(np.array([case.c, 0, 0, 0]), case.edot, case.delta, 9)
    assert ei.value.status == G.GAP_ECONTACT
    s.assemble(case.e, case.edot, case.delta, 9)
    with pytest.raises(G.GapError) as ei:
        s.solve(eps=1e-10, max_iter=3)
    assert ei.value.status == G.GAP_ENOCONV and ei.value.info.iterations == 3
    with pytest.raises(G.GapError) as ei:
        s.solve(eps=1e-10, omega=2.0)
    assert ei.value.status == G.GAP_EINVAL
    s.close()
    s1 = JointGapSolver.from_case(case, max_cond=1)
    with pytest.raises(G.GapError) as ei:
        s1.assemble(case.e, case.edot, case.delta, 9)
    assert ei.value.status == G.GAP_EINVAL
    s1.assemble(case.e, case.edot, None, 1)
    s1.solve(eps=1e-10, omega=case.omega)
    s1.integrate()
    with pytest.raises(G.GapError) as ei:
        s1.jacobian_fd()
    assert ei.value.status == G.GAP_ESTATE
    s1.close()


def test_split_forces_and_rebuilt_field():
    """Pressure / shear split with the axial force and torque, and the full field with its
    boundary rows, against the oracle (axial sliding V != 0 so that every shear term is on)."""
    case = synth.textured_case(80, 36, 4)
    log(f"case: {case.label}, 9 conditions, split forces and rebuilt field")
    V = 0.15
    gap, tex = gap_of(case, V=V), texture_of(case)
    s = JointGapSolver(case.R, case.c, case.L, case.mu, case.U, V, case.p_in, case.p_out, case.n_theta, case.n_axial,
                       dimples=(case.dimple_theta, case.dimple_z, case.dimple_radius, case.dimple_depth), max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    s.solve(omega=case.omega, eps=EPS_PARITY)
    Fs = s.integrate_split().cpu().numpy()
    F = s.integrate().cpu().numpy()
    full = s.full_pressure().cpu().numpy()
    full_c = s.full_pressure(G.GAP_CAVITATION_CLAMP, 0.0).cpu().numpy()
    p_gpu = s.pressure().reshape(9, -1).cpu().numpy()
    s.close()
    for k, (ek, edk) in enumerate(oracle.conditions(case.e, case.edot, case.delta)):
        _, p_ref = oracle.condition_forces(gap, ek, edk, tex)
        ref = oracle.forces_split_for_condition(gap, ek, p_ref, tex)
        for sl in (slice(0, 2), slice(2, 4), slice(4, 6), slice(6, 8)):
            assert np.linalg.norm(Fs[k, sl] - ref[sl]) <= F_TOL * np.linalg.norm(ref[sl]), (k, sl)
        assert abs(Fs[k, 8] - ref[8]) <= F_TOL * abs(ref[8]) and abs(Fs[k, 9] - ref[9]) <= F_TOL * abs(ref[9])
        np.testing.assert_allclose(Fs[k, 0:4] + Fs[k, 4:8], F[k], rtol=1e-12, atol=1e-12 * np.abs(F[k]).max())
        np.testing.assert_array_equal(full[k], oracle.rebuild_field(gap, p_gpu[k]))
        np.testing.assert_array_equal(full_c[k], oracle.rebuild_field(gap, p_gpu[k], "clamp", 0.0))


def test_true_residual_reported_at_exit():
    """The true residual ||S - A p|| / ||S|| the library recomputes at exit, against the same
    quantity on the CPU: with the library's own assembled system (read back) to 1e-4 (at a
    residual of 1e-10 the subtraction S - A p cancels, so the summation order alone moves the
    norm by ~1e-6), and with the oracle's system to 5e-2 (entry differences of 1e-13..1e-12
    between the two assemblies move a 1e-10 residual by up to ~1e-2)."""
    case = synth.textured_case(70, 30, 8)
    log(f"case: {case.label}, true residual at exit")
    gap, tex = gap_of(case), texture_of(case)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    p, info = s.solve(omega=case.omega, eps=1e-10)
    p = p.reshape(9, -1).cpu().numpy()
    systems = [[t.cpu().numpy() for t in s.read_system(k)] for k in range(9)]
    s.close()
    rr = ss = 0.0
    for k, (ek, edk) in enumerate(oracle.conditions(case.e, case.edot, case.delta)):
        kx, kz, Sg = systems[k]
        r = Sg.ravel() - oracle.stencil_matrix(gap, kx, kz) @ p[k]
        rel = np.linalg.norm(r) / np.linalg.norm(Sg)
        assert abs(info.true_rel_residual_cond[k] - rel) <= 1e-4 * rel, (k, info.true_rel_residual_cond[k], rel)
        A, S = oracle.assemble(gap, ek, edk, tex)
        rel_o = np.linalg.norm(S - A @ p[k]) / np.linalg.norm(S)
        assert abs(info.true_rel_residual_cond[k] - rel_o) <= 5e-2 * rel_o
        rr += r @ r
        ss += Sg.ravel() @ Sg.ravel()
    assert abs(info.true_rel_residual - np.sqrt(rr / ss)) <= 1e-4 * np.sqrt(rr / ss)
    assert info.true_rel_residual <= 10 * info.rel_residual      # the recurrence tracks it
