"""GPU parity of GMAF step V (the general iteration of Eq 2.12, with the conventional scheme of
Eq 2.20-2.22 as an option) and of the operating-point update used by the pump kinematics,
through the C ABI, against the oracle."""

import math

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
from paper_2511_06824_amd.dynamics import PumpKinematics, equilibrium, simulate  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402

DT = 1e-4
MASS = np.diag([0.154, 0.154, 2e-5, 2e-5])


def log(msg):
    print(msg, flush=True)


def state(seed):
    rng = np.random.default_rng(seed)
    ed_prev = rng.uniform(-1e-4, 1e-4, 4)
    ed = ed_prev + rng.uniform(-5e-5, 5e-5, 4)
    F_ext = np.array([rng.uniform(-50, 50), rng.uniform(-50, 50), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)])
    return ed_prev, ed, F_ext


@pytest.mark.parametrize("scheme,name", [(G.GAP_SCHEME_GENERAL, "general"), (G.GAP_SCHEME_CONVENTIONAL, "conventional")])
@pytest.mark.parametrize("case", [synth.smooth_case(48, 24, 1), synth.textured_case(64, 32, 2)], ids=["smooth48", "tex64"])
def test_step_matches_oracle(case, scheme, name):
    log(f"case: {case.label}, general iteration step ({name}, FD Jacobian)")
    gap, tex = gap_of(case), texture_of(case)
    ed_prev, ed, F_ext = state(3)
    e = np.array(case.e) * 0.5
    e_ref, ed_ref, F_ref, _ = oracle.dynamics.step(gap, e, ed, case.delta, F_ext, MASS, ed_prev, DT, tex, name)
    s = JointGapSolver.from_case(case, max_cond=9)
    opts = s.options(omega=case.omega, eps=1e-13)
    e_new, ed_new, F, J, info = s.general_iteration_step(e, ed, case.delta, DT, ed_prev, F_ext, MASS, opts,
                                                         scheme=scheme)
    s.close()
    dF = np.linalg.norm(np.array(F) - F_ref) / np.linalg.norm(F_ref)
    d_ed = np.linalg.norm(np.array(ed_new) - ed_ref) / np.linalg.norm(ed_ref - ed)
    d_e = np.linalg.norm(np.array(e_new) - e_ref) / np.linalg.norm(e_ref - e)
    log(f"  residual {dF:.1e}, d(edot) {d_ed:.1e}, de {d_e:.1e}")
    assert dF <= 1e-8 and d_ed <= 1e-5 and d_e <= 1e-5


def test_adjoint_step_uses_the_exact_jacobian():
    case = synth.textured_case(40, 20, 4)
    log(f"case: {case.label}, general iteration step (adjoint Jacobian)")
    gap, tex = gap_of(case), texture_of(case)
    ed_prev, ed, F_ext = state(5)
    e = np.array(case.e) * 0.3
    F_O, _ = oracle.condition_forces(gap, e, ed, tex)
    F_ref = oracle.dynamics.residual(F_O, F_ext, MASS, ed, ed_prev, DT)
    J_cs = oracle.jacobian_complex_step(gap, e, ed, tex)
    de_ref, ded_ref = oracle.dynamics.update(F_ref, J_cs, MASS, DT, "general")
    s = JointGapSolver.from_case(case, max_cond=9)
    opts = s.options(omega=case.omega, eps=1e-13)
    e_new, ed_new, F, J, _ = s.general_iteration_step(e, ed, None, DT, ed_prev, F_ext, MASS, opts,
                                                      jacobian=G.GAP_JACOBIAN_ADJOINT)
    s.close()
    assert np.linalg.norm(np.array(F) - F_ref) <= 1e-8 * np.linalg.norm(F_ref)
    assert np.linalg.norm(np.array(ed_new) - ed - ded_ref) <= 1e-6 * np.linalg.norm(ded_ref)
    assert np.linalg.norm(np.array(e_new) - e - de_ref) <= 1e-6 * np.linalg.norm(de_ref)


def test_general_iteration_returns_to_a_known_equilibrium():
    """Loads chosen by the oracle so that (e*, edot*) is in equilibrium; three GPU steps with
    warm-started solves return to it."""
    case = synth.smooth_case(64, 32, 3)
    log(f"case: {case.label}, Picard iteration to a known equilibrium")
    gap = gap_of(case)
    ed_prev = np.zeros(4)
    e_prev = np.array(case.e) * 0.5
    ed_star = np.array([2e-5, -1e-5, -3e-5, 1.5e-5])
    F_star, _ = oracle.condition_forces(gap, e_prev + DT * ed_star, ed_star)
    F_ext = -(F_star - MASS @ (ed_star - ed_prev) / DT)
    s = JointGapSolver.from_case(case, max_cond=9)
    e, ed, hist, its = equilibrium(s, e_prev, ed_prev, DT, F_ext, MASS, case.delta, tol=1e-12, max_picard=4,
                                   opts=s.options(omega=case.omega, eps=1e-13))
    s.close()
    log(f"  residuals {[f'{h:.1e}' for h in hist]}, PCG iterations {its}")
    assert np.linalg.norm(ed - ed_star) <= 1e-6 * np.linalg.norm(ed_star)
    assert its[-1] < its[0]                                     # warm starts


def test_operating_point_matches_oracle():
    case = synth.textured_case(96, 40, 6)
    log(f"case: {case.label}, operating point U, V, p_in, p_out changed")
    U, V, p_in, p_out = 0.9, -0.07, 4.5e6, 0.5e6
    s = JointGapSolver.from_case(case, max_cond=9)
    s.set_operating_point(U, V, p_in, p_out)
    with pytest.raises(G.GapError):
        s.solve()                                                # needs a new assembly
    s.assemble(case.e, case.edot, case.delta, 9)
    p, _ = s.solve(omega=case.omega, eps=1e-13)
    F = s.integrate().cpu().numpy()
    p = p.reshape(9, -1).cpu().numpy()
    s.close()
    gap = oracle.Gap(case.R, case.c, case.L, case.mu, U, V, p_in, p_out, case.n_theta, case.n_axial)
    tex = texture_of(case)
    for k, (ek, edk) in enumerate(oracle.conditions(case.e, case.edot, case.delta)):
        F_ref, p_ref = oracle.condition_forces(gap, ek, edk, tex)
        assert np.linalg.norm(p[k] - p_ref) <= 1e-9 * np.linalg.norm(p_ref)
        assert np.linalg.norm(F[k, :2] - F_ref[:2]) <= 1e-8 * np.linalg.norm(F_ref[:2])
        assert np.linalg.norm(F[k, 2:] - F_ref[2:]) <= 1e-8 * np.linalg.norm(F_ref[2:])


def test_pump_simulation_converges_every_time_step():
    """Twelve 1-degree time steps of the synthetic pump (600 rpm, swashplate 10 degrees, inlet
    pressure ramping into delivery): every time point reaches equilibrium."""
    case = synth.smooth_case(64, 32, 0)
    log(f"case: {case.label}, 12 time steps of the synthetic pump")
    kin = PumpKinematics()
    s = JointGapSolver.from_case(case, max_cond=9)
    U = kin.omega * case.R
    traj = simulate(s, kin, 12, 0.1 / 360, case.delta, np.zeros(4), np.zeros(4), tol=1e-6, max_picard=8, U=U)
    s.close()
    for r in traj:
        log(f"  phi {math.degrees(r['phi']):5.1f} p_in {r['p_in'] / 1e6:5.2f} MPa picard {r['picard']} "
            f"residual {r['residual']:.1e} |e|/c {np.max(np.abs(r['e'])) / case.c:.3f}")
    assert all(r["picard"] < 8 for r in traj)
    assert all(np.max(np.abs(r["e"])) < case.c for r in traj)
