"""Pins for the oracle's general-iteration step (paper Sec 2.3, Eq 2.10, 2.12, 2.20-2.22):
exactness on an affine force model, the term the conventional scheme drops, the
backward-difference constraint, and convergence to a known equilibrium with the real film
forces."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of

D = oracle.dynamics


def affine_model(seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=4) * 50.0
    A = rng.normal(size=(4, 4)) * 1e6 + np.eye(4) * 5e6       # N/m
    B = rng.normal(size=(4, 4)) * 1e4 + np.eye(4) * 2e5       # N/(m/s)
    return c, A, B


def mass_matrix(seed):
    rng = np.random.default_rng(seed + 7)
    Q = rng.normal(size=(4, 4))
    return Q @ Q.T * 0.01 + np.eye(4) * 0.15


@pytest.mark.parametrize("seed", range(3))
def test_general_step_is_exact_for_an_affine_force(seed):
    """Eq 2.12 is the first-order expansion: for F_O affine in (e, edot) with the exact
    Jacobian, one step from a backward-difference-consistent state lands on F = 0."""
    c, A, B = affine_model(seed)
    M = mass_matrix(seed)
    dt = 2e-4
    rng = np.random.default_rng(seed + 1)
    e_prev, ed_prev = rng.normal(size=4) * 1e-6, rng.normal(size=4) * 1e-4
    ed = ed_prev + rng.normal(size=4) * 1e-4
    e = e_prev + dt * ed
    F_ext = rng.normal(size=4) * 30.0
    F = D.residual(c + A @ e + B @ ed, F_ext, M, ed, ed_prev, dt)
    de, d_ed = D.update(F, np.hstack([A, B]), M, dt, "general")
    e1, ed1 = e + de, ed + d_ed
    F1 = D.residual(c + A @ e1 + B @ ed1, F_ext, M, ed1, ed_prev, dt)
    assert np.linalg.norm(F1) <= 1e-10 * np.linalg.norm(F)
    np.testing.assert_allclose(e1 - e_prev - dt * ed1, e - e_prev - dt * ed, atol=1e-20)


def test_conventional_step_drops_the_eccentricity_jacobian():
    """Eq 2.20-2.22: exact when F_O does not depend on e; with A != 0 the residual left after
    one step is exactly dt A d(edot), the term Eq 2.12 keeps."""
    c, A, B = affine_model(4)
    M = mass_matrix(4)
    dt = 1e-4
    e_prev, ed_prev = np.full(4, 1e-7), np.full(4, 2e-5)
    ed = ed_prev + 3e-5
    e = e_prev + dt * ed
    F_ext = np.array([10.0, -5.0, 0.2, 0.1])
    for AA in (np.zeros((4, 4)), A):
        F = D.residual(c + AA @ e + B @ ed, F_ext, M, ed, ed_prev, dt)
        de, d_ed = D.update(F, np.hstack([AA, B]), M, dt, "conventional")
        F1 = D.residual(c + AA @ (e + de) + B @ (ed + d_ed), F_ext, M, ed + d_ed, ed_prev, dt)
        np.testing.assert_allclose(F1, dt * AA @ d_ed, rtol=1e-9, atol=1e-12 * np.linalg.norm(F))
    assert np.linalg.norm(dt * A @ d_ed) > 1e-3 * np.linalg.norm(F)


def test_general_iteration_converges_to_a_known_equilibrium():
    """Real film forces (32 x 16 smooth gap): loads chosen so that (e*, edot*) is in
    equilibrium; the general iteration with forward-difference Jacobians returns to it."""
    case = synth.smooth_case(32, 16, 3)
    gap = gap_of(case)
    dt = 1e-4
    M = np.diag([0.154, 0.154, 2e-5, 2e-5])
    ed_prev = np.zeros(4)
    e_prev = np.array(case.e) * 0.5
    ed_star = np.array([2e-5, -1e-5, -3e-5, 1.5e-5])
    e_star = e_prev + dt * ed_star
    F_star, _ = oracle.condition_forces(gap, e_star, ed_star)
    F_ext = -(F_star - M @ (ed_star - ed_prev) / dt)
    ed = ed_prev.copy()
    e = e_prev + dt * ed
    err0 = np.linalg.norm(ed - ed_star)
    errs = []
    for _ in range(3):
        e, ed, F, _ = D.step(gap, e, ed, case.delta, F_ext, M, ed_prev, dt)
        errs.append(np.linalg.norm(ed - ed_star))
    assert errs[0] < 1e-2 * err0 and errs[2] < 1e-7 * err0
    np.testing.assert_allclose(e, e_prev + dt * ed, rtol=0, atol=1e-18)
