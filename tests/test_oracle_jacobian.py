"""Pins for the oracle's Jacobians (paper Eq 2.13-2.19): affine rate dependence, central
and complex-step derivatives, first-order behaviour of the forward difference."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of, texture_of


def forces9(gap, case, tex, delta):
    return np.array([oracle.condition_forces(gap, ek, edk, tex)[0]
                     for ek, edk in oracle.conditions(case.e, case.edot, delta)])


def blocks(J):
    return [J[0:2, 0:4], J[0:2, 4:8], J[2:4, 0:4], J[2:4, 4:8]]


def block_err(J, ref):
    return max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(blocks(J), blocks(ref)))


def test_fd_formula_on_synthetic_forces():
    F9 = np.arange(36, dtype=float).reshape(9, 4) ** 1.5
    delta = np.linspace(1, 2, 8)
    J = oracle.jacobian_fd(F9, delta)
    for k in range(8):
        assert np.allclose(J[:, k], (F9[k + 1] - F9[0]) / delta[k], rtol=1e-15)


@pytest.fixture(scope="module")
def small():
    case = synth.textured_case(32, 16, 0)
    gap = gap_of(case)
    tex = texture_of(case)
    cs = oracle.jacobian_complex_step(gap, case.e, case.edot, tex)
    return case, gap, tex, cs


def test_rate_columns_are_exact_for_forward_difference(small):
    """Rates enter A p = S only through S, linearly: F is affine in edot."""
    case, gap, tex, cs = small
    J1 = oracle.jacobian_fd(forces9(gap, case, tex, case.delta), case.delta)
    J10 = oracle.jacobian_fd(forces9(gap, case, tex, 10 * case.delta), 10 * case.delta)
    for J in (J1, J10):
        assert np.linalg.norm(J[:, 4:] - cs[:, 4:]) <= 1e-7 * np.linalg.norm(cs[:, 4:])


def test_complex_step_agrees_with_central_difference(small):
    case, gap, tex, cs = small
    Jc = oracle.jacobian_central(gap, case.e, case.edot, case.delta, tex)
    Jc2 = oracle.jacobian_central(gap, case.e, case.edot, case.delta / 2, tex)
    e1 = np.linalg.norm(Jc[:, :4] - cs[:, :4])
    e2 = np.linalg.norm(Jc2[:, :4] - cs[:, :4])
    assert e1 <= 1e-4 * np.linalg.norm(cs[:, :4])
    assert 3.0 < e1 / e2 < 5.0          # second order: the gap shrinks 4x when delta halves


def test_forward_difference_is_first_order(small):
    case, gap, tex, cs = small
    Jf = oracle.jacobian_fd(forces9(gap, case, tex, case.delta), case.delta)
    Jh = oracle.jacobian_fd(forces9(gap, case, tex, case.delta / 2), case.delta / 2)
    e1 = np.linalg.norm(Jf[:, :4] - cs[:, :4])
    e2 = np.linalg.norm(Jh[:, :4] - cs[:, :4])
    assert 1.7 < e1 / e2 < 2.3
    assert block_err(Jf, cs) < 1e-2
