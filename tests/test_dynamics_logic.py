"""Host-side logic of the dynamics driver (no GPU): swashplate kinematics, the synthetic inlet
pressure and loads, and the inertia matrix of the rigid piston."""

import math

import numpy as np

from paper_2511_06824_amd.dynamics import PumpKinematics


def test_axial_speed_is_the_derivative_of_the_stroke():
    """V = omega R_b tan(beta) sin(phi) is d/dt of the stroke R_b tan(beta) (1 - cos(phi))."""
    k = PumpKinematics()
    stroke = lambda phi: k.R_b * math.tan(math.radians(k.beta_deg)) * (1.0 - math.cos(phi))
    for phi in np.linspace(0.1, 6.0, 7):
        h = 1e-6
        dsdt = (stroke(phi + h) - stroke(phi - h)) / (2 * h) * k.omega
        assert abs(k.V(phi) - dsdt) <= 1e-8 * max(1.0, abs(dsdt))
    assert abs(k.omega - 2 * math.pi * 10.0) < 1e-12            # 600 rpm


def test_inlet_pressure_levels_and_continuity():
    k = PumpKinematics()
    assert abs(k.p_in(math.radians(90.0)) - k.p_high) < 1e-6
    assert abs(k.p_in(math.radians(270.0)) - k.p_low) < 1e-6
    assert abs(k.p_in(0.0) - 0.5 * (k.p_low + k.p_high)) < 1e-6
    assert abs(k.p_in(math.pi) - 0.5 * (k.p_low + k.p_high)) < 1e-3
    phis = np.linspace(0.0, 4 * math.pi, 7201)
    p = np.array([k.p_in(x) for x in phis])
    assert np.max(np.abs(np.diff(p))) < 0.01 * (k.p_high - k.p_low)   # no jumps
    assert np.all(p >= k.p_low - 1e-9) and np.all(p <= k.p_high + 1e-9)


def test_external_load_is_the_swashplate_reaction_and_centrifugal_force():
    k = PumpKinematics()
    R, L = 0.01, 0.04
    phi = math.radians(90.0)
    F = k.external_load(phi, R, L, lever=0.015)
    side = k.p_high * math.pi * R * R * math.tan(math.radians(10.0))
    cf = (0.128 + 0.0259) * k.omega ** 2 * 40.5e-3
    np.testing.assert_allclose(F, [cf - side, 0.0, 0.0, -(0.02 + 0.015) * side], rtol=1e-12)


def test_mass_matrix_translation_and_tilt():
    """A translation a = (a, 0, a, 0) gives Fx = -m a and no moment; a tilt about the gap
    centre (e1 = -e3) gives only a moment, of size I * (2a / L)."""
    k = PumpKinematics()
    L = 0.04
    M = k.mass_matrix(L)
    m = 0.128 + 0.0259
    Irot = 0.128 * L ** 2 / 12
    a = 3.0
    np.testing.assert_allclose(-M @ [a, 0, a, 0], [-m * a, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(-M @ [0, a, 0, a], [0, -m * a, 0, 0], atol=1e-15)
    # tilt in the x-z plane, theta_y = (e3 - e1) / L: My = -I theta_y''
    np.testing.assert_allclose(-M @ [-a, 0, a, 0], [0, 0, 0, -Irot * 2 * a / L], atol=1e-15)
    # tilt in the y-z plane, theta_x = -(e4 - e2) / L: Mx = -I theta_x''
    np.testing.assert_allclose(-M @ [0, -a, 0, a], [0, 0, Irot * 2 * a / L, 0], atol=1e-15)
