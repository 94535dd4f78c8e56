"""Pins for the oracle's force and moment integration on synthetic fields with closed-form
integrals (midpoint sums of trigonometric polynomials over a periodic grid are exact)."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of


def grid(gap):
    th, z, dth, dz = oracle.cell_centers(gap)
    TH, Z = np.meshgrid(th, z)
    return TH, Z


@pytest.fixture
def gap():
    return gap_of(synth.smooth_case(64, 32, 0), U=0.0, V=0.0)


def test_pressure_terms_cos_sin(gap):
    TH, Z = grid(gap)
    P = 3e6
    h = np.full(TH.shape, 1e-30)          # shear terms scale with h -> negligible
    F = oracle.force_moment(gap, P * np.cos(TH), h)
    area = np.pi * gap.R * gap.L
    assert F[0] == pytest.approx(-P * area, rel=1e-13)
    assert abs(F[1]) < 1e-12 * P * area
    F = oracle.force_moment(gap, P * np.sin(TH), h)
    assert F[1] == pytest.approx(-P * area, rel=1e-13)
    assert abs(F[0]) < 1e-12 * P * area


def test_pressure_moments(gap):
    TH, Z = grid(gap)
    P = 1e8
    h = np.full(TH.shape, 1e-30)
    _, _, dth, dz = oracle.cell_centers(gap)
    nz = gap.n_axial
    s2 = dz ** 3 * nz * (nz * nz - 1) / 12.0          # sum_j (z_j - L/2)^2 dz
    F = oracle.force_moment(gap, P * (Z - gap.L / 2) * np.cos(TH), h)
    assert F[3] == pytest.approx(-P * np.pi * gap.R * s2, rel=1e-12)
    assert abs(F[2]) < 1e-12 * abs(F[3])
    F = oracle.force_moment(gap, P * (Z - gap.L / 2) * np.sin(TH), h)
    assert F[2] == pytest.approx(P * np.pi * gap.R * s2, rel=1e-12)


def test_shear_terms_closed_form():
    """p linear in z (gradients exact on every row), h = c (1 + eps cos theta):
    Fy = mu U R L (2 pi / c)(1 - 1/sqrt(1-eps^2))/eps, Fx = Mx = 0,
    My = (R G / 2) R L c eps pi - mu V R^2 L (2 pi / c)(1 - 1/sqrt(1-eps^2))/eps."""
    base = synth.smooth_case(128, 16, 0)
    gap = gap_of(base, U=1.7, V=0.6)
    TH, Z = grid(gap)
    c, eps = gap.c, 0.4
    h = c * (1 + eps * np.cos(TH))
    G = (gap.p_out - gap.p_in) / gap.L
    p = gap.p_in + G * Z
    F = oracle.force_moment(gap, p, h)
    I1 = (2 * np.pi / c) * (1 - 1 / np.sqrt(1 - eps * eps)) / eps     # int cos/h dtheta
    R, L, mu = gap.R, gap.L, gap.mu
    assert F[1] == pytest.approx(mu * gap.U * R * L * I1, rel=1e-10)
    My = 0.5 * R * G * R * L * c * eps * np.pi - mu * gap.V * R * R * L * I1
    assert F[3] == pytest.approx(My, rel=1e-10)
    scale = abs(G) * R * R * L * c
    assert abs(F[0]) < 1e-10 * abs(F[1]) and abs(F[2]) < 1e-12 * scale


def test_cavitation_clamp(gap):
    TH, Z = grid(gap)
    h = np.full(TH.shape, gap.c)
    p = 2e6 + 1e6 * np.cos(TH)
    assert np.array_equal(oracle.effective_pressure(p, "clamp", 0.0), p)
    q = -5e5 + 0.0 * p
    assert np.all(oracle.effective_pressure(q, "clamp", 0.0) == 0.0)
    F = oracle.force_moment(gap, oracle.effective_pressure(-1e6 * np.cos(TH) - 2e6, "clamp", 0.0), h)
    assert F[0] == 0.0 and F[1] == 0.0
    with pytest.raises(ValueError):
        oracle.effective_pressure(p, "elrod")


def test_circumferential_gradient_shear():
    """p = P sin(theta), h = h0: the periodic central difference gives exactly
    dp/dx = P cos(theta) sin(dtheta) / (dtheta R), so the Poiseuille part of tau_theta adds
    -(h0/2) P (sin(dtheta)/dtheta) pi L to Fy on top of the pressure term -P pi R L."""
    gap = gap_of(synth.smooth_case(48, 16, 0), U=0.0, V=0.0)
    TH, Z = grid(gap)
    P, h0 = 2e6, 30e-6
    _, _, dth, _ = oracle.cell_centers(gap)
    F = oracle.force_moment(gap, P * np.sin(TH), np.full(TH.shape, h0))
    expect = -P * np.pi * gap.R * gap.L - 0.5 * h0 * P * np.sin(dth) / dth * np.pi * gap.L
    assert F[1] == pytest.approx(expect, rel=1e-13)
    assert abs(F[1] + P * np.pi * gap.R * gap.L) > 1e3 * 1e-13 * abs(expect)   # term is visible


def test_split_couette_torque_and_no_pressure_force():
    """Concentric gap at uniform pressure with the wall sliding at U: tau_theta = mu U / c,
    so the torque is R mu U / c times the area 2 pi R L; the pressure part of (Fx, Fy, Mx, My)
    vanishes and there is no axial shear."""
    g = oracle.Gap(0.01, 2e-5, 0.04, 0.04, 1.7, 0.0, 3e6, 3e6, 48, 20)
    p = np.full((20, 48), 3e6)
    h = np.full((20, 48), g.c)
    Fs = oracle.force_moment_split(g, p, h)
    torque = g.R * g.mu * g.U / g.c * 2 * np.pi * g.R * g.L
    assert abs(Fs[9] - torque) <= 1e-12 * torque
    assert np.all(np.abs(Fs[:4]) <= 1e-9 * 3e6 * g.R * g.L) and abs(Fs[8]) <= 1e-12 * torque
    np.testing.assert_allclose(Fs[4:8], 0.0, atol=1e-12 * torque)


def test_split_axial_poiseuille_force():
    """Concentric gap with the linear axial profile (no sliding): dp/dz = (p_out - p_in)/L on
    every row (the end rows see the Dirichlet face 1.5 dz away), tau_z = -(c/2) dp/dz, so the
    axial force is -(c/2) (p_out - p_in)/L times 2 pi R L; adding V adds mu V / c per area."""
    for V in (0.0, 0.3):
        g = oracle.Gap(0.01, 2e-5, 0.04, 0.04, 0.0, V, 8e6, 1e5, 32, 25)
        _, z, _, _ = oracle.cell_centers(g)
        p = np.repeat((g.p_in + (g.p_out - g.p_in) * z / g.L)[:, None], 32, axis=1)
        Fs = oracle.force_moment_split(g, p, np.full((25, 32), g.c))
        area = 2 * np.pi * g.R * g.L
        fz = (-0.5 * g.c * (g.p_out - g.p_in) / g.L + g.mu * V / g.c) * area
        assert abs(Fs[8] - fz) <= 1e-12 * abs(fz)
        assert abs(Fs[9]) <= 1e-12 * abs(fz)


def test_split_parts_add_up_to_the_total():
    case = synth.textured_case(40, 18, 2)
    from conftest import texture_of
    gap, tex = gap_of(case), texture_of(case)
    F, p = oracle.condition_forces(gap, case.e, case.edot, tex)
    Fs = oracle.forces_split_for_condition(gap, case.e, p, tex)
    np.testing.assert_allclose(Fs[0:4] + Fs[4:8], F, rtol=1e-12, atol=1e-12 * np.max(np.abs(F)))


def test_rebuilt_field_is_linear_for_the_linear_profile():
    """The rebuilt field of the linear axial solution is linear in z through both boundary
    rows (at z = 0 and z = L, half a cell beyond the end centres)."""
    g = oracle.Gap(0.01, 2e-5, 0.04, 0.04, 0.0, 0.0, 5e6, 2e5, 16, 10)
    _, z, _, dz = oracle.cell_centers(g)
    p = np.repeat((g.p_in + (g.p_out - g.p_in) * z / g.L)[:, None], 16, axis=1)
    full = oracle.rebuild_field(g, p)
    zz = np.concatenate([[0.0], z, [g.L]])
    np.testing.assert_allclose(full, np.repeat((g.p_in + (g.p_out - g.p_in) * zz / g.L)[:, None], 16, axis=1),
                               rtol=1e-13)
    clamped = oracle.rebuild_field(g, p - 4e6, cavitation="clamp", p_cav=0.0)
    assert clamped.min() >= 0.0 and clamped[0, 0] == g.p_in
