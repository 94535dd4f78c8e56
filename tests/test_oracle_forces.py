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
