"""Pins for the oracle's assembly and exact solve: closed forms, textbook limits,
invariants and brute force (paper Eq 2.1, 2.4-2.7, 2.17-2.19, 3.7)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from conftest import gap_of, texture_of


def solve(gap, e, edot, texture=oracle.no_texture):
    A, S = oracle.assemble(gap, e, edot, texture)
    return oracle.solve_band(A, S, gap.n_theta).reshape(gap.n_axial, gap.n_theta)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("seed", range(3))
def test_matrix_symmetric_m_matrix_spd(seed):
    case = synth.textured_case(48, 24, seed)
    gap = gap_of(case)
    A, _ = oracle.assemble(gap, case.e, case.edot, texture_of(case))
    assert abs(A - A.T).max() == 0.0
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0.0
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    assert np.all(rowsum >= -1e-12 * A.diagonal())
    bnd = np.r_[0:gap.n_theta, A.shape[0] - gap.n_theta:A.shape[0]]
    assert np.all(rowsum[bnd] > 0)
    ev = np.linalg.eigvalsh(np.asarray(A.todense()))
    assert ev.min() > 0


@pytest.mark.parametrize("ecc", [(0, 0, 0, 0), (6e-6, -3e-6, 6e-6, -3e-6)])
def test_linear_axial_profile_closed_form(ecc):
    """No wedge, squeeze or texture and h independent of z: p = p_in + (p_out-p_in) z/L."""
    case = synth.smooth_case(64, 32, 0)
    U = 0.0 if any(ecc) else case.U      # concentric: h constant, the wedge term vanishes anyway
    gap = gap_of(case, U=U)
    p = solve(gap, np.array(ecc, float), np.zeros(4))
    _, z, _, _ = oracle.cell_centers(gap)
    exact = gap.p_in + (gap.p_out - gap.p_in) * z / gap.L
    assert np.max(np.abs(p - exact[:, None])) <= 1e-13 * gap.p_in


def test_axisymmetric_groove_series_resistance():
    """Concentric piston with an axial groove profile h_text(z): the axial flux is the same
    through every face, so p follows the cumulative face resistances (discrete closed form)."""
    case = synth.smooth_case(32, 40, 0)
    gap = gap_of(case)

    def groove(theta, z):
        return 8e-6 * np.exp(-((z - 0.4 * gap.L) / (0.1 * gap.L)) ** 2) + 0.0 * theta

    p = solve(gap, np.zeros(4), np.zeros(4), groove)
    _, _, dth, dz = oracle.cell_centers(gap)
    dx = gap.R * dth
    zf = np.arange(gap.n_axial + 1) * dz
    h = gap.c + groove(0.0, zf)
    cond = h ** 3 / (12 * gap.mu) * dx / dz
    cond[0] *= 2
    cond[-1] *= 2
    res = 1.0 / cond
    q = (gap.p_in - gap.p_out) / res.sum()
    exact = gap.p_in - q * np.cumsum(res)[:-1]
    assert np.max(np.abs(p - exact[:, None])) <= 1e-12 * gap.p_in


def test_short_bearing_limit_wedge_and_squeeze():
    """L << R (Ocvirk's short-bearing approximation, textbook): the circumferential flow
    is negligible and p = (3 mu U dh/dx + 6 mu dh/dt) z (z - L) / h^3 with p = 0 at both ends."""
    case = synth.smooth_case(256, 64, 0)
    gap = gap_of(case, L=0.2e-3, p_in=0.0, p_out=0.0)
    e = np.array([8e-6, 3e-6, 8e-6, 3e-6])          # parallel: h independent of z
    edot = np.array([4e-4, -2e-4, 4e-4, -2e-4])
    p = solve(gap, e, edot)
    th, z, _, _ = oracle.cell_centers(gap)
    TH, Z = np.meshgrid(th, z)
    h = oracle.film(gap, e, TH, Z)
    t = 1e-7
    hx = (oracle.film(gap, e, TH + t, Z) - oracle.film(gap, e, TH - t, Z)) / (2 * t) / gap.R
    ht = (oracle.film(gap, e + t * edot, TH, Z) - oracle.film(gap, e - t * edot, TH, Z)) / (2 * t)
    exact = (3 * gap.mu * gap.U * hx + 6 * gap.mu * ht) * Z * (Z - gap.L) / h ** 3
    err = np.max(np.abs(p - exact)) / np.max(np.abs(exact))
    assert err < 2e-3, err      # observed 2.4e-4 (z-discretisation floor at 64 rows)
    # the sign pins: converging wedge / approaching walls raise the pressure
    i_peak = np.unravel_index(np.argmax(exact), exact.shape)
    assert p[i_peak] > 0


@pytest.mark.parametrize("k", [5, 16])
def test_rotation_invariance(k):
    case = synth.smooth_case(64, 32, 3)
    gap = gap_of(case)
    phi = 2 * np.pi * k / gap.n_theta
    Rm = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])

    def rot(v):
        return np.r_[Rm @ v[:2], Rm @ v[2:]]

    p0 = solve(gap, case.e, case.edot)
    p1 = solve(gap, rot(case.e), rot(case.edot))
    assert rel(p1, np.roll(p0, k, axis=1)) < 1e-12
    F0 = oracle.forces_for_condition(gap, case.e, p0)
    F1 = oracle.forces_for_condition(gap, rot(case.e), p1)
    assert np.allclose(F1[:2], Rm @ F0[:2], rtol=0, atol=1e-9 * np.abs(F0[:2]).max())
    assert np.allclose(F1[2:], Rm @ F0[2:], rtol=0, atol=1e-9 * np.abs(F0[2:]).max())


def test_reflection_invariance():
    case = synth.smooth_case(64, 32, 4)
    gap = gap_of(case)
    flip = np.array([1, -1, 1, -1])
    p0 = solve(gap, case.e, case.edot)
    gap_m = gap_of(case, U=-case.U)
    p1 = solve(gap_m, flip * case.e, flip * case.edot)
    assert rel(p1, p0[:, ::-1]) < 1e-12
    F0 = oracle.forces_for_condition(gap, case.e, p0)
    F1 = oracle.forces_for_condition(gap_m, flip * case.e, p1)
    assert np.allclose(F1, F0 * np.array([1, -1, -1, 1]), rtol=1e-9, atol=1e-9 * np.abs(F0).max())


def test_superposition_in_sources():
    case = synth.smooth_case(48, 24, 5)
    full = gap_of(case, V=0.7)
    e, ed = case.e, case.edot
    z4 = np.zeros(4)
    parts = [solve(gap_of(case, V=0.0, U=0.0, p_out=0.0), e, z4),
             solve(gap_of(case, V=0.0, U=0.0, p_in=0.0), e, z4),
             solve(gap_of(case, V=0.0, p_in=0.0, p_out=0.0), e, z4),
             solve(gap_of(case, V=0.7, U=0.0, p_in=0.0, p_out=0.0), e, z4),
             solve(gap_of(case, V=0.0, U=0.0, p_in=0.0, p_out=0.0), e, ed)]
    assert rel(sum(parts), solve(full, e, ed)) < 1e-12


def test_global_flux_balance():
    """Summing all rows: net outflow through both Dirichlet ends equals minus the volume
    rate of the film (squeeze) minus the axial-wedge term of the sliding axial wall."""
    case = synth.textured_case(64, 32, 1)
    gap = gap_of(case, V=0.5)
    tex = texture_of(case)
    kx, kz = oracle.face_conductances(gap, case.e, tex)
    p = solve(gap, case.e, case.edot, tex)
    out = np.sum(kz[0] * (p[0] - gap.p_in)) + np.sum(kz[-1] * (p[-1] - gap.p_out))
    th, z, dth, dz = oracle.cell_centers(gap)
    dx = gap.R * dth
    TH, Z = np.meshgrid(th, z)
    hdot = oracle.film_rate(gap, case.e, case.edot, TH, Z)
    hL = oracle.film(gap, case.e, th, gap.L + 0 * th, tex)
    h0 = oracle.film(gap, case.e, th, 0 * th, tex)
    expect = -np.sum(hdot) * dx * dz - 0.5 * gap.V * dx * np.sum(hL - h0)
    scale = np.sum(np.abs(kz[0] * (p[0] - gap.p_in)))
    assert abs(out - expect) <= 1e-10 * scale


@pytest.mark.parametrize("shape", [(8, 4), (16, 8), (32, 16), (3, 2)])
def test_brute_force_dense_band_sor_agree(shape):
    case = synth.textured_case(*shape, 2)
    gap = gap_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot, texture_of(case))
    pd = oracle.solve_dense(A, S)
    pb = oracle.solve_band(A, S, gap.n_theta)
    ps, sweeps, rr = oracle.sor_solve(A, S, omega=1.0 if shape[0] < 8 else 1.7, tol=1e-15)
    assert rel(pb, pd) < 1e-12
    assert rel(ps, pd) < 1e-11, (sweeps, rr)


@pytest.mark.parametrize("shape", [(256, 128), (512, 256)])
def test_band_matches_sparse_lu(shape):
    case = synth.smooth_case(*shape, 0)
    gap = gap_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot)
    pb = oracle.solve_band(A, S, gap.n_theta)
    pl = spla.spsolve(A.tocsc(), S)
    assert rel(pb, pl) < 1e-10
    assert np.linalg.norm(A @ pb - S) / np.linalg.norm(S) < 1e-12


def test_conditions_and_shared_operators():
    case = synth.smooth_case(32, 16, 0)
    gap = gap_of(case)
    conds = oracle.conditions(case.e, case.edot, case.delta)
    assert len(conds) == 9
    for k in range(1, 5):
        de = conds[k][0] - case.e
        assert np.count_nonzero(de) == 1 and de[k - 1] == pytest.approx(case.delta[k - 1], rel=1e-6)
        assert np.array_equal(conds[k][1], case.edot)
    for k in range(5, 9):
        assert np.array_equal(conds[k][0], case.e)
        dd = conds[k][1] - case.edot
        assert np.count_nonzero(dd) == 1 and dd[k - 5] == pytest.approx(case.delta[k - 1], rel=1e-6)
    A0, _ = oracle.assemble(gap, *conds[0])
    for k in range(5, 9):                 # rates enter only the source
        Ak, _ = oracle.assemble(gap, *conds[k])
        assert (Ak != A0).nnz == 0
    AG, SG = oracle.assemble_joint(gap, case.e, case.edot, case.delta)
    n = gap.n_theta * gap.n_axial
    A3, S3 = oracle.assemble(gap, *conds[3])
    assert abs(AG[3 * n:4 * n, 3 * n:4 * n] - A3).max() == 0
    assert np.array_equal(SG[3 * n:4 * n], S3)


def test_cell_values_equal_full_assembly_everywhere():
    """The cell-by-cell entries (used to spot-check grids too large to assemble) are the
    full-array entries, bitwise, at every cell of a textured grid including both Dirichlet
    rows and both wrap columns."""
    case = synth.textured_case(40, 17, 3)
    gap = gap_of(case)
    tex = texture_of(case)
    kx_r, kz_r = oracle.face_conductances(gap, case.e, tex)
    S_r = oracle.source(gap, case.e, case.edot, tex)
    J, I = np.meshgrid(np.arange(gap.n_axial), np.arange(gap.n_theta), indexing="ij")
    kx, kz_s, kz_n, S = oracle.cell_values(gap, case.e, case.edot, I, J, tex)
    assert np.array_equal(kx, kx_r)
    assert np.array_equal(kz_s, kz_r[:-1])
    assert np.array_equal(kz_n, kz_r[1:])
    assert np.array_equal(S, S_r)
