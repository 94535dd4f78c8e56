"""Mutation check of the oracle's pins: each case plants one plausible mistake (a sign, a
dropped or wrong factor, a wrong index, a swapped operand) in a copy of ``oracle/`` and
requires that at least one of the pins below fails on the mutated copy, while all of them
pass on the unmodified oracle.  The pins are closed forms, invariants and textbook limits,
the same kinds of fact the ``test_oracle_*`` files pin (paper Eq 2.3, 2.4-2.7, 2.13-2.19,
3.4-3.6, Table 1, Sec 2.4-III)."""

import importlib
import os
import shutil
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from conftest import gap_of

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gap(O, case, **over):
    d = dict(R=case.R, c=case.c, L=case.L, mu=case.mu, U=case.U, V=case.V, p_in=case.p_in,
             p_out=case.p_out, n_theta=case.n_theta, n_axial=case.n_axial)
    d.update(over)
    return O.Gap(**d)


# ---- pins (each raises AssertionError on failure) --------------------------------------
def pin_film(O):
    """Eq 2.3: e = 0 gives h = c; the stable form equals the literal one; dh/dt is the rate of h."""
    case = synth.smooth_case(16, 8, 1)
    gap = _gap(O, case)
    th, z, _, _ = O.cell_centers(gap)
    TH, Z = np.meshgrid(th, z)
    assert np.allclose(O.film(gap, np.zeros(4), TH, Z), gap.c, rtol=1e-12, atol=0)
    e = np.array([5e-6, -4e-6, -3e-6, 6e-6])
    ed = np.array([2e-4, 1e-4, -3e-4, 5e-5])
    assert np.allclose(O.film(gap, e, TH, Z), O.film_naive(gap, e, TH, Z), rtol=1e-9, atol=0)
    t = 1e-3
    fd = (O.film(gap, e + t * ed, TH, Z) - O.film(gap, e - t * ed, TH, Z)) / (2 * t)
    assert np.allclose(O.film_rate(gap, e, ed, TH, Z), fd, rtol=1e-6, atol=1e-12)


def pin_linear_profile(O):
    """z-independent film, no wedge or squeeze: p = p_in + (p_out - p_in) z / L exactly."""
    case = synth.smooth_case(32, 16, 0)
    for ecc in ((0, 0, 0, 0), (6e-6, -3e-6, 6e-6, -3e-6)):
        gap = _gap(O, case, U=0.0, V=0.0)
        A, S = O.assemble(gap, np.array(ecc, float), np.zeros(4))
        p = O.solve_band(A, S, gap.n_theta).reshape(gap.n_axial, gap.n_theta)
        _, z, _, _ = O.cell_centers(gap)
        exact = gap.p_in + (gap.p_out - gap.p_in) * z / gap.L
        assert np.max(np.abs(p - exact[:, None])) <= 1e-12 * gap.p_in


def pin_symmetric_m_matrix(O):
    case = synth.textured_case(24, 12, 2)
    gap = _gap(O, case)
    tex = O.dimple_texture(case.R, case.dimple_theta, case.dimple_z, case.dimple_radius, case.dimple_depth)
    A, _ = O.assemble(gap, case.e, case.edot, tex)
    assert abs(A - A.T).max() == 0.0
    assert (A - sp.diags(A.diagonal())).max() <= 0.0


def pin_ring_mode(O):
    """Constant film: the ring operator on p = cos(m theta) (any z) returns
    k (dz / dx) (2 - 2 cos(m dtheta)) p on the interior rows (discrete eigenfunction)."""
    case = synth.smooth_case(20, 10, 0)
    gap = _gap(O, case)
    kx, kz = O.face_conductances(gap, np.zeros(4))
    A = O.stencil_matrix(gap, kx, kz)
    th, _, dth, dz = O.cell_centers(gap)
    dx = gap.R * dth
    m = 3
    p = np.tile(np.cos(m * th), (gap.n_axial, 1))
    Ap = (A @ p.ravel()).reshape(p.shape)
    k = gap.c ** 3 / (12 * gap.mu)
    exact = k * (dz / dx) * (2 - 2 * np.cos(m * dth)) * p
    assert np.allclose(Ap[1:-1], exact[1:-1], rtol=1e-9, atol=1e-12 * np.abs(exact).max())


def pin_short_bearing(O):
    """Ocvirk's short-bearing limit with wedge and squeeze (textbook), and its sign."""
    case = synth.smooth_case(128, 32, 0)
    gap = _gap(O, case, L=0.2e-3, p_in=0.0, p_out=0.0)
    e = np.array([8e-6, 3e-6, 8e-6, 3e-6])
    edot = np.array([4e-4, -2e-4, 4e-4, -2e-4])
    A, S = O.assemble(gap, e, edot)
    p = O.solve_band(A, S, gap.n_theta).reshape(gap.n_axial, gap.n_theta)
    th, z, _, _ = O.cell_centers(gap)
    TH, Z = np.meshgrid(th, z)
    Rc = gap.R + gap.c
    ax, ay = Rc * np.cos(TH) - e[0], Rc * np.sin(TH) - e[1]
    h = np.hypot(ax, ay) - gap.R                      # Eq 2.3 for a parallel axis
    hx = (e[0] * np.sin(TH) - e[1] * np.cos(TH)) * Rc / np.hypot(ax, ay) / gap.R
    ht = -(ax * edot[0] + ay * edot[1]) / np.hypot(ax, ay)
    exact = (3 * gap.mu * gap.U * hx + 6 * gap.mu * ht) * Z * (Z - gap.L) / h ** 3
    assert np.max(np.abs(p - exact)) / np.max(np.abs(exact)) < 5e-3


def pin_rate_step(O):
    """The condition list of Eq 2.17-2.19 steps e_j by delta_j and edot_j by delta_{4+j}."""
    d = np.arange(1, 9) * 1e-3
    conds = O.conditions(np.zeros(4), np.zeros(4), d)
    for j in range(4):
        assert np.array_equal(conds[1 + j][0], np.eye(4)[j] * d[j])
        assert np.array_equal(conds[5 + j][1], np.eye(4)[j] * d[4 + j])


def pin_assor(O):
    """Eq 3.5-3.6 applied in two steps equal the explicit Eq 3.4 matrix."""
    case = synth.textured_case(6, 4, 1)
    gap = _gap(O, case)
    A, _ = O.assemble(gap, case.e, case.edot)
    Me = O.assor2_explicit(A, 1.3)
    apply = O.assor2_precond(A, 1.3)
    rng = np.random.default_rng(0)
    for _ in range(3):
        r = rng.standard_normal(A.shape[0])
        assert np.allclose(apply(r), Me @ r, rtol=1e-12, atol=1e-12 * np.abs(Me @ r).max())


def pin_cg(O):
    """Table 1 without preconditioning takes the conjugate-gradient iterates (SciPy's CG)."""
    case = synth.smooth_case(16, 8, 3)
    gap = _gap(O, case)
    A, S = O.assemble(gap, case.e, case.edot)
    p, it, _ = O.pcg(A, S, lambda r: r.copy(), 1e-300, 12)
    ref, _ = spla.cg(A, S, x0=np.zeros_like(S), rtol=1e-300, atol=0.0, maxiter=12)
    assert it == 12 and np.linalg.norm(p - ref) <= 1e-8 * np.linalg.norm(ref)


def pin_forces(O):
    """p = cos(theta) on a concentric gap at rest: Fx = -dA n_axial (n_theta / 2)
    (1 + (h / 2) sin(dtheta) / (R dtheta)) (the shear of the circumferential gradient), and
    Mx = My = 0 about the mid-length point (the field does not depend on z)."""
    case = synth.smooth_case(24, 10, 0)
    gap = _gap(O, case, U=0.0, V=0.0, p_in=0.0, p_out=0.0)
    th, z, dth, dz = O.cell_centers(gap)
    p = np.tile(np.cos(th), (gap.n_axial, 1))
    F = O.forces_for_condition(gap, np.zeros(4), p)
    dA = gap.R * dth * dz
    fx = -dA * gap.n_axial * (gap.n_theta / 2) * (1 + 0.5 * gap.c * np.sin(dth) / (gap.R * dth))
    assert abs(F[0] - fx) <= 1e-12 * abs(fx)
    assert abs(F[1]) <= 1e-12 * abs(fx)
    assert abs(F[2]) <= 1e-12 * abs(fx) * gap.L and abs(F[3]) <= 1e-12 * abs(fx) * gap.L


def pin_jacobian(O):
    """Forward differences of Eq 2.13-2.14 are exact in the rate columns (F is affine in the
    rates): against the complex-step derivative."""
    case = synth.smooth_case(12, 8, 4)
    gap = _gap(O, case)
    F9 = np.array([O.condition_forces(gap, ek, edk)[0] for ek, edk in O.conditions(case.e, case.edot, case.delta)])
    J = O.jacobian_fd(F9, case.delta)
    Jc = O.jacobian_complex_step(gap, case.e, case.edot)
    assert np.linalg.norm(J[:, 4:] - Jc[:, 4:]) <= 1e-6 * np.linalg.norm(Jc[:, 4:])
    assert np.linalg.norm(J[:, :4] - Jc[:, :4]) <= 5e-2 * np.linalg.norm(Jc[:, :4])


PINS = [pin_film, pin_linear_profile, pin_symmetric_m_matrix, pin_ring_mode, pin_short_bearing, pin_rate_step,
        pin_assor, pin_cg, pin_forces, pin_jacobian]

# (file, original text, mutated text, what the mistake is); the first occurrence is replaced
MUTATIONS = [
    ("film.py", "q = (Rc * Rc - R * R) - 2.0 * Rc *", "q = (Rc * Rc - R * R) + 2.0 * Rc *", "eccentricity sign in h"),
    ("film.py", "return -(ax * exd + ay * eyd) / d", "return (ax * exd + ay * eyd) / d", "squeeze sign"),
    ("film.py", "ex = e1 + (e3 - e1) * z / L", "ex = e1 + (e3 - e2) * z / L", "axis-offset index"),
    ("film.py", "d = np.sqrt(R * R + q)", "d = np.sqrt(R * R - q)", "sign under the root"),
    ("fvm.py", "kx = h_east ** 3 / (12.0 * gap.mu) * (dz / dx)", "kx = h_east ** 3 / (12.0 * gap.mu) * (dx / dz)",
     "east-face aspect ratio"),
    ("fvm.py", "    kz[0, :] *= 2.0\n", "    kz[0, :] *= 1.0\n", "half-cell Dirichlet face dropped"),
    ("fvm.py", "S = -(0.5 * gap.U) * (h_e - h_w) * dz", "S = (0.5 * gap.U) * (h_e - h_w) * dz", "wedge sign"),
    ("fvm.py", "- hdot * dx * dz\n    _, kz", "+ hdot * dx * dz\n    _, kz", "squeeze sign in the source"),
    ("fvm.py", "dirichlet[0, :] += kz[0, :] * gap.p_in", "dirichlet[0, :] += kz[0, :] * gap.p_out", "inlet value"),
    ("fvm.py", "kx_w = kx[:, (np.arange(nt) - 1) % nt]", "kx_w = kx[:, (np.arange(nt) + 1) % nt]",
     "west-face index"),
    ("fvm.py", "edj[j] += delta[4 + j]", "edj[j] += delta[j]", "rate step"),
    ("pcg.py", "            t = -omega * (L @ t) / D\n", "            t = -omega * (LT @ t) / D\n",
     "L^T in the first sweep"),
    ("pcg.py", "        return omega * (2.0 - omega) * z\n", "        return omega * z\n", "ASSOR scale factor"),
    ("pcg.py", "        beta = d_new / d\n", "        beta = d / d_new\n", "beta inverted"),
    ("pcg.py", "    r = S - A @ p\n    hist", "    r = A @ p - S\n    hist", "initial residual sign"),
    ("forces.py", "    Fx = np.sum(-p * c - tau_t * s) * dA", "    Fx = np.sum(-p * c + tau_t * s) * dA",
     "shear sign in Fx"),
    ("forces.py", "    zr = Z - 0.5 * gap.L\n    Fx", "    zr = Z\n    Fx", "moment reference point"),
    ("forces.py", "    tau_t = -0.5 * h * dpdx + gap.mu * gap.U / h\n    tau_z = -0.5 * h * dpdz + gap.mu * gap.V / h\n"
     "    c, s = np.cos(TH), np.sin(TH)\n    zr = Z - 0.5 * gap.L\n    Fx",
     "    tau_t = 0.5 * h * dpdx + gap.mu * gap.U / h\n    tau_z = -0.5 * h * dpdz + gap.mu * gap.V / h\n"
     "    c, s = np.cos(TH), np.sin(TH)\n    zr = Z - 0.5 * gap.L\n    Fx", "pressure-gradient shear sign"),
    ("jacobian.py", "    return (F9[1:9, :] - F9[0:1, :]).T / delta[None, :]",
     "    return (F9[1:9, :] - F9[0:1, :]).T / delta[::-1][None, :]", "FD steps in the wrong order"),
]


def load_copy(tmp_path, name, mutation=None):
    """A copy of oracle/ as package `name`, with one text replacement applied."""
    dst = tmp_path / name
    shutil.copytree(os.path.join(ROOT, "oracle"), dst / name,
                    ignore=shutil.ignore_patterns("__pycache__", "*.so"))
    if mutation:
        f, old, new, _ = mutation
        path = dst / name / f
        text = path.read_text()
        assert text.count(old) >= 1, (f, old)
        path.write_text(text.replace(old, new, 1))
    sys.path.insert(0, str(dst))
    try:
        return importlib.import_module(name)
    finally:
        sys.path.remove(str(dst))


def failing_pins(O):
    failed = []
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(O)
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError, np.linalg.LinAlgError):
            failed.append(pin.__name__)
    return failed


def test_pins_pass_on_the_oracle(tmp_path):
    assert failing_pins(load_copy(tmp_path, "oracle_copy_clean")) == []


@pytest.mark.parametrize("k", range(len(MUTATIONS)), ids=[m[3].replace(" ", "_") for m in MUTATIONS])
def test_a_planted_mistake_fails_a_pin(tmp_path, k):
    O = load_copy(tmp_path, f"oracle_copy_m{k}", MUTATIONS[k])
    failed = failing_pins(O)
    assert failed, f"no pin caught: {MUTATIONS[k][3]}"
