"""Oracle: condition solves, forces and the double Jacobian (paper Eq 2.13-2.19).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``jacobian_fd``      : Eq 2.13-2.14 from the forces of the 9 conditions of Eq 2.17-2.19,
                         J[:, k] = (F_k - F_0) / delta_k, columns (e1..e4, edot1..edot4),
                         rows (Fx, Fy, Mx, My).
* ``jacobian_central`` : (F(x + delta_k) - F(x - delta_k)) / (2 delta_k), second-order.
* ``jacobian_complex_step`` : Im F(x + i h_k) / h_k, h_k tiny; exact to round-off for the
                         analytic map x -> F (cavitation mode "none"), computed with a
                         complex sparse LU solve.
"""

import numpy as np
import scipy.sparse.linalg as spla

from .direct import solve_band, solve_dense
from .film import Gap, no_texture
from .fvm import assemble, conditions
from .forces import forces_for_condition


def solve_condition(gap: Gap, e, edot, texture=no_texture, method="band"):
    """Exact discrete pressure of one condition (flat, natural order)."""
    A, S = assemble(gap, e, edot, texture)
    if method == "band":
        return solve_band(A, S, gap.n_theta)
    if method == "dense":
        return solve_dense(A, S)
    if method == "splu":
        return spla.spsolve(A.tocsc(), S)
    raise ValueError(method)


def condition_forces(gap: Gap, e, edot, texture=no_texture, cavitation="none", p_cav=0.0,
                     method="band"):
    p = solve_condition(gap, e, edot, texture, method)
    return forces_for_condition(gap, e, p, texture, cavitation, p_cav), p


def jacobian_fd(F9, delta):
    """Eq 2.13-2.14: forward differences from the 9 condition forces F9 (9, 4)."""
    F9 = np.asarray(F9, dtype=float)
    delta = np.asarray(delta, dtype=float)
    return (F9[1:9, :] - F9[0:1, :]).T / delta[None, :]


def _perturbed(e, edot, k, step):
    e = np.array(e, dtype=np.result_type(float, step))
    edot = np.array(edot, dtype=np.result_type(float, step))
    if k < 4:
        e[k] = e[k] + step
    else:
        edot[k - 4] = edot[k - 4] + step
    return e, edot


def jacobian_central(gap: Gap, e, edot, delta, texture=no_texture, cavitation="none", p_cav=0.0,
                     method="band"):
    J = np.zeros((4, 8))
    for k in range(8):
        ep, edp = _perturbed(e, edot, k, delta[k])
        em, edm = _perturbed(e, edot, k, -delta[k])
        Fp, _ = condition_forces(gap, ep, edp, texture, cavitation, p_cav, method)
        Fm, _ = condition_forces(gap, em, edm, texture, cavitation, p_cav, method)
        J[:, k] = (Fp - Fm) / (2.0 * delta[k])
    return J


def jacobian_complex_step(gap: Gap, e, edot, texture=no_texture, scale=(1e-5, 1e-3)):
    """Exact Jacobian by complex-step differentiation (cavitation mode "none" only)."""
    J = np.zeros((4, 8))
    for k in range(8):
        h = 1e-30 * (scale[0] if k < 4 else scale[1])
        ec, edc = _perturbed(e, edot, k, 1j * h)
        A, S = assemble(gap, ec, edc, texture)
        p = spla.spsolve(A.tocsc(), S)
        F = forces_for_condition(gap, ec, p, texture, "none")
        J[:, k] = np.imag(F) / h
    return J


def joint_conditions(e, edot, delta):
    return conditions(e, edot, delta)
