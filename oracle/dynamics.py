"""Oracle: one general-iteration step of the piston equilibrium (paper Sec 2.3, Eq 2.10,
2.12-2.14, 2.20-2.22).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Equilibrium (Eq 2.10): F = F_E + F_I + F_O = 0, with F = (Fx, Fy, Mx, My) (Eq 2.11), F_O the
oil-film force of the base condition, F_E an external load and F_I the inertia force.
Readings taken (the paper gives neither loads nor an inertia model):
  * F_I = -M (edot - edot_prev) / dt: a constant 4 x 4 mass matrix M acting on the
    backward-difference acceleration of the eccentricities;
  * the eccentricities follow the backward-difference scheme e = e_prev + dt edot (the
    scheme under Eq 2.22), so an update keeps de = dt d(edot).
Then Eq 2.12, 0 = F + F_,e de + F_,edot d(edot), becomes
  general (both Jacobians):      (F_,edot + dt F_,e) d(edot) = -F,   de = dt d(edot);
  conventional (Eq 2.20-2.22):    F_,edot d(edot) = -F,              de = dt d(edot),
with F_,e = dF_O/de and F_,edot = dF_O/dedot - M / dt, the oil-film parts by the forward
differences of Eq 2.13-2.14.
"""

import numpy as np

from .fvm import conditions
from .jacobian import condition_forces, jacobian_fd


def residual(F_O, F_ext, mass, edot, edot_prev, dt):
    """F = F_E + F_I + F_O with F_I = -M (edot - edot_prev) / dt."""
    mass = np.asarray(mass, dtype=float).reshape(4, 4)
    F_I = -mass @ (np.asarray(edot, float) - np.asarray(edot_prev, float)) / dt
    return np.asarray(F_ext, float) + F_I + np.asarray(F_O, float)


def update(F, J_O, mass, dt, scheme="general"):
    """The increments (de, d(edot)) of Eq 2.12 (scheme "general") or Eq 2.20-2.22 ("conventional")
    from the residual F and the 4 x 8 oil-film Jacobian J_O = [dF_O/de | dF_O/dedot]."""
    J_O = np.asarray(J_O, dtype=float).reshape(4, 8)
    mass = np.asarray(mass, dtype=float).reshape(4, 4)
    F_e = J_O[:, :4]
    F_ed = J_O[:, 4:] - mass / dt
    K = F_ed + dt * F_e if scheme == "general" else F_ed
    d_edot = np.linalg.solve(K, -np.asarray(F, float))
    return dt * d_edot, d_edot


def step(gap, e, edot, delta, F_ext, mass, edot_prev, dt, texture=None, scheme="general"):
    """One step from (e, edot): the 9 conditions solved exactly, forces, the FD Jacobian, the
    update.  Returns (e_new, edot_new, F at the input state, J_O)."""
    kw = {} if texture is None else {"texture": texture}
    F9 = np.array([condition_forces(gap, ek, edk, **kw)[0] for ek, edk in conditions(e, edot, delta)])
    J_O = jacobian_fd(F9, delta)
    F = residual(F9[0], F_ext, mass, edot, edot_prev, dt)
    de, d_edot = update(F, J_O, mass, dt, scheme)
    return np.asarray(e, float) + de, np.asarray(edot, float) + d_edot, F, J_O
