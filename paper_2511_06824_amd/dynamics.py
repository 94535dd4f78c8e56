"""GMAF step V on the GPU path: the general (Picard) iteration of the piston equilibrium
F_E + F_I + F_O = 0 at successive time points (Sec 2.3, Eq 2.10-2.12), with the axial sliding
speed of a swashplate pump and a time-varying inlet pressure (NEXT to the hot path: the paper's
measured inlet trace and loads are not given, so both are synthetic here).

Each Picard iteration is one call of ``general_iteration_step`` in the HIP library: assembly,
joint PCG solve, forces and the Jacobian on the device, then the 4 x 4 update of Eq 2.12 on the
host.  The pressure field of the previous iteration is the warm start of the next.

Kinematics (textbook swashplate pump; the paper gives only the parameters of Table 8): a piston
on pitch radius R_b, swashplate angle beta, shaft speed omega, slides axially with
V(phi) = omega R_b tan(beta) sin(phi).  The inlet pressure p_in(phi) (bottom of the piston) rises
from p_low to p_high over the delivery half-turn with cosine ramps; the outlet end stays at
p_out (0.5 MPa in the paper's set-up).  The external load is the lateral swashplate reaction
p_in pi R^2 tan(beta) acting at the ball joint a distance `lever` beyond the gap centre, plus the
centrifugal force of piston and slipper, m omega^2 R_b.
"""

import math
from dataclasses import dataclass

import numpy as np

from . import gapsolve as G


@dataclass
class PumpKinematics:
    rpm: float = 600.0
    R_b: float = 40.5e-3            # pitch radius of the cylinder block (Table 8)
    beta_deg: float = 10.0          # swashplate angle (Table 8)
    p_low: float = 0.5e6
    p_high: float = 10.0e6
    p_out: float = 0.5e6            # outlet end (paper Sec 4.3)
    ramp_deg: float = 30.0
    m_piston: float = 0.128         # Table 8
    m_slipper: float = 0.0259       # Table 8

    @property
    def omega(self):
        return 2.0 * math.pi * self.rpm / 60.0

    def phi(self, t):
        return self.omega * t

    def V(self, phi):
        return self.omega * self.R_b * math.tan(math.radians(self.beta_deg)) * math.sin(phi)

    def p_in(self, phi):
        """p_high over the delivery half-turn (0 <= phi mod 2 pi < pi), p_low over suction,
        joined by cosine ramps of ramp_deg centred on 0 and pi."""
        x = math.degrees(phi) % 360.0
        w = self.ramp_deg

        def up(d):   # 0 -> 1 across [-w/2, w/2]
            if d <= -w / 2:
                return 0.0
            if d >= w / 2:
                return 1.0
            return 0.5 - 0.5 * math.cos(math.pi * (d + w / 2) / w)

        d0 = x if x < 180.0 else x - 360.0      # distance to the start of delivery
        s = up(d0) if abs(d0) <= 90.0 else (1.0 - up(x - 180.0))
        return self.p_low + (self.p_high - self.p_low) * s

    def external_load(self, phi, R, length, lever=0.015):
        """F_E = (Fx, Fy, Mx, My): lateral swashplate reaction in -x at the ball joint and the
        centrifugal force in +x (radial direction of the piston)."""
        side = self.p_in(phi) * math.pi * R * R * math.tan(math.radians(self.beta_deg))
        centrifugal = (self.m_piston + self.m_slipper) * self.omega ** 2 * self.R_b
        arm = 0.5 * length + lever          # ball joint beyond the outlet end, from z_ref = L/2
        # the side force (-side, 0, 0) at (x, 0, arm) has the moment arm * (-side) about y
        return np.array([centrifugal - side, 0.0, 0.0, -arm * side])

    def mass_matrix(self, length):
        """F_I = -M (edot - edot_prev)/dt in (Fx, Fy, Mx, My) for a rigid piston whose axis passes
        through (e1, e2) at z = 0 and (e3, e4) at z = L: translation of the gap centre with the
        piston and slipper mass, tilt with the piston's moment of inertia m L^2 / 12."""
        m = self.m_piston + self.m_slipper
        Irot = self.m_piston * length ** 2 / 12.0
        M = np.zeros((4, 4))
        M[0, 0] = M[0, 2] = 0.5 * m                   # Fx = -m (a1 + a3)/2
        M[1, 1] = M[1, 3] = 0.5 * m                   # Fy = -m (a2 + a4)/2
        M[2, 1], M[2, 3] = Irot / length, -Irot / length      # Mx =  I (a4 - a2)/L
        M[3, 0], M[3, 2] = -Irot / length, Irot / length      # My = -I (a3 - a1)/L
        return M


def step_params(dt, edot_prev, F_ext, mass, scheme=G.GAP_SCHEME_GENERAL, jacobian=G.GAP_JACOBIAN_FD):
    prm = G.gap_step_params()
    prm.dt = float(dt)
    for k in range(4):
        prm.edot_prev[k] = float(edot_prev[k])
        prm.F_ext[k] = float(F_ext[k])
    for k, v in enumerate(np.asarray(mass, dtype=float).ravel()):
        prm.mass[k] = float(v)
    prm.scheme, prm.jacobian = int(scheme), int(jacobian)
    return prm


def equilibrium(solver, e_prev, edot_prev, dt, F_ext, mass, delta, tol=1e-6, max_picard=8,
                scheme=G.GAP_SCHEME_GENERAL, jacobian=G.GAP_JACOBIAN_FD, opts=None, edot_guess=None):
    """Picard iterations of one time point: start from edot_guess (default edot_prev) with
    e = e_prev + dt edot, iterate general_iteration_step until the residual satisfies
    |F| <= tol (|F_ext| + |F_O scale|) or max_picard iterations.  Returns (e, edot, history of
    |F|, PCG iterations per Picard iteration)."""
    opts = opts or solver.options()          # warm_start is managed here
    edot = np.array(edot_guess if edot_guess is not None else edot_prev, dtype=float)
    e = np.asarray(e_prev, float) + dt * edot
    prm = step_params(dt, edot_prev, F_ext, mass, scheme, jacobian)
    hist, its = [], []
    opts.warm_start = 0
    for _ in range(max_picard):
        e_new, ed_new, F, J, info = G.general_iteration_step(solver.handle, opts, prm, delta, solver.p.data_ptr(),
                                                              e, edot, _stream(solver))
        its.append(info.iterations)
        nF = float(np.linalg.norm(F[:2])) + float(np.linalg.norm(F[2:])) / solver.geom.length
        hist.append(nF)
        e, edot = np.array(e_new), np.array(ed_new)
        opts.warm_start = 1 if jacobian == G.GAP_JACOBIAN_FD else 0
        scale = float(np.linalg.norm(np.asarray(F_ext)[:2])) + 1.0
        if nF <= tol * scale:
            break
    return e, edot, hist, its


def simulate(solver, kin, n_steps, dt, delta, e0, edot0, tol=1e-6, max_picard=8, scheme=G.GAP_SCHEME_GENERAL,
             jacobian=G.GAP_JACOBIAN_FD, U=None):
    """Time points t_1 .. t_n: operating point from the kinematics, synthetic loads, Picard
    equilibrium.  Returns a list of dicts (t, phi, V, p_in, e, edot, picard, pcg)."""
    U = solver.geom.U if U is None else U
    M = kin.mass_matrix(solver.geom.length)
    e, edot = np.array(e0, float), np.array(edot0, float)
    out = []
    for s in range(1, n_steps + 1):
        t = s * dt
        phi = kin.phi(t)
        V, p_in = kin.V(phi), kin.p_in(phi)
        solver.set_operating_point(U, V, p_in, kin.p_out)
        F_ext = kin.external_load(phi, solver.geom.R, solver.geom.length)
        e, edot, hist, its = equilibrium(solver, e, edot, dt, F_ext, M, delta, tol, max_picard, scheme, jacobian,
                                         edot_guess=edot)
        out.append({"t": t, "phi": phi, "V": V, "p_in": p_in, "e": e.tolist(), "edot": edot.tolist(),
                    "picard": len(hist), "residual": hist[-1], "pcg_iterations": its})
    return out


def _stream(solver):
    import torch
    return torch.cuda.current_stream(solver.device).cuda_stream
