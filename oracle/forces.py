"""Oracle: force and moment of the oil film on the piston (paper Sec 2.4-III, Eq 2.11).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper integrates "pressure and viscous shear stress" per surface element but gives no
formulas and no cavitation rule.  Readings taken:

* Cavitation: mode "none" uses p as solved; mode "clamp" uses max(p, p_cav) everywhere
  below (gradients included).
* Wall shear on the (stationary) piston surface for a film whose other wall slides at
  (U, V):  tau_theta = -(h/2) dp/dx + mu U / h,   tau_z = -(h/2) dp/dz + mu V / h,
  with h at the cell centre.  dp/dx: central difference, periodic; dp/dz: central
  difference inside, and on the end rows the Dirichlet value at the boundary face,
  (p_1 - p_in)/(1.5 dz) and (p_out - p_{n-2})/(1.5 dz).
* Midpoint rule, dA = dx dz, moments about the axis point z_ref = L/2.  With the outward
  normal (cos, sin, 0) and tangent (-sin, cos, 0) the surface traction is
  f = (-p cos - tau_theta sin, -p sin + tau_theta cos, tau_z), and
  (F1, F2, F3, F4) = (Fx, Fy, Mx, My) = (sum f_x dA, sum f_y dA,
  sum [(z - z_ref)(p sin - tau_theta cos) + tau_z R sin] dA,
  sum [-(z - z_ref)(p cos + tau_theta sin) - tau_z R cos] dA).
* Split (the paper reports the forces of normal pressure and of viscous shear separately,
  Sec 4.3): the pressure part keeps the p terms, the shear part the tau terms; the shear
  part also has the axial force Fz = sum tau_z dA and the torque Mz = sum R tau_theta dA
  (the pressure has neither on a cylinder).
* Rebuilt field (GMAF step II): the cell-centre pressure with the two Dirichlet rows added,
  p_in at z = 0 and p_out at z = L, (n_axial + 2) x n_theta, after the cavitation rule.
"""

import numpy as np

from .film import Gap, cell_centers, film, no_texture


def effective_pressure(p, mode="none", p_cav=0.0):
    if mode == "none":
        return p
    if mode == "clamp":
        return np.maximum(p, p_cav)
    raise ValueError("cavitation mode must be 'none' or 'clamp'")


def force_moment(gap: Gap, p, h):
    """(Fx, Fy, Mx, My) from the cell-centre pressure p and film h, both (n_axial, n_theta)."""
    nt, nz = gap.n_theta, gap.n_axial
    p = np.asarray(p).reshape(nz, nt)
    h = np.asarray(h).reshape(nz, nt)
    th, z, dth, dz = cell_centers(gap)
    dx = gap.R * dth
    dA = dx * dz
    TH, Z = np.meshgrid(th, z)
    dpdx = (np.roll(p, -1, axis=1) - np.roll(p, 1, axis=1)) / (2.0 * dx)
    dpdz = np.zeros_like(p)
    if nz > 2:
        dpdz[1:-1, :] = (p[2:, :] - p[:-2, :]) / (2.0 * dz)
    dpdz[0, :] = (p[1, :] - gap.p_in) / (1.5 * dz)
    dpdz[-1, :] = (gap.p_out - p[-2, :]) / (1.5 * dz)
    tau_t = -0.5 * h * dpdx + gap.mu * gap.U / h
    tau_z = -0.5 * h * dpdz + gap.mu * gap.V / h
    c, s = np.cos(TH), np.sin(TH)
    zr = Z - 0.5 * gap.L
    Fx = np.sum(-p * c - tau_t * s) * dA
    Fy = np.sum(-p * s + tau_t * c) * dA
    Mx = np.sum(zr * (p * s - tau_t * c) + tau_z * gap.R * s) * dA
    My = np.sum(-zr * (p * c + tau_t * s) - tau_z * gap.R * c) * dA
    return np.array([Fx, Fy, Mx, My])


def forces_for_condition(gap: Gap, e, p, texture=no_texture, cavitation="none", p_cav=0.0):
    """Forces of one solved condition: film at the cell centres, cavitation rule, integrals."""
    th, z, _, _ = cell_centers(gap)
    TH, Z = np.meshgrid(th, z)
    h = film(gap, e, TH, Z, texture)
    return force_moment(gap, effective_pressure(np.asarray(p).reshape(gap.n_axial, gap.n_theta),
                                                cavitation, p_cav), h)


def _gradients(gap: Gap, p):
    nt, nz = gap.n_theta, gap.n_axial
    _, _, dth, dz = cell_centers(gap)
    dx = gap.R * dth
    dpdx = (np.roll(p, -1, axis=1) - np.roll(p, 1, axis=1)) / (2.0 * dx)
    dpdz = np.zeros_like(p)
    if nz > 2:
        dpdz[1:-1, :] = (p[2:, :] - p[:-2, :]) / (2.0 * dz)
    dpdz[0, :] = (p[1, :] - gap.p_in) / (1.5 * dz)
    dpdz[-1, :] = (gap.p_out - p[-2, :]) / (1.5 * dz)
    return dpdx, dpdz


def force_moment_split(gap: Gap, p, h):
    """(Fx, Fy, Mx, My) of the pressure, then (Fx, Fy, Mx, My, Fz, Mz) of the viscous shear:
    10 values, from the cell-centre pressure p and film h, both (n_axial, n_theta)."""
    nt, nz = gap.n_theta, gap.n_axial
    p = np.asarray(p).reshape(nz, nt)
    h = np.asarray(h).reshape(nz, nt)
    th, z, dth, dz = cell_centers(gap)
    dA = gap.R * dth * dz
    TH, Z = np.meshgrid(th, z)
    dpdx, dpdz = _gradients(gap, p)
    tau_t = -0.5 * h * dpdx + gap.mu * gap.U / h
    tau_z = -0.5 * h * dpdz + gap.mu * gap.V / h
    c, s = np.cos(TH), np.sin(TH)
    zr = Z - 0.5 * gap.L
    pressure = [np.sum(-p * c), np.sum(-p * s), np.sum(zr * p * s), np.sum(-zr * p * c)]
    shear = [np.sum(-tau_t * s), np.sum(tau_t * c), np.sum(-zr * tau_t * c + tau_z * gap.R * s),
             np.sum(-zr * tau_t * s - tau_z * gap.R * c), np.sum(tau_z), np.sum(gap.R * tau_t)]
    return np.array(pressure + shear) * dA


def forces_split_for_condition(gap: Gap, e, p, texture=no_texture, cavitation="none", p_cav=0.0):
    th, z, _, _ = cell_centers(gap)
    TH, Z = np.meshgrid(th, z)
    h = film(gap, e, TH, Z, texture)
    return force_moment_split(gap, effective_pressure(np.asarray(p).reshape(gap.n_axial, gap.n_theta),
                                                      cavitation, p_cav), h)


def rebuild_field(gap: Gap, p, cavitation="none", p_cav=0.0):
    """(n_axial + 2) x n_theta: p_in row, the cell-centre pressure (cavitation rule applied), p_out row."""
    pe = effective_pressure(np.asarray(p).reshape(gap.n_axial, gap.n_theta), cavitation, p_cav)
    out = np.empty((gap.n_axial + 2, gap.n_theta))
    out[0, :] = gap.p_in
    out[1:-1, :] = pe
    out[-1, :] = gap.p_out
    return out
