"""Oracle: grid, film thickness and its rate (paper Sec 2.1, Eq 2.3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings taken where the paper is silent:

* Grid: cell-centred, theta_i = (i+1/2) dtheta with dtheta = 2 pi / n_theta
  (periodic, circumferential, fastest index); z_j = (j+1/2) dz with
  dz = L / n_axial.  The paper's axial coordinate y of Eq 2.3 is z here.
* Eq 2.3 with R_c = R + c: the eccentricity of the piston axis varies linearly
  along the gap, e_x(z) = e1 + (e3 - e1) z / L, e_y(z) = e2 + (e4 - e2) z / L.
  ``film_naive`` evaluates Eq 2.3 literally; ``film`` uses the algebraically
  identical form h = q / (sqrt(R^2 + q) + R) with
  q = R_c^2 - R^2 - 2 R_c (e_x cos + e_y sin) + e_x^2 + e_y^2, which avoids
  the cancellation of two ~1e-2 m quantities.
* Eq 2.3 writes h(e, edot) but contains no rate: the rates enter only through
  the squeeze term dh/dt = sum_j (dh/de_j) edot_j (``film_rate``).
* Texture: an additive depth h_text(theta, z) >= 0 on the piston (Eq 2.3's
  h_Text).  The synthetic dimples are spherical caps (``dimple_texture``).
"""

from typing import Callable, NamedTuple

import numpy as np


class Gap(NamedTuple):
    """Geometry, fluid and boundary data of one piston/bore gap (SI units)."""
    R: float          # piston radius R_k
    c: float          # radial clearance, R_c = R + c
    L: float          # gap length L_F
    mu: float         # dynamic viscosity
    U: float          # circumferential sliding speed of the bore relative to the piston
    V: float          # axial sliding speed
    p_in: float       # Dirichlet pressure at z = 0
    p_out: float      # Dirichlet pressure at z = L
    n_theta: int
    n_axial: int


def cell_centers(gap: Gap):
    """Cell-centre coordinates: theta (n_theta,), z (n_axial,) and dtheta, dz."""
    dth = 2.0 * np.pi / gap.n_theta
    dz = gap.L / gap.n_axial
    th = (np.arange(gap.n_theta) + 0.5) * dth
    z = (np.arange(gap.n_axial) + 0.5) * dz
    return th, z, dth, dz


def axis_offset(e, z, L):
    """Piston-axis offset (e_x, e_y) at axial position z: linear between the two ends."""
    e1, e2, e3, e4 = e[0], e[1], e[2], e[3]
    ex = e1 + (e3 - e1) * z / L
    ey = e2 + (e4 - e2) * z / L
    return ex, ey


def no_texture(theta, z):
    return np.zeros(np.broadcast(theta, z).shape)


def film_naive(gap: Gap, e, theta, z):
    """Eq 2.3 evaluated literally (no texture)."""
    Rc = gap.R + gap.c
    ex, ey = axis_offset(e, z, gap.L)
    return np.sqrt((Rc * np.cos(theta) - ex) ** 2 + (Rc * np.sin(theta) - ey) ** 2) - gap.R


def film(gap: Gap, e, theta, z, texture: Callable = no_texture):
    """Eq 2.3 in cancellation-free form, plus the texture depth.

    Complex eccentricities are allowed (complex-step differentiation)."""
    R = gap.R
    Rc = R + gap.c
    ex, ey = axis_offset(e, z, gap.L)
    q = (Rc * Rc - R * R) - 2.0 * Rc * (ex * np.cos(theta) + ey * np.sin(theta)) + ex * ex + ey * ey
    d = np.sqrt(R * R + q)
    return q / (d + R) + texture(theta, z)


def film_rate(gap: Gap, e, edot, theta, z):
    """Squeeze term dh/dt = sum_j (dh/de_j) edot_j.

    d = |bore point - axis point|, h = d - R, so dh/d(e_x) = -(R_c cos - e_x)/d and
    likewise for e_y; e_x, e_y and their rates are linear in z.  The texture is fixed
    to the piston and adds nothing."""
    R = gap.R
    Rc = R + gap.c
    ex, ey = axis_offset(e, z, gap.L)
    exd, eyd = axis_offset(edot, z, gap.L)
    ax = Rc * np.cos(theta) - ex
    ay = Rc * np.sin(theta) - ey
    d = np.sqrt(ax * ax + ay * ay)
    return -(ax * exd + ay * eyd) / d


def dimple_texture(R, theta_c, z_c, radius, depth):
    """Spherical-cap dimples on the piston surface, combined by max where they overlap.

    A cap of footprint radius a and depth d has sphere radius rho = (a^2 + d^2)/(2 d);
    its depth at in-surface distance r < a is sqrt(rho^2 - r^2) - (rho - d), zero
    outside.  The in-surface distance uses the wrapped arc R * dtheta and dz."""
    theta_c = np.asarray(theta_c, dtype=float).ravel()
    z_c = np.asarray(z_c, dtype=float).ravel()
    radius = np.broadcast_to(np.asarray(radius, dtype=float), theta_c.shape).ravel()
    depth = np.broadcast_to(np.asarray(depth, dtype=float), theta_c.shape).ravel()

    def tex(theta, z):
        theta, z = np.broadcast_arrays(np.asarray(theta, dtype=float), np.asarray(z, dtype=float))
        shape = theta.shape
        theta, z = theta.ravel(), z.ravel()
        out = np.zeros(theta.shape)
        for tc, zc, a, d in zip(theta_c, z_c, radius, depth):
            near = np.nonzero(np.abs(z - zc) < a)[0]      # only points in the cap's axial band
            dth = np.mod(theta[near] - tc + np.pi, 2.0 * np.pi) - np.pi
            r2 = (R * dth) ** 2 + (z[near] - zc) ** 2
            rho = (a * a + d * d) / (2.0 * d)
            inside = r2 < a * a
            cap = np.where(inside, np.sqrt(np.maximum(rho * rho - r2, 0.0)) - (rho - d), 0.0)
            out[near] = np.maximum(out[near], cap)
        return out.reshape(shape)

    return tex
