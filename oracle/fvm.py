"""Oracle: finite-volume assembly of the Reynolds system (paper Eq 2.1, 2.4-2.7, 2.17-2.19, 3.7).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper gives the discrete row form A_P p_P + A_E p_E + A_W p_W + A_S p_S + A_N p_N = S_P
(Eq 2.4), Dirichlet ends (south = inlet at z = 0, north = outlet at z = L) folded in
"via linear transform", and a periodic circumferential axis (the A_EB / A_WB
diagonals of Eq 2.7).  It does not state the PDE.  Reading taken: the isoviscous,
incompressible Reynolds equation in the piston frame,

    d/dx(k dp/dx) + d/dz(k dp/dz) = (U/2) dh/dx + (V/2) dh/dz + dh/dt,   k = h^3 / (12 mu),

with x = R theta.  Integrating over cell (i, j) of size dx * dz gives

    sum_faces kf (p_P - p_nb) = S_P,
    kx(i, j)  = k(theta_i + dtheta/2, z_j) dz/dx        (east face; wraps at i = n_theta-1)
    kz(i, f)  = k(theta_i, f dz) dx/dz,  f = 0..n_axial (f = 0 and f = n_axial are the
                Dirichlet faces, at half a cell from the centre: doubled)
    S_P = -(U/2)(h_e - h_w) dz - (V/2)(h_n - h_s) dx - (dh/dt)_P dx dz
          + [j = 0] kz(i, 0) p_in + [j = n_axial-1] kz(i, n_axial) p_out.

Matrix entries: A_PP = kx(i) + kx(i-1) + kz(f=j) + kz(f=j+1); off-diagonals are the
negated face conductances.  The matrix is symmetric, an M-matrix, and SPD whenever h > 0.
Unknown ordering (Eq 3.8 reading): g = i + j * n_theta (+ k * n for condition k).
"""

import numpy as np
import scipy.sparse as sp

from .film import Gap, cell_centers, film, film_rate, no_texture


def face_conductances(gap: Gap, e, texture=no_texture):
    """kx (n_axial, n_theta) on east faces and kz (n_axial+1, n_theta) on axial faces."""
    th, z, dth, dz = cell_centers(gap)
    dx = gap.R * dth
    TH, Z = np.meshgrid(th, z)
    h_east = film(gap, e, TH + 0.5 * dth, Z, texture)
    kx = h_east ** 3 / (12.0 * gap.mu) * (dz / dx)
    zf = np.arange(gap.n_axial + 1) * dz
    THf, ZF = np.meshgrid(th, zf)
    h_face = film(gap, e, THf, ZF, texture)
    kz = h_face ** 3 / (12.0 * gap.mu) * (dx / dz)
    kz[0, :] *= 2.0
    kz[-1, :] *= 2.0
    return kx, kz


def source(gap: Gap, e, edot, texture=no_texture):
    """Right-hand side S (n_axial, n_theta): wedge, axial wedge, squeeze, Dirichlet terms."""
    th, z, dth, dz = cell_centers(gap)
    dx = gap.R * dth
    TH, Z = np.meshgrid(th, z)
    h_e = film(gap, e, TH + 0.5 * dth, Z, texture)
    h_w = film(gap, e, TH - 0.5 * dth, Z, texture)
    h_n = film(gap, e, TH, Z + 0.5 * dz, texture)
    h_s = film(gap, e, TH, Z - 0.5 * dz, texture)
    hdot = film_rate(gap, e, edot, TH, Z)
    S = -(0.5 * gap.U) * (h_e - h_w) * dz - (0.5 * gap.V) * (h_n - h_s) * dx - hdot * dx * dz
    _, kz = face_conductances(gap, e, texture)
    dirichlet = np.zeros(S.shape, dtype=np.result_type(S, kz))
    dirichlet[0, :] += kz[0, :] * gap.p_in
    dirichlet[-1, :] += kz[-1, :] * gap.p_out
    return S + dirichlet


def cell_values(gap: Gap, e, edot, i, j, texture=no_texture):
    """Entries of the assembled system at the cells (i, j) (index arrays of one shape):
    kx(i, j), kz on the south face j and on the north face j + 1 of the cell, and S(i, j).
    The same expressions as ``face_conductances`` and ``source``, evaluated cell by cell, so
    that a grid too large to assemble here can be checked at sampled cells."""
    th, z, dth, dz = cell_centers(gap)
    dx = gap.R * dth
    i = np.asarray(i)
    j = np.asarray(j)
    TH, Z = th[i], z[j]
    zf = np.arange(gap.n_axial + 1) * dz
    kx = film(gap, e, TH + 0.5 * dth, Z, texture) ** 3 / (12.0 * gap.mu) * (dz / dx)
    kz_s = film(gap, e, TH, zf[j], texture) ** 3 / (12.0 * gap.mu) * (dx / dz)
    kz_n = film(gap, e, TH, zf[j + 1], texture) ** 3 / (12.0 * gap.mu) * (dx / dz)
    kz_s = np.where(j == 0, 2.0 * kz_s, kz_s)
    kz_n = np.where(j == gap.n_axial - 1, 2.0 * kz_n, kz_n)
    h_e = film(gap, e, TH + 0.5 * dth, Z, texture)
    h_w = film(gap, e, TH - 0.5 * dth, Z, texture)
    h_n = film(gap, e, TH, Z + 0.5 * dz, texture)
    h_s = film(gap, e, TH, Z - 0.5 * dz, texture)
    hdot = film_rate(gap, e, edot, TH, Z)
    S = -(0.5 * gap.U) * (h_e - h_w) * dz - (0.5 * gap.V) * (h_n - h_s) * dx - hdot * dx * dz
    S = S + np.where(j == 0, kz_s * gap.p_in, 0.0) + np.where(j == gap.n_axial - 1, kz_n * gap.p_out, 0.0)
    return kx, kz_s, kz_n, S


def stencil_matrix(gap: Gap, kx, kz):
    """Sparse n x n matrix from the face conductances (natural order, theta fastest)."""
    nt, nz = gap.n_theta, gap.n_axial
    n = nt * nz
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(nz, nt)
    east = idx[:, (np.arange(nt) + 1) % nt]
    west = idx[:, (np.arange(nt) - 1) % nt]
    kx_w = kx[:, (np.arange(nt) - 1) % nt]
    diag = kx + kx_w + kz[:-1, :] + kz[1:, :]
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    rows.append(idx.ravel()); cols.append(east.ravel()); vals.append(-kx.ravel())
    rows.append(idx.ravel()); cols.append(west.ravel()); vals.append(-kx_w.ravel())
    if nz > 1:
        rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(-kz[1:-1, :].ravel())
        rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(-kz[1:-1, :].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def assemble(gap: Gap, e, edot, texture=no_texture):
    """One working condition: (A csr n x n, S flat n)."""
    kx, kz = face_conductances(gap, e, texture)
    A = stencil_matrix(gap, kx, kz)
    S = source(gap, e, edot, texture).ravel()
    return A, S


def conditions(e, edot, delta):
    """The 9 working conditions of Eq 2.17-2.19: k=0 base; k=1..4 e_k + delta_k;
    k=5..8 edot_{k-4} + delta_k.  Returns a list of (e, edot) pairs."""
    e = np.asarray(e, dtype=float)
    edot = np.asarray(edot, dtype=float)
    out = [(e.copy(), edot.copy())]
    for j in range(4):
        ej = e.copy()
        ej[j] += delta[j]
        out.append((ej, edot.copy()))
    for j in range(4):
        edj = edot.copy()
        edj[j] += delta[4 + j]
        out.append((e.copy(), edj))
    return out


def assemble_joint(gap: Gap, e, edot, delta, texture=no_texture):
    """Joint block-diagonal system A_G p_G = S_G of Eq 3.7 over the 9 conditions."""
    blocks, rhs = [], []
    for ek, edk in conditions(e, edot, delta):
        A, S = assemble(gap, ek, edk, texture)
        blocks.append(A)
        rhs.append(S)
    return sp.block_diag(blocks, format="csr"), np.concatenate(rhs)
