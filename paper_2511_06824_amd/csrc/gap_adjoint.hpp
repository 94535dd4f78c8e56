// Adjoint (reverse-mode) Jacobian of the force/moment integrals of condition 0 with respect
// to the eccentricities e and their rates edot (the double Jacobian of Eq 2.13-2.14 without
// finite differences).
//
// F_i = f_i(p, e) with A(e) p = S(e, edot):
//   dF_i/dx_k = df_i/dx_k |_p + lambda_i^T (dS/dx_k - dA/dx_k p),   A lambda_i = g_i = df_i/dp,
// A is symmetric, so the 4 adjoint solves use the operator of condition 0 itself.
// dA/dx_k p is assembled face by face: a face of conductance k_f between cells a and b
// contributes dk_f (p_a - p_b)(lambda_a - lambda_b); a Dirichlet face contributes
// dk_b (p_bnd - p_a) lambda_a together with its source term.  Rates enter only the
// squeeze source, dS/d(edot_k) = -(dh/de_k) dx dz.
#pragma once

#include "gap_kernels.hpp"

// First and second derivatives of the film thickness with respect to the axis offset
// (e_x, e_y) at angle (cs, sn): h = d - R, d = |R_c (cs, sn) - (e_x, e_y)|.
struct FilmDeriv {
    double h;                 // film including texture
    double hx, hy;            // dh/de_x, dh/de_y
    double hxx, hxy, hyy;     // second derivatives
    double t;                 // z / L: de_x/de1 = 1 - t, de_x/de3 = t (likewise e_y)
};

__device__ __forceinline__ FilmDeriv film_deriv(const GeomDev& g, const double* e, double cs, double sn, double z,
                                                double tex)
{
    FilmDeriv f;
    f.t = z / g.L;
    const double ex = e[0] + (e[2] - e[0]) * f.t;
    const double ey = e[1] + (e[3] - e[1]) * f.t;
    const double a = g.Rc * cs - ex, b = g.Rc * sn - ey;
    const double d = sqrt(a * a + b * b);
    const double q = g.c2R - 2.0 * g.Rc * (ex * cs + ey * sn) + ex * ex + ey * ey;
    f.h = q / (sqrt(g.R * g.R + q) + g.R) + tex;
    f.hx = -a / d;
    f.hy = -b / d;
    const double d3 = d * d * d;
    f.hxx = b * b / d3;
    f.hyy = a * a / d3;
    f.hxy = -a * b / d3;
    return f;
}

// dh/de_k, k = 0..3 (e1..e4)
__device__ __forceinline__ void dh_de(const FilmDeriv& f, double (&out)[4])
{
    out[0] = f.hx * (1.0 - f.t);
    out[1] = f.hy * (1.0 - f.t);
    out[2] = f.hx * f.t;
    out[3] = f.hy * f.t;
}

__device__ __forceinline__ double mask_of(double p, int cav, double pc) { return (cav && !(p > pc)) ? 0.0 : 1.0; }

// g_i = dF_i/dp per cell (transpose of the force stencil of k_forces), i = Fx, Fy, Mx, My.
// With weights w (4 values, nw = 1) the single right-hand side sum_i w_i g_i is written.
// CLAMP mode multiplies by the derivative of max(p, p_cav): 1 where p > p_cav.
__global__ __launch_bounds__(GAP_BLOCK) void k_adjoint_rhs(GeomDev g, CondDev cd, TablesDev tb, const double* __restrict__ p0, int cav,
                              double p_cav, int weighted, double w0, double w1, double w2, double w3,
                              double* __restrict__ out)
{
    const int nt = g.nt, nz = g.nz;
    const int n = nt * nz;
    const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (gidx >= n) return;
    const int j = gidx / nt, i = gidx - j * nt;
    const int iw = i ? i - 1 : nt - 1;
    const int ie = (i + 1 < nt) ? i + 1 : 0;
    const double* e = cd.e[0];
    const double zj = (j + 0.5) * g.dz;
    const double zr = zj - 0.5 * g.L;
    const double dA = g.dx * g.dz;
    const double cw = tb.cos_c[iw], sw = tb.sin_c[iw], ce = tb.cos_c[ie], se = tb.sin_c[ie];
    const double cs = tb.cos_c[i], sn = tb.sin_c[i];
    const double hw = film_h(g, e, cw, sw, zj, tb.tex_c[j * nt + iw]);
    const double he = film_h(g, e, ce, se, zj, tb.tex_c[j * nt + ie]);
    // ring part of the Poiseuille shear: T_f = (f_w h_w - f_e h_e) / (4 dx)
    const double Ts = (sw * hw - se * he) / (4.0 * g.dx);
    const double Tc = (cw * hw - ce * he) / (4.0 * g.dx);
    // axial part: cells below / above that use p at this cell in their dp/dz
    double zb = 0.0;   // sum over those cells of h_c * d(dp/dz)_c / dp_here (same column)
    if (j >= 1) {
        const double hb = film_h(g, e, cs, sn, (j - 0.5) * g.dz, tb.tex_c[(j - 1) * nt + i]);
        zb += hb * ((j - 1 == 0) ? 1.0 / (1.5 * g.dz) : 1.0 / (2.0 * g.dz));
    }
    if (j + 1 <= nz - 1) {
        const double ha = film_h(g, e, cs, sn, (j + 1.5) * g.dz, tb.tex_c[(j + 1) * nt + i]);
        zb -= ha * ((j + 1 == nz - 1) ? 1.0 / (1.5 * g.dz) : 1.0 / (2.0 * g.dz));
    }
    // sum_c f_c dtau_z,c / dp_here = -(f / 2) zb
    const double m = mask_of(p0 ? p0[gidx] : 0.0, cav, p_cav) * dA;
    const double gx = m * (-cs + Ts);
    const double gy = m * (-sn - Tc);
    const double gmx = m * (zr * sn + zr * Tc + g.R * (-0.5 * sn * zb));
    const double gmy = m * (-zr * cs + zr * Ts - g.R * (-0.5 * cs * zb));
    if (weighted) {
        out[gidx] = w0 * gx + w1 * gy + w2 * gmx + w3 * gmy;
    } else {
        out[gidx] = gx;
        out[n + gidx] = gy;
        out[2 * n + gidx] = gmx;
        out[3 * n + gidx] = gmy;
    }
}

// Sensitivity pass.  Per chunk, partial sums of J[i][k] (n_out = 4 rows, or 1 weighted row)
// for k = 0..7 (e1..e4, edot1..edot4).  lam: n_out adjoint fields, condition-major.
template <int NOUT>
__global__ __launch_bounds__(GAP_BLOCK) void k_adjoint_sens(GeomDev g, CondDev cd, ChunkMap cm, TablesDev tb, const double* __restrict__ p0,
                               const double* __restrict__ lam, int cav, double p_cav, double w0, double w1, double w2,
                               double w3, double* __restrict__ partial)
{
    const int nt = g.nt, nz = g.nz;
    const int n = nt * nz;
    int c, j0, j1;
    chunk_rows(cm, nz, blockIdx.x, c, j0, j1);
    const double* e = cd.e[0];
    const double* ed = cd.ed[0];
    const double dA = g.dx * g.dz;
    const double cxk = g.dz / g.dx / (12.0 * g.mu);   // east-face conductance per h^3
    const double czk = g.dx / g.dz / (12.0 * g.mu);   // axial-face conductance per h^3
    const double wv[4] = {w0, w1, w2, w3};
    double acc[NOUT][8];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[o][k] = 0.0;

    for (int j = j0; j < j1; ++j) {
        const double zj = (j + 0.5) * g.dz;
        const double zr = zj - 0.5 * g.L;
        for (int i = threadIdx.x; i < nt; i += blockDim.x) {
            const int gi = j * nt + i;
            const int iw = i ? i - 1 : nt - 1;
            const int ie = (i + 1 < nt) ? i + 1 : 0;
            const double cs = tb.cos_c[i], sn = tb.sin_c[i];
            double lc[NOUT], le[NOUT], ln[NOUT];
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                lc[o] = lam[(size_t)o * n + gi];
                le[o] = lam[(size_t)o * n + j * nt + ie];
                ln[o] = (j + 1 < nz) ? lam[(size_t)o * n + gi + nt] : 0.0;
            }
            const double pc = p0[gi];
            const double pe = p0[j * nt + ie];
            // ---- explicit dependence of the integrals on e through h (shear terms)
            const FilmDeriv fc = film_deriv(g, e, cs, sn, zj, tb.tex_c[gi]);
            double dhc[4];
            dh_de(fc, dhc);
            {
                const double dpdx = (peff(pe, cav, p_cav) - peff(p0[j * nt + iw], cav, p_cav)) / (2.0 * g.dx);
                double dpdz;
                if (j == 0) dpdz = (peff(p0[gi + nt], cav, p_cav) - g.p_in) / (1.5 * g.dz);
                else if (j == nz - 1) dpdz = (g.p_out - peff(p0[gi - nt], cav, p_cav)) / (1.5 * g.dz);
                else dpdz = (peff(p0[gi + nt], cav, p_cav) - peff(p0[gi - nt], cav, p_cav)) / (2.0 * g.dz);
                const double h2 = fc.h * fc.h;
                const double at = -0.5 * dpdx - g.mu * g.U / h2;   // d tau_theta / dh
                const double az = -0.5 * dpdz - g.mu * g.V / h2;   // d tau_z / dh
                const double ef[4] = {-sn * at, cs * at, -zr * cs * at + g.R * sn * az, -zr * sn * at - g.R * cs * az};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (NOUT == 4) {
#pragma unroll
                        for (int o = 0; o < NOUT; ++o) acc[o][k] += ef[o] * dhc[k] * dA;
                    } else {
                        acc[0][k] += (wv[0] * ef[0] + wv[1] * ef[1] + wv[2] * ef[2] + wv[3] * ef[3]) * dhc[k] * dA;
                    }
                }
            }
            // ---- source: wedge terms through the face films, squeeze term through dh/dt
            const FilmDeriv fe = film_deriv(g, e, tb.cos_e[i], tb.sin_e[i], zj, tb.tex_e[gi]);
            const FilmDeriv fw = film_deriv(g, e, tb.cos_e[iw], tb.sin_e[iw], zj, tb.tex_e[j * nt + iw]);
            const FilmDeriv fs = film_deriv(g, e, cs, sn, j * g.dz, tb.tex_f[gi]);
            const FilmDeriv fn = film_deriv(g, e, cs, sn, (j + 1) * g.dz, tb.tex_f[gi + nt]);
            double dhe[4], dhw[4], dhs[4], dhn[4];
            dh_de(fe, dhe);
            dh_de(fw, dhw);
            dh_de(fs, dhs);
            dh_de(fn, dhn);
            // d(dh/dt)/de_k: dh/dt = hx ex' + hy ey', ex' = ed1 (1-t) + ed3 t, ey' likewise
            const double exd = ed[0] + (ed[2] - ed[0]) * fc.t, eyd = ed[1] + (ed[3] - ed[1]) * fc.t;
            const double dhdot_x = fc.hxx * exd + fc.hxy * eyd;
            const double dhdot_y = fc.hxy * exd + fc.hyy * eyd;
            const double dhdot[4] = {dhdot_x * (1.0 - fc.t), dhdot_y * (1.0 - fc.t), dhdot_x * fc.t,
                                     dhdot_y * fc.t};
            double dS[8];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                dS[k] = -(0.5 * g.U) * (dhe[k] - dhw[k]) * g.dz - (0.5 * g.V) * (dhn[k] - dhs[k]) * g.dx -
                        dhdot[k] * dA;
                dS[4 + k] = -dhc[k] * dA;
            }
            // ---- operator: east face (to ie) and north face (to the row above or the boundary)
            double dAe[4], dAn[4];
            const double ke3 = 3.0 * fe.h * fe.h * cxk;
            const double kn3 = 3.0 * fn.h * fn.h * czk * (j == nz - 1 ? 2.0 : 1.0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                dAe[k] = ke3 * dhe[k];
                dAn[k] = kn3 * dhn[k];
            }
            const double dpe = pc - pe;
            const double dpn = (j + 1 < nz) ? pc - p0[gi + nt] : pc - g.p_out;
            // south Dirichlet face of the first row
            double dAs[4] = {0.0, 0.0, 0.0, 0.0};
            if (j == 0) {
                const double ks3 = 2.0 * 3.0 * fs.h * fs.h * czk;
#pragma unroll
                for (int k = 0; k < 4; ++k) dAs[k] = ks3 * dhs[k];
            }
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                const double dle = lc[o] - le[o];
                const double dln = (j + 1 < nz) ? lc[o] - ln[o] : lc[o];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    double v = lc[o] * dS[k] - dAe[k] * dpe * dle - dAn[k] * dpn * dln;
                    if (j == 0) v += dAs[k] * (g.p_in - pc) * lc[o];
                    acc[o][k] += v;
                    acc[o][4 + k] += lc[o] * dS[4 + k];
                }
            }
        }
    }
    // fixed-order block reductions, 8 values at a time
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        block_sum<8>(acc[o]);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 8; ++k) partial[(size_t)(o * 8 + k) * cm.total + blockIdx.x] = acc[o][k];
    }
}

// J[q] = sum over chunks of partial q, q = 0 .. nq-1 (fixed order).
__global__ __launch_bounds__(GAP_BLOCK) void k_adjoint_finalize(ChunkMap cm, int nq, const double* __restrict__ part, double* __restrict__ J)
{
    for (int q = 0; q < nq; ++q) {
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < cm.total; b += blockDim.x) v[0] += part[(size_t)q * cm.total + b];
        block_sum<1>(v);
        if (threadIdx.x == 0) J[q] = v[0];
    }
}
