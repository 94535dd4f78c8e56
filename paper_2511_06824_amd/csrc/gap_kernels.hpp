// HIP kernels of the joint piston-gap solve (gfx950, FP64, no MFMA: bandwidth-bound sparse work).
//
// Work decomposition shared by the solve kernels: the rows of every condition are cut into
// `per_cond` chunks of `rows` consecutive rows; block b works on chunk b (condition
// b / per_cond).  Every chunk writes one partial sum per reduced quantity to a fixed slot,
// and a one-block finalize kernel adds the slots of each condition in a fixed order, so
// all reductions are deterministic and independent of scheduling.
#pragma once

#include "gap_device.hpp"

struct ChunkMap {
    int per_cond;   // chunks per condition
    int rows;       // rows per chunk (the last chunk of a condition may hold fewer)
    int total;      // per_cond * n_cond
};

__device__ __forceinline__ void chunk_rows(const ChunkMap& cm, int nz, int b, int& c, int& j0, int& j1)
{
    c = b / cm.per_cond;
    j0 = (b - c * cm.per_cond) * cm.rows;
    j1 = min(j0 + cm.rows, nz);
}

// ---------------------------------------------------------------------------------------
// Texture: spherical caps scattered over their footprint boxes, overlaps combined by max.
// Depths are >= 0, so their IEEE bit patterns order like unsigned integers.
// plane 0: cell centres, plane 1: east faces, plane 2: axial faces (nz + 1 rows).
__global__ __launch_bounds__(GAP_BLOCK) void k_texture(GeomDev g, int count, const double* __restrict__ th_c,
                          const double* __restrict__ z_c, const double* __restrict__ rad,
                          const double* __restrict__ dep, double* tex_c, double* tex_e, double* tex_f)
{
    const int k = blockIdx.x;
    const int plane = blockIdx.y;
    if (k >= count) return;
    const double tc = th_c[k], zc = z_c[k], a = rad[k], d = dep[k];
    const double rho = (a * a + d * d) / (2.0 * d);
    const double half_ang = a / g.R;
    const int span_i = (int)ceil(half_ang / g.dth) + 2;
    int ncol = 2 * span_i + 1;
    if (ncol > g.nt) ncol = g.nt;
    const int ic0 = (int)floor(tc / g.dth) - span_i;
    const int nrows = (plane == 2) ? g.nz + 1 : g.nz;
    int jlo = (int)floor((zc - a) / g.dz) - 2;
    int jhi = (int)ceil((zc + a) / g.dz) + 2;
    if (jlo < 0) jlo = 0;
    if (jhi > nrows - 1) jhi = nrows - 1;
    if (jhi < jlo) return;
    double* dst = plane == 0 ? tex_c : (plane == 1 ? tex_e : tex_f);
    const double two_pi = 2.0 * 3.14159265358979323846;
    const long long cells = (long long)ncol * (jhi - jlo + 1);
    for (long long q = threadIdx.x; q < cells; q += blockDim.x) {
        const int jr = jlo + (int)(q / ncol);
        int i = (ic0 + (int)(q % ncol)) % g.nt;
        if (i < 0) i += g.nt;
        const double th = (plane == 1) ? (i + 1.0) * g.dth : (i + 0.5) * g.dth;
        const double z = (plane == 2) ? jr * g.dz : (jr + 0.5) * g.dz;
        double dt = th - tc + 0.5 * two_pi;
        dt = dt - two_pi * floor(dt / two_pi) - 0.5 * two_pi;
        const double ds = g.R * dt, dzz = z - zc;
        const double r2 = ds * ds + dzz * dzz;
        if (r2 < a * a) {
            const double v = sqrt(fmax(rho * rho - r2, 0.0)) - (rho - d);
            if (v > 0.0)
                atomicMax((unsigned long long*)&dst[(size_t)jr * g.nt + i],
                          (unsigned long long)__double_as_longlong(v));
        }
    }
}

// ---------------------------------------------------------------------------------------
// Assembly (step I): one thread per (cell, condition).  Writes the source of every
// condition and, for conditions that own an operator, its face conductances.
// The faces each row owns, as pairs for the strip iteration: pair (r + 1, i) holds the east
// face of cell (r, i) and the axial face above it, (kx(r, i), kz(r + 1, i)), for rows
// r = -1 .. n_axial - 1 (row -1: (0, the inlet face kz(0, i))), per operator.  A row step then
// reads its conductances with one 16-byte load per lane.
__global__ __launch_bounds__(GAP_BLOCK) void k_pair_ops(int nt, int nz, const double* __restrict__ kx,
                                                        const double* __restrict__ kz, double* __restrict__ kxz)
{
    const int op = blockIdx.y;
    const size_t n = (size_t)nt * nz, nf = n + nt;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;     // pair (r + 1, i)
    if (idx >= nf) return;
    const double e = idx >= (size_t)nt ? kx[op * n + idx - nt] : 0.0;
    kxz[op * 2 * nf + 2 * idx] = e;
    kxz[op * 2 * nf + 2 * idx + 1] = kz[op * nf + idx];
}

__global__ __launch_bounds__(GAP_BLOCK) void k_assemble(GeomDev g, CondDev cd, TablesDev tb, double* __restrict__ kx,
                           double* __restrict__ kz, double* __restrict__ S)
{
    const int c = blockIdx.y;
    const int n = g.nt * g.nz;
    const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (gidx >= n) return;
    const int j = gidx / g.nt, i = gidx - j * g.nt;
    const int iw = i ? i - 1 : g.nt - 1;
    const double* e = cd.e[c];
    const double zj = (j + 0.5) * g.dz;
    const double h_e = film_h(g, e, tb.cos_e[i], tb.sin_e[i], zj, tb.tex_e[gidx]);
    const double h_w = film_h(g, e, tb.cos_e[iw], tb.sin_e[iw], zj, tb.tex_e[j * g.nt + iw]);
    const double h_s = film_h(g, e, tb.cos_c[i], tb.sin_c[i], j * g.dz, tb.tex_f[j * g.nt + i]);
    const double h_n = film_h(g, e, tb.cos_c[i], tb.sin_c[i], (j + 1) * g.dz, tb.tex_f[(j + 1) * g.nt + i]);
    const double hdot = film_rate(g, e, cd.ed[c], tb.cos_c[i], tb.sin_c[i], zj);
    const double kfz = g.dx / g.dz / (12.0 * g.mu);
    double s = -(0.5 * g.U) * (h_e - h_w) * g.dz - (0.5 * g.V) * (h_n - h_s) * g.dx - hdot * g.dx * g.dz;
    if (j == 0) s += 2.0 * (h_s * h_s * h_s) * kfz * g.p_in;
    if (j == g.nz - 1) s += 2.0 * (h_n * h_n * h_n) * kfz * g.p_out;
    S[(size_t)c * n + gidx] = s;
    if (c < cd.n_op) {
        const double kfx = g.dz / g.dx / (12.0 * g.mu);
        kx[(size_t)c * n + gidx] = (h_e * h_e * h_e) * kfx;
        double* kzo = kz + (size_t)c * (n + g.nt);
        kzo[gidx] = (j == 0 ? 2.0 : 1.0) * (h_s * h_s * h_s) * kfz;
        if (j == g.nz - 1) kzo[n + i] = 2.0 * (h_n * h_n * h_n) * kfz;
    }
}

// Diagonal A_PP = kx(i) + kx(i-1) + kz(j) + kz(j+1) (Dirichlet faces included).
__device__ __forceinline__ double diag_at(const double* kx, const double* kz, int i, int j, int nt)
{
    const int iw = i ? i - 1 : nt - 1;
    return ((kx[j * nt + i] + kx[j * nt + iw]) + kz[j * nt + i]) + kz[(j + 1) * nt + i];
}

// (A x)(i, j) with x given by a functor of (i, j).
template <class X>
__device__ __forceinline__ double apply_A(const double* kx, const double* kz, int i, int j, int nt,
                                          int nz, X x)
{
    const int iw = i ? i - 1 : nt - 1;
    const int ie = (i + 1 < nt) ? i + 1 : 0;
    const double kE = kx[j * nt + i], kW = kx[j * nt + iw];
    const double kS = kz[j * nt + i], kN = kz[(j + 1) * nt + i];
    double a = (((kE + kW) + kS) + kN) * x(i, j) - kE * x(ie, j) - kW * x(iw, j);
    if (j > 0) a -= kS * x(i, j - 1);
    if (j < nz - 1) a -= kN * x(i, j + 1);
    return a;
}

// Diagonal preconditioners: Jacobi (Eq 2.8) and ASSOR I (Eq 3.2), stored as M^{-1}_ii per
// operator.  ASSOR I: w(2-w) / (D_ii + w^2 sum_k L_ik^2 / D_kk), L the strict lower
// triangle in the natural order (west, south, and the east wrap of the last column).
__global__ __launch_bounds__(GAP_BLOCK) void k_diag_precond(GeomDev g, int kind, double omega, const double* __restrict__ kx_all,
                               const double* __restrict__ kz_all, double* __restrict__ minv, int n_op)
{
    const int o = blockIdx.y;
    const int n = g.nt * g.nz;
    const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (gidx >= n || o >= n_op) return;
    const double* kx = kx_all + (size_t)o * n;
    const double* kz = kz_all + (size_t)o * (n + g.nt);
    const int nt = g.nt, j = gidx / nt, i = gidx - j * nt;
    const double D = diag_at(kx, kz, i, j, nt);
    double val;
    if (kind == 0) {
        val = 1.0 / D;
    } else {
        double s = 0.0;
        if (i > 0) { const double l = kx[j * nt + i - 1]; s += l * l / diag_at(kx, kz, i - 1, j, nt); }
        if (i == nt - 1) { const double l = kx[j * nt + i]; s += l * l / diag_at(kx, kz, 0, j, nt); }
        if (j > 0) { const double l = kz[j * nt + i]; s += l * l / diag_at(kx, kz, i, j - 1, nt); }
        val = omega * (2.0 - omega) / (D + omega * omega * s);
    }
    minv[(size_t)o * n + gidx] = val;
}

// ---------------------------------------------------------------------------------------
// Force and moment integration (step III) with the cavitation rule; partials 0..3 are
// Fx, Fy, Mx, My per chunk before the factor dA.
__device__ __forceinline__ double peff(double p, int cav, double pc) { return (cav && p < pc) ? pc : p; }

// NV = 4: (Fx, Fy, Mx, My) of pressure and shear together.  NV = 10: the pressure part
// (Fx, Fy, Mx, My), then the shear part (Fx, Fy, Mx, My, Fz, Mz) with the axial force and the
// torque of the wall shear.
template <int NV>
__global__ __launch_bounds__(GAP_BLOCK) void k_forces(GeomDev g, CondDev cd, ChunkMap cm, TablesDev tb,
                                                      const double* __restrict__ p_all, int cav, double p_cav,
                                                      double* __restrict__ partial)
{
    int c, j0, j1;
    chunk_rows(cm, g.nz, blockIdx.x, c, j0, j1);
    const int nt = g.nt, nz = g.nz;
    const size_t n = (size_t)nt * nz;
    const double* p = p_all + (size_t)c * n;
    const double* e = cd.e[c];
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double zj = (j + 0.5) * g.dz;
        const double zr = zj - 0.5 * g.L;
        for (int i = threadIdx.x; i < nt; i += blockDim.x) {
            const int gi = j * nt + i;
            const int iw = i ? i - 1 : nt - 1;
            const int ie = (i + 1 < nt) ? i + 1 : 0;
            const double pc = peff(p[gi], cav, p_cav);
            const double dpdx = (peff(p[j * nt + ie], cav, p_cav) - peff(p[j * nt + iw], cav, p_cav)) / (2.0 * g.dx);
            double dpdz;
            if (j == 0) dpdz = (peff(p[gi + nt], cav, p_cav) - g.p_in) / (1.5 * g.dz);
            else if (j == nz - 1) dpdz = (g.p_out - peff(p[gi - nt], cav, p_cav)) / (1.5 * g.dz);
            else dpdz = (peff(p[gi + nt], cav, p_cav) - peff(p[gi - nt], cav, p_cav)) / (2.0 * g.dz);
            const double cs = tb.cos_c[i], sn = tb.sin_c[i];
            const double h = film_h(g, e, cs, sn, zj, tb.tex_c ? tb.tex_c[gi] : 0.0);
            const double tt = -0.5 * h * dpdx + g.mu * g.U / h;
            const double tz = -0.5 * h * dpdz + g.mu * g.V / h;
            if (NV == 4) {
                acc[0] += -pc * cs - tt * sn;
                acc[1] += -pc * sn + tt * cs;
                acc[2] += zr * (pc * sn - tt * cs) + tz * g.R * sn;
                acc[3] += -zr * (pc * cs + tt * sn) - tz * g.R * cs;
            } else {
                acc[0] += -pc * cs;
                acc[1] += -pc * sn;
                acc[2] += zr * pc * sn;
                acc[3] += -zr * pc * cs;
                acc[4 % NV] += -tt * sn;
                acc[5 % NV] += tt * cs;
                acc[6 % NV] += -zr * tt * cs + tz * g.R * sn;
                acc[7 % NV] += -zr * tt * sn - tz * g.R * cs;
                acc[8 % NV] += tz;
                acc[9 % NV] += g.R * tt;
            }
        }
    }
    block_sum<NV>(acc);
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) partial[q * cm.total + blockIdx.x] = acc[q];
}

// cos and sin of the cell-centre angles theta_i = (i + 1/2) dtheta, i < nt, formed on the
// device (the handle-free force integration has no host-built table).
__global__ __launch_bounds__(GAP_BLOCK) void k_trig_centres(int nt, double dth, double* __restrict__ cs,
                                                            double* __restrict__ sn)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const double th = (i + 0.5) * dth;
    cs[i] = cos(th);
    sn[i] = sin(th);
}

__device__ __forceinline__ double cond_sum(const double* part, const ChunkMap& cm, int c)
{
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < cm.per_cond; b += blockDim.x) v[0] += part[c * cm.per_cond + b];
    block_sum<1>(v);
    return v[0];   // valid in thread 0
}

__global__ __launch_bounds__(GAP_BLOCK) void k_forces_finalize(ChunkMap cm, int n_cond, int nv, double dA,
                                                               const double* __restrict__ part, double* __restrict__ F)
{
    for (int c = 0; c < n_cond; ++c)
        for (int q = 0; q < nv; ++q) {
            const double s = cond_sum(part + q * cm.total, cm, c);
            if (threadIdx.x == 0) F[c * nv + q] = s * dA;
        }
}

// ||S - A p||^2 and ||S||^2 per chunk of rows, the true residual of a returned solution.
__global__ __launch_bounds__(GAP_BLOCK) void k_true_residual(GeomDev g, CondDev cd, ChunkMap cm,
                                                             const double* __restrict__ kx_all,
                                                             const double* __restrict__ kz_all,
                                                             const double* __restrict__ S_all,
                                                             const double* __restrict__ p_all, double* __restrict__ partial)
{
    int c, j0, j1;
    chunk_rows(cm, g.nz, blockIdx.x, c, j0, j1);
    const int nt = g.nt, nz = g.nz;
    const size_t n = (size_t)nt * nz;
    const int op = cd.op[c];
    const double* kx = kx_all + (size_t)op * n;
    const double* kz = kz_all + (size_t)op * (n + nt);
    const double* S = S_all + (size_t)c * n;
    const double* p = p_all + (size_t)c * n;
    double acc[2] = {0.0, 0.0};
    for (int j = j0; j < j1; ++j) {
        for (int i = threadIdx.x; i < nt; i += blockDim.x) {
            const size_t gi = (size_t)j * nt + i;
            const int iw = i ? i - 1 : nt - 1;
            const int ie = (i + 1 < nt) ? i + 1 : 0;
            const double kE = kx[gi], kW = kx[(size_t)j * nt + iw];
            const double kS = kz[gi], kN = kz[gi + nt];
            double Ap = (((kE + kW) + kS) + kN) * p[gi] - kE * p[(size_t)j * nt + ie] - kW * p[(size_t)j * nt + iw];
            if (j > 0) Ap -= kS * p[gi - nt];
            if (j < nz - 1) Ap -= kN * p[gi + nt];
            const double r = S[gi] - Ap;
            acc[0] += r * r;
            acc[1] += S[gi] * S[gi];
        }
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = acc[0];
        partial[cm.total + blockIdx.x] = acc[1];
    }
}

// GMAF step II: the full field with its boundary rows, out[c][j][i] for j = 0 .. n_axial + 1
// (row 0: p_in at z = 0, rows 1 .. n_axial: the cell centres after the cavitation rule, last
// row: p_out at z = L).
__global__ __launch_bounds__(GAP_BLOCK) void k_rebuild(GeomDev g, int n_cond, const double* __restrict__ p_all, int cav,
                                                       double p_cav, double* __restrict__ out)
{
    const size_t nt = g.nt, nz = g.nz;
    const size_t per = (nz + 2) * nt;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * (size_t)n_cond) return;
    const size_t c = idx / per, r = idx - c * per;
    const size_t j = r / nt, i = r - j * nt;
    double v;
    if (j == 0) v = g.p_in;
    else if (j == nz + 1) v = g.p_out;
    else v = peff(p_all[c * nz * nt + (j - 1) * nt + i], cav, p_cav);
    out[idx] = v;
}

// Eq 2.13-2.14: J[i][k] = (F_{k+1,i} - F_{0,i}) / delta_k.
struct Delta8 { double d[8]; };
__global__ void k_jacobian_fd(const double* __restrict__ F, Delta8 dl, double* __restrict__ J)
{
    const int t = threadIdx.x;
    if (t >= 32) return;
    const int i = t / 8, k = t % 8;
    J[t] = (F[(k + 1) * 4 + i] - F[i]) / dl.d[k];
}
