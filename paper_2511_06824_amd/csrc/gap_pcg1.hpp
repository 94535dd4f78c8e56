// One-launch PCG iteration for gfx950, FP64: Table 1 with ASSOR II (Eq 3.4-3.6), Jacobi
// (Eq 2.8, 1/D formed from the conductances) or the stored diagonal of ASSOR I (Eq 3.2).
//
// Table 1 needs two grid-wide reductions per iteration: alpha's denominator u^T A u depends
// on the new search direction u = z + beta u_prev over the whole grid, so p and r cannot move
// in the launch that forms u.  With A symmetric the denominator expands into
//     u^T A u = z^T A z + 2 beta z^T A u_prev + beta^2 u_prev^T A u_prev,
// three sums the previous launch can form: it produces z (z^T A z), holds A u_prev from its
// own SpMV (z^T A u_prev) and u_prev itself (u_prev^T A u_prev).  So one launch per
// iteration suffices.  It reduces the partials of the previous launch into beta, alpha and
// the stopping test (Eq 3.9 / 3.10), then forms u = z + beta u_prev, A u,
// r' = r - alpha A u, z' = M^-1 r', and the partials r'.z', r'.r', z'^T A z', z'^T A u,
// u^T A u; p += alpha u is folded into every other launch (below).  The iterates are
// Table 1's up to rounding: the expansion cancels by the ratio z^T A z / u^T A u, a few
// units on the gap systems.
//
// z'^T A z' is summed face by face: k_f (z_i - z_j)^2 over interior faces plus k_f z_i^2 over
// the two Dirichlet end faces, a sum of non-negative terms.  A row owns its east faces (the
// periodic wrap face included) and its north face.  The chunk of rows [j0, j1) therefore
// needs z' on row j1 as well, which takes r' on rows [j0 - 1, j1 + 1] (each ASSOR sweep
// reaches one row) and u on rows [j0 - 2, j1 + 2].
//
// p is not read by the recurrence, so it moves every other iteration: a launch of odd j adds
// alpha_{j-1} u_{j-1} + alpha_j u_j when a row's z_j and u_{j-1} arrive, and a launch of even j
// leaves its term pending.  The launch that stops or freezes a condition right after an even
// iteration settles the pending term over the condition's rows.  The iterates (alpha, beta, r, z, u) are unchanged; p differs only in the
// order of its additions.
//
// Bytes per condition-DOF: reads z, u_prev, r and writes u, r', z' (48 B), plus p read and
// written on odd iterations (56 B on average), plus the face conductances once per operator.
// The two-launch iteration of gap_pcg.hpp moves 72 B and reads the conductances in both
// launches.
//
// Buffers that one launch both reads (with halo rows) and writes alternate by iteration
// parity: u, r, z and the partial sums.  The iteration index and the per-condition r.z that
// the next launch divides by sit in the device record by launch parity `par`: launch j reads
// slot [par] and its record writer fills [par ^ 1].  The host alternates the launch parity,
// starting at 0 after the initial launch; a batch, whose requests join at different launches,
// gives each request an offset (par = launch parity xor par_off).  Launches after a solve has
// stopped return at once.
//
// Row pipeline, one row step s per loop trip, two barriers per step:
//   P1  u and the east-face conductances of row s to LDS; loads of step s + 1 issued
//   P2  A u, r' and y = D^-1 r' of row s; stores of u and r' on owned rows; the east faces
//       of row s - 2 for z'^T A z' (z' of that row reached LDS in the previous step)
//   P3  first ASSOR sweep (Eq 3.5) of row s; second sweep (Eq 3.6) and z' of row s - 1;
//       the axial faces of z'^T A z' below row s - 1; then u of row s + 2 from its loads, and
//       on odd iterations its p
// Steps s = nz and nz + 1 (last chunk of a ring) only drain the lagged stages.
#pragma once

#include "gap_pcg.hpp"

constexpr int kOnePassParts = 5;   // r.z, r.r, z^T A z, z^T A u, u^T A u

// INIT = true: r_0 = S - A p_0 (p_0 = 0 on a cold start), z_0 = M^-1 r_0 and the partials
// r.z, r.r, z^T A z, S.S; the record is reset and the next launch runs with par = 0.
template <int NT, int Q, bool INIT>
__global__ __launch_bounds__(NT, (Q >= 4 ? 2 : 4)) void k_pcg_f(const PcgDev* __restrict__ reqs,
                                                                 const int* __restrict__ work, int launch_par)
{
    int req, c, kc;
    if (!pcg_work(work, blockIdx.x, req, c, kc)) return;
    const PcgDev& a = reqs[req];
    const int par = (launch_par ^ a.par_off) & 1;
    const bool writer_ = (c == 0 && kc == 0);
    // stopped: return at once; the record writer carries the flag into the other parity slot
    if (!INIT && a.sc->done_f[par]) {
        if (writer_ && threadIdx.x == 0) a.sc->done_f[par ^ 1] = 1;
        return;
    }
    const int nt = a.nt, nz = a.nz;
    const int j0 = kc * a.rows_b, j1 = min(j0 + a.rows_b, nz), slot = c * a.chunks_b + kc;
    const bool writer = writer_;               // publishes the request's device record
    const size_t fs = (size_t)a.fstride;
    double* wpart = a.fpart[INIT ? 0 : (par ^ 1)];
    const int t = threadIdx.x;
    // A condition frozen by the asynchronized test in an earlier launch carries its partials
    // into the set the next launch reads, so that its residual stays the one it froze at.
    if (!INIT && a.async && !writer && !((a.sc->act_f[par] >> c) & 1)) {
        if (t == 0)
            for (int q = 0; q < kOnePassParts; ++q) wpart[q * fs + slot] = a.fpart[par][q * fs + slot];
        return;
    }
    const int j = INIT ? -1 : a.sc->iter_f[par];
    const size_t n = (size_t)nt * nz;
    const bool assor = (a.precond == 2);
    const bool spmv = !INIT || a.warm;
    const bool has_prev = !INIT && j > 0;
    const int op = a.op[c];
    const GAP_AS1 double* kx = as_global(a.kx + (size_t)op * n);
    const GAP_AS1 double* kz = as_global(a.kz + (size_t)op * (n + nt));
    const GAP_AS1 double* mv = as_global(assor ? a.kx : a.minv + (size_t)op * n);   // read by ASSOR I only
    const size_t co = (size_t)c * n;
    // cell indices within one condition's vector are 32-bit (n <= 2^27): the loads and stores
    // then take a scalar base and a 32-bit vector offset
    const GAP_AS1 double* zin = as_global((INIT ? a.p : a.zf[j & 1]) + co);    // the vector A multiplies: z_j (u_j after beta), p_0
    const GAP_AS1 double* uin = as_global(a.u[(j + 1) & 1] + co);              // u_{j-1}
    GAP_AS1 double* uout = as_global(a.u[j & 1] + co);
    const GAP_AS1 double* rin = as_global((INIT ? a.S : a.r[j & 1]) + co);
    GAP_AS1 double* rout = as_global(a.r[(j + 1) & 1] + co);
    GAP_AS1 double* zout = as_global(a.zf[(j + 1) & 1] + co);
    GAP_AS1 double* pp = as_global(a.p + co);

    const int s_begin = max(j0 - 1, 0);
    const int s_stop = j1 + 1;              // steps s >= nz only drain the lagged stages
    const int z_hi = min(j1, nz - 1);       // z' is produced on rows [j0, z_hi]
    const int u_hi = min(j1 + 2, nz - 1);   // u is needed on rows [s_begin - 1, u_hi]

    extern __shared__ double lds[];
    double* su = lds;              // u, row s
    double* sy = lds + nt;         // y = D^-1 r', row s
    double* sv = lds + 2 * nt;     // [2][nt] first-sweep rows, by row parity
    double* sz = lds + 4 * nt;     // [2][nt] z' rows, by row parity
    double* skx = lds + 6 * nt;    // [3][nt] east-face conductances of rows s, s-1, s-2 (ring)

    // registers per column: u of rows s-1, s, s+1; axial faces s, s+1 and s-1; r, p of row
    // s; the lagged values of row s-1 (y, r', A u) and z' of row s-2; the loads of the next
    // row step.  The east-face conductances live in the LDS ring (the western neighbour and
    // the two earlier rows come from there), v of row s-1 in its LDS row, and 1/D of row
    // s-1 is recomputed from the same four conductances in the same order.
    double um[Q], uc[Q], up[Q], kzS[Q], kzN[Q], kzSprev[Q], rc[Q];
    double yprev[Q], rpprev[Q], aup[Q], zprev[Q];
    double kxn[Q], nzl[Q], nul[Q], nkz[Q], nr[Q], np[Q];
    double um_[Q], uc_[Q], up_[Q];          // u_{j-1} of the first rows, combined after beta
    // p moves on odd iterations only, by alpha_{j-1} u_{j-1} + alpha_j u_j, when the row's z_j
    // and u_{j-1} arrive (a launch of even j leaves its term pending)
    const bool odd = !INIT && (j & 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = t + q * NT;
        um[q] = uc[q] = up[q] = kzS[q] = kzN[q] = kzSprev[q] = rc[q] = 0.0;
        yprev[q] = rpprev[q] = aup[q] = zprev[q] = 0.0;
        kxn[q] = nzl[q] = nul[q] = nkz[q] = nr[q] = np[q] = 0.0;
        um_[q] = uc_[q] = up_[q] = 0.0;
        if (i < nt) {
            const unsigned g = (unsigned)s_begin * nt + i;
            if (spmv) {
                if (s_begin > 0) {
                    um[q] = zin[g - nt];
                    if (has_prev) um_[q] = uin[g - nt];
                }
                uc[q] = zin[g];
                if (has_prev) uc_[q] = uin[g];
                if (s_begin + 1 < nz) {
                    up[q] = zin[g + nt];
                    if (has_prev) up_[q] = uin[g + nt];
                }
            }
            kzS[q] = kz[g];
            kzN[q] = kz[g + nt];
            kxn[q] = kx[g];
            rc[q] = rin[g];
        }
    }

    // ---- scalars -----------------------------------------------------------------------
    double alpha = 1.0, beta = 0.0, a_prev = 0.0;
    if (!INIT) {
        __shared__ double sums[kOnePassParts + 1][GAP_MAXC];
        {
            const double* rp = a.fpart[par];
            const double* src[kOnePassParts + 1] = {rp, rp + fs, rp + 2 * fs, rp + 3 * fs, rp + 4 * fs, a.part_ss};
            const int cnt[kOnePassParts + 1] = {a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b};
            cond_sums<NT, kOnePassParts + 1>(a.n_cond, cnt, src, sums);
        }
        // sums: 0 r.z (d_j), 1 r.r, 2 z^T A z, 3 z^T A u_{j-1}, 4 u_{j-1}^T A u_{j-1}, 5 S.S
        const double* gprev = a.sc->gam[par];   // d_{j-1} per condition
        const unsigned was_active = (unsigned)a.sc->act_f[par];
        unsigned active = 0;
        double rr = 0.0, ss = 0.0;
        for (int k = 0; k < a.n_cond; ++k) {
            const double sk = sums[5][k] > 0.0 ? sums[5][k] : 1.0;
            const bool act = !a.async || (((was_active >> k) & 1) && sqrt(sums[1][k] / sk) > a.eps_c[k]);
            if (act) active |= 1u << k;
            rr += sums[1][k];
            ss += sums[5][k];
        }
        const double rel = sqrt(rr / (ss > 0.0 ? ss : 1.0));
        const bool converged = a.async ? (active == 0) : (rel <= a.eps);
        bool bad = !finite_d(rel);
        double alk[GAP_MAXC];                  // alpha_j per condition
        for (int k = 0; k < GAP_MAXC; ++k) alk[k] = 0.0;
        if (!converged && j < a.max_iter) {
            // u_j^T A u_j from the three sums, per condition for beta b
            auto den = [&](int k, double b) {
                return j > 0 ? sums[2][k] + 2.0 * b * sums[3][k] + b * b * sums[4][k] : sums[2][k];
            };
            if (a.per_cond) {
                for (int k = 0; k < a.n_cond; ++k) {
                    if (!(active & (1u << k))) continue;
                    const double bk = j > 0 ? sums[0][k] / gprev[k] : 0.0;
                    alk[k] = sums[0][k] / den(k, bk);
                    bad |= !finite_d(bk) || !finite_d(alk[k]);
                }
                beta = j > 0 ? sums[0][c] / gprev[c] : 0.0;
                alpha = sums[0][c] / den(c, beta);
            } else {
                double dn = 0.0, dp = 0.0, uau = 0.0;
                for (int k = 0; k < a.n_cond; ++k)
                    if (active & (1u << k)) {
                        dn += sums[0][k];
                        dp += gprev[k];
                    }
                beta = j > 0 ? dn / dp : 0.0;
                for (int k = 0; k < a.n_cond; ++k)
                    if (active & (1u << k)) uau += den(k, beta);
                alpha = dn / uau;
                bad |= !finite_d(beta) || !finite_d(alpha);
                for (int k = 0; k < a.n_cond; ++k) alk[k] = alpha;
            }
        }
        const bool stop = bad || converged || j >= a.max_iter;
        if (writer && t == 0) {
            PcgScalars* s = a.sc;
            s->iterations = j;
            s->rel = rel;
            for (int k = 0; k < a.n_cond; ++k) {
                const double sk = sums[5][k] > 0.0 ? sums[5][k] : 1.0;
                s->rel_cond[k] = sqrt(sums[1][k] / sk);
                s->gam[par ^ 1][k] = sums[0][k];
            }
            s->iter_f[par ^ 1] = j + 1;
            s->active_b = (int)active;
            s->act_f[par ^ 1] = (int)active;
            for (int k = 0; k < a.n_cond; ++k) s->alf[par ^ 1][k] = alk[k];
            s->status = bad ? -4 : (converged ? 0 : (j >= a.max_iter ? -3 : 0));
            if (stop) {
                s->done = 1;
                s->done_f[par ^ 1] = 1;
            }
            if (a.hist && !stop && j < a.hist_cap) {
                a.hist[2 * j] = alpha;
                a.hist[2 * j + 1] = beta;
            }
        }
        a_prev = odd ? a.sc->alf[par][c] : 0.0;
        if (stop || !(active & (1u << c))) {
            if (!stop && t == 0)
                for (int q = 0; q < kOnePassParts; ++q) wpart[q * fs + slot] = a.fpart[par][q * fs + slot];
            // this condition stops here: after an even iteration, alpha_{j-1} u_{j-1} is still
            // pending in p (a condition frozen earlier settled it in its own last launch)
            if (odd && ((was_active >> c) & 1)) {
                for (int s = j0; s < j1; ++s) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int i = t + q * NT;
                        if (i < nt) {
                            const unsigned g = (unsigned)s * nt + i;
                            pp[g] = pp[g] + a_prev * uin[g];
                        }
                    }
                }
            }
            return;
        }
    } else if (writer && t == 0) {
        PcgScalars* s = a.sc;
        s->iter_f[0] = 0;
        s->done = 0;
        s->status = 0;
        s->iterations = 0;
        s->active_b = (1 << a.n_cond) - 1;
        s->act_f[0] = s->act_f[1] = (1 << a.n_cond) - 1;
        s->done_f[0] = s->done_f[1] = 0;
    }

    // the scalars are alike in every lane: keep them in scalar registers
    alpha = wave_uniform(alpha);
    beta = wave_uniform(beta);
    a_prev = wave_uniform(a_prev);
    if (has_prev) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] += beta * um_[q];
            uc[q] += beta * uc_[q];
            up[q] += beta * up_[q];
        }
    }
    if (odd) {
        // the first rows (s_begin <= j0, so row s_begin - 1 is never owned)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt) {
                const unsigned g = (unsigned)s_begin * nt + i;
                if (s_begin >= j0) pp[g] = pp[g] + (a_prev * uc_[q] + alpha * uc[q]);
                if (s_begin + 1 >= j0 && s_begin + 1 < j1) pp[g + nt] = pp[g + nt] + (a_prev * up_[q] + alpha * up[q]);
            }
        }
    }

    const double om = a.omega;
    const double scale = om * (2.0 - om);
    double acc_rz = 0.0, acc_rr = 0.0, acc_zaz = 0.0, acc_zau = 0.0, acc_uau = 0.0, acc_ss = 0.0;
    int k0 = s_begin % 3;                 // ring slot of row s; row s-1 at (k0 + 2) % 3, row s-2 at (k0 + 1) % 3

    for (int s = s_begin; s <= s_stop; ++s) {
        const bool real = s < nz;
        const bool own = s >= j0 && s < j1;
        double* skc = skx + k0 * nt;
        const double* skp = skx + (k0 == 0 ? 2 : k0 - 1) * nt;
        const double* skq = skx + (k0 == 2 ? 0 : k0 + 1) * nt;
        // ---- P1 -------------------------------------------------------------------------
        const bool next = real && s + 1 < nz && s + 1 <= s_stop;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt && real) {
                su[i] = uc[q];
                skc[i] = kxn[q];
            }
            nzl[q] = nul[q] = kxn[q] = nkz[q] = nr[q] = np[q] = 0.0;
            if (i < nt && next) {
                const unsigned g1 = (unsigned)(s + 1) * nt + i;
                kxn[q] = kx[g1];
                nkz[q] = kz[g1 + nt];
                nr[q] = rin[g1];
                if (odd && s + 2 >= j0 && s + 2 < j1) np[q] = __builtin_nontemporal_load(&pp[g1 + nt]);
                if (spmv && s + 2 <= u_hi) {
                    nzl[q] = __builtin_nontemporal_load(&zin[g1 + nt]);
                    if (has_prev) nul[q] = __builtin_nontemporal_load(&uin[g1 + nt]);
                }
            }
        }
        __syncthreads();
        // ---- P2 -------------------------------------------------------------------------
        double rp[Q], dinv[Q], au[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            rp[q] = dinv[q] = au[q] = 0.0;
            if (i < nt) {
                const int ie = (i + 1 < nt) ? i + 1 : 0;
                if (real) {
                    const int iw = i ? i - 1 : nt - 1;
                    const double kxc = skc[i], kW = skc[iw];
                    const double D = ((kxc + kW) + kzS[q]) + kzN[q];
                    double r1 = rc[q];
                    if (spmv) {
                        double v = D * uc[q] - kxc * su[ie] - kW * su[iw];
                        if (s > 0) v -= kzS[q] * um[q];
                        if (s < nz - 1) v -= kzN[q] * up[q];
                        au[q] = v;
                        r1 -= alpha * v;
                    }
                    rp[q] = r1;
                    dinv[q] = 1.0 / D;
                    if (own) {
                        const unsigned g = (unsigned)s * nt + i;
                        rout[g] = r1;
                        acc_rr += r1 * r1;
                        if (INIT) {
                            acc_ss += rc[q] * rc[q];
                            if (!a.warm) pp[g] = 0.0;
                        } else {
                            __builtin_nontemporal_store(uc[q], &uout[g]);
                            acc_uau += uc[q] * au[q];
                        }
                    }
                    if (assor) sy[i] = r1 * dinv[q];
                }
                // east face of row s - 2
                if (s - 2 >= j0 && s - 2 < j1) {
                    const double d = zprev[q] - sz[((s - 2) & 1) * nt + ie];
                    acc_zaz += skq[i] * d * d;
                }
            }
        }
        __syncthreads();
        // ---- P3 -------------------------------------------------------------------------
        const bool make_z = (s - 1 >= j0 && s - 1 <= z_hi);
        const bool own_z = make_z && (s - 1 < j1);
        double* svc = sv + (s & 1) * nt;
        const double* svp = sv + ((s + 1) & 1) * nt;
        double* szc = sz + ((s - 1) & 1) * nt;
        const double kxwrap_prev = skp[nt - 1];      // west wrap of column 0 in row s - 1
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i >= nt) continue;
            double zv = 0.0;
            if (assor) {
                // Eq 3.5: v = y + w D^-1 (couplings to west, south and the east wrap); zero
                // beyond the last row
                double v = 0.0, y = 0.0;
                if (real) {
                    y = sy[i];
                    double lo = 0.0;
                    if (i > 0) lo += skc[i - 1] * sy[i - 1];            // west face of row s
                    if (i == nt - 1) lo += skc[i] * sy[0];              // east wrap face
                    if (s > 0) lo += kzS[q] * yprev[q];
                    v = y + om * dinv[q] * lo;
                }
                svc[i] = v;
                // Eq 3.6 for row s - 1: z = w(2-w)(v + w D^-1 (east, north, west wrap))
                if (make_z) {
                    const int iw = i ? i - 1 : nt - 1;
                    const double kxp = skp[i];
                    const double dinvprev = 1.0 / (((kxp + skp[iw]) + kzSprev[q]) + kzS[q]);
                    double hi = kzS[q] * v;
                    if (i < nt - 1) hi += kxp * svp[i + 1];
                    if (i == 0) hi += kxwrap_prev * svp[nt - 1];
                    zv = scale * (svp[i] + om * dinvprev * hi);
                }
                yprev[q] = y;
            } else if (make_z) {
                if (a.precond == 0) {
                    // Jacobi (Eq 2.8): 1/D of row s - 1 from its four conductances, added in the
                    // order the stored diagonal was formed, so z is the same to the bit
                    const int iw = i ? i - 1 : nt - 1;
                    zv = (1.0 / (((skp[i] + skp[iw]) + kzSprev[q]) + kzS[q])) * rpprev[q];
                } else {
                    zv = mv[(unsigned)(s - 1) * nt + i] * rpprev[q];
                }
            }
            if (make_z) {
                if (own_z) {
                    __builtin_nontemporal_store(zv, &zout[(unsigned)(s - 1) * nt + i]);
                    acc_rz += rpprev[q] * zv;
                    acc_zau += zv * aup[q];
                }
                szc[i] = zv;
                // axial faces of z'^T A z': the Dirichlet face below row 0, the face between
                // rows s - 2 and s - 1 (owned by row s - 2), the Dirichlet face above row nz - 1
                if (s - 1 == 0) {
                    acc_zaz += kzSprev[q] * zv * zv;
                } else if (s - 2 >= j0 && s - 2 < j1) {
                    const double d = zprev[q] - zv;
                    acc_zaz += kzSprev[q] * d * d;
                }
                if (own_z && s - 1 == nz - 1) acc_zaz += kzS[q] * zv * zv;
                zprev[q] = zv;
            }
        }
        // ---- advance one row ------------------------------------------------------------
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] = uc[q];
            uc[q] = up[q];
            up[q] = has_prev ? nzl[q] + beta * nul[q] : nzl[q];
            if (odd && s + 2 >= j0 && s + 2 < j1 && t + q * NT < nt)
                pp[(unsigned)(s + 2) * nt + t + q * NT] = np[q] + (a_prev * nul[q] + alpha * up[q]);
            kzSprev[q] = kzS[q];
            kzS[q] = kzN[q];
            kzN[q] = nkz[q];
            rc[q] = nr[q];
            rpprev[q] = rp[q];
            aup[q] = au[q];
        }
        k0 = (k0 == 2) ? 0 : k0 + 1;
    }
    double v6[6] = {acc_rz, acc_rr, acc_zaz, acc_zau, acc_uau, acc_ss};
    wg_sum<NT, 6>(v6);
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < kOnePassParts; ++q) wpart[q * fs + slot] = v6[q];
        if (INIT) a.part_ss[slot] = v6[5];
    }
}
