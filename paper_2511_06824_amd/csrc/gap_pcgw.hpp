// One-launch PCG iteration on wavefront strips, for gfx950, FP64: Table 1 with ASSOR II
// (Eq 3.4-3.6), Jacobi (Eq 2.8) or the stored diagonal of ASSOR I (Eq 3.2).
//
// Same scalar scheme as the ring kernel of gap_pcg1.hpp: u^T A u of the new direction is
//     z^T A z + 2 beta z^T A u_prev + beta^2 u_prev^T A u_prev,
// three sums the previous launch forms, so alpha is known at the start of a launch and one
// launch per iteration suffices.  What differs is the work decomposition and what is stored.
//
// * z is not stored.  Launch j reads r_j and u_{j-1} (and p on odd iterations), recomputes
//   z_j = M^-1 r_j, forms u_j = z_j + beta u_{j-1}, A u_j, r_{j+1} = r_j - alpha A u_j and
//   z_{j+1} = M^-1 r_{j+1} (for the partials only), and writes u_j and r_{j+1}: 32 B per
//   condition-DOF plus 16 B of p every other iteration (40 B on average) against the ring
//   kernel's 56 B, at the price of applying the preconditioner twice.  z_j is formed from
//   r_j with the same operations in the same order as the previous launch formed z_{j+1},
//   so it is the same vector to the bit.
// * Each wavefront owns a strip of one ring: a block of columns, with a halo of columns on
//   either side, and marches a chunk of rows.  Lane l holds the columns l, l + 64, ...,
//   l + 64 (Q - 1) of its strip, so every row load is 64 consecutive doubles per instruction.
//   Ring neighbours come from the neighbouring lane through DPP wave shifts (v_mov_b32_dpp
//   wave_shr:1 / wave_shl:1, with lane 0 / 63 filled from the next column block by
//   readlane); axial neighbours are earlier rows held in registers.  No LDS rows, no
//   barriers in the row march, and any ring width: a ring is cut into as many strips as it
//   needs.
// * Neumann order M (Eq 3.4 is M = 1): the inverses of (I + w D^-1 L) and (I + w D^-1 L^T)
//   keep M terms of their series.  The first sweep adds t_k = -w D^-1 L t_{k-1} on the row
//   being read (south and west couplings: earlier rows and lanes); the second adds
//   w_k = -w D^-1 L^T w_{k-1}, whose north coupling makes each term lag one more row, so
//   z of row r is complete M rows after r was read.
// * Halo.  The chain from r_j to the faces of z_{j+1}^T A z_{j+1} reaches 1/D one column,
//   each sweep of either application M columns, A u_j one and the east faces one:
//   values within 4M + 2 columns of a strip edge are not valid, so a strip owns the columns
//   at least that far from both of its edges.  Along the axis the chain reaches 2M + 1 rows
//   below a chunk and 2M + 2 above; those halo rows are recomputed by both chunks at a seam.
// * The strip's columns map to ring columns modulo n_theta, so the periodic wrap is plain
//   index arithmetic, and the split of the wrap entries between L and L^T (the east wrap of
//   the last column is in L, the west wrap of the first column in L^T) is decided by the
//   ring column a lane holds.
//
// Row pipeline of one wavefront, one row step s per loop trip (registers only):
//   S1  1/D and y = D^-1 r_j of row s
//   S2  first ASSOR sweep (Eq 3.5) of row s
//   S3  second sweep (Eq 3.6): its k-th term on row s - k; z_j and u_j = z_j + beta u_{j-1}
//       of row s - M
//   S4  A u_j, r_{j+1} and y' = D^-1 r_{j+1} of row a = s - M - 1; stores of u_j and r_{j+1};
//       p on odd iterations; partials u^T A u and r'.r'
//   S5  first sweep of z_{j+1} on row a
//   S6  second sweep and z_{j+1} of row b = s - 2M - 1; partials r'.z' and z'^T A u
//   S7  faces of z'^T A z': east faces of row b, the axial face below it (owned by the row
//       below), the Dirichlet faces
// The loads of row step s + 2 (one column per lane) or s + 1 are issued before the
// arithmetic of step s; with loads two steps ahead, S1 of row s + 1 is formed at the end of
// step s, off the dependency chain of the next step.
//
// Buffers, parities, the device record, frozen and stopped conditions and the pending p term
// follow the ring kernel exactly; the partial-sum slot of a workgroup is
// c * chunks + (row chunk) * groups + (strip group).
#pragma once

#include "gap_pcg.hpp"

constexpr int kStripWaves = 4;                      // strips (wavefronts) per workgroup
constexpr int kStripThreads = 64 * kStripWaves;
constexpr int kStripParts = 5;                      // r.z, r.r, z^T A z, z^T A u, u^T A u
constexpr int kStripMaxNeumann = 3;                 // Neumann orders M = 1 .. 3 are instantiated

// Halo columns on each side of a strip with Neumann order M: 1/D reaches one column, each
// sweep of each preconditioner application M, A u one and the east faces one.
__host__ __device__ constexpr int strip_halo(int M) { return 4 * M + 2; }

// Columns a strip of Q columns per lane owns at most.
__host__ __device__ constexpr int strip_owned_max(int Q, int M) { return 64 * Q - 2 * strip_halo(M); }

// One 32-bit DPP move.  ctrl 0x138: wave_shr:1 (lane i reads lane i - 1), 0x130: wave_shl:1
// (lane i reads lane i + 1); the lane without a source keeps `fill`.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double x, double fill)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned long long f = (unsigned long long)__double_as_longlong(fill);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)(f & 0xffffffffull), (int)(unsigned)(b & 0xffffffffull),
                                               CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf,
                                               false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double read_lane(double x, int l)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Value of the strip column one to the west (m - 1) of each lane's column m = lane + 64 q:
// lane l - 1 of the same block, lane 63 of block q - 1 for lane 0 (0 at the strip's west end).
template <int Q>
__device__ __forceinline__ void west_of(const double (&x)[Q], double (&w)[Q])
{
#pragma unroll
    for (int q = 0; q < Q; ++q) w[q] = dpp_shift<0x138>(x[q], q > 0 ? read_lane(x[q - 1], 63) : 0.0);
}

// Value one to the east (m + 1): lane l + 1, lane 0 of block q + 1 for lane 63 (0 at the east end).
template <int Q>
__device__ __forceinline__ void east_of(const double (&x)[Q], double (&e)[Q])
{
#pragma unroll
    for (int q = 0; q < Q; ++q) e[q] = dpp_shift<0x130>(x[q], q < Q - 1 ? read_lane(x[q + 1], 0) : 0.0);
}

// PK: the preconditioner fixed at compile time (0 Jacobi, 1 ASSOR I, 2 ASSOR II), or -1 to
// read it from the request (a batch whose requests differ).  M: the Neumann order of ASSOR II
// (1 is Eq 3.4; the diagonal preconditioners run with M = 1).
template <int Q, int PK, int M, bool INIT>
__global__ __launch_bounds__(kStripThreads, 2) void k_pcg_w(const PcgDev* __restrict__ reqs,
                                                            const int* __restrict__ work, int launch_par)
{
    int req, c, kc;
    if (!pcg_work(work, blockIdx.x, req, c, kc)) return;
    const PcgDev& a = reqs[req];
    const int par = (launch_par ^ a.par_off) & 1;
    const bool writer = (c == 0 && kc == 0);    // publishes the request's device record
    if (!INIT && a.sc->done_f[par]) {
        if (writer && threadIdx.x == 0) a.sc->done_f[par ^ 1] = 1;
        return;
    }
    const int t = threadIdx.x;
    const size_t fs = (size_t)a.fstride;
    const int slot = c * a.chunks_b + kc;
    double* wpart = a.fpart[INIT ? 0 : (par ^ 1)];
    if (!INIT && a.async && !writer && !((a.sc->act_f[par] >> c) & 1)) {
        if (t == 0)
            for (int q = 0; q < kStripParts; ++q) wpart[q * fs + slot] = a.fpart[par][q * fs + slot];
        return;
    }
    const int nt = a.nt, nz = a.nz;
    const int rchunk = kc / a.strip_groups, grp = kc - rchunk * a.strip_groups;
    const int j0 = rchunk * a.rows_b, j1 = min(j0 + a.rows_b, nz);
    const int lane = t & 63;
    const int strip = grp * kStripWaves + (t >> 6);
    const bool has_strip = strip < a.n_strips;
    // owned ring columns [oc0, oc1); strip column m is ring column (oc0 - halo + m) mod nt
    const int oc0 = (int)(((long long)strip * nt) / a.n_strips);
    const int oc1 = (int)(((long long)(strip + 1) * nt) / a.n_strips);
    int gcol[Q];
    bool ownc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int m = lane + 64 * q;
        int gc = (oc0 - strip_halo(M) + m) % nt;
        if (gc < 0) gc += nt;
        gcol[q] = gc;
        ownc[q] = has_strip && m >= strip_halo(M) && m < strip_halo(M) + (oc1 - oc0);
    }

    const int j = INIT ? -1 : a.sc->iter_f[par];
    const size_t n = (size_t)nt * nz;
    const int pk = PK >= 0 ? PK : a.precond;  // 0 Jacobi, 1 ASSOR I, 2 ASSOR II
    const bool spmv = !INIT || a.warm;
    const bool has_prev = !INIT && j > 0;
    const bool odd = !INIT && (j & 1);
    const int op = a.op[c];
    const GAP_AS1 double* kx = as_global(a.kx + (size_t)op * n);
    const GAP_AS1 double* kz = as_global(a.kz + (size_t)op * (n + nt));
    const GAP_AS1 double* mv = as_global(pk == 1 ? a.minv + (size_t)op * n : a.kx);   // read by ASSOR I only
    const size_t co = (size_t)c * n;
    // the vector that u_j is formed against: u_{j-1}, or p_0 for the initial residual
    const GAP_AS1 double* uin = as_global((INIT ? a.p : a.u[(j + 1) & 1]) + co);
    GAP_AS1 double* uout = as_global(a.u[(j & 1)] + co);
    const GAP_AS1 double* rin = as_global((INIT ? a.S : a.r[j & 1]) + co);
    GAP_AS1 double* rout = as_global(a.r[(j + 1) & 1] + co);
    GAP_AS1 double* pp = as_global(a.p + co);

    // Row pipeline with Neumann order M (the lags grow with M): S1, S2 on row s; the second
    // sweep of z_j reaches row s - M; S4, S5 run on row a = s - M - 1; z_{j+1} and the faces on
    // row b = s - 2M - 1.  S1 runs on [s_begin, s_last - 2M - 1]; z_{j+1} is needed on rows
    // [j0, min(j1, nz - 1)], which takes r_j on rows [j0 - 2M - 1, j1 + 2M + 1].
    constexpr int LB = 2 * M + 1;                // lag of the last stage
    const int s_begin = max(j0 - LB, 0);
    const int s_last = min(j1, nz - 1) + LB;
    // register rings, index d = row s - d (faces: d = face s + 1 - d)
    double R[M + 2][Q];                         // r_j (S for the initial residual)
    double KX[LB + 1][Q];                       // east-face conductances
    double DI[LB + 1][Q];                       // 1/D
    double F[LB + 2][Q];                        // axial faces
    double T[M][Q];                             // first-sweep terms t_k of row s - 1 (z_j)
    double V[M + 1][Q];                         // v of rows s .. s - M (z_j)
    double W[M][M + 1][Q];                      // W[k][e]: second-sweep term w_k of row s - k - e (z_j), k >= 1
    double U[3][Q];                             // u_j of rows s - M, s - M - 1, s - M - 2
    double UP[2][Q];                            // u_{j-1} (p_0 at the start) of rows s - M, s - M - 1
    double TQ[M][Q];                            // first-sweep terms of row a - 1 (z_{j+1})
    double VQ[M + 1][Q];                        // v' of rows a .. a - M
    double WQ[M][M + 1][Q];                     // w'_k of row a - k - e
    double RQ[M + 1][Q], AU[M + 1][Q];          // r_{j+1} and A u_j of rows a .. a - M
    double ZQ[Q];                               // z_{j+1} of row b - 1
    double MV1[Q], MV3[Q];                      // ASSOR I diagonal of rows s - 1, s - 3 (M = 1)
    double pp2[Q];                              // p of row a (odd iterations)
    // loads of the next two row steps (a: step s + 1, b: step s + 2)
    double ar[Q], akx[Q], af[Q], aup[Q], app[Q], amv[Q], amv3[Q];
    double br[Q], bkx[Q], bf[Q], bup[Q], bpp[Q], bmv[Q], bmv3[Q];
    double kwn[Q], din[Q], yn[Q];               // S1 of row s + 1 (loads two steps ahead)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int d = 0; d < M + 2; ++d) R[d][q] = 0.0;
#pragma unroll
        for (int d = 0; d <= LB; ++d) KX[d][q] = DI[d][q] = 0.0;
#pragma unroll
        for (int d = 0; d <= LB + 1; ++d) F[d][q] = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            T[k][q] = TQ[k][q] = 0.0;
#pragma unroll
            for (int e = 0; e <= M; ++e) W[k][e][q] = WQ[k][e][q] = 0.0;
        }
#pragma unroll
        for (int e = 0; e <= M; ++e) V[e][q] = VQ[e][q] = RQ[e][q] = AU[e][q] = 0.0;
        U[0][q] = U[1][q] = U[2][q] = UP[0][q] = UP[1][q] = 0.0;
        ZQ[q] = MV1[q] = MV3[q] = pp2[q] = 0.0;
        kwn[q] = din[q] = yn[q] = 0.0;
    }
    // loads of row step s: r, kx of row s; face s + 1; u_prev of row s - M; p of row s - M - 1;
    // the ASSOR I diagonal of rows s - 1 and s - 3
    auto issue = [&](int s, double (&nr)[Q], double (&nkx)[Q], double (&nf)[Q], double (&nup)[Q],
                     double (&npp)[Q], double (&nmv)[Q], double (&nmv3)[Q]) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            nr[q] = nkx[q] = nf[q] = nup[q] = npp[q] = nmv[q] = nmv3[q] = 0.0;
            const unsigned gc = (unsigned)gcol[q];
            if (s < nz) {
                const unsigned g = (unsigned)s * nt + gc;
                nr[q] = rin[g];
                nkx[q] = kx[g];
            }
            if (s + 1 <= nz) nf[q] = kz[(unsigned)(s + 1) * nt + gc];
            if (s - M >= 0 && s - M < nz && spmv) nup[q] = __builtin_nontemporal_load(&uin[(unsigned)(s - M) * nt + gc]);
            if (odd && ownc[q] && s - M - 1 >= j0 && s - M - 1 < j1)
                npp[q] = __builtin_nontemporal_load(&pp[(unsigned)(s - M - 1) * nt + gc]);
            if (pk == 1) {
                if (s - 1 >= 0 && s - 1 < nz) nmv[q] = mv[(unsigned)(s - 1) * nt + gc];
                if (s - 3 >= 0 && s - 3 < nz) nmv3[q] = mv[(unsigned)(s - 3) * nt + gc];
            }
        }
    };
    // one column per lane: loads two row steps ahead; more columns per lane: one step ahead
    // (the registers of a second stage would spill).  The loads of the first steps go out
    // before the reduction of the scalars, whose latency they overlap; they do not depend on
    // alpha or beta.
    constexpr int kAhead = Q == 1 ? 2 : 1;
    if (has_strip) {
        // face s_begin, the south face of the first row (it reaches F[1] at the first shift)
#pragma unroll
        for (int q = 0; q < Q; ++q) F[0][q] = kz[(unsigned)s_begin * nt + gcol[q]];
        issue(s_begin, ar, akx, af, aup, app, amv, amv3);
        if constexpr (kAhead == 2) issue(s_begin + 1, br, bkx, bf, bup, bpp, bmv, bmv3);
    }

    // ---- scalars (as in the ring kernel) ------------------------------------------------
    double alpha = 1.0, beta = 0.0, a_prev = 0.0;
    if (!INIT) {
        __shared__ double sums[kStripParts + 1][GAP_MAXC];
        {
            const double* rp = a.fpart[par];
            const double* src[kStripParts + 1] = {rp, rp + fs, rp + 2 * fs, rp + 3 * fs, rp + 4 * fs, a.part_ss};
            const int cnt[kStripParts + 1] = {a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b};
            cond_sums<kStripThreads, kStripParts + 1>(a.n_cond, cnt, src, sums);
        }
        const double* gprev = a.sc->gam[par];
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
        double alk[GAP_MAXC];
        for (int k = 0; k < GAP_MAXC; ++k) alk[k] = 0.0;
        if (!converged && j < a.max_iter) {
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
                for (int q = 0; q < kStripParts; ++q) wpart[q * fs + slot] = a.fpart[par][q * fs + slot];
            // the condition stops here: after an even iteration alpha_{j-1} u_{j-1} is still
            // pending in p (a condition frozen earlier settled it in its own last launch)
            if (odd && ((was_active >> c) & 1) && has_strip) {
                a_prev = wave_uniform(a_prev);
                for (int s = j0; s < j1; ++s) {
#pragma unroll
                    for (int q = 0; q < Q; ++q)
                        if (ownc[q]) {
                            const unsigned g = (unsigned)s * nt + gcol[q];
                            pp[g] = pp[g] + a_prev * uin[g];
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
    alpha = wave_uniform(alpha);
    beta = wave_uniform(beta);
    a_prev = wave_uniform(a_prev);

    const double om = a.omega;
    const double scale = om * (2.0 - om);
    double acc_rz = 0.0, acc_rr = 0.0, acc_zaz = 0.0, acc_zau = 0.0, acc_uau = 0.0, acc_ss = 0.0;

    if (has_strip) {
        for (int s = s_begin; s <= s_last; ++s) {
            // ---- shift the rings by one row, take the loads of this step ------------------
#pragma unroll
            for (int q = 0; q < Q; ++q) {
#pragma unroll
                for (int d = M + 1; d > 0; --d) R[d][q] = R[d - 1][q];
#pragma unroll
                for (int d = LB; d > 0; --d) {
                    KX[d][q] = KX[d - 1][q];
                    DI[d][q] = DI[d - 1][q];
                }
#pragma unroll
                for (int d = LB + 1; d > 0; --d) F[d][q] = F[d - 1][q];
#pragma unroll
                for (int e = M; e > 0; --e) {
                    V[e][q] = V[e - 1][q];
                    VQ[e][q] = VQ[e - 1][q];
                    RQ[e][q] = RQ[e - 1][q];
                    AU[e][q] = AU[e - 1][q];
                }
#pragma unroll
                for (int k = 1; k < M; ++k) {
#pragma unroll
                    for (int e = M - k; e > 0; --e) {
                        W[k][e][q] = W[k][e - 1][q];
                        WQ[k][e][q] = WQ[k][e - 1][q];
                    }
                }
                U[2][q] = U[1][q];
                U[1][q] = U[0][q];
                UP[1][q] = UP[0][q];
                R[0][q] = ar[q];
                KX[0][q] = akx[q];
                F[0][q] = af[q];
                UP[0][q] = aup[q];
                pp2[q] = app[q];
                MV1[q] = amv[q];
                MV3[q] = amv3[q];
                if constexpr (kAhead == 2) {
                    ar[q] = br[q];
                    akx[q] = bkx[q];
                    af[q] = bf[q];
                    aup[q] = bup[q];
                    app[q] = bpp[q];
                    amv[q] = bmv[q];
                    amv3[q] = bmv3[q];
                }
            }
            if constexpr (kAhead == 2) {
                if (s + 2 <= s_last) issue(s + 2, br, bkx, bf, bup, bpp, bmv, bmv3);
            } else {
                if (s + 1 <= s_last) issue(s + 1, ar, akx, af, aup, app, amv, amv3);
            }
            const int ra = s - M - 1;               // row of S4, S5
            const int rb = s - LB;                  // row of z_{j+1} and the faces
            const bool row0 = s < nz;
            const bool rowz = s - M >= 0 && s - M < nz;
            const bool rowa = ra >= 0 && ra < nz;
            const bool rowb = rb >= 0 && rb < nz;

            // ---- S1: 1/D and y of row s (with loads two steps ahead, formed in the previous
            // step, off the dependency chain of this one) ------------------------------------
            double kw0[Q], y0[Q];
            if (kAhead == 1 || s == s_begin) {
                west_of<Q>(KX[0], kw0);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    y0[q] = 0.0;
                    DI[0][q] = 0.0;
                    if (row0) {
                        const double D = ((KX[0][q] + kw0[q]) + F[1][q]) + F[0][q];
                        DI[0][q] = 1.0 / D;
                        y0[q] = R[0][q] * DI[0][q];
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    kw0[q] = kwn[q];
                    DI[0][q] = din[q];
                    y0[q] = yn[q];
                }
            }
            // ---- S2, S3: z_j of row s - M (Eq 3.5, 3.6 with M Neumann terms) --------------
            double un[Q];                           // u_j of row s - M
            if (INIT) {
#pragma unroll
                for (int q = 0; q < Q; ++q) un[q] = rowz ? UP[0][q] : 0.0;   // p_0 (zero on a cold start)
            } else if (pk == 2) {
                // first sweep on row s: v = y + t_1 + ... + t_M, t_k = w D^-1 (west, south and
                // east-wrap couplings of t_{k-1})
                double t[Q], v[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) t[q] = v[q] = y0[q];
#pragma unroll
                for (int k = 1; k <= M; ++k) {
                    double tw[Q], te[Q];
                    west_of<Q>(t, tw);
                    east_of<Q>(t, te);
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        double nt_ = 0.0;
                        if (row0) {
                            double lo = 0.0;
                            if (gcol[q] > 0) lo += kw0[q] * tw[q];
                            if (gcol[q] == nt - 1) lo += KX[0][q] * te[q];
                            if (s > 0) lo += F[1][q] * T[k - 1][q];
                            nt_ = om * DI[0][q] * lo;
                        }
                        T[k - 1][q] = t[q];         // t_{k-1} of row s, the south neighbour next step
                        t[q] = nt_;
                        v[q] += nt_;
                    }
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) V[0][q] = row0 ? v[q] : 0.0;
                // second sweep: w_k of row s - k from w_{k-1} of rows s - k + 1 (north) and
                // s - k (east, west wrap); z = w(2-w)(v + w_1 + ... + w_M) on row s - M
                double wl[Q];                       // w_M of row s - M
#pragma unroll
                for (int k = 1; k <= M; ++k) {
                    double here[Q], he[Q], hw[Q], kwk[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) here[q] = k == 1 ? V[1][q] : W[k - 1][1][q];
                    east_of<Q>(here, he);
                    west_of<Q>(here, hw);
                    west_of<Q>(KX[k], kwk);
                    const bool rowk = s - k >= 0 && s - k < nz;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        double hi = F[k][q] * (k == 1 ? V[0][q] : W[k - 1][0][q]);
                        if (gcol[q] < nt - 1) hi += KX[k][q] * he[q];
                        if (gcol[q] == 0) hi += kwk[q] * hw[q];
                        const double w = rowk ? om * DI[k][q] * hi : 0.0;
                        if (k < M) W[k][0][q] = w;
                        else wl[q] = w;
                    }
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double zs = V[M][q];
#pragma unroll
                    for (int k = 1; k < M; ++k) zs += W[k][M - k][q];
                    zs += wl[q];
                    const double zj = scale * zs;
                    un[q] = rowz ? (has_prev ? zj + beta * UP[0][q] : zj) : 0.0;
                }
            } else {
                // Jacobi (Eq 2.8) or ASSOR I: z_j = diag r_j of row s - 1 (M = 1)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const double zj = (pk == 0 ? DI[1][q] : MV1[q]) * R[1][q];
                    un[q] = rowz ? (has_prev ? zj + beta * UP[0][q] : zj) : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) U[0][q] = un[q];
            // ---- S4: A u_j, r_{j+1}, y' of row a ---------------------------------------
            constexpr int DA = M + 1;               // ring index of row a
            double yq[Q], kwa[Q];
            west_of<Q>(KX[DA], kwa);
            {
                double ue[Q], uw[Q];
                east_of<Q>(U[1], ue);
                west_of<Q>(U[1], uw);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    yq[q] = RQ[0][q] = AU[0][q] = 0.0;
                    if (!rowa) continue;
                    double r1v = R[DA][q];
                    if (spmv) {
                        const double D = ((KX[DA][q] + kwa[q]) + F[DA + 1][q]) + F[DA][q];
                        double v = D * U[1][q] - KX[DA][q] * ue[q] - kwa[q] * uw[q];
                        if (ra > 0) v -= F[DA + 1][q] * U[2][q];
                        if (ra < nz - 1) v -= F[DA][q] * U[0][q];
                        AU[0][q] = v;
                        r1v -= alpha * v;
                    }
                    RQ[0][q] = r1v;
                    yq[q] = r1v * DI[DA][q];
                    if (ownc[q] && ra >= j0 && ra < j1) {
                        const unsigned g = (unsigned)ra * nt + gcol[q];
                        rout[g] = r1v;
                        acc_rr += r1v * r1v;
                        if (INIT) {
                            acc_ss += R[DA][q] * R[DA][q];
                            if (!a.warm) pp[g] = 0.0;
                        } else {
                            __builtin_nontemporal_store(U[1][q], &uout[g]);
                            acc_uau += U[1][q] * AU[0][q];
                            if (odd) pp[g] = pp2[q] + (a_prev * UP[1][q] + alpha * U[1][q]);
                        }
                    }
                }
            }
            // ---- S5, S6: z_{j+1} of row b ---------------------------------------------
            double zq[Q];
            if (pk == 2) {
                double t[Q], v[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) t[q] = v[q] = yq[q];
#pragma unroll
                for (int k = 1; k <= M; ++k) {
                    double tw[Q], te[Q];
                    west_of<Q>(t, tw);
                    east_of<Q>(t, te);
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        double nt_ = 0.0;
                        if (rowa) {
                            double lo = 0.0;
                            if (gcol[q] > 0) lo += kwa[q] * tw[q];
                            if (gcol[q] == nt - 1) lo += KX[DA][q] * te[q];
                            if (ra > 0) lo += F[DA + 1][q] * TQ[k - 1][q];
                            nt_ = om * DI[DA][q] * lo;
                        }
                        TQ[k - 1][q] = t[q];
                        t[q] = nt_;
                        v[q] += nt_;
                    }
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) VQ[0][q] = rowa ? v[q] : 0.0;
                double wl[Q];
#pragma unroll
                for (int k = 1; k <= M; ++k) {
                    constexpr int D0 = M + 1;
                    const int d = D0 + k;               // ring index of row a - k
                    double here[Q], he[Q], hw[Q], kwk[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) here[q] = k == 1 ? VQ[1][q] : WQ[k - 1][1][q];
                    east_of<Q>(here, he);
                    west_of<Q>(here, hw);
                    west_of<Q>(KX[d], kwk);
                    const bool rowk = ra - k >= 0 && ra - k < nz;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        double hi = F[d][q] * (k == 1 ? VQ[0][q] : WQ[k - 1][0][q]);
                        if (gcol[q] < nt - 1) hi += KX[d][q] * he[q];
                        if (gcol[q] == 0) hi += kwk[q] * hw[q];
                        const double w = rowk ? om * DI[d][q] * hi : 0.0;
                        if (k < M) WQ[k][0][q] = w;
                        else wl[q] = w;
                    }
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double zs = VQ[M][q];
#pragma unroll
                    for (int k = 1; k < M; ++k) zs += WQ[k][M - k][q];
                    zs += wl[q];
                    zq[q] = rowb ? scale * zs : 0.0;
                }
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q) zq[q] = rowb ? (pk == 0 ? DI[LB][q] : MV3[q]) * RQ[M][q] : 0.0;
            }
            // ---- S7: partials and faces of z'^T A z' on row b ---------------------------
            {
                double ze[Q];
                east_of<Q>(zq, ze);
                const bool ownb = rowb && rb >= j0 && rb < j1;
                const bool own_below = rb - 1 >= j0 && rb - 1 < j1;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if (!ownc[q] || !rowb) continue;
                    if (ownb) {
                        acc_rz += RQ[M][q] * zq[q];
                        acc_zau += zq[q] * AU[M][q];
                        const double d = zq[q] - ze[q];
                        acc_zaz += KX[LB][q] * d * d;
                        if (rb == nz - 1) acc_zaz += F[LB][q] * zq[q] * zq[q];
                    }
                    if (rb == 0) {
                        if (ownb) acc_zaz += F[LB + 1][q] * zq[q] * zq[q];
                    } else if (own_below) {
                        const double d = ZQ[q] - zq[q];
                        acc_zaz += F[LB + 1][q] * d * d;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) ZQ[q] = zq[q];
            // ---- S1 of row s + 1 from its loads (already in registers) -------------------
            if constexpr (kAhead == 2) {
                west_of<Q>(akx, kwn);
                const bool rown = s + 1 < nz;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    din[q] = yn[q] = 0.0;
                    if (rown) {
                        const double D = ((akx[q] + kwn[q]) + F[0][q]) + af[q];
                        din[q] = 1.0 / D;
                        yn[q] = ar[q] * din[q];
                    }
                }
            }
        }
    }
    double v6[6] = {acc_rz, acc_rr, acc_zaz, acc_zau, acc_uau, acc_ss};
    wg_sum<kStripThreads, 6>(v6);
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < kStripParts; ++q) wpart[q * fs + slot] = v6[q];
        if (INIT) a.part_ss[slot] = v6[5];
    }
}
