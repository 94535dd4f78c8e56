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
//   readlane); axial neighbours are earlier rows held in registers.  No LDS rows, no data
//   exchange in the row march, and any ring width: a ring is cut into as many strips as it
//   needs.  On large systems at order 1 the wavefronts of a workgroup, which march
//   neighbouring strips of the same rows, meet at a barrier once per unrolled period of the
//   march, so that the columns two of them read are more often still in the caches when the
//   second one reads them.
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

#include <type_traits>

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

// The same move with BOUND_CTRL set: the lane without a source reads 0, so no fill value has
// to be placed in the destination first.
template <int CTRL>
__device__ __forceinline__ double dpp_shift0(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
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
    for (int q = 0; q < Q; ++q) w[q] = q > 0 ? dpp_shift<0x138>(x[q], read_lane(x[q - 1], 63)) : dpp_shift0<0x138>(x[q]);
}

// Value one to the east (m + 1): lane l + 1, lane 0 of block q + 1 for lane 63 (0 at the east end).
template <int Q>
__device__ __forceinline__ void east_of(const double (&x)[Q], double (&e)[Q])
{
#pragma unroll
    for (int q = 0; q < Q; ++q) e[q] = q < Q - 1 ? dpp_shift<0x130>(x[q], read_lane(x[q + 1], 0)) : dpp_shift0<0x130>(x[q]);
}

// Per-condition sums of NQ partial arrays of `chunks` slots each, in the order of cond_sums
// (wave w takes conditions w, w + NW, ...; lane l adds slots l, l + 64, ... to a zero start;
// then the same shuffle tree), so the sums are the same to the bit.  The loads of a round of
// 64 slots go out for all of a wave's conditions and arrays together: one memory latency per
// round instead of one per condition and array.  Threads 0 .. n_cond - 1 also copy gsrc[t]
// to gout[t] on the way.  Results in out[q][c] and gout, valid after the trailing barrier.
template <int NT, int NQ>
__device__ __forceinline__ void strip_cond_sums(int n_cond, int chunks, const double* const (&src)[NQ],
                                                double (*out)[GAP_MAXC], const double* gsrc, double* gout)
{
    constexpr int NW = NT / 64;
    constexpr int R = (GAP_MAXC + NW - 1) / NW;     // conditions per wavefront at most
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool gcopy = (int)threadIdx.x < n_cond;
    double g = 0.0;
    if (gcopy) g = gsrc[threadIdx.x];
    double v[R][NQ];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[r][q] = 0.0;
    for (int k0 = 0; k0 < chunks; k0 += 64) {
        const int k = k0 + lane;
        double x[R][NQ];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool ok = w + r * NW < n_cond && k < chunks;
#pragma unroll
            for (int q = 0; q < NQ; ++q) x[r][q] = ok ? src[q][(w + r * NW) * chunks + k] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool ok = w + r * NW < n_cond && k < chunks;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (ok) v[r][q] += x[r][q];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[r][q] += __shfl_xor(v[r][q], off, 64);
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (w + r * NW < n_cond) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[q][w + r * NW] = v[r][q];
            }
    }
    if (gcopy) gout[threadIdx.x] = g;
    __syncthreads();
}

// Runs the row steps of phases PH .. P - 1 (fn(s, phase) each), advancing s; false once s has
// passed s_last.  Unrolled at compile time, so each step sees its phase as a constant.
template <int PH, int P, class Fn>
__device__ __forceinline__ bool strip_steps(Fn& fn, int& s, int s_last)
{
    fn(s, std::integral_constant<int, PH>{});
    if (++s > s_last) return false;
    if constexpr (PH + 1 < P) return strip_steps<PH + 1, P>(fn, s, s_last);
    else return true;
}

// PK: the preconditioner fixed at compile time (0 Jacobi, 1 ASSOR I, 2 ASSOR II), or -1 to
// read it from the request (a batch whose requests differ).  M: the Neumann order of ASSOR II
// (1 is Eq 3.4; the diagonal preconditioners run with M = 1).  SYNC (order 1 only): the
// wavefronts of a workgroup meet at a barrier after each period of the row march.
template <int Q, int PK, int M, bool INIT, bool SYNC = false>
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
    const GAP_AS1 double* kxz = as_global(a.kxz + (size_t)op * 2 * (n + nt));   // pairs (orders 1, 2)
    const GAP_AS1 double* mv = as_global(pk == 1 ? a.minv + (size_t)op * n : a.kx);   // read by ASSOR I only
    const size_t co = (size_t)c * n;
    // Orders 1 and 2 keep r and u as interleaved pairs: the block of parity k holds
    // (r_k, u_{k-1}) per cell, so a launch reads the pair it needs with one 16-byte load per
    // lane and writes (r_{j+1}, u_j) with one store; the initial residual reads S and p_0 from
    // their own arrays and writes (r_0, 0).  They read the conductances as the row pairs of
    // kxz the same way.  u_{j-1} of row s then waits M + 1 steps in registers, which order 3
    // cannot afford (its registers are full): it keeps r and u in separate arrays (the halves
    // of the same blocks), reads u_{j-1} of row s - M where it is needed, and reads kx and kz.
    constexpr bool kPairs = (M <= 2);
    constexpr int DU = kPairs ? M : 0;           // ring index of u_{j-1} of row s - M
    const GAP_AS1 double* ruin = as_global(a.r[j & 1] + 2 * co);       // pair g at [2g], [2g + 1]
    GAP_AS1 double* ruout = as_global(a.r[(j + 1) & 1] + 2 * co);
    const GAP_AS1 double* rin = as_global((INIT ? a.S : a.r[j & 1]) + co);   // separate arrays
    GAP_AS1 double* rout = as_global(a.r[(j + 1) & 1] + co);
    const GAP_AS1 double* uin = as_global((INIT ? a.p : a.u[(j + 1) & 1]) + co);
    GAP_AS1 double* uout = as_global(a.u[j & 1] + co);
    GAP_AS1 double* pp = as_global(a.p + co);

    // Row pipeline with Neumann order M (the lags grow with M): S1, S2 on row s; the second
    // sweep of z_j reaches row s - M; S4, S5 run on row a = s - M - 1; z_{j+1} and the faces on
    // row b = s - 2M - 1.  S1 runs on [s_begin, s_last - 2M - 1]; z_{j+1} is needed on rows
    // [j0, min(j1, nz - 1)], which takes r_j on rows [j0 - 2M - 1, j1 + 2M + 1].
    constexpr int LB = 2 * M + 1;                // lag of the last stage
    const int s_begin = max(j0 - LB, 0);
    const int s_last = min(j1, nz - 1) + LB;
    // Register rings.  Row step s runs in phase PH = (s - s_begin) mod P, and the value of the
    // row d steps behind s (faces: face s + 1 - d) sits in slot (PH - d) mod P of its ring.
    // The march is unrolled by P, so every slot index is a constant and the rings rotate by
    // renaming instead of moves.  Loads land kAhead steps ahead (d = -kAhead) and 1/D of the
    // next row one step ahead, so P exceeds the deepest read (faces, d = 2M + 2) by more
    // than kAhead.  Rows outside the grid or before the chunk's first row hold zeros and
    // 1/D = 0, which zeroes every term they would feed.
    constexpr int P = 2 * M + 5;
    constexpr int kAhead = Q == 1 ? 2 : 1;      // one column per lane: loads two steps ahead
    double R[P][Q];                             // r_j (S for the initial residual)
    double KX[P][Q];                            // east-face conductances
    double DI[P][Q];                            // 1/D
    double F[P][Q];                             // axial faces
    double UP[P][Q];                            // u_{j-1} (p_0 at the start) of row s - d (pairs), s - M - d
    double PP[P][Q];                            // loaded with step s: p of row s - M - 1 (odd iterations)
    double MV1[P][Q], MV3[P][Q];                // loaded with step s: ASSOR I diagonal of rows s - 1, s - 3
    double V[P][Q];                             // v of row s - d (z_j)
    double W[M][P][Q];                          // W[k]: second-sweep term w_k of row s - k - d (z_j), k >= 1
    double U[P][Q];                             // u_j of row s - M - d
    double VQ[P][Q];                            // v' of row a - d (z_{j+1})
    double WQ[M][P][Q];                         // w'_k of row a - k - d
    double RQ[P][Q], AU[P][Q];                  // r_{j+1} and A u_j of row a - d
    double T[M][Q], TQ[M][Q];                   // first-sweep terms of the previous row (z_j, z_{j+1})
    double ZQ[Q];                               // z_{j+1} of row b - 1
    double kwc[Q], yc[Q];                       // S1 of the current row: west conductance, D^-1 r
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int d = 0; d < P; ++d) {
            R[d][q] = KX[d][q] = DI[d][q] = F[d][q] = UP[d][q] = PP[d][q] = MV1[d][q] = MV3[d][q] = 0.0;
            V[d][q] = U[d][q] = VQ[d][q] = RQ[d][q] = AU[d][q] = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) W[k][d][q] = WQ[k][d][q] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < M; ++k) T[k][q] = TQ[k][q] = 0.0;
        ZQ[q] = kwc[q] = yc[q] = 0.0;
    }
    // u_{j-1} is read from the second iteration on (beta = 0 before), p_0 on a warm start
    const bool need_up = INIT ? a.warm != 0 : has_prev;
    // loads of row step s into ring slot SL: r, u_prev (p_0), kx of row s; face s + 1; p of
    // row s - M - 1; the ASSOR I diagonal of rows s - 1 and s - 3
    auto issue = [&](int s, auto SLc) {
        constexpr int sl = decltype(SLc)::value;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            R[sl][q] = KX[sl][q] = F[sl][q] = UP[sl][q] = PP[sl][q] = MV1[sl][q] = MV3[sl][q] = 0.0;
            const unsigned gc = (unsigned)gcol[q];
            if (s < nz) {
                const unsigned g = (unsigned)s * nt + gc;
                if (INIT || !kPairs) {
                    R[sl][q] = rin[g];
                    if (kPairs && need_up) UP[sl][q] = uin[g];
                } else {
                    R[sl][q] = ruin[2 * g];         // u_{j-1} is 0 at j = 0 (written so by the initial residual)
                    UP[sl][q] = ruin[2 * g + 1];
                }
                if (kPairs) {
                    const unsigned h = g + (unsigned)nt;   // pair (s + 1, column): kx of row s, face s + 1
                    KX[sl][q] = kxz[2 * h];
                    F[sl][q] = kxz[2 * h + 1];
                } else {
                    KX[sl][q] = kx[g];
                }
            }
            if (!kPairs && s - M >= 0 && s - M < nz && need_up)
                UP[sl][q] = __builtin_nontemporal_load(&uin[(unsigned)(s - M) * nt + gc]);
            if (!kPairs && s + 1 <= nz) F[sl][q] = kz[(unsigned)(s + 1) * nt + gc];
            if (odd && ownc[q] && s - M - 1 >= j0 && s - M - 1 < j1)
                PP[sl][q] = __builtin_nontemporal_load(&pp[(unsigned)(s - M - 1) * nt + gc]);
            if (pk == 1) {
                if (s - 1 >= 0 && s - 1 < nz) MV1[sl][q] = mv[(unsigned)(s - 1) * nt + gc];
                if (s - 3 >= 0 && s - 3 < nz) MV3[sl][q] = mv[(unsigned)(s - 3) * nt + gc];
            }
        }
    };
    // The loads of the first steps go out before the reduction of the scalars, whose latency
    // they overlap; they do not depend on alpha or beta.
    if (has_strip) {
        // face s_begin, the south face of the first row (d = 1 in phase 0)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const unsigned h = (unsigned)s_begin * nt + gcol[q];
            F[P - 1][q] = kPairs ? kxz[2 * h + 1] : kz[h];
        }
        issue(s_begin, std::integral_constant<int, 0>{});
        if constexpr (kAhead == 2) issue(s_begin + 1, std::integral_constant<int, 1>{});
    }

    // ---- scalars (as in the ring kernel) ------------------------------------------------
    double alpha = 1.0, beta = 0.0, a_prev = 0.0;
    if (!INIT) {
        // the device record's fields are read before the reduction's barrier, so that their
        // latency overlaps that of the partial sums; r.z of the previous launch goes through LDS
        __shared__ double sums[kStripParts + 1][GAP_MAXC];
        __shared__ double gprev[GAP_MAXC];
        const unsigned was_active = (unsigned)a.sc->act_f[par];
        const double alf_prev = odd ? a.sc->alf[par][c] : 0.0;
        {
            const double* rp = a.fpart[par];
            const double* src[kStripParts + 1] = {rp, rp + fs, rp + 2 * fs, rp + 3 * fs, rp + 4 * fs, a.part_ss};
            strip_cond_sums<kStripThreads, kStripParts + 1>(a.n_cond, a.chunks_b, src, sums, a.sc->gam[par], gprev);
        }
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
        a_prev = alf_prev;
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
                            pp[g] = pp[g] + a_prev * (kPairs ? ruin[2 * g + 1] : uin[g]);
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

    // S1 of row r, whose loads sit in slot SL (face r + 1 there, face r one slot before): the
    // west conductance, 1/D (0 outside the grid) and y = D^-1 r
    auto s1 = [&](int r, auto SLc) {
        constexpr int sl = decltype(SLc)::value, sf = (sl + P - 1) % P;
        west_of<Q>(KX[sl], kwc);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double D = ((KX[sl][q] + kwc[q]) + F[sf][q]) + F[sl][q];
            DI[sl][q] = r < nz ? 1.0 / D : 0.0;
            yc[q] = R[sl][q] * DI[sl][q];
        }
    };
    // One row step in phase PH.  WRAP: the strip holds ring column 0 or n_theta - 1, whose
    // periodic couplings split between L and L^T (Eq 3.5, 3.6); elsewhere the west coupling
    // is in L and the east one in L^T, with no per-column tests.
    auto step = [&](int s, auto PHc, auto WRc) {
        constexpr int PH = decltype(PHc)::value;
        constexpr bool WRAP = decltype(WRc)::value;
        auto S = [](int d) constexpr { return ((PH - d) % P + P) % P; };
        if (s + kAhead <= s_last) issue(s + kAhead, std::integral_constant<int, S(-kAhead)>{});
        if constexpr (kAhead == 1) s1(s, std::integral_constant<int, S(0)>{});
        const int ra = s - M - 1;               // row of S4, S5
        const int rb = s - LB;                  // row of z_{j+1} and the faces
        constexpr int DA = M + 1;               // ring index of row a

        // ---- S2, S3: z_j and u_j of row s - M (Eq 3.5, 3.6 with M Neumann terms) --------
        double un[Q];
        if constexpr (INIT) {
#pragma unroll
            for (int q = 0; q < Q; ++q) un[q] = UP[S(DU)][q];  // p_0 (zero on a cold start)
        } else if (pk == 2) {
            // first sweep on row s: v = y + t_1 + ... + t_M, t_k = w D^-1 (west, south and
            // east-wrap couplings of t_{k-1})
            double t[Q], v[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) t[q] = v[q] = yc[q];
#pragma unroll
            for (int k = 1; k <= M; ++k) {
                double tw[Q], te[Q];
                west_of<Q>(t, tw);
                if constexpr (WRAP) east_of<Q>(t, te);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double lo;
                    if constexpr (WRAP)
                        lo = (gcol[q] > 0 ? kwc[q] * tw[q] : 0.0) + (gcol[q] == nt - 1 ? KX[S(0)][q] * te[q] : 0.0);
                    else
                        lo = kwc[q] * tw[q];
                    lo += F[S(1)][q] * T[k - 1][q];
                    const double nt_ = om * DI[S(0)][q] * lo;
                    T[k - 1][q] = t[q];         // t_{k-1} of row s, the south neighbour next step
                    t[q] = nt_;
                    v[q] += nt_;
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) V[S(0)][q] = v[q];
            // second sweep: w_k of row s - k from w_{k-1} of rows s - k + 1 (north) and
            // s - k (east, west wrap); z = w(2-w)(v + w_1 + ... + w_M) on row s - M
            double wl[Q];                       // w_M of row s - M
#pragma unroll
            for (int k = 1; k <= M; ++k) {
                double here[Q], he[Q], hw[Q], kwk[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) here[q] = k == 1 ? V[S(1)][q] : W[k - 1][S(1)][q];
                east_of<Q>(here, he);
                if constexpr (WRAP) {
                    west_of<Q>(here, hw);
                    west_of<Q>(KX[S(k)], kwk);
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double hi = F[S(k)][q] * (k == 1 ? V[S(0)][q] : W[k - 1][S(0)][q]);
                    if constexpr (WRAP) {
                        if (gcol[q] < nt - 1) hi += KX[S(k)][q] * he[q];
                        if (gcol[q] == 0) hi += kwk[q] * hw[q];
                    } else {
                        hi += KX[S(k)][q] * he[q];
                    }
                    const double w = om * DI[S(k)][q] * hi;
                    if (k < M) W[k][S(0)][q] = w;
                    else wl[q] = w;
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double zs = V[S(M)][q];
#pragma unroll
                for (int k = 1; k < M; ++k) zs += W[k][S(M - k)][q];
                zs += wl[q];
                const double zj = scale * zs;
                un[q] = zj + beta * UP[S(DU)][q];       // u_{j-1} reads 0 while beta = 0
            }
        } else {
            // Jacobi (Eq 2.8) or ASSOR I: z_j = diag r_j of row s - 1 (M = 1)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const double zj = (pk == 0 ? DI[S(1)][q] : MV1[S(0)][q]) * R[S(1)][q];
                un[q] = zj + beta * UP[S(DU)][q];
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) U[S(0)][q] = un[q];

        // ---- S4: A u_j, r_{j+1}, y' of row a (rows outside the grid: u = 0 there, so the
        // Dirichlet faces of the end rows drop out of the products) ------------------------
        double yq[Q], kwa[Q];
        west_of<Q>(KX[S(DA)], kwa);
        {
            double ue[Q], uw[Q];
            east_of<Q>(U[S(1)], ue);
            west_of<Q>(U[S(1)], uw);
            const bool own_a = ra >= j0 && ra < j1;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double r1v = R[S(DA)][q];
                AU[S(0)][q] = 0.0;
                if (spmv) {
                    const double D = ((KX[S(DA)][q] + kwa[q]) + F[S(DA + 1)][q]) + F[S(DA)][q];
                    double v = D * U[S(1)][q] - KX[S(DA)][q] * ue[q] - kwa[q] * uw[q];
                    v -= F[S(DA + 1)][q] * U[S(2)][q];
                    v -= F[S(DA)][q] * U[S(0)][q];
                    AU[S(0)][q] = v;
                    r1v -= alpha * v;
                }
                RQ[S(0)][q] = r1v;
                yq[q] = r1v * DI[S(DA)][q];
                if (ownc[q] && own_a) {
                    const unsigned g = (unsigned)ra * nt + gcol[q];
                    if (kPairs) {
                        ruout[2 * g] = r1v;
                        ruout[2 * g + 1] = INIT ? 0.0 : U[S(1)][q];
                    } else {
                        rout[g] = r1v;
                        if (!INIT) __builtin_nontemporal_store(U[S(1)][q], &uout[g]);
                    }
                    acc_rr += r1v * r1v;
                    if (INIT) {
                        acc_ss += R[S(DA)][q] * R[S(DA)][q];
                        if (!a.warm) pp[g] = 0.0;
                    } else {
                        acc_uau += U[S(1)][q] * AU[S(0)][q];
                        if (odd) pp[g] = PP[S(0)][q] + (a_prev * UP[S(DU + 1)][q] + alpha * U[S(1)][q]);
                    }
                }
            }
        }
        // ---- S5, S6: z_{j+1} of row b ---------------------------------------------------
        double zq[Q];
        if (pk == 2) {
            double t[Q], v[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) t[q] = v[q] = yq[q];
#pragma unroll
            for (int k = 1; k <= M; ++k) {
                double tw[Q], te[Q];
                west_of<Q>(t, tw);
                if constexpr (WRAP) east_of<Q>(t, te);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double lo;
                    if constexpr (WRAP)
                        lo = (gcol[q] > 0 ? kwa[q] * tw[q] : 0.0) + (gcol[q] == nt - 1 ? KX[S(DA)][q] * te[q] : 0.0);
                    else
                        lo = kwa[q] * tw[q];
                    lo += F[S(DA + 1)][q] * TQ[k - 1][q];
                    const double nt_ = om * DI[S(DA)][q] * lo;
                    TQ[k - 1][q] = t[q];
                    t[q] = nt_;
                    v[q] += nt_;
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) VQ[S(0)][q] = v[q];
            double wl[Q];
#pragma unroll
            for (int k = 1; k <= M; ++k) {
                const int d = DA + k;           // ring index of row a - k
                double here[Q], he[Q], hw[Q], kwk[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) here[q] = k == 1 ? VQ[S(1)][q] : WQ[k - 1][S(1)][q];
                east_of<Q>(here, he);
                if constexpr (WRAP) {
                    west_of<Q>(here, hw);
                    west_of<Q>(KX[S(d)], kwk);
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    double hi = F[S(d)][q] * (k == 1 ? VQ[S(0)][q] : WQ[k - 1][S(0)][q]);
                    if constexpr (WRAP) {
                        if (gcol[q] < nt - 1) hi += KX[S(d)][q] * he[q];
                        if (gcol[q] == 0) hi += kwk[q] * hw[q];
                    } else {
                        hi += KX[S(d)][q] * he[q];
                    }
                    const double w = om * DI[S(d)][q] * hi;
                    if (k < M) WQ[k][S(0)][q] = w;
                    else wl[q] = w;
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double zs = VQ[S(M)][q];
#pragma unroll
                for (int k = 1; k < M; ++k) zs += WQ[k][S(M - k)][q];
                zs += wl[q];
                zq[q] = scale * zs;
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) zq[q] = (pk == 0 ? DI[S(LB)][q] : MV3[S(0)][q]) * RQ[S(M)][q];
        }
        // ---- S7: partials and faces of z'^T A z' on row b -------------------------------
        {
            double ze[Q];
            east_of<Q>(zq, ze);
            const bool rowb = rb >= 0 && rb < nz;
            const bool ownb = rowb && rb >= j0 && rb < j1;
            const bool own_below = rb - 1 >= j0 && rb - 1 < j1;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (!ownc[q] || !rowb) continue;
                if (ownb) {
                    acc_rz += RQ[S(M)][q] * zq[q];
                    acc_zau += zq[q] * AU[S(M)][q];
                    const double d = zq[q] - ze[q];
                    acc_zaz += KX[S(LB)][q] * d * d;
                    if (rb == nz - 1) acc_zaz += F[S(LB)][q] * zq[q] * zq[q];
                }
                if (rb == 0) {
                    if (ownb) acc_zaz += F[S(LB + 1)][q] * zq[q] * zq[q];
                } else if (own_below) {
                    const double d = ZQ[q] - zq[q];
                    acc_zaz += F[S(LB + 1)][q] * d * d;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) ZQ[q] = zq[q];
        // ---- S1 of row s + 1 from its loads (already in registers) ----------------------
        if constexpr (kAhead == 2) s1(s + 1, std::integral_constant<int, S(-1)>{});
    };

    if constexpr (SYNC) {
        static_assert(M == 1, "the synchronized march is built for order 1");
        auto nowrap = [&](int sv, auto PHc) { step(sv, PHc, std::false_type{}); };
        auto withwrap = [&](int sv, auto PHc) { step(sv, PHc, std::true_type{}); };
        int s = s_begin;
        // the strip's columns lie inside [1, n_theta - 2]: no wrap coupling in it
        const int w0 = oc0 - strip_halo(M);
        const bool wrap = !(w0 >= 1 && w0 + 64 * Q - 1 <= nt - 2);
        if (has_strip && kAhead == 2) s1(s_begin, std::integral_constant<int, 0>{});
        // The wavefronts of the workgroup meet at a barrier after each period of P row steps
        // (periods - 1 full ones, then the last of 1 .. P steps).  The trip count is the same
        // for all of them (one row chunk), and the barrier sits where every wavefront, with a
        // strip or without, passes it once per trip.  They exchange nothing there: held within
        // a period of each other, the edge columns two of them read are more often still in
        // the caches at the second read.  Measured on the 9-condition 2048 x 1024 system:
        // 3 % less time and 2 % less HBM traffic per launch; on 1024 x 512, whose vectors and
        // operators fit the last-level cache, this form of the march costs 3-5 %, so the host
        // picks it for requests that stream more than that cache holds.
        const int periods = (s_last - s_begin + P) / P;
        for (int it = 0; it < periods; ++it) {
            if (has_strip) {
                if (!wrap) strip_steps<0, P>(nowrap, s, s_last);
                else strip_steps<0, P>(withwrap, s, s_last);
            }
            __syncthreads();
        }
    } else if (has_strip) {
        if constexpr (kAhead == 2) s1(s_begin, std::integral_constant<int, 0>{});
        // the strip's columns lie inside [1, n_theta - 2]: no wrap coupling in it
        const int w0 = oc0 - strip_halo(M);
        const bool wrap = !(w0 >= 1 && w0 + 64 * Q - 1 <= nt - 2);
        int s = s_begin;
        auto march = [&](auto WRc) {
            auto one = [&](int sv, auto PHc) { step(sv, PHc, WRc); };
            while (strip_steps<0, P>(one, s, s_last)) {
            }
        };
        if constexpr (M == 1) {
            if (!wrap) march(std::false_type{});
            else march(std::true_type{});
        } else {
            march(std::true_type{});
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
