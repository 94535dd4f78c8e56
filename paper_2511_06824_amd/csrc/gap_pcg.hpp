// Fused PCG iteration kernels (Table 1 with ASSOR II, Eq 3.4-3.6) for gfx950, FP64.
//
// Two kernels per iteration:
//   A(j): beta from the previous r.z sums; stopping test (Eq 3.9); u_j = z_j + beta u_{j-1};
//         partial u_j^T A u_j.
//   B(j): alpha = d_j / (u_j^T A u_j); p += alpha u_j; r_{j+1} = r_j - alpha A u_j (A u_j
//         recomputed from u_j); z_{j+1} = M^{-1} r_{j+1}; partials r.z and r.r.
//   B in "init" mode computes r_0 = S - A p_0 and z_0 instead.
//
// Work decomposition: a workgroup owns the whole ring of one condition (all n_theta
// columns; thread t handles columns t, t + NT, ..., t + (Q-1) NT) and marches over a chunk
// of consecutive rows.  Ring neighbours come from LDS, axial neighbours from registers of
// the previous/next row, so the periodic wrap and the ASSOR split of the wrap entries
// (east wrap of the last column in L, west wrap of the first column in L^T) stay inside one
// workgroup.  The chunk of rows [j0, j1) reads one or two halo rows on each side.
//
// Buffer addresses come from the request record in device memory; the kernels access them
// through global-memory views (as_global), so that waits for LDS reads do not also wait for
// the loads in flight.
//
// Cache hints: the row-by-row z and u_prev loads and the u stores of A, and the p loads and z
// stores of B, are non-temporal.  Those streams are not re-read within a launch (the first
// rows of a chunk, which neighbouring chunks also read as halo, keep normal loads), and
// keeping them out of L2 and the Infinity Cache leaves both to what is re-read: the operator
// rows shared by conditions and the halo rows.  On the 2048 x 1024 joint workload this subset
// measured fastest of the combinations tried (iteration 379 -> 347 us together with the
// early first-row loads).
//
// Scalars: every workgroup reduces the per-chunk partial sums it needs at its start, in a
// fixed order, so all workgroups of a launch derive identical alpha / beta / stopping
// decisions without atomics or an extra launch; workgroup 0 publishes the host-visible
// record.  Iteration indices live in device memory (iter_a read by A and written by B,
// iter_b read by B and written by A), so the launches take identical arguments every
// iteration and can be replayed from a captured graph.
#pragma once

#include "gap_device.hpp"

struct PcgScalars {
    int iter_a;                 // iteration index the next A launch runs (written by B, init)
    int iter_b;                 // iteration index the next B launch runs (written by A)
    int done;                   // nonzero: every launch returns at once
    int status;                 // 0, -3 (no convergence), -4 (non-finite)
    int iterations;             // completed iterations (written by A)
    int active_b;               // conditions still iterating, bit c (written by A, read by B)
    double rel;                 // ||r_G|| / ||S_G|| of the last completed iteration
    double rel_cond[GAP_MAXC];  // per condition
    // one-launch iteration (gap_pcg1.hpp): iteration index and per-condition r.z of the
    // launch's own iteration, both by launch parity (read from [par], written to [par ^ 1])
    int iter_f[2];
    double gam[2][GAP_MAXC];
    // one-launch iteration, also by launch parity: the stop flag and the active mask that the
    // next launch reads (so that no workgroup of a launch sees that launch's own update), and
    // alpha_j per condition (the term a launch of even j leaves pending in p)
    int done_f[2];
    int act_f[2];
    double alf[2][GAP_MAXC];
};

struct PcgDev {
    // operator (face conductances) and diagonal preconditioner, per distinct operator
    const double* kx;           // [n_op][n]
    const double* kz;           // [n_op][n + nt]
    const double* kxz;          // [n_op][n + nt][2]: (kx of row r, kz of face r + 1) at pair r + 1
    const double* minv;         // [n_op][n]  (Jacobi / ASSOR I), or null
    // vectors, condition-major
    const double* S;            // [n_cond][n]
    double* p;                  // [n_cond][n]  caller memory
    double* r[2];               // residual, ping-pong by iteration parity
    double* u[2];               // search direction, ping-pong by iteration parity
    double* z;                  // preconditioned residual
    double* zf[2];              // one-launch iteration: z by iteration parity (zf[0] == z)
    // partial sums, one slot per chunk: slot = c * chunks + k
    double* part_rz[2];         // r.z, parity of the iteration that consumes it as d_j
    double* part_rr;            // ||r||^2
    double* part_ss;            // ||S||^2 (init)
    double* part_uau;           // u^T A u
    // one-launch iteration: partial sums by launch parity, 5 arrays each (r.z, r.r, z^T A z,
    // z^T A u, u^T A u) of fstride slots
    double* fpart[2];
    int fstride;
    int par_off;                // one-launch iteration: the request's iteration parity is the
                                // launch parity xor par_off (batches; 0 for a solve of its own)
    double* hist;               // or null: alpha_j at [2j], beta_{j-1} at [2j+1], j < hist_cap
    int hist_cap;               // (measurement: the scalars of condition 0's recurrence)
    PcgScalars* sc;
    int op[GAP_MAXC];
    int nt, nz, n_cond;
    int chunks_a, rows_a;       // row chunks per condition of the A launch
    int chunks_b, rows_b;       // row chunks per condition of the B launches
    double omega, eps;
    double eps_c[GAP_MAXC];     // per-condition tolerance of the asynchronized test (Eq 3.10)
    int max_iter, per_cond, warm, precond;   // precond: 0 Jacobi, 1 ASSOR I, 2 ASSOR II
    int async;                  // 1: each condition stops at its own test (Eq 3.10) and is frozen
    // strip iteration (gap_pcgw.hpp): strips per ring and strip groups (workgroups) per row
    // chunk; chunks_b counts row chunks x groups, rows_b the rows of a row chunk
    int n_strips, strip_groups;
};

// A launch covers one or more joint systems ("requests"), each described by a PcgDev in
// device memory.  Block b takes work entry work[b] = request << 24 | chunk << 4 | condition
// (-1: idle padding) from a schedule table built on the host: workgroups reach the XCDs
// round-robin, and the table places the conditions of a request that share an operator on
// one XCD, so that their face-conductance reads meet in its L2.
// slot = c * chunks + k indexes the request's partial sums.
__device__ __forceinline__ bool pcg_work(const int* work, int b, int& req, int& c, int& k)
{
    const int w = work[b];
    if (w < 0) return false;
    req = w >> 24;
    k = (w >> 4) & 0xFFFFF;
    c = w & 15;
    return true;
}

// Per-condition sums of up to NQ partial arrays, in a fixed order: wave w handles
// conditions w, w + NW, ...; lane l adds slots l, l + 64, ... to a zero start, then a fixed
// shuffle tree.  The loads of one round of 64 slots go out for all arrays together, so a
// condition waits for one memory latency per round, not one per array.  Results land in
// out[q][c] (shared memory), valid after the trailing barrier.
template <int NT, int NQ>
__device__ __forceinline__ void cond_sums(int n_cond, const int (&chunks)[NQ], const double* const (&src)[NQ],
                                          double (*out)[GAP_MAXC])
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int kmax = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) kmax = chunks[q] > kmax ? chunks[q] : kmax;
    for (int c = w; c < n_cond; c += NW) {
        double v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = 0.0;
        for (int k0 = 0; k0 < kmax; k0 += 64) {
            const int k = k0 + lane;
            double x[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) x[q] = k < chunks[q] ? src[q][c * chunks[q] + k] : 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (k < chunks[q]) v[q] += x[q];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) out[q][c] = v[q];
        }
    }
    __syncthreads();
}

// Sum of NV values over the workgroup (fixed order), result valid in thread 0.
template <int NT, int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV])
{
    constexpr int NW = NT / 64;
    __shared__ double part[NV][NW];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = part[k][0];
            for (int i = 1; i < NW; ++i) s += part[k][i];
            v[k] = s;
        }
    }
}

// ---------------------------------------------------------------------------------------
// A(j): u = z + beta u_prev, partial u^T A u.
// Register budgets: at least 4 waves per SIMD (<= 128 VGPRs) for A and for B with up to two
// columns per thread; B with four columns per thread keeps 20 row values per column live and
// runs at 2 waves per SIMD.
template <int NT, int Q>
__global__ __launch_bounds__(NT, 4) void k_pcg_a(const PcgDev* __restrict__ reqs, const int* __restrict__ work)
{
    int req, c, kc;
    if (!pcg_work(work, blockIdx.x, req, c, kc)) return;
    const PcgDev& a = reqs[req];
    if (a.sc->done) return;
    const int j0 = kc * a.rows_a, j1 = min(j0 + a.rows_a, a.nz), slot = c * a.chunks_a + kc;
    const bool writer = (c == 0 && kc == 0);   // publishes the request's device record
    // A condition frozen by the asynchronized test stays frozen: skip it before any load
    // (the mask of the previous iteration; the writer always runs)
    if (a.async && !writer && !((a.sc->active_b >> c) & 1)) return;
    const int j = a.sc->iter_a;
    const int nt = a.nt, nz = a.nz;
    const size_t n = (size_t)nt * nz;

    // ---- rows of the chunk: operands of the first rows (issued before the scalars) -----
    extern __shared__ double lds[];
    double* su = lds;             // [2][nt]  u of the current row, by row parity
    const int op = a.op[c];
    const GAP_AS1 double* kx = as_global(a.kx + (size_t)op * n);
    const GAP_AS1 double* kz = as_global(a.kz + (size_t)op * (n + nt));
    const GAP_AS1 double* zc = as_global(a.z + (size_t)c * n);
    const GAP_AS1 double* ui = as_global(a.u[(j + 1) & 1] + (size_t)c * n);
    GAP_AS1 double* uo = as_global(a.u[j & 1] + (size_t)c * n);
    const bool first = (j == 0);
    const int t = threadIdx.x;

    // registers: u of rows s-1, s, s+1; face conductances of faces s, s+1; kx of row s at
    // the own and at the western column (periodic; a second load of the same cache lines).
    // The loads of the next PF row steps are in flight in the stages: stage k holds row step
    // s + 1 + k (kx of that row, its northern face, z and u_prev of the row after it).  Two
    // steps ahead where registers allow: a row step of this kernel moves little data, so one
    // step of lead does not cover the memory latency.
    constexpr int PF = (Q <= 2) ? 2 : 1;
    double um[Q], uc[Q], up[Q], kzS[Q], kzN[Q], kxc[Q], kwc[Q];
    double pz[PF][Q], pu[PF][Q], pkx[PF][Q], pkw[PF][Q], pkz[PF][Q];
    // the loads of the first rows do not depend on the scalars: they are issued before the
    // reduction below and combined with beta after it (um/uc/up hold z, um_/uc_/up_ u_prev)
    double um_[Q], uc_[Q], up_[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = t + q * NT;
        const int dw = i ? -1 : nt - 1;
        um[q] = uc[q] = up[q] = kzS[q] = kzN[q] = kxc[q] = kwc[q] = 0.0;
        um_[q] = uc_[q] = up_[q] = 0.0;
#pragma unroll
        for (int k = 0; k < PF; ++k) pz[k][q] = pu[k][q] = pkx[k][q] = pkw[k][q] = pkz[k][q] = 0.0;
        if (i < nt) {
            if (j0 > 0) {
                const size_t g = (size_t)(j0 - 1) * nt + i;
                um[q] = zc[g];
                if (!first) um_[q] = ui[g];
            }
            size_t g = (size_t)j0 * nt + i;
            uc[q] = zc[g];
            if (!first) uc_[q] = ui[g];
            kzS[q] = kz[g];
            kxc[q] = kx[g];
            kwc[q] = kx[g + dw];
            g += nt;
            kzN[q] = kz[g];
            if (j0 + 1 < nz) {
                up[q] = zc[g];
                if (!first) up_[q] = ui[g];
            }
        }
    }
    // prologue: stages 0 .. PF-2 receive row steps j0+1 .. j0+PF-1
#pragma unroll
    for (int k = 0; k < PF - 1; ++k) {
        const int r = j0 + 1 + k;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt && r < j1) {
                const size_t g1 = (size_t)r * nt + i;
                pkx[k][q] = kx[g1];
                pkw[k][q] = kx[g1 + (i ? -1 : nt - 1)];
                pkz[k][q] = kz[g1 + nt];
                if (r + 1 < nz) {
                    pz[k][q] = zc[g1 + nt];
                    if (!first) pu[k][q] = ui[g1 + nt];
                }
            }
        }
    }
    // ---- scalars: beta_{j-1} = d_j / d_{j-1}, stopping test on ||r_j|| -----------------
    __shared__ double sums[4][GAP_MAXC];
    {
        const double* src[4] = {a.part_rz[j & 1], a.part_rz[(j + 1) & 1], a.part_rr, a.part_ss};
        const int cnt[4] = {a.chunks_b, a.chunks_b, a.chunks_b, a.chunks_b};
        cond_sums<NT, 4>(a.n_cond, cnt, src, sums);
    }
    // Active conditions: all (synchronized test, Eq 3.9) or those whose own relative residual
    // is above eps (asynchronized test, Eq 3.10; a converged condition is frozen, so its
    // residual and the decision stay fixed).  Scalars of the joint recurrence run over the
    // active conditions.
    unsigned active = 0;
    double dn = 0.0, dp = 0.0, rr = 0.0, ss = 0.0;
    for (int k = 0; k < a.n_cond; ++k) {
        const double sk = sums[3][k] > 0.0 ? sums[3][k] : 1.0;
        const bool act = !a.async || sqrt(sums[2][k] / sk) > a.eps_c[k];
        if (act) {
            active |= 1u << k;
            dn += sums[0][k];
            dp += sums[1][k];
        }
        rr += sums[2][k];
        ss += sums[3][k];
    }
    const double rel = sqrt(rr / (ss > 0.0 ? ss : 1.0));
    double beta = 0.0;
    if (j > 0) beta = a.per_cond ? sums[0][c] / sums[1][c] : dn / dp;
    bool bad = !finite_d(rel);
    if (j > 0)
        for (int k = 0; k < a.n_cond; ++k)
            if (active & (1u << k)) bad |= !finite_d(a.per_cond ? sums[0][k] / sums[1][k] : dn / dp);
    const bool converged = a.async ? (active == 0) : (rel <= a.eps);
    const bool stop = bad || converged || j >= a.max_iter;
    if (writer && threadIdx.x == 0) {
        PcgScalars* s = a.sc;
        s->iterations = j;
        s->rel = rel;
        for (int k = 0; k < a.n_cond; ++k) {
            const double sk = sums[3][k] > 0.0 ? sums[3][k] : 1.0;
            s->rel_cond[k] = sqrt(sums[2][k] / sk);
        }
        s->iter_b = j;
        s->active_b = (int)active;
        s->status = bad ? -4 : (converged ? 0 : (j >= a.max_iter ? -3 : 0));
        if (stop) s->done = 1;
        if (a.hist && !stop && j < a.hist_cap) a.hist[2 * j + 1] = beta;
    }
    if (stop || !(active & (1u << c))) return;

    // u = z + beta u_prev on the first rows
    if (!first) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] += beta * um_[q];
            uc[q] += beta * uc_[q];
            up[q] += beta * up_[q];
        }
    }
    double acc = 0.0;
    for (int s = j0; s < j1; ++s) {
        const int buf = s & 1;
        // issue the loads of row step s + PF into the last stage
        {
            const int r = s + PF;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = t + q * NT;
                if (i < nt && r < j1) {
                    const size_t g1 = (size_t)r * nt + i;
                    pkx[PF - 1][q] = kx[g1];
                    pkw[PF - 1][q] = kx[g1 + (i ? -1 : nt - 1)];
                    pkz[PF - 1][q] = kz[g1 + nt];
                    if (r + 1 < nz) {
                        pz[PF - 1][q] = __builtin_nontemporal_load(&zc[g1 + nt]);
                        if (!first) pu[PF - 1][q] = __builtin_nontemporal_load(&ui[g1 + nt]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt) su[buf * nt + i] = uc[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt) {
                const int iw = i ? i - 1 : nt - 1;
                const int ie = (i + 1 < nt) ? i + 1 : 0;
                const double kW = kwc[q];
                const double D = ((kxc[q] + kW) + kzS[q]) + kzN[q];
                double v = D * uc[q] - kxc[q] * su[buf * nt + ie] - kW * su[buf * nt + iw];
                if (s > 0) v -= kzS[q] * um[q];
                if (s < nz - 1) v -= kzN[q] * up[q];
                acc += uc[q] * v;
                __builtin_nontemporal_store(uc[q], &uo[(size_t)s * nt + i]);
            }
        }
        // advance one row: the current state takes stage 0 (row step s + 1), the stages shift
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] = uc[q];
            uc[q] = up[q];
            kzS[q] = kzN[q];
            kzN[q] = pkz[0][q];
            kxc[q] = pkx[0][q];
            kwc[q] = pkw[0][q];
            up[q] = (s + 2 < nz) ? (first ? pz[0][q] : pz[0][q] + beta * pu[0][q]) : 0.0;
#pragma unroll
            for (int k = 0; k + 1 < PF; ++k) {
                pz[k][q] = pz[k + 1][q];
                pu[k][q] = pu[k + 1][q];
                pkx[k][q] = pkx[k + 1][q];
                pkw[k][q] = pkw[k + 1][q];
                pkz[k][q] = pkz[k + 1][q];
            }
        }
    }
    double v1[1] = {acc};
    wg_sum<NT, 1>(v1);
    if (threadIdx.x == 0) a.part_uau[slot] = v1[0];
}

// ---------------------------------------------------------------------------------------
// B(j) (INIT = false) or the initial residual (INIT = true).
template <int NT, int Q, bool INIT>
__global__ __launch_bounds__(NT, (Q >= 4 ? 2 : 4)) void k_pcg_b(const PcgDev* __restrict__ reqs, const int* __restrict__ work)
{
    int req, c, kc;
    if (!pcg_work(work, blockIdx.x, req, c, kc)) return;
    const PcgDev& a = reqs[req];
    if (!INIT && a.sc->done) return;
    const int j0 = kc * a.rows_b, j1 = min(j0 + a.rows_b, a.nz), slot = c * a.chunks_b + kc;
    const bool writer = (c == 0 && kc == 0);   // publishes the request's device record
    if (!INIT && !writer && !((a.sc->active_b >> c) & 1)) return;   // frozen condition
    const int j = INIT ? -1 : a.sc->iter_b;
    const int nt = a.nt, nz = a.nz;
    const size_t n = (size_t)nt * nz;

    // ---- operands of the first rows: they do not depend on alpha and are issued before the
    // reduction of the scalars ------------------------------------------------------------
    const bool spmv = !INIT || a.warm;
    const bool assor = (a.precond == 2);
    const int op = a.op[c];
    const GAP_AS1 double* kx = as_global(a.kx + (size_t)op * n);
    const GAP_AS1 double* kz = as_global(a.kz + (size_t)op * (n + nt));
    const GAP_AS1 double* mv = as_global(assor ? a.kx : a.minv + (size_t)op * n);   // read only when !assor
    const GAP_AS1 double* uu = as_global((INIT ? a.p : a.u[j & 1]) + (size_t)c * n);
    const GAP_AS1 double* rin = as_global((INIT ? a.S : a.r[j & 1]) + (size_t)c * n);
    GAP_AS1 double* rout = as_global(a.r[(j + 1) & 1] + (size_t)c * n);
    GAP_AS1 double* pp = as_global(a.p + (size_t)c * n);
    GAP_AS1 double* zz = as_global(a.z + (size_t)c * n);
    const double om = a.omega;
    const double scale = om * (2.0 - om);

    extern __shared__ double lds[];
    double* su = lds;             // u row s
    double* sy = lds + nt;        // y = D^-1 r' row s
    double* sv = lds + 2 * nt;    // [2][nt]: (I - w D^-1 L) y, rows by parity

    // rows visited: the chunk plus, for the ASSOR sweeps, one halo row on each side
    const int s_begin = assor ? max(j0 - 1, 0) : j0;
    const int s_last = assor ? min(j1, nz - 1) : j1 - 1;
    const bool updates_p = !INIT || !a.warm;   // B writes p += alpha u; cold init writes p = 0

    const int t = threadIdx.x;
    // state of rows s-1, s, s+1 and of the row below (for the lagged Eq 3.6 sweep); kwc is
    // kx of the western column (periodic), a second load of the same cache lines as kxc
    double um[Q], uc[Q], up[Q], kzS[Q], kzN[Q], kxc[Q], kwc[Q], rc[Q], pc[Q];
    double yprev[Q], vprev[Q], dinvprev[Q], kxprev[Q], rpprev[Q];
    // loads of the next row step, issued one step ahead
    double nu[Q], nkx[Q], nkw[Q], nkz[Q], nr[Q], np[Q];
    double kxwrap_prev = 0.0;     // thread 0: kx(nt-1) of the previous row, the west wrap of column 0
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = t + q * NT;
        um[q] = uc[q] = up[q] = kzS[q] = kzN[q] = kxc[q] = kwc[q] = rc[q] = pc[q] = 0.0;
        yprev[q] = vprev[q] = dinvprev[q] = kxprev[q] = rpprev[q] = 0.0;
        nu[q] = nkx[q] = nkw[q] = nkz[q] = nr[q] = np[q] = 0.0;
        if (i < nt) {
            const size_t g = (size_t)s_begin * nt + i;
            if (spmv) {
                if (s_begin > 0) um[q] = uu[g - nt];
                uc[q] = uu[g];
                if (s_begin + 1 < nz) up[q] = uu[g + nt];
            }
            kzS[q] = kz[g];
            kzN[q] = kz[g + nt];
            kxc[q] = kx[g];
            kwc[q] = kx[g + (i ? -1 : nt - 1)];
            rc[q] = rin[g];
            if (!INIT && s_begin >= j0) pc[q] = __builtin_nontemporal_load(&pp[g]);
        }
    }
    // ---- scalars: alpha_j = d_j / (u_j^T A u_j) ------------------------------------------
    double alpha = 1.0;
    if (!INIT) {
        __shared__ double sums[2][GAP_MAXC];
        const double* src[2] = {a.part_rz[j & 1], a.part_uau};
        const int cnt[2] = {a.chunks_b, a.chunks_a};
        cond_sums<NT, 2>(a.n_cond, cnt, src, sums);
        const unsigned active = (unsigned)a.sc->active_b;
        double num = 0.0, den = 0.0;
        bool bad = false;
        for (int k = 0; k < a.n_cond; ++k) {
            if (!(active & (1u << k))) continue;
            num += sums[0][k];
            den += sums[1][k];
            if (a.per_cond) bad |= !finite_d(sums[0][k] / sums[1][k]);
        }
        if (!a.per_cond) bad |= !finite_d(num / den);
        alpha = a.per_cond ? sums[0][c] / sums[1][c] : num / den;
        if (bad) {
            if (writer && threadIdx.x == 0) {
                a.sc->status = -4;
                a.sc->done = 1;
            }
            return;
        }
        if (writer && threadIdx.x == 0) {
            a.sc->iter_a = j + 1;
            if (a.hist && j < a.hist_cap) a.hist[2 * j] = alpha;
        }
        if (!(active & (1u << c))) return;
    } else if (writer && threadIdx.x == 0) {
        a.sc->iter_a = 0;
        a.sc->iter_b = 0;
        a.sc->done = 0;
        a.sc->status = 0;
        a.sc->iterations = 0;
        a.sc->active_b = (1 << a.n_cond) - 1;
    }

    double acc_rz = 0.0, acc_rr = 0.0, acc_ss = 0.0;

    for (int s = s_begin; s <= s_last; ++s) {
        const bool own = (s >= j0 && s < j1);
        // issue the loads of row s + 1 (u of row s + 2, face s + 2)
        if (s + 1 <= s_last) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = t + q * NT;
                if (i < nt) {
                    const size_t g1 = (size_t)(s + 1) * nt + i;
                    nu[q] = (spmv && s + 2 < nz) ? uu[g1 + nt] : 0.0;
                    nkx[q] = kx[g1];
                    nkw[q] = kx[g1 + (i ? -1 : nt - 1)];
                    nkz[q] = kz[g1 + nt];
                    nr[q] = rin[g1];
                    np[q] = (!INIT && s + 1 >= j0 && s + 1 < j1) ? __builtin_nontemporal_load(&pp[g1]) : 0.0;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt) su[i] = uc[q];
        }
        __syncthreads();
        double rp[Q], dinv[Q], y[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            rp[q] = dinv[q] = y[q] = 0.0;
            if (i < nt) {
                const size_t g = (size_t)s * nt + i;
                const int iw = i ? i - 1 : nt - 1;
                const int ie = (i + 1 < nt) ? i + 1 : 0;
                const double kW = kwc[q];
                const double D = ((kxc[q] + kW) + kzS[q]) + kzN[q];
                const double r0 = rc[q];
                double r1 = r0;
                if (spmv) {
                    double v = D * uc[q] - kxc[q] * su[ie] - kW * su[iw];
                    if (s > 0) v -= kzS[q] * um[q];
                    if (s < nz - 1) v -= kzN[q] * up[q];
                    r1 = r0 - alpha * v;
                }
                rp[q] = r1;
                dinv[q] = 1.0 / D;
                if (own) {
                    rout[g] = r1;
                    acc_rr += r1 * r1;
                    if (INIT) acc_ss += r0 * r0;
                    if (updates_p) pp[g] = INIT ? 0.0 : pc[q] + alpha * uc[q];
                    if (!assor) {
                        const double zv = mv[g] * r1;
                        zz[g] = zv;
                        acc_rz += r1 * zv;
                    }
                }
                if (assor) {
                    y[q] = r1 * dinv[q];
                    sy[i] = y[q];
                }
            }
        }
        if (assor) {
            __syncthreads();
            double* svc = sv + (s & 1) * nt;
            const double* svp = sv + ((s + 1) & 1) * nt;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = t + q * NT;
                if (i < nt) {
                    // Eq 3.5: v = y + w D^-1 (couplings to west, south and the east wrap)
                    double lo = 0.0;
                    if (i > 0) lo += kwc[q] * sy[i - 1];
                    if (i == nt - 1) lo += kxc[q] * sy[0];
                    if (s > 0) lo += kzS[q] * yprev[q];
                    const double v = y[q] + om * dinv[q] * lo;
                    svc[i] = v;
                    // Eq 3.6 for the row below: z = w(2-w)(v + w D^-1 (east, north, west wrap))
                    if (s - 1 >= j0 && s - 1 < j1) {
                        double hi = kzS[q] * v;
                        if (i < nt - 1) hi += kxprev[q] * svp[i + 1];
                        if (i == 0) hi += kxwrap_prev * svp[nt - 1];
                        const double zv = scale * (vprev[q] + om * dinvprev[q] * hi);
                        __builtin_nontemporal_store(zv, &zz[(size_t)(s - 1) * nt + i]);
                        acc_rz += rpprev[q] * zv;
                    }
                    yprev[q] = y[q];
                    vprev[q] = v;
                }
            }
        } else {
            __syncthreads();   // the LDS rows are rewritten by the next row step
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            um[q] = uc[q];
            uc[q] = up[q];
            up[q] = nu[q];
            kzS[q] = kzN[q];
            kzN[q] = nkz[q];
            dinvprev[q] = dinv[q];
            kxprev[q] = kxc[q];
            kxc[q] = nkx[q];
            rpprev[q] = rp[q];
            rc[q] = nr[q];
            pc[q] = np[q];
        }
        kxwrap_prev = kwc[0];
#pragma unroll
        for (int q = 0; q < Q; ++q) kwc[q] = nkw[q];
    }
    // last row of the ring: no northern neighbour
    if (assor && j1 == nz) {
        __syncthreads();
        const double* svp = sv + ((nz - 1) & 1) * nt;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + q * NT;
            if (i < nt) {
                double hi = 0.0;
                if (i < nt - 1) hi += kxprev[q] * svp[i + 1];
                if (i == 0) hi += kxwrap_prev * svp[nt - 1];
                const double zv = scale * (vprev[q] + om * dinvprev[q] * hi);
                __builtin_nontemporal_store(zv, &zz[(size_t)(nz - 1) * nt + i]);
                acc_rz += rpprev[q] * zv;
            }
        }
    }
    double v3[3] = {acc_rz, acc_rr, acc_ss};
    wg_sum<NT, 3>(v3);
    if (threadIdx.x == 0) {
        a.part_rz[(j + 1) & 1][slot] = v3[0];
        a.part_rr[slot] = v3[1];
        if (INIT) a.part_ss[slot] = v3[2];
    }
}
