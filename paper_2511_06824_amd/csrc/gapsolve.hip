// Host side of the gapsolve C ABI: handle management, validation, launches and the device-
// resident PCG loop.  See include/gapsolve.h for the contract of every entry point.
#include "gapsolve.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gap_kernels.hpp"
#include "gap_pcg.hpp"
#include "gap_pcg1.hpp"
#include "gap_pcgw.hpp"
#include "gap_adjoint.hpp"

namespace {

thread_local std::string g_err;

gap_status fail(gap_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(GAP_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));              \
    } while (0)

#define HIPLAUNCHCHK(what)                                                                  \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess)                                                               \
            return fail(GAP_EDEVICE, "launch of %s: %s", what, hipGetErrorString(e_));     \
    } while (0)

bool is_finite(double x) { return std::isfinite(x); }

// A handle in a batch lends its Krylov buffers and device record to the batch: no other use
// until gap_batch_remove.
#define GAP_NOT_IN_BATCH(g, what)                                                                  \
    do {                                                                                           \
        if ((g)->batch) return fail(GAP_ESTATE, "%s on a grid that is in a batch (gap_batch_remove it first)", what); \
    } while (0)

constexpr int kTargetChunks = 2048;
constexpr int kMaxThetaCells = 16384;
constexpr int kMaxRingCells = 2048;     // kernels whose workgroups hold whole rings
constexpr int kMaxAxialCells = 65536;

ChunkMap make_chunks(int nz, int n_cond)
{
    ChunkMap cm;
    int per = (kTargetChunks + n_cond - 1) / n_cond;
    if (per > nz) per = nz;
    cm.rows = (nz + per - 1) / per;
    cm.per_cond = (nz + cm.rows - 1) / cm.rows;
    cm.total = cm.per_cond * n_cond;
    return cm;
}

// Kernel shape of the PCG iteration kernels: NT threads per workgroup, Q ring columns per
// thread (thread t handles columns t, t + NT, ...), NT * Q >= n_theta.
struct PcgShape {
    int NT = 512, Q = 4;
    int pk = -1;    // strip kernel: the preconditioner compiled in (-1: read from each request)
    int M = 1;      // strip kernel: the Neumann order of ASSOR II
    int sync = 0;   // strip kernel at order 1: the march with a workgroup barrier per period
};

// Every instantiated shape.
#define GAP_PCG_SHAPES(X) \
    X(64, 1) X(128, 1) X(128, 2) X(256, 1) X(256, 2) X(256, 4) X(512, 1) X(512, 2) X(512, 4) X(1024, 1) X(1024, 2)

bool shape_known(PcgShape sh)
{
#define GAP_SHAPE_CASE(nt_, q_) if (sh.NT == nt_ && sh.Q == q_) return true;
    GAP_PCG_SHAPES(GAP_SHAPE_CASE)
#undef GAP_SHAPE_CASE
    return false;
}

// Candidate shapes for a ring of nt cells, the default first: at most one idle column slot
// in two, and wavefront-multiple workgroups.
std::vector<PcgShape> pcg_candidates(int nt)
{
    if (nt <= 64) return {{64, 1}};
    if (nt <= 128) return {{128, 1}};
    if (nt <= 256) return {{256, 1}, {128, 2}};
    if (nt <= 512) return {{512, 1}, {256, 2}};
    if (nt <= 1024) return {{512, 2}, {1024, 1}, {256, 4}};
    return {{1024, 2}, {512, 4}};        // n_theta <= 2048 (validated at create)
}

// Kernels of the PCG iteration, by the `which` argument of the launch helpers.
enum { kPcgA = 0, kPcgB = 1, kPcgInit = 2, kPcgOne = 3, kPcgOneInit = 4, kPcgStrip = 5, kPcgStripInit = 6 };

// Dynamic LDS: A (u row, double-buffered); B and its init (u and y rows, two rows of the
// first ASSOR sweep); the one-launch kernel and its init (those four, two z rows and a ring
// of three rows of east-face conductances).
size_t pcg_lds_bytes(int which, int nt)
{
    const int rows = which == kPcgA ? 2 : (which <= kPcgInit ? 4 : 9);
    return (size_t)rows * nt * sizeof(double);
}

// Row chunks per condition: as many workgroups as the device holds at once (occupancy x CUs),
// so that one launch runs in a single round; but at least kMinChunkCells cells per chunk and
// at most kMaxChunks workgroups per request.  Every workgroup reduces all chunk partials of
// its request at its start (work ~ NQ x chunks^2 per launch), and a chunk of a row or two is
// mostly halo: narrow rings (small n_theta) would otherwise get thousands of one-row chunks.
constexpr int kMinChunkCells = 1024;
constexpr int kMaxChunks = 1024;

void pcg_chunks(int nz, int nt, int n_cond, int slots, int& chunks, int& rows)
{
    int per = std::min(slots, kMaxChunks) / n_cond;
    const int min_rows = (kMinChunkCells + nt - 1) / nt;
    per = std::min(per, std::max(1, nz / min_rows));
    if (per < 1) per = 1;
    if (per > nz) per = nz;
    rows = (nz + per - 1) / per;
    chunks = (nz + rows - 1) / rows;
}

// Packed work entry of a PCG launch: request << 24 | chunk << 4 | condition.
inline int pcg_entry(int req, int k, int c) { return (req << 24) | (k << 4) | c; }

// Work groups of one request: per run of `span` consecutive chunk slots, the conditions that
// share an operator.  span = 1 for the whole-ring kernels; the strip kernel passes its strip
// groups per row chunk, so that the workgroups of one row chunk, whose strips read each
// other's edge columns, land on one XCD with the conditions that share their operator.
void pcg_groups(int req, int chunks, int n_cond, const int* op, std::vector<std::vector<int>>& groups, int span = 1)
{
    for (int k0 = 0; k0 < chunks; k0 += span) {
        std::vector<std::vector<int>> by_op(GAP_MAXC);
        for (int k = k0; k < std::min(k0 + span, chunks); ++k)
            for (int c = 0; c < n_cond; ++c) by_op[op[c]].push_back(pcg_entry(req, k, c));
        for (auto& gcl : by_op)
            if (!gcl.empty()) groups.push_back(gcl);
    }
}

// Schedule table of one PCG launch.  Workgroup b is dispatched to XCD b % 8.  Groups go
// largest first to the least loaded XCD and stay on it (the conditions in a group read the
// same operator, so the repeats hit that XCD's L2) as far as they fit: no XCD takes more than
// its even share, ceil(entries / 8), so that a launch that fills the chip in one round does
// so on every XCD; the part of a group beyond that share goes on to the next least loaded
// XCD.  Idle entries (-1) pad the XCD lists to equal length.
std::vector<int> pcg_schedule(std::vector<std::vector<int>> groups)
{
    constexpr int X = 8;
    std::vector<std::vector<int>> lists(X);
    std::vector<int> load(X, 0);
    std::stable_sort(groups.begin(), groups.end(),
                     [](const std::vector<int>& x, const std::vector<int>& y) { return x.size() > y.size(); });
    size_t total = 0;
    for (const auto& gcl : groups) total += gcl.size();
    const int share = (int)((total + X - 1) / X);
    for (const auto& gcl : groups) {
        size_t i = 0;
        while (i < gcl.size()) {
            int best = 0;
            for (int x = 1; x < X; ++x)
                if (load[x] < load[best]) best = x;
            const size_t take = std::min(gcl.size() - i, (size_t)std::max(1, share - load[best]));
            for (size_t m = 0; m < take; ++m) lists[best].push_back(gcl[i + m]);
            load[best] += (int)take;
            i += take;
        }
    }
    size_t len = 0;
    for (auto& l : lists) len = std::max(len, l.size());
    std::vector<int> table(X * len, -1);
    for (int x = 0; x < X; ++x)
        for (size_t m = 0; m < lists[x].size(); ++m) table[m * X + x] = lists[x][m];
    return table;
}

// ---- strip kernel (gap_pcgw.hpp): shape = (kStripThreads, Q columns per lane) ----------
// One column per lane only: with two, the unrolled row march needs more than the 256 VGPRs a
// lane has and spills (three times slower).
constexpr int kStripMaxQ = 1;
constexpr int kStripDefaultQ = 1;
constexpr int kMinStripRows = 16;      // a row chunk recomputes 7 halo rows
// A request that streams at least this many bytes per iteration runs the order-1 strip
// kernel whose wavefronts meet at a barrier once per period: 3 % faster on the 9-condition
// 2048 x 1024 system (0.92 GB per iteration).  Where the vectors and operators fit the
// 256 MB last-level cache the barrier only costs: 1024 x 512 (0.23 GB) runs 3-5 % faster
// without it.  Both forms compute the same values in the same order.
constexpr double kStripSyncBytes = 512.0 * 1024 * 1024;

// Bytes the strip iteration streams for a request per launch: 40 B per condition-DOF on
// average (r and u_prev read, u and r' written, p every other launch) and 16 B per
// operator-DOF (the conductance pairs).
inline double strip_request_bytes(const PcgDev& a)
{
    int n_op = 0;
    for (int c = 0; c < a.n_cond; ++c) n_op = std::max(n_op, a.op[c] + 1);
    return (double)a.nt * a.nz * (40.0 * a.n_cond + 16.0 * n_op);
}

// Whether a request of order M runs the synchronized march.
inline bool strip_sync(int M, const PcgDev& a) { return M == 1 && strip_request_bytes(a) >= kStripSyncBytes; }

bool strip_q_known(int Q) { return Q >= 1 && Q <= kStripMaxQ; }

// Columns per lane the strip kernel runs with for the configured Q and Neumann order M: order
// 3 has one column per lane only.
inline int strip_q(int Q, int M) { return M >= 3 ? 1 : Q; }

// Strips per ring and strip groups (workgroups of kStripWaves strips) per row chunk, for Q
// columns per lane and Neumann order M.
void strip_layout(int nt, int Q, int M, int& strips, int& groups)
{
    const int w = strip_owned_max(Q, M);
    strips = (nt + w - 1) / w;
    groups = (strips + kStripWaves - 1) / kStripWaves;
}

// Row chunks of a strip launch: about `slots` workgroups in all (occupancy x CUs, a single
// round), at least kMinStripRows rows per chunk, at most kMaxChunks partial-sum slots per
// request and at most n_axial per condition (the partial arrays hold that many).
void strip_chunks(int nz, int nt, int n_cond, int Q, int M, int slots, PcgDev& a)
{
    int strips = 1, groups = 1;
    strip_layout(nt, Q, M, strips, groups);
    int per = slots / (n_cond * groups);
    per = std::min(per, std::max(1, nz / kMinStripRows));
    per = std::min(per, std::max(1, nz / groups));
    per = std::min(per, std::max(1, kMaxChunks / (n_cond * groups)));
    if (per < 1) per = 1;
    const int rows = (nz + per - 1) / per;
    const int chunks = (nz + rows - 1) / rows;
    a.n_strips = strips;
    a.strip_groups = groups;
    a.rows_b = a.rows_a = rows;
    a.chunks_b = a.chunks_a = chunks * groups;
}

// The strip kernels of Q columns per lane: the initial residual (preconditioner read from
// the request) for each Neumann order, and the iteration for each preconditioner, fixed or
// read from the request; ASSOR II with Neumann orders 1 .. kStripMaxNeumann.
template <int Q>
const void* strip_fn(bool init, int pk, int M, bool sync = false)
{
    // two columns per lane at order 3 would spill most of its registers: not instantiated
    if (Q >= 2 && M >= 3) return nullptr;
    if (sync) {
        if (M != 1) return nullptr;
        if (init) return (const void*)k_pcg_w<Q, -1, 1, true, true>;
        switch (pk) {
        case 0: return (const void*)k_pcg_w<Q, 0, 1, false, true>;
        case 1: return (const void*)k_pcg_w<Q, 1, 1, false, true>;
        case 2: return (const void*)k_pcg_w<Q, 2, 1, false, true>;
        default: return (const void*)k_pcg_w<Q, -1, 1, false, true>;
        }
    }
    if (init) {
        switch (M) {
        case 1: return (const void*)k_pcg_w<Q, -1, 1, true>;
        case 2: return (const void*)k_pcg_w<Q, -1, 2, true>;
        case 3: return (const void*)k_pcg_w<(Q < 2 ? Q : 1), -1, 3, true>;
        default: return nullptr;
        }
    }
    if (pk == 2) {
        switch (M) {
        case 1: return (const void*)k_pcg_w<Q, 2, 1, false>;
        case 2: return (const void*)k_pcg_w<Q, 2, 2, false>;
        case 3: return (const void*)k_pcg_w<(Q < 2 ? Q : 1), 2, 3, false>;
        default: return nullptr;
        }
    }
    if (M != 1) return nullptr;
    switch (pk) {
    case 0: return (const void*)k_pcg_w<Q, 0, 1, false>;
    case 1: return (const void*)k_pcg_w<Q, 1, 1, false>;
    default: return (const void*)k_pcg_w<Q, -1, 1, false>;
    }
}

template <int Q>
hipError_t strip_prepare_t(int M, int* occupancy)
{
    // the occupancy of the ASSOR II iteration of order M and of its initial residual, in
    // both forms of the march at order 1
    int occ = 1 << 20;
    for (int sync = 0; sync < (M == 1 ? 2 : 1); ++sync)
        for (int init = 0; init < 2; ++init) {
            int nb = 0;
            const void* fn = strip_fn<Q>(init != 0, 2, M, sync != 0);
            if (!fn) return hipErrorInvalidValue;
            const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kStripThreads, 0);
            if (e != hipSuccess) return e;
            occ = std::min(occ, nb > 0 ? nb : 1);
        }
    *occupancy = occ;
    return hipSuccess;
}

// Workgroups of the strip kernel of order M (and its initial residual) that fit on one CU.
hipError_t strip_prepare(int Q, int M, int* occupancy)
{
    switch (Q) {
    case 1: return strip_prepare_t<1>(M, occupancy);
    default: return hipErrorInvalidValue;
    }
}

// pk: the preconditioner of every request in the launch (0, 1, 2), or -1 if they differ;
// M: their Neumann order; sync: the march with a barrier per period (order 1).
hipError_t launch_strip(int Q, int pk, int M, bool sync, bool init, const PcgDev* reqs, const int* work, int blocks,
                        hipStream_t st, int par)
{
    const void* fn = nullptr;
    switch (Q) {
    case 1: fn = strip_fn<1>(init, pk, M, sync); break;
    default: return hipErrorInvalidValue;
    }
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {(void*)&reqs, (void*)&work, (void*)&par};
    return hipLaunchKernel(fn, dim3(blocks), dim3(kStripThreads), args, 0, st);
}

template <int NT, int Q>
const void* pcg_fn(int which)
{
    switch (which) {
    case kPcgA: return (const void*)k_pcg_a<NT, Q>;
    case kPcgB: return (const void*)k_pcg_b<NT, Q, false>;
    case kPcgInit: return (const void*)k_pcg_b<NT, Q, true>;
    case kPcgOne: return (const void*)k_pcg_f<NT, Q, false>;
    default: return (const void*)k_pcg_f<NT, Q, true>;
    }
}

template <int NT, int Q>
hipError_t pcg_prepare_t(int which, int nt, int* occupancy)
{
    const void* fn = pcg_fn<NT, Q>(which);
    const size_t lds = pcg_lds_bytes(which, nt);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)pcg_lds_bytes(which, NT * Q));
    if (e != hipSuccess) return e;
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, NT, lds);
    if (e != hipSuccess) return e;
    *occupancy = nb > 0 ? nb : 1;
    return hipSuccess;
}

template <int NT, int Q>
hipError_t launch_pcg_t(int which, int lds_nt, const PcgDev* reqs, const int* work, int blocks, hipStream_t st,
                        int par)
{
    const size_t lds = pcg_lds_bytes(which, lds_nt);
    switch (which) {
    case kPcgA: hipLaunchKernelGGL((k_pcg_a<NT, Q>), dim3(blocks), dim3(NT), lds, st, reqs, work); break;
    case kPcgB: hipLaunchKernelGGL((k_pcg_b<NT, Q, false>), dim3(blocks), dim3(NT), lds, st, reqs, work); break;
    case kPcgInit: hipLaunchKernelGGL((k_pcg_b<NT, Q, true>), dim3(blocks), dim3(NT), lds, st, reqs, work); break;
    case kPcgOne: hipLaunchKernelGGL((k_pcg_f<NT, Q, false>), dim3(blocks), dim3(NT), lds, st, reqs, work, par); break;
    default: hipLaunchKernelGGL((k_pcg_f<NT, Q, true>), dim3(blocks), dim3(NT), lds, st, reqs, work, 0); break;
    }
    return hipGetLastError();
}

// Set the LDS attribute of a kernel of shape sh and read how many of its workgroups fit on
// one CU when its rings have nt cells.
hipError_t pcg_prepare(PcgShape sh, int which, int nt, int* occupancy)
{
#define GAP_SHAPE_CASE(nt_, q_) \
    if (sh.NT == nt_ && sh.Q == q_) return pcg_prepare_t<nt_, q_>(which, nt, occupancy);
    GAP_PCG_SHAPES(GAP_SHAPE_CASE)
#undef GAP_SHAPE_CASE
    return hipErrorInvalidValue;
}

// which: kPcgA = A(j), kPcgB = B(j), kPcgInit = initial residual of the two-launch
// iteration; kPcgOne / kPcgOneInit the one-launch iteration and its initial residual, par
// the launch parity.  lds_nt: the largest ring of the requests in the launch; blocks =
// entries of the work table.
hipError_t launch_pcg(PcgShape sh, int which, int lds_nt, const PcgDev* reqs, const int* work, int blocks,
                      hipStream_t st, int par = 0)
{
    if (which == kPcgStrip || which == kPcgStripInit)
        return launch_strip(sh.Q, sh.pk, sh.M, sh.sync != 0, which == kPcgStripInit, reqs, work, blocks, st, par);
#define GAP_SHAPE_CASE(nt_, q_) \
    if (sh.NT == nt_ && sh.Q == q_) return launch_pcg_t<nt_, q_>(which, lds_nt, reqs, work, blocks, st, par);
    GAP_PCG_SHAPES(GAP_SHAPE_CASE)
#undef GAP_SHAPE_CASE
    return hipErrorInvalidValue;
}

// Capture `iters` iterations into a graph: A, B launch pairs, or (one_which = kPcgOne or
// kPcgStrip) launches of that one-launch kernel with parities par0, par0 ^ 1, ... on work_b.
hipError_t capture_block(hipStream_t cap, int iters, PcgShape sh_a, PcgShape sh_b, int lds_nt, const PcgDev* reqs,
                         const int* work_a,
                         int blocks_a, const int* work_b, int blocks_b, hipGraphExec_t* exec, int one_which = 0,
                         int par0 = 0)
{
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int it = 0; it < iters && le == hipSuccess; ++it) {
        if (one_which) {
            le = launch_pcg(sh_b, one_which, lds_nt, reqs, work_b, blocks_b, cap, (par0 + it) & 1);
            continue;
        }
        le = launch_pcg(sh_a, kPcgA, lds_nt, reqs, work_a, blocks_a, cap);
        if (le == hipSuccess) le = launch_pcg(sh_b, kPcgB, lds_nt, reqs, work_b, blocks_b, cap);
    }
    e = hipStreamEndCapture(cap, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return le != hipSuccess ? le : e;
    }
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return e;
}

}  // namespace

struct gap_grid_s {
    gap_geom geom{};
    GeomDev gd{};
    int nt = 0, nz = 0;
    size_t n = 0;
    int max_cond = 0, max_op = 0;
    int n_cond = 0, n_op = 0;
    bool assembled = false;
    double delta[8] = {0};
    CondDev cd{};
    ChunkMap cm{};
    // device memory
    double *trig = nullptr;                                  // cos_c, sin_c, cos_e, sin_e
    double *tex = nullptr;                                   // centres, east faces, axial faces
    double *dim_dev = nullptr, *dim_host = nullptr;          // dimple parameters for set_gap_dimples (host: pinned)
    int dim_cap = 0;                                         // dimples they hold
    double *kx = nullptr, *kz = nullptr, *minv = nullptr;
    double *kxz = nullptr;                                   // kx and kz as the pairs of k_pair_ops
    double *S = nullptr, *r0 = nullptr, *r1 = nullptr, *u0 = nullptr, *u1 = nullptr, *z = nullptr;
    double *z1 = nullptr;                                    // second z of the one-launch iteration
    double *partial = nullptr;                               // force-integration partials
    double *pcg_part = nullptr;                              // PCG partials: 15 arrays of max_cond * nz (5 two-launch, 2 x 5 one-launch)
    size_t pcg_part_stride = 0;
    PcgScalars *sc = nullptr;
    PcgScalars *sc_host = nullptr;                           // pinned
    struct Sched {                                           // PCG schedule tables (device), by key
        std::vector<int> key;                                // (n_cond, chunks_a, chunks_b, ops...)
        int* table = nullptr;
        int blocks_a = 0, blocks_b = 0;
    };
    std::vector<Sched> scheds;
    PcgDev *req_dev = nullptr, *req_host = nullptr;          // the request record of this handle's launches
    double *adj_rhs = nullptr, *adj_lam = nullptr;           // adjoint right-hand sides and solutions
    double *adj_part = nullptr;                              // sensitivity partials
    double *step_buf = nullptr;                              // general iteration: F (9 x 4) and J (4 x 8)
    double *hist = nullptr;                                  // PCG scalars per iteration (measurement), or null
    int hist_cap = 0;
    gap_batch_s* batch = nullptr;                            // the batch this handle is in (its buffers are lent)
    int cus = 256;                                           // compute units of the device
    PcgShape shape_a{}, shape_b{};                           // PCG kernel shapes in use (A; B and init)
    int occ[3] = {1, 1, 1};                                  // workgroups per CU of the PCG kernels A, B, init
    int wg_a = 1, wg_b = 1;                                  // workgroups per CU the row chunking targets
    PcgShape shape_f{};                                      // the one-launch kernel (and its init)
    int occ_f = 1, wg_f = 1;
    PcgShape shape_w{kStripThreads, kStripDefaultQ};         // the strip kernel (and its init)
    int occ_w = 1, wg_w = 1;
    int occ_wm[kStripMaxQ + 1][kStripMaxNeumann + 1] = {};  // strip occupancy by (Q, Neumann order), 0: not asked yet
    bool rings_ok = true;                                    // n_theta fits the whole-ring kernels
    int lds_max = 65536;                                     // bytes of LDS one workgroup may use
    int minv_kind = -1;
    double minv_omega = 0.0;
    // kernel timing (measurement support)
    bool timing = false;
    int timing_period = 1;                                   // time one launch in timing_period
    long long ev_tick = 0;                                   // iteration-kernel launches since enabling
    bool ev_open = false;                                    // the current launch is timed
    std::vector<hipEvent_t> ev;                              // pairs: start, stop
    std::vector<int> ev_kind;                                // kernel kind of each used pair
    int ev_used = 0;
    long long launches[GAP_KERNEL_COUNT] = {0};
    double total_ms[GAP_KERNEL_COUNT] = {0};
    // captured iteration blocks (graph replay), by launch arguments; oldest evicted
    struct Graph {
        const int* table = nullptr;                          // schedule the graph was captured with
        int block = 0;
        int par0 = -1;                                       // one-launch: parity of the first launch; -1: two-launch
        hipGraphExec_t exec = nullptr;
    };
    hipStream_t cap_stream = nullptr;
    std::vector<Graph> graphs;

    TablesDev tables() const
    {
        TablesDev t;
        t.cos_c = trig;
        t.sin_c = trig + nt;
        t.cos_e = trig + 2 * nt;
        t.sin_e = trig + 3 * nt;
        t.tex_c = tex;
        t.tex_e = tex + n;
        t.tex_f = tex + 2 * n;
        return t;
    }
};

namespace {

void release(gap_grid_t g)
{
    double* bufs[] = {g->trig, g->tex, g->kx, g->kz, g->kxz, g->minv, g->S, g->r0, g->r1, g->z, g->z1, g->partial,
                      g->pcg_part, g->adj_rhs, g->adj_lam, g->adj_part, g->step_buf, g->hist};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& gr : g->graphs)
        if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    for (auto& sc : g->scheds)
        if (sc.table) (void)hipFree(sc.table);
    if (g->req_dev) (void)hipFree(g->req_dev);
    if (g->req_host) (void)hipHostFree(g->req_host);
    if (g->sc) (void)hipFree(g->sc);
    if (g->sc_host) (void)hipHostFree(g->sc_host);
    if (g->dim_dev) (void)hipFree(g->dim_dev);
    if (g->dim_host) (void)hipHostFree(g->dim_host);
    delete g;
}

gap_status dmalloc(double** p, size_t count)
{
    hipError_t e = hipMalloc((void**)p, count * sizeof(double));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GAP_ENOMEM, "hipMalloc of %zu bytes: %s", count * sizeof(double), hipGetErrorString(e));
    }
    return GAP_OK;
}

// Kernel timing: reserve event pairs for the next block of launches.
gap_status timing_reserve(gap_grid_t g, int pairs)
{
    while ((int)g->ev.size() < 2 * pairs) {
        // timing-only events: no system-scope fence (no cache writeback / invalidate per event)
        hipEvent_t e;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        if (r != hipSuccess) return fail(GAP_EDEVICE, "hipEventCreate: %s", hipGetErrorString(r));
        g->ev.push_back(e);
    }
    g->ev_kind.resize(pairs);
    g->ev_used = 0;
    return GAP_OK;
}

// Record the start (before) or stop (after) event of a launch; while timing, one launch in
// timing_period is timed, counted over the iteration-kernel launches since enabling.
inline void timing_mark(gap_grid_t g, int kind, bool start, hipStream_t st)
{
    if (!g->timing) return;
    if (start) {
        g->ev_open = (g->ev_tick++ % g->timing_period) == 0;
        if (!g->ev_open) return;
        g->ev_kind[g->ev_used] = kind;
        (void)hipEventRecord(g->ev[2 * g->ev_used], st);
    } else if (g->ev_open) {
        (void)hipEventRecord(g->ev[2 * g->ev_used + 1], st);
        ++g->ev_used;
        g->ev_open = false;
    }
}

// After the stream has been synchronized: add the elapsed times of the recorded pairs.
gap_status timing_collect(gap_grid_t g)
{
    for (int k = 0; k < g->ev_used; ++k) {
        float ms = 0.f;
        hipError_t r = hipEventElapsedTime(&ms, g->ev[2 * k], g->ev[2 * k + 1]);
        if (r != hipSuccess) return fail(GAP_EDEVICE, "hipEventElapsedTime: %s", hipGetErrorString(r));
        g->launches[g->ev_kind[k]] += 1;
        g->total_ms[g->ev_kind[k]] += ms;
    }
    g->ev_used = 0;
    return GAP_OK;
}

// Run the PCG of Table 1 on the conditions described by `a` (operators, sources, solution,
// scalar and stopping variants already set): Krylov buffers, partial sums, schedule,
// initial residual, then blocks of check_every iterations (captured once into a hipGraph and
// replayed, unless disabled or kernel timing is on) until the device record says done.
// Leaves the final record in g->sc_host.
// Fill the per-request fields of a PcgDev that come from the handle and the options.
void fill_pcg(gap_grid_t g, PcgDev& a, const gap_solver_opts* o)
{
    a.r[0] = g->r0;
    a.r[1] = g->r1;
    a.u[0] = g->u0;
    a.u[1] = g->u1;
    a.z = g->z;
    a.zf[0] = g->z;
    a.zf[1] = g->z1;
    const size_t ps = g->pcg_part_stride;
    a.part_rz[0] = g->pcg_part;
    a.part_rz[1] = g->pcg_part + ps;
    a.part_rr = g->pcg_part + 2 * ps;
    a.part_ss = g->pcg_part + 3 * ps;
    a.part_uau = g->pcg_part + 4 * ps;
    a.fpart[0] = g->pcg_part + 5 * ps;
    a.fpart[1] = g->pcg_part + 10 * ps;
    a.fstride = (int)ps;
    a.hist = g->hist;
    a.hist_cap = g->hist_cap;
    a.sc = g->sc;
    a.nt = g->nt;
    a.nz = g->nz;
    a.omega = o->omega;
    a.eps = o->eps;
    for (int k = 0; k < GAP_MAXC; ++k)          // a caller's per-condition tolerances stay
        if (!(a.eps_c[k] > 0.0)) a.eps_c[k] = o->eps;
    a.max_iter = o->max_iter;
    a.precond = o->precond;
}

gap_status run_pcg(gap_grid_t g, PcgDev& a, const gap_solver_opts* o, hipStream_t st)
{
    const int check_every = o->check_every ? o->check_every : 32;
    const bool strip = o->iteration == GAP_ITERATION_STRIPS;
    const bool one = o->iteration != GAP_ITERATION_TWO_LAUNCH;
    const int one_which = strip ? kPcgStrip : (one ? kPcgOne : 0);
    const int kernel_one = strip ? GAP_KERNEL_PCG_STRIPS : GAP_KERNEL_PCG_ONE;
    fill_pcg(g, a, o);
    a.n_strips = a.strip_groups = 1;
    if (strip) {
        const int M = o->neumann, Q = strip_q(g->shape_w.Q, M);
        if (!g->occ_wm[Q][M]) {
            int occ = 1;
            const hipError_t oe = strip_prepare(Q, M, &occ);
            if (oe != hipSuccess) return fail(GAP_EDEVICE, "preparing the strip kernel: %s", hipGetErrorString(oe));
            g->occ_wm[Q][M] = occ;
        }
        strip_chunks(g->nz, g->nt, a.n_cond, Q, M, std::min(g->wg_w, g->occ_wm[Q][M]) * g->cus, a);
    } else if (one) {
        // one launch per iteration on the B chunking fields
        pcg_chunks(g->nz, g->nt, a.n_cond, g->wg_f * g->cus, a.chunks_b, a.rows_b);
        a.chunks_a = a.chunks_b;
        a.rows_a = a.rows_b;
    } else {
        pcg_chunks(g->nz, g->nt, a.n_cond, g->wg_a * g->cus, a.chunks_a, a.rows_a);
        pcg_chunks(g->nz, g->nt, a.n_cond, g->wg_b * g->cus, a.chunks_b, a.rows_b);
    }
    PcgShape sh_b = strip ? g->shape_w : (one ? g->shape_f : g->shape_b);
    if (strip) {
        sh_b.pk = o->precond;
        sh_b.M = o->neumann;
        sh_b.Q = strip_q(sh_b.Q, sh_b.M);
        sh_b.sync = strip_sync(sh_b.M, a) ? 1 : 0;
    }

    // schedule tables for this (iteration kind, kernel shapes, n_cond, chunk counts, operator
    // map); graphs are cached by table, so the shapes belong to the key
    std::vector<int> key = {o->iteration, one ? 0 : g->shape_a.NT, one ? 0 : g->shape_a.Q, sh_b.NT, sh_b.Q, sh_b.pk,
                            sh_b.M, sh_b.sync, a.n_cond, a.chunks_a, a.chunks_b};
    for (int c = 0; c < a.n_cond; ++c) key.push_back(a.op[c]);
    gap_grid_s::Sched* sch = nullptr;
    for (auto& e : g->scheds)
        if (e.key == key) sch = &e;
    if (!sch) {
        std::vector<std::vector<int>> ga, gb;
        if (!one) pcg_groups(0, a.chunks_a, a.n_cond, a.op, ga);
        pcg_groups(0, a.chunks_b, a.n_cond, a.op, gb, strip ? a.strip_groups : 1);
        const std::vector<int> ta = pcg_schedule(ga), tb = pcg_schedule(gb);
        gap_grid_s::Sched e;
        e.key = key;
        if (hipMalloc((void**)&e.table, (ta.size() + tb.size()) * sizeof(int)) != hipSuccess)
            return fail(GAP_ENOMEM, "hipMalloc of a PCG schedule failed");
        e.blocks_a = (int)ta.size();
        e.blocks_b = (int)tb.size();
        g->scheds.push_back(e);
        sch = &g->scheds.back();
        if (!ta.empty())
            HIPCHK(hipMemcpyAsync(sch->table, ta.data(), ta.size() * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(sch->table + ta.size(), tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    const int* work_a = sch->table;
    const int* work_b = sch->table + sch->blocks_a;
    // the request record the kernels read (pinned staging, stream-ordered copy)
    if (!g->req_dev) {
        if (hipMalloc((void**)&g->req_dev, sizeof(PcgDev)) != hipSuccess) {
            g->req_dev = nullptr;
            return fail(GAP_ENOMEM, "hipMalloc of the request record failed");
        }
        if (hipHostMalloc((void**)&g->req_host, sizeof(PcgDev), hipHostMallocDefault) != hipSuccess) {
            g->req_host = nullptr;
            return fail(GAP_ENOMEM, "hipHostMalloc of the request record failed");
        }
    }
    HIPCHK(hipStreamSynchronize(st));           // the staging record may still feed an earlier copy
    *g->req_host = a;
    HIPCHK(hipMemcpyAsync(g->req_dev, g->req_host, sizeof(PcgDev), hipMemcpyHostToDevice, st));

    hipError_t le = launch_pcg(sh_b, strip ? kPcgStripInit : (one ? kPcgOneInit : kPcgInit), g->nt, g->req_dev, work_b,
                               sch->blocks_b, st);
    if (le != hipSuccess) return fail(GAP_EDEVICE, "launch of the initial residual kernel: %s", hipGetErrorString(le));

    // One block = check_every iterations; after each block the host reads the device record.
    // Launches after convergence return at once.  `closing`: one more launch (A, or the
    // one-launch kernel), which ends a solve that has reached max_iter.  The one-launch kernel
    // takes the parity of its launch count since the initial residual.
    long launched = 0;
    auto enqueue_block = [&](hipStream_t s, int iters, bool closing) -> hipError_t {
        for (int it = 0; it < iters + (closing ? 1 : 0); ++it) {
            if (one) {
                timing_mark(g, kernel_one, true, s);
                hipError_t e1 = launch_pcg(sh_b, one_which, g->nt, g->req_dev, work_b, sch->blocks_b, s, (int)(launched & 1));
                timing_mark(g, kernel_one, false, s);
                ++launched;
                if (e1 != hipSuccess) return e1;
                continue;
            }
            timing_mark(g, GAP_KERNEL_PCG_A, true, s);
            hipError_t e1 = launch_pcg(g->shape_a, kPcgA, g->nt, g->req_dev, work_a, sch->blocks_a, s);
            timing_mark(g, GAP_KERNEL_PCG_A, false, s);
            if (e1 != hipSuccess) return e1;
            if (it == iters) break;
            timing_mark(g, GAP_KERNEL_PCG_B, true, s);
            e1 = launch_pcg(g->shape_b, kPcgB, g->nt, g->req_dev, work_b, sch->blocks_b, s);
            timing_mark(g, GAP_KERNEL_PCG_B, false, s);
            if (e1 != hipSuccess) return e1;
        }
        return hipSuccess;
    };
    // Event pairs around each launch need plain launches: events recorded by graph nodes
    // cannot be read back with hipEventElapsedTime.  The kernels read the request record
    // from device memory, so one graph per (schedule, block size, starting parity) serves
    // every solve.
    const bool use_graph = o->graph != 0 && !g->timing;
    auto graph_for = [&](int par0, hipGraphExec_t* out) -> gap_status {
        const int want = one ? par0 : -1;
        for (auto& gr : g->graphs)
            if (gr.block == check_every && gr.table == sch->table && gr.par0 == want) {
                *out = gr.exec;
                return GAP_OK;
            }
        if (!g->cap_stream) HIPCHK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
        hipGraphExec_t exec = nullptr;
        hipError_t ce = capture_block(g->cap_stream, check_every, g->shape_a, sh_b, g->nt, g->req_dev, work_a,
                                      sch->blocks_a, work_b, sch->blocks_b, &exec, one_which, par0);
        if (ce != hipSuccess) return fail(GAP_EDEVICE, "capturing the PCG block: %s", hipGetErrorString(ce));
        if (g->graphs.size() >= 4) {
            (void)hipGraphExecDestroy(g->graphs.front().exec);
            g->graphs.erase(g->graphs.begin());
        }
        gap_grid_s::Graph gr;
        gr.table = sch->table;
        gr.block = check_every;
        gr.par0 = want;
        gr.exec = exec;
        g->graphs.push_back(gr);
        *out = exec;
        return GAP_OK;
    };
    // Full blocks while at least check_every iterations remain before max_iter; then the
    // remaining iterations and the closing launch, so that a solve limited by max_iter
    // launches no idle block.
    const long max_blocks = o->max_iter / check_every + 2;
    long enqueued = 0;
    for (long blk = 0; blk < max_blocks; ++blk) {
        const long remaining = (long)o->max_iter - enqueued;
        const bool last = remaining < check_every;
        const int iters = last ? (int)remaining : check_every;
        if (use_graph && !last) {
            hipGraphExec_t exec = nullptr;
            gap_status gs = graph_for((int)(launched & 1), &exec);
            if (gs != GAP_OK) return gs;
            HIPCHK(hipGraphLaunch(exec, st));
            launched += one ? iters : 0;
        } else {
            if (g->timing) {
                gap_status ts = timing_reserve(g, 2 * iters + 1);
                if (ts != GAP_OK) return ts;
            }
            le = enqueue_block(st, iters, last);
            if (le != hipSuccess) return fail(GAP_EDEVICE, "launch of a PCG iteration: %s", hipGetErrorString(le));
        }
        enqueued += iters;
        HIPCHK(hipMemcpyAsync(g->sc_host, g->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (g->timing) {
            gap_status ts = timing_collect(g);
            if (ts != GAP_OK) return ts;
        }
        if (g->sc_host->done) break;
    }
    return GAP_OK;
}

// Adjoint buffers: right-hand sides and solutions of up to 5 systems (a base system and 4
// adjoint systems), and the sensitivity partials.
gap_status ensure_adjoint(gap_grid_t g)
{
    if (g->adj_rhs) return GAP_OK;
    const ChunkMap cm1 = make_chunks(g->nz, 1);
    gap_status s1 = dmalloc(&g->adj_rhs, 5 * g->n);
    if (s1 == GAP_OK) s1 = dmalloc(&g->adj_lam, 5 * g->n);
    if (s1 == GAP_OK) s1 = dmalloc(&g->adj_part, 32 * (size_t)cm1.total);
    return s1;
}

// Switch the handle to kernel shapes sa (A) and sb (B, init); wg_a / wg_b: workgroups per
// CU the row chunking targets (0: as many as fit, i.e. the occupancy).
hipError_t use_shape(gap_grid_t g, PcgShape sa, PcgShape sb, int wg_a, int wg_b)
{
    int occ[3];
    for (int which = 0; which < 3; ++which) {
        hipError_t e = pcg_prepare(which == 0 ? sa : sb, which, g->nt, &occ[which]);
        if (e != hipSuccess) return e;
    }
    g->shape_a = sa;
    g->shape_b = sb;
    for (int k = 0; k < 3; ++k) g->occ[k] = occ[k];
    g->wg_a = wg_a > 0 ? wg_a : occ[0];
    g->wg_b = wg_b > 0 ? wg_b : std::min(occ[1], occ[2]);
    return hipSuccess;
}

// Switch the handle's one-launch kernel to shape sf; wg_f as for use_shape.
hipError_t use_shape_f(gap_grid_t g, PcgShape sf, int wg_f)
{
    int occ[2];
    for (int k = 0; k < 2; ++k) {
        hipError_t e = pcg_prepare(sf, k ? kPcgOneInit : kPcgOne, g->nt, &occ[k]);
        if (e != hipSuccess) return e;
    }
    g->shape_f = sf;
    g->occ_f = std::min(occ[0], occ[1]);
    g->wg_f = wg_f > 0 ? wg_f : g->occ_f;
    return hipSuccess;
}

// Switch the handle's strip kernel to Q columns per lane; wg_w as for use_shape.
hipError_t use_shape_w(gap_grid_t g, int Q, int wg_w)
{
    int occ = 1;
    const hipError_t e = strip_prepare(Q, 1, &occ);
    if (e != hipSuccess) return e;
    g->shape_w = PcgShape{kStripThreads, Q};
    g->occ_w = occ;
    g->wg_w = wg_w > 0 ? wg_w : occ;
    return hipSuccess;
}

gap_status validate_opts(gap_grid_t g, const gap_solver_opts* o)
{
    if (!o) return fail(GAP_EINVAL, "opts is NULL");
    if (!g->rings_ok && o->iteration != GAP_ITERATION_STRIPS)
        return fail(GAP_EINVAL, "n_theta = %d > %d needs iteration = GAP_ITERATION_STRIPS", g->nt, kMaxRingCells);
    if (!is_finite(o->omega) || !(o->omega > 0.0 && o->omega < 2.0)) return fail(GAP_EINVAL, "omega must lie in (0, 2)");
    if (!is_finite(o->eps) || !(o->eps > 0.0)) return fail(GAP_EINVAL, "eps must be > 0");
    if (!is_finite(o->eps_adjoint) || o->eps_adjoint < 0.0) return fail(GAP_EINVAL, "eps_adjoint must be >= 0");
    if (o->max_iter < 1) return fail(GAP_EINVAL, "max_iter must be >= 1");
    if (o->precond < GAP_PRECOND_JACOBI || o->precond > GAP_PRECOND_ASSOR2) return fail(GAP_EINVAL, "unknown precond");
    if (o->neumann < 1 || o->neumann > kStripMaxNeumann) return fail(GAP_EINVAL, "neumann must lie in [1, %d]", kStripMaxNeumann);
    if (o->neumann != 1 && (o->precond != GAP_PRECOND_ASSOR2 || o->iteration != GAP_ITERATION_STRIPS))
        return fail(GAP_EINVAL, "Neumann orders above 1 need precond = GAP_PRECOND_ASSOR2 and iteration = GAP_ITERATION_STRIPS");
    if (o->scalars != GAP_SCALARS_GLOBAL && o->scalars != GAP_SCALARS_PER_COND)
        return fail(GAP_EINVAL, "unknown scalars mode");
    if (o->check_every < 0) return fail(GAP_EINVAL, "check_every must be >= 0");
    if (o->strategy != GAP_STRATEGY_SYNC && o->strategy != GAP_STRATEGY_ASYNC)
        return fail(GAP_EINVAL, "unknown strategy");
    if (o->iteration != GAP_ITERATION_TWO_LAUNCH && o->iteration != GAP_ITERATION_ONE_LAUNCH &&
        o->iteration != GAP_ITERATION_STRIPS)
        return fail(GAP_EINVAL, "unknown iteration kind");
    return GAP_OK;
}

// Diagonal preconditioners (Jacobi, ASSOR I) are stored per operator; rebuilt when the kind,
// omega or the assembled operators change.
gap_status prepare_precond(gap_grid_t g, const gap_solver_opts* o, hipStream_t st)
{
    if (o->precond == GAP_PRECOND_ASSOR2 || (g->minv_kind == o->precond && g->minv_omega == o->omega)) return GAP_OK;
    if (!g->minv) {
        gap_status s = dmalloc(&g->minv, g->max_op * g->n);
        if (s != GAP_OK) return s;
    }
    hipLaunchKernelGGL(k_diag_precond, dim3((unsigned)((g->n + GAP_BLOCK - 1) / GAP_BLOCK), g->n_op), dim3(GAP_BLOCK),
                       0, st, g->gd, o->precond, o->omega, g->kx, g->kz, g->minv, g->n_op);
    HIPLAUNCHCHK("k_diag_precond");
    g->minv_kind = o->precond;
    g->minv_omega = o->omega;
    return GAP_OK;
}

// Translate the device record of the last solve into info and a status.
gap_status finish_solve(gap_grid_t g, int n_cond, gap_solve_info* info)
{
    const PcgScalars& h = *g->sc_host;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iterations = h.iterations;
        info->n_cond = n_cond;
        info->rel_residual = h.rel;
        for (int c = 0; c < n_cond; ++c) info->rel_residual_cond[c] = h.rel_cond[c];
        info->true_rel_residual = -1.0;
        for (int c = 0; c < GAP_MAX_COND; ++c) info->true_rel_residual_cond[c] = -1.0;
    }
    gap_status result = GAP_OK;
    if (h.status == -4) result = fail(GAP_ENONFINITE, "non-finite value in the PCG reductions at iteration %d", h.iterations);
    else if (h.status == -3 || !h.done) result = fail(GAP_ENOCONV, "no convergence after %d iterations (rel %.3e)", h.iterations, h.rel);
    if (info) info->status = result;
    return result;
}

// The geometry as the kernels see it.
GeomDev geom_dev(const gap_geom& geom)
{
    GeomDev d{};
    d.R = geom.R;
    d.Rc = geom.R + geom.clearance;
    d.c2R = geom.clearance * (2.0 * geom.R + geom.clearance);
    d.L = geom.length;
    d.mu = geom.mu;
    d.U = geom.U;
    d.V = geom.V;
    d.p_in = geom.p_in;
    d.p_out = geom.p_out;
    d.nt = geom.n_theta;
    d.nz = geom.n_axial;
    d.dth = 2.0 * M_PI / d.nt;
    d.dz = geom.length / d.nz;
    d.dx = geom.R * d.dth;
    return d;
}

gap_status validate_geom(const gap_geom* g)
{
    if (!g) return fail(GAP_EINVAL, "geom is NULL");
    if (g->n_theta < 3 || g->n_theta > kMaxThetaCells)
        return fail(GAP_EINVAL, "n_theta = %d outside [3, %d]", g->n_theta, kMaxThetaCells);
    if (g->n_axial < 2 || g->n_axial > kMaxAxialCells)
        return fail(GAP_EINVAL, "n_axial = %d outside [2, %d]", g->n_axial, kMaxAxialCells);
    const double pos[] = {g->R, g->clearance, g->length, g->mu};
    const char* names[] = {"R", "clearance", "length", "mu"};
    for (int k = 0; k < 4; ++k)
        if (!is_finite(pos[k]) || !(pos[k] > 0.0)) return fail(GAP_EINVAL, "%s must be finite and > 0", names[k]);
    if (!is_finite(g->U) || !is_finite(g->V) || !is_finite(g->p_in) || !is_finite(g->p_out))
        return fail(GAP_EINVAL, "U, V, p_in and p_out must be finite");
    return GAP_OK;
}

}  // namespace

extern "C" {

const char* gap_last_error(void) { return g_err.c_str(); }

gap_status gap_default_opts(gap_solver_opts* o)
{
    if (!o) return fail(GAP_EINVAL, "opts is NULL");
    o->omega = 1.6;
    o->eps = 1e-10;
    o->max_iter = 100000;
    o->precond = GAP_PRECOND_ASSOR2;
    o->neumann = 1;
    o->scalars = GAP_SCALARS_GLOBAL;
    o->warm_start = 0;
    o->check_every = 32;
    o->graph = 1;
    o->strategy = GAP_STRATEGY_SYNC;
    o->iteration = GAP_ITERATION_STRIPS;
    o->reserved = 0;
    o->eps_adjoint = 0.0;
    return GAP_OK;
}

namespace {

// One non-blocking stream per device for the initialisation copies of new handles (created
// on first use, kept until the process ends): a handle gets no stream of its own until it
// captures a graph, so that creating many handles does not multiply the streams that share
// the hardware queues.
std::mutex g_init_mu;
hipStream_t g_init_stream[64] = {};

hipError_t init_stream(hipStream_t* out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_init_mu);
    if (!g_init_stream[dev]) {
        e = hipStreamCreateWithFlags(&g_init_stream[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            g_init_stream[dev] = nullptr;
            return e;
        }
    }
    *out = g_init_stream[dev];
    return hipSuccess;
}

gap_status check_dimples(const gap_geom* geom, const gap_dimples* dimples)
{
    const int count = dimples ? dimples->count : 0;
    if (count < 0) return fail(GAP_EINVAL, "dimple count < 0");
    if (count > 0) {
        if (!dimples->theta || !dimples->z || !dimples->radius || !dimples->depth)
            return fail(GAP_EINVAL, "dimple arrays must be non-NULL when count > 0");
        for (int k = 0; k < count; ++k) {
            const double a = dimples->radius[k], d = dimples->depth[k];
            const double th = dimples->theta[k], zc = dimples->z[k];
            if (!is_finite(th) || !is_finite(zc) || !is_finite(a) || !is_finite(d) || !(a > 0.0) || !(d > 0.0) ||
                d > a)
                return fail(GAP_EINVAL, "dimple %d: need finite centre, radius > 0 and 0 < depth <= radius", k);
            // keeps every index the texture kernel derives from a dimple inside int range
            if (std::fabs(th) > 1e3 || zc < -geom->length || zc > 2.0 * geom->length || a > geom->length ||
                a > M_PI * geom->R)
                return fail(GAP_EINVAL, "dimple %d: |theta| <= 1e3, -L <= z <= 2L, radius <= min(L, pi R)", k);
        }
    }
    return GAP_OK;
}

}  // namespace

gap_status create_gap_grid(const gap_geom* geom, const gap_dimples* dimples, int32_t max_cond, gap_grid_t* out)
{
    if (!out) return fail(GAP_EINVAL, "out is NULL");
    *out = nullptr;
    gap_status st = validate_geom(geom);
    if (st != GAP_OK) return st;
    if (max_cond != 1 && max_cond != GAP_MAX_COND) return fail(GAP_EINVAL, "max_cond must be 1 or 9");
    st = check_dimples(geom, dimples);
    if (st != GAP_OK) return st;

    gap_grid_t g = new gap_grid_s;
    g->geom = *geom;
    g->nt = geom->n_theta;
    g->nz = geom->n_axial;
    g->n = (size_t)g->nt * g->nz;
    g->max_cond = max_cond;
    g->max_op = (max_cond == GAP_MAX_COND) ? 5 : 1;
    g->gd = geom_dev(*geom);
    const GeomDev& d = g->gd;

    const size_t n = g->n, nt = g->nt;
    const ChunkMap cm_max = make_chunks(g->nz, 1);
    const ChunkMap cm9 = make_chunks(g->nz, GAP_MAX_COND);
    const size_t max_chunks = (size_t)std::max(cm_max.total, cm9.total);
#define ALLOC(ptr, cnt)                                   \
    do {                                                  \
        gap_status s_ = dmalloc(&(ptr), (cnt));           \
        if (s_ != GAP_OK) { release(g); return s_; }      \
    } while (0)
    ALLOC(g->trig, 4 * nt);
    ALLOC(g->tex, 2 * n + (g->nz + 1) * nt);
    ALLOC(g->kx, g->max_op * n);
    ALLOC(g->kz, g->max_op * (n + nt));
    ALLOC(g->kxz, g->max_op * 2 * (n + nt));
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || g->cus < 1)
            g->cus = 256;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            g->lds_max = lds;
        g->rings_ok = g->nt <= kMaxRingCells;
        if (g->rings_ok) {
            g->shape_a = g->shape_b = g->shape_f = pcg_candidates(g->nt)[0];
            const size_t need = pcg_lds_bytes(kPcgOne, g->shape_f.NT * g->shape_f.Q) + 2048;
            if (need > (size_t)g->lds_max) {
                release(g);
                return fail(GAP_EINVAL, "n_theta = %d needs %zu bytes of LDS per workgroup, the device allows %d",
                            geom->n_theta, need, g->lds_max);
            }
        }
    }
    // PCG partial sums: at most one slot per row of every condition, or per strip group of
    // the narrowest strips when a ring has more of those than rows
    int strips1 = 1, groups1 = 1;
    strip_layout(g->nt, 1, kStripMaxNeumann, strips1, groups1);
    const size_t max_pcg = (size_t)max_cond * std::max(g->nz, groups1);
    g->pcg_part_stride = max_pcg;
    {
        hipError_t pe = hipSuccess;
        if (g->rings_ok) {
            pe = use_shape(g, g->shape_a, g->shape_b, 0, 0);
            if (pe == hipSuccess) pe = use_shape_f(g, g->shape_f, 0);
        }
        if (pe == hipSuccess) pe = use_shape_w(g, kStripDefaultQ, 0);
        if (pe != hipSuccess) {
            release(g);
            return fail(GAP_EDEVICE, "preparing the PCG kernels: %s", hipGetErrorString(pe));
        }
    }
    ALLOC(g->S, max_cond * n);
    // r and u of one parity share a block: the ring kernels use its halves, the strip kernel
    // reads it as interleaved (r, u) pairs (a solve uses one iteration kind)
    ALLOC(g->r0, 2 * max_cond * n);
    ALLOC(g->r1, 2 * max_cond * n);
    g->u0 = g->r0 + max_cond * n;
    g->u1 = g->r1 + max_cond * n;
    ALLOC(g->z, max_cond * n);
    ALLOC(g->z1, max_cond * n);
    ALLOC(g->partial, 10 * max_chunks);
    ALLOC(g->pcg_part, 15 * max_pcg);
#undef ALLOC
    if (hipMalloc((void**)&g->sc, sizeof(PcgScalars)) != hipSuccess) {
        g->sc = nullptr;
        release(g);
        return fail(GAP_ENOMEM, "hipMalloc of the scalar block failed");
    }
    if (hipHostMalloc((void**)&g->sc_host, sizeof(PcgScalars), hipHostMallocDefault) != hipSuccess) {
        g->sc_host = nullptr;
        release(g);
        return fail(GAP_ENOMEM, "hipHostMalloc of the scalar block failed");
    }

    std::vector<double> trig(4 * nt);
    for (size_t i = 0; i < nt; ++i) {
        const double tc = (i + 0.5) * d.dth, te = (i + 1.0) * d.dth;
        trig[i] = std::cos(tc);
        trig[nt + i] = std::sin(tc);
        trig[2 * nt + i] = std::cos(te);
        trig[3 * nt + i] = std::sin(te);
    }
    // initialisation on a stream of its own (no device-wide synchronization, so a handle may
    // be created beside the work and graph captures of other threads); concurrent creations
    // share it, serialized
    hipStream_t s0 = nullptr;
    hipError_t e = init_stream(&s0);
    if (e != hipSuccess) {
        release(g);
        return fail(GAP_EDEVICE, "creating the initialisation stream: %s", hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> init_lock(g_init_mu);
    e = hipMemcpyAsync(g->trig, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice, s0);
    if (e == hipSuccess) e = hipMemsetAsync(g->sc, 0, sizeof(PcgScalars), s0);
    if (e == hipSuccess) e = hipMemsetAsync(g->pcg_part, 0, 15 * g->pcg_part_stride * sizeof(double), s0);
    if (e == hipSuccess) e = hipStreamSynchronize(s0);
    if (e != hipSuccess) {
        release(g);
        return fail(GAP_EDEVICE, "initialising tables: %s", hipGetErrorString(e));
    }
    st = set_gap_dimples(g, dimples, s0);
    if (st != GAP_OK) {
        release(g);
        return st;
    }
    *out = g;
    return GAP_OK;
}

gap_status create_gap_grid_field(const gap_geom* geom, const double* tex_c, const double* tex_e, const double* tex_f,
                                 int32_t max_cond, gap_grid_t* out)
{
    if (!out) return fail(GAP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tex_c || !tex_e || !tex_f) return fail(GAP_EINVAL, "tex_c, tex_e and tex_f must be non-NULL");
    gap_grid_t g = nullptr;
    gap_status st = create_gap_grid(geom, nullptr, max_cond, &g);
    if (st != GAP_OK) return st;
    const size_t n = g->n, nf = (size_t)(g->nz + 1) * g->nt;
    const TablesDev t = g->tables();
    hipError_t e = hipMemcpy((double*)t.tex_c, tex_c, n * sizeof(double), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy((double*)t.tex_e, tex_e, n * sizeof(double), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy((double*)t.tex_f, tex_f, nf * sizeof(double), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
        release(g);
        return fail(GAP_EDEVICE, "copying the texture field: %s", hipGetErrorString(e));
    }
    // a depth must be finite and >= 0 (a pocket in the piston surface): checked once, here
    std::vector<double> host(2 * n + nf);
    e = hipMemcpy(host.data(), t.tex_c, host.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        release(g);
        return fail(GAP_EDEVICE, "reading the texture field back: %s", hipGetErrorString(e));
    }
    for (size_t k = 0; k < host.size(); ++k)
        if (!is_finite(host[k]) || host[k] < 0.0) {
            const char* which = k < n ? "tex_c" : (k < 2 * n ? "tex_e" : "tex_f");
            const size_t at = k < n ? k : (k < 2 * n ? k - n : k - 2 * n);
            release(g);
            return fail(GAP_EINVAL, "%s[%zu] = %g: texture depths must be finite and >= 0", which, at, host[k]);
        }
    *out = g;
    return GAP_OK;
}

gap_status destroy_gap_grid(gap_grid_t g)
{
    if (!g) return GAP_OK;
    GAP_NOT_IN_BATCH(g, "destroy_gap_grid");
    (void)hipDeviceSynchronize();
    release(g);
    return GAP_OK;
}

gap_status set_gap_dimples(gap_grid_t g, const gap_dimples* dimples, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "set_gap_dimples");
    gap_status st = check_dimples(&g->geom, dimples);
    if (st != GAP_OK) return st;
    const int count = dimples ? dimples->count : 0;
    hipStream_t s = (hipStream_t)stream;
    // the parameter buffers grow to a multiple of 256 dimples (once, in the usual case)
    if (count > g->dim_cap) {
        HIPCHK(hipStreamSynchronize(s));
        if (g->dim_dev) (void)hipFree(g->dim_dev);
        if (g->dim_host) (void)hipHostFree(g->dim_host);
        g->dim_dev = g->dim_host = nullptr;
        g->dim_cap = 0;
        const int cap = (count + 255) / 256 * 256;
        if (hipMalloc((void**)&g->dim_dev, 4 * (size_t)cap * sizeof(double)) != hipSuccess) {
            g->dim_dev = nullptr;
            return fail(GAP_ENOMEM, "hipMalloc of the dimple parameters failed");
        }
        if (hipHostMalloc((void**)&g->dim_host, 4 * (size_t)cap * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            g->dim_host = nullptr;
            return fail(GAP_ENOMEM, "hipHostMalloc of the dimple parameters failed");
        }
        g->dim_cap = cap;
    }
    g->assembled = false;
    const size_t nt = g->nt, n = g->n;
    HIPCHK(hipMemsetAsync(g->tex, 0, (2 * n + (g->nz + 1) * nt) * sizeof(double), s));
    if (count > 0) {
        const double* src[4] = {dimples->theta, dimples->z, dimples->radius, dimples->depth};
        for (int k = 0; k < 4; ++k) std::memcpy(g->dim_host + (size_t)k * count, src[k], count * sizeof(double));
        double* dm = g->dim_dev;
        HIPCHK(hipMemcpyAsync(dm, g->dim_host, 4 * (size_t)count * sizeof(double), hipMemcpyHostToDevice, s));
        const TablesDev t = g->tables();
        hipLaunchKernelGGL(k_texture, dim3(count, 3), dim3(GAP_BLOCK), 0, s, g->gd, count, dm, dm + count,
                           dm + 2 * count, dm + 3 * count, (double*)t.tex_c, (double*)t.tex_e, (double*)t.tex_f);
        HIPLAUNCHCHK("k_texture");
    }
    HIPCHK(hipStreamSynchronize(s));           // the pinned parameters may be overwritten after this
    return GAP_OK;
}

gap_status assemble_joint_system(gap_grid_t g, const double e[4], const double edot[4], const double delta[8],
                                 int32_t n_cond, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "assemble_joint_system");
    if (!e || !edot) return fail(GAP_EINVAL, "e and edot must be non-NULL");
    if (n_cond != 1 && n_cond != GAP_MAX_COND) return fail(GAP_EINVAL, "n_cond must be 1 or 9");
    if (n_cond > g->max_cond) return fail(GAP_EINVAL, "n_cond = %d exceeds max_cond = %d", n_cond, g->max_cond);
    if (n_cond == GAP_MAX_COND && !delta) return fail(GAP_EINVAL, "delta is required for 9 conditions");
    for (int k = 0; k < 4; ++k)
        if (!is_finite(e[k]) || !is_finite(edot[k])) return fail(GAP_EINVAL, "e and edot must be finite");
    if (n_cond == GAP_MAX_COND)
        for (int k = 0; k < 8; ++k)
            if (!is_finite(delta[k]) || delta[k] == 0.0) return fail(GAP_EINVAL, "delta[%d] must be finite and nonzero", k);

    CondDev cd{};
    cd.n_cond = n_cond;
    cd.n_op = (n_cond == GAP_MAX_COND) ? 5 : 1;
    for (int c = 0; c < n_cond; ++c) {
        for (int k = 0; k < 4; ++k) {
            cd.e[c][k] = e[k];
            cd.ed[c][k] = edot[k];
        }
        if (c >= 1 && c <= 4) cd.e[c][c - 1] += delta[c - 1];
        if (c >= 5) cd.ed[c][c - 5] += delta[c - 1];
        cd.op[c] = (c < 5) ? c : 0;
        const double c0 = std::hypot(cd.e[c][0], cd.e[c][1]);
        const double c1 = std::hypot(cd.e[c][2], cd.e[c][3]);
        if (c0 >= g->geom.clearance || c1 >= g->geom.clearance)
            return fail(GAP_ECONTACT, "condition %d: |e| at a gap end (%.6g, %.6g) >= clearance %.6g", c, c0, c1,
                        g->geom.clearance);
    }
    hipStream_t st = (hipStream_t)stream;
    const TablesDev t = g->tables();
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((g->n + GAP_BLOCK - 1) / GAP_BLOCK), n_cond), dim3(GAP_BLOCK), 0, st,
                       g->gd, cd, t, g->kx, g->kz, g->S);
    HIPLAUNCHCHK("k_assemble");
    hipLaunchKernelGGL(k_pair_ops, dim3((unsigned)((g->n + g->nt + GAP_BLOCK - 1) / GAP_BLOCK), cd.n_op),
                       dim3(GAP_BLOCK), 0, st, g->nt, g->nz, (const double*)g->kx, (const double*)g->kz, g->kxz);
    HIPLAUNCHCHK("k_pair_ops");
    g->cd = cd;
    g->n_cond = n_cond;
    g->n_op = cd.n_op;
    g->cm = make_chunks(g->nz, n_cond);
    if (delta)
        for (int k = 0; k < 8; ++k) g->delta[k] = delta[k];
    g->assembled = true;
    g->minv_kind = -1;
    return GAP_OK;
}

gap_status solve_joint_pcg(gap_grid_t g, const gap_solver_opts* o, double* p, gap_solve_info* info, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "solve_joint_pcg");
    if (!p) return fail(GAP_EINVAL, "p is NULL");
    gap_status vs = validate_opts(g, o);
    if (vs != GAP_OK) return vs;
    if (!g->assembled) return fail(GAP_ESTATE, "solve_joint_pcg before assemble_joint_system");
    hipStream_t st = (hipStream_t)stream;
    gap_status ps = prepare_precond(g, o, st);
    if (ps != GAP_OK) return ps;

    PcgDev a{};
    a.kx = g->kx;
    a.kxz = g->kxz;
    a.kz = g->kz;
    a.minv = g->minv;
    a.S = g->S;
    a.p = p;
    for (int c = 0; c < GAP_MAXC; ++c) a.op[c] = g->cd.op[c];
    a.n_cond = g->n_cond;
    a.per_cond = o->scalars == GAP_SCALARS_PER_COND;
    a.async = o->strategy == GAP_STRATEGY_ASYNC;
    a.warm = o->warm_start ? 1 : 0;
    gap_status rs = run_pcg(g, a, o, st);
    if (rs != GAP_OK) return rs;
    const gap_status result = finish_solve(g, g->n_cond, info);
    if (info) {
        // the true residual of the returned p, once (Table 1 tests the recurrence residual)
        const ChunkMap cm = g->cm;
        hipLaunchKernelGGL(k_true_residual, dim3(cm.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm,
                           (const double*)g->kx, (const double*)g->kz, (const double*)g->S, (const double*)p,
                           g->partial);
        HIPLAUNCHCHK("k_true_residual");
        if (!g->step_buf) {
            gap_status s1 = dmalloc(&g->step_buf, 36 + 32);
            if (s1 != GAP_OK) return s1;
        }
        hipLaunchKernelGGL(k_forces_finalize, dim3(1), dim3(GAP_BLOCK), 0, st, cm, g->n_cond, 2, 1.0,
                           (const double*)g->partial, g->step_buf);
        HIPLAUNCHCHK("residual sums");
        double sums[2 * GAP_MAX_COND];
        HIPCHK(hipMemcpyAsync(sums, g->step_buf, 2 * g->n_cond * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double rr = 0.0, ss = 0.0;
        for (int c = 0; c < g->n_cond; ++c) {
            rr += sums[2 * c];
            ss += sums[2 * c + 1];
            info->true_rel_residual_cond[c] = sqrt(sums[2 * c] / (sums[2 * c + 1] > 0.0 ? sums[2 * c + 1] : 1.0));
        }
        info->true_rel_residual = sqrt(rr / (ss > 0.0 ? ss : 1.0));
    }
    return result;
}

gap_status jacobian_adjoint(gap_grid_t g, const gap_solver_opts* o, const double* p0, int32_t cavitation, double p_cav,
                            const double* w, double* J, gap_solve_info* info, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "jacobian_adjoint");
    if (!p0 || !J) return fail(GAP_EINVAL, "p0 and J must be non-NULL");
    gap_status vs = validate_opts(g, o);
    if (vs != GAP_OK) return vs;
    if (!g->assembled) return fail(GAP_ESTATE, "jacobian_adjoint before assemble_joint_system");
    if (cavitation != GAP_CAVITATION_NONE && cavitation != GAP_CAVITATION_CLAMP)
        return fail(GAP_EINVAL, "unknown cavitation mode");
    if (!is_finite(p_cav)) return fail(GAP_EINVAL, "p_cav must be finite");
    if (w)
        for (int i = 0; i < 4; ++i)
            if (!is_finite(w[i])) return fail(GAP_EINVAL, "w must be finite");
    const int n_rhs = w ? 1 : 4;
    if (n_rhs > g->max_cond)
        return fail(GAP_EINVAL, "the full adjoint Jacobian needs a handle created for 9 conditions (pass w for a "
                                "vector-Jacobian product)");
    hipStream_t st = (hipStream_t)stream;
    gap_status ps = prepare_precond(g, o, st);
    if (ps != GAP_OK) return ps;
    const size_t n = g->n;
    const ChunkMap cm1 = make_chunks(g->nz, 1);
    gap_status as = ensure_adjoint(g);
    if (as != GAP_OK) return as;
    const double w0 = w ? w[0] : 0.0, w1 = w ? w[1] : 0.0, w2 = w ? w[2] : 0.0, w3 = w ? w[3] : 0.0;
    hipLaunchKernelGGL(k_adjoint_rhs, dim3((unsigned)((n + GAP_BLOCK - 1) / GAP_BLOCK)), dim3(GAP_BLOCK), 0, st, g->gd,
                       g->cd, g->tables(), p0, cavitation, p_cav, w ? 1 : 0, w0, w1, w2, w3, g->adj_rhs);
    HIPLAUNCHCHK("k_adjoint_rhs");

    // A lambda_i = g_i on the operator of condition 0: one recurrence per right-hand side,
    // each stopped by its own relative residual.
    gap_solver_opts oa = *o;
    if (o->eps_adjoint > 0.0) oa.eps = o->eps_adjoint;
    oa.scalars = GAP_SCALARS_PER_COND;
    oa.strategy = GAP_STRATEGY_ASYNC;
    oa.warm_start = 0;
    PcgDev a{};
    a.kx = g->kx;
    a.kxz = g->kxz;
    a.kz = g->kz;
    a.minv = g->minv;
    a.S = g->adj_rhs;
    a.p = g->adj_lam;
    for (int c = 0; c < GAP_MAXC; ++c) a.op[c] = 0;
    a.n_cond = n_rhs;
    a.per_cond = 1;
    a.async = 1;
    a.warm = 0;
    gap_status rs = run_pcg(g, a, &oa, st);
    if (rs != GAP_OK) return rs;
    gap_status fs = finish_solve(g, n_rhs, info);
    if (fs != GAP_OK) return fs;

    if (w)
        hipLaunchKernelGGL((k_adjoint_sens<1>), dim3(cm1.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm1, g->tables(),
                           p0, (const double*)g->adj_lam, cavitation, p_cav, w0, w1, w2, w3, g->adj_part);
    else
        hipLaunchKernelGGL((k_adjoint_sens<4>), dim3(cm1.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm1, g->tables(),
                           p0, (const double*)g->adj_lam, cavitation, p_cav, 0.0, 0.0, 0.0, 0.0, g->adj_part);
    HIPLAUNCHCHK("k_adjoint_sens");
    hipLaunchKernelGGL(k_adjoint_finalize, dim3(1), dim3(GAP_BLOCK), 0, st, cm1, w ? 8 : 32,
                       (const double*)g->adj_part, J);
    HIPLAUNCHCHK("k_adjoint_finalize");
    HIPCHK(hipStreamSynchronize(st));
    return GAP_OK;
}

gap_status solve_with_adjoint(gap_grid_t g, const gap_solver_opts* o, double* p0, const double* w, double* J,
                              gap_solve_info* info, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "solve_with_adjoint");
    if (!p0 || !J) return fail(GAP_EINVAL, "p0 and J must be non-NULL");
    gap_status vs = validate_opts(g, o);
    if (vs != GAP_OK) return vs;
    if (!g->assembled) return fail(GAP_ESTATE, "solve_with_adjoint before assemble_joint_system");
    if (w)
        for (int i = 0; i < 4; ++i)
            if (!is_finite(w[i])) return fail(GAP_EINVAL, "w must be finite");
    const int n_rhs = w ? 1 : 4;
    const int n_sys = 1 + n_rhs;
    if (n_sys > g->max_cond)
        return fail(GAP_EINVAL, "the joint base + adjoint solve of %d systems needs a handle created for at least %d "
                                "conditions", n_sys, n_sys);
    hipStream_t st = (hipStream_t)stream;
    gap_status ps = prepare_precond(g, o, st);
    if (ps != GAP_OK) return ps;
    const size_t n = g->n;
    const ChunkMap cm1 = make_chunks(g->nz, 1);
    gap_status as = ensure_adjoint(g);
    if (as != GAP_OK) return as;
    const double w0 = w ? w[0] : 0.0, w1 = w ? w[1] : 0.0, w2 = w ? w[2] : 0.0, w3 = w ? w[3] : 0.0;
    // right-hand sides: S of condition 0, then df_i/dp (no clamp: independent of p0)
    HIPCHK(hipMemcpyAsync(g->adj_rhs, g->S, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_adjoint_rhs, dim3((unsigned)((n + GAP_BLOCK - 1) / GAP_BLOCK)), dim3(GAP_BLOCK), 0, st, g->gd,
                       g->cd, g->tables(), (const double*)nullptr, (int)GAP_CAVITATION_NONE, 0.0, w ? 1 : 0, w0, w1, w2,
                       w3, g->adj_rhs + n);
    HIPLAUNCHCHK("k_adjoint_rhs");

    gap_solver_opts oa = *o;
    oa.scalars = GAP_SCALARS_PER_COND;
    oa.strategy = GAP_STRATEGY_ASYNC;
    oa.warm_start = 0;
    PcgDev a{};
    a.kx = g->kx;
    a.kxz = g->kxz;
    a.kz = g->kz;
    a.minv = g->minv;
    a.S = g->adj_rhs;
    a.p = g->adj_lam;
    for (int c = 0; c < GAP_MAXC; ++c) a.op[c] = 0;
    for (int c = 1; c < n_sys; ++c) a.eps_c[c] = o->eps_adjoint;   // 0: the base system's eps
    a.n_cond = n_sys;
    a.per_cond = 1;
    a.async = 1;
    a.warm = 0;
    gap_status rs = run_pcg(g, a, &oa, st);
    if (rs != GAP_OK) return rs;
    gap_status fs = finish_solve(g, n_sys, info);
    if (fs != GAP_OK) return fs;

    const double* lam = g->adj_lam + n;
    if (w)
        hipLaunchKernelGGL((k_adjoint_sens<1>), dim3(cm1.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm1, g->tables(),
                           (const double*)g->adj_lam, lam, (int)GAP_CAVITATION_NONE, 0.0, w0, w1, w2, w3, g->adj_part);
    else
        hipLaunchKernelGGL((k_adjoint_sens<4>), dim3(cm1.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm1, g->tables(),
                           (const double*)g->adj_lam, lam, (int)GAP_CAVITATION_NONE, 0.0, 0.0, 0.0, 0.0, 0.0,
                           g->adj_part);
    HIPLAUNCHCHK("k_adjoint_sens");
    hipLaunchKernelGGL(k_adjoint_finalize, dim3(1), dim3(GAP_BLOCK), 0, st, cm1, w ? 8 : 32,
                       (const double*)g->adj_part, J);
    HIPLAUNCHCHK("k_adjoint_finalize");
    HIPCHK(hipMemcpyAsync(p0, g->adj_lam, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return GAP_OK;
}

gap_status set_operating_point(gap_grid_t g, double U, double V, double p_in, double p_out)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "set_operating_point");
    if (!is_finite(U) || !is_finite(V) || !is_finite(p_in) || !is_finite(p_out))
        return fail(GAP_EINVAL, "U, V, p_in and p_out must be finite");
    g->geom.U = g->gd.U = U;
    g->geom.V = g->gd.V = V;
    g->geom.p_in = g->gd.p_in = p_in;
    g->geom.p_out = g->gd.p_out = p_out;
    g->assembled = false;
    return GAP_OK;
}

gap_status general_iteration_step(gap_grid_t g, const gap_solver_opts* o, const gap_step_params* prm,
                                  const double* delta, double* p, double* e, double* edot, double* F, double* J,
                                  gap_solve_info* info, void* stream)
{
    if (!g || !o || !prm || !p || !e || !edot || !F) return fail(GAP_EINVAL, "grid, opts, prm, p, e, edot and F must be non-NULL");
    GAP_NOT_IN_BATCH(g, "general_iteration_step");
    if (!is_finite(prm->dt) || !(prm->dt > 0.0)) return fail(GAP_EINVAL, "dt must be finite and > 0");
    for (int k = 0; k < 4; ++k)
        if (!is_finite(prm->edot_prev[k]) || !is_finite(prm->F_ext[k])) return fail(GAP_EINVAL, "edot_prev and F_ext must be finite");
    for (int k = 0; k < 16; ++k)
        if (!is_finite(prm->mass[k])) return fail(GAP_EINVAL, "mass must be finite");
    if (prm->scheme != GAP_SCHEME_GENERAL && prm->scheme != GAP_SCHEME_CONVENTIONAL) return fail(GAP_EINVAL, "unknown scheme");
    if (prm->jacobian != GAP_JACOBIAN_FD && prm->jacobian != GAP_JACOBIAN_ADJOINT) return fail(GAP_EINVAL, "unknown jacobian");
    if (prm->jacobian == GAP_JACOBIAN_FD && (g->max_cond != GAP_MAX_COND || !delta))
        return fail(GAP_EINVAL, "the FD Jacobian needs a 9-condition handle and delta");
    hipStream_t st = (hipStream_t)stream;
    if (!g->step_buf) {
        gap_status s1 = dmalloc(&g->step_buf, 36 + 32);
        if (s1 != GAP_OK) return s1;
    }
    double* F_dev = g->step_buf;
    double* J_dev = g->step_buf + 36;
    gap_status s1;
    if (prm->jacobian == GAP_JACOBIAN_FD) {
        s1 = assemble_joint_system(g, e, edot, delta, GAP_MAX_COND, stream);
        if (s1 == GAP_OK) s1 = solve_joint_pcg(g, o, p, info, stream);
        if (s1 == GAP_OK) s1 = integrate_force_moment(g, p, GAP_CAVITATION_NONE, 0.0, F_dev, stream);
        if (s1 == GAP_OK) s1 = jacobian_fd(g, F_dev, J_dev, stream);
    } else {
        s1 = assemble_joint_system(g, e, edot, nullptr, 1, stream);
        if (s1 == GAP_OK) s1 = solve_with_adjoint(g, o, p, nullptr, J_dev, info, stream);
        if (s1 == GAP_OK) s1 = integrate_force_moment(g, p, GAP_CAVITATION_NONE, 0.0, F_dev, stream);
    }
    if (s1 != GAP_OK) return s1;
    double Fo[4], Jo[32];
    HIPCHK(hipMemcpyAsync(Fo, F_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(Jo, J_dev, 32 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // residual F = F_E + F_I + F_O and the update matrix (Eq 2.12 or Eq 2.20)
    const double dt = prm->dt;
    const double* M = prm->mass;
    double R[4], K[4][4];
    for (int i = 0; i < 4; ++i) {
        double fi = 0.0;
        for (int k = 0; k < 4; ++k) fi -= M[4 * i + k] * (edot[k] - prm->edot_prev[k]);
        R[i] = prm->F_ext[i] + fi / dt + Fo[i];
        for (int k = 0; k < 4; ++k) {
            K[i][k] = Jo[8 * i + 4 + k] - M[4 * i + k] / dt;
            if (prm->scheme == GAP_SCHEME_GENERAL) K[i][k] += dt * Jo[8 * i + k];
        }
    }
    for (int i = 0; i < 4; ++i) F[i] = R[i];
    if (J)
        for (int k = 0; k < 32; ++k) J[k] = Jo[k];
    // K d(edot) = -R by Gaussian elimination with partial pivoting
    double b[4] = {-R[0], -R[1], -R[2], -R[3]};
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(K[r][c]) > std::fabs(K[piv][c])) piv = r;
        if (!(std::fabs(K[piv][c]) > 0.0) || !is_finite(K[piv][c]))
            return fail(GAP_ENONFINITE, "the update matrix of the general iteration is singular");
        if (piv != c) {
            for (int k = 0; k < 4; ++k) std::swap(K[c][k], K[piv][k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < 4; ++r) {
            const double f = K[r][c] / K[c][c];
            for (int k = c; k < 4; ++k) K[r][k] -= f * K[c][k];
            b[r] -= f * b[c];
        }
    }
    double d_edot[4];
    for (int r = 3; r >= 0; --r) {
        double v = b[r];
        for (int k = r + 1; k < 4; ++k) v -= K[r][k] * d_edot[k];
        d_edot[r] = v / K[r][r];
    }
    for (int k = 0; k < 4; ++k)
        if (!is_finite(d_edot[k])) return fail(GAP_ENONFINITE, "non-finite update of the general iteration");
    for (int k = 0; k < 4; ++k) {
        e[k] += dt * d_edot[k];
        edot[k] += d_edot[k];
    }
    return GAP_OK;
}

namespace {

gap_status check_integrate(gap_grid_t g, const double* p, const double* out, int32_t cavitation, double p_cav,
                           const char* what)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    if (!p || !out) return fail(GAP_EINVAL, "p and the output must be non-NULL");
    if (!g->assembled) return fail(GAP_ESTATE, "%s before assemble_joint_system", what);
    if (cavitation != GAP_CAVITATION_NONE && cavitation != GAP_CAVITATION_CLAMP)
        return fail(GAP_EINVAL, "unknown cavitation mode");
    if (!is_finite(p_cav)) return fail(GAP_EINVAL, "p_cav must be finite");
    return GAP_OK;
}

}  // namespace

gap_status integrate_force_moment(gap_grid_t g, const double* p, int32_t cavitation, double p_cav, double* F,
                                  void* stream)
{
    gap_status cs = check_integrate(g, p, F, cavitation, p_cav, "integrate_force_moment");
    if (cs != GAP_OK) return cs;
    hipStream_t st = (hipStream_t)stream;
    const ChunkMap cm = g->cm;
    hipLaunchKernelGGL((k_forces<4>), dim3(cm.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm, g->tables(), p,
                       cavitation, p_cav, g->partial);
    hipLaunchKernelGGL(k_forces_finalize, dim3(1), dim3(GAP_BLOCK), 0, st, cm, g->n_cond, 4, g->gd.dx * g->gd.dz,
                       (const double*)g->partial, F);
    HIPLAUNCHCHK("force integration");
    return GAP_OK;
}

gap_status integrate_force_moment_split(gap_grid_t g, const double* p, int32_t cavitation, double p_cav, double* F,
                                        void* stream)
{
    gap_status cs = check_integrate(g, p, F, cavitation, p_cav, "integrate_force_moment_split");
    if (cs != GAP_OK) return cs;
    hipStream_t st = (hipStream_t)stream;
    const ChunkMap cm = g->cm;
    hipLaunchKernelGGL((k_forces<10>), dim3(cm.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm, g->tables(), p,
                       cavitation, p_cav, g->partial);
    hipLaunchKernelGGL(k_forces_finalize, dim3(1), dim3(GAP_BLOCK), 0, st, cm, g->n_cond, 10, g->gd.dx * g->gd.dz,
                       (const double*)g->partial, F);
    HIPLAUNCHCHK("split force integration");
    return GAP_OK;
}

}  // extern "C"

namespace {

// Device scratch of integrate_force_moment_noalloc: the cos / sin table of the cell centres
// (2 n_theta doubles) followed by the per-chunk partial sums (4 per row chunk).  Each GPU holds
// its own copy for the life of the process.  In host code `scratch` is only a stand-in for the
// symbol: every use goes through the device address that hipGetSymbolAddress returns.
constexpr size_t kScratchDoubles = 49152;   // 384 KiB
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per device.
gap_status scratch_address(double** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GAP_EDEVICE, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(GAP_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return GAP_OK;
}

}  // namespace

extern "C" {

gap_status integrate_force_moment_noalloc(const gap_geom* geom, int32_t n_cond, const double* e, const double* tex_c,
                                          const double* p, int32_t cavitation, double p_cav, double* F, void* stream)
{
    gap_status st = validate_geom(geom);
    if (st != GAP_OK) return st;
    if (n_cond < 1 || n_cond > GAP_MAX_COND) return fail(GAP_EINVAL, "n_cond = %d outside [1, %d]", n_cond, GAP_MAX_COND);
    if (!e || !p || !F) return fail(GAP_EINVAL, "e, p and F must be non-NULL");
    if (cavitation != GAP_CAVITATION_NONE && cavitation != GAP_CAVITATION_CLAMP)
        return fail(GAP_EINVAL, "unknown cavitation mode");
    if (!is_finite(p_cav)) return fail(GAP_EINVAL, "p_cav must be finite");
    CondDev cd{};
    for (int c = 0; c < n_cond; ++c) {
        for (int q = 0; q < 4; ++q) {
            if (!is_finite(e[4 * c + q])) return fail(GAP_EINVAL, "e of condition %d is not finite", c);
            cd.e[c][q] = e[4 * c + q];
        }
        const double c0 = std::hypot(cd.e[c][0], cd.e[c][1]);
        const double c1 = std::hypot(cd.e[c][2], cd.e[c][3]);
        if (c0 >= geom->clearance || c1 >= geom->clearance)
            return fail(GAP_ECONTACT, "condition %d: |e| at a gap end (%.6g, %.6g) >= clearance %.6g", c, c0, c1,
                        geom->clearance);
    }
    cd.n_cond = n_cond;
    const int nt = geom->n_theta;
    const ChunkMap cm = make_chunks(geom->n_axial, n_cond);
    const size_t need = 2 * (size_t)nt + 4 * (size_t)cm.total;
    if (need > kScratchDoubles)
        return fail(GAP_EINVAL, "n_theta = %d, n_axial = %d, %d conditions need %zu scratch doubles, the limit is %zu",
                    nt, geom->n_axial, n_cond, need, kScratchDoubles);
    double* ws = nullptr;
    st = scratch_address(&ws);
    if (st != GAP_OK) return st;
    const GeomDev gd = geom_dev(*geom);
    TablesDev tb{};
    tb.cos_c = ws;
    tb.sin_c = ws + nt;
    tb.tex_c = tex_c;
    double* part = ws + 2 * nt;
    hipStream_t hs = (hipStream_t)stream;
    hipLaunchKernelGGL(k_trig_centres, dim3((nt + GAP_BLOCK - 1) / GAP_BLOCK), dim3(GAP_BLOCK), 0, hs, nt, gd.dth, ws,
                       ws + nt);
    hipLaunchKernelGGL((k_forces<4>), dim3(cm.total), dim3(GAP_BLOCK), 0, hs, gd, cd, cm, tb, p, cavitation, p_cav,
                       part);
    hipLaunchKernelGGL(k_forces_finalize, dim3(1), dim3(GAP_BLOCK), 0, hs, cm, n_cond, 4, gd.dx * gd.dz,
                       (const double*)part, F);
    HIPLAUNCHCHK("handle-free force integration");
    return GAP_OK;
}

gap_status rebuild_pressure_field(gap_grid_t g, const double* p, int32_t cavitation, double p_cav, double* out,
                                  void* stream)
{
    gap_status cs = check_integrate(g, p, out, cavitation, p_cav, "rebuild_pressure_field");
    if (cs != GAP_OK) return cs;
    hipStream_t st = (hipStream_t)stream;
    const size_t total = (size_t)g->n_cond * (g->nz + 2) * g->nt;
    hipLaunchKernelGGL(k_rebuild, dim3((unsigned)((total + GAP_BLOCK - 1) / GAP_BLOCK)), dim3(GAP_BLOCK), 0, st, g->gd,
                       g->n_cond, p, cavitation, p_cav, out);
    HIPLAUNCHCHK("k_rebuild");
    return GAP_OK;
}

gap_status jacobian_fd(gap_grid_t g, const double* F, double* J, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    if (!F || !J) return fail(GAP_EINVAL, "F and J must be non-NULL");
    if (!g->assembled || g->n_cond != GAP_MAX_COND) return fail(GAP_ESTATE, "jacobian_fd needs 9 assembled conditions");
    Delta8 dl;
    for (int k = 0; k < 8; ++k) dl.d[k] = g->delta[k];
    hipLaunchKernelGGL(k_jacobian_fd, dim3(1), dim3(64), 0, (hipStream_t)stream, F, dl, J);
    HIPLAUNCHCHK("k_jacobian_fd");
    return GAP_OK;
}

gap_status gap_kernel_timing(gap_grid_t g, int32_t enable)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    if (enable < 0) return fail(GAP_EINVAL, "kernel timing period %d is negative", enable);
    if (enable) {
        for (int k = 0; k < GAP_KERNEL_COUNT; ++k) {
            g->launches[k] = 0;
            g->total_ms[k] = 0.0;
        }
        g->timing_period = enable;
        g->ev_tick = 0;
    }
    g->timing = enable != 0;
    g->ev_used = 0;
    g->ev_open = false;
    return GAP_OK;
}

gap_status gap_kernel_stats(gap_grid_t g, int32_t kernel, int64_t* launches, double* total_ms)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    if (kernel < 0 || kernel >= GAP_KERNEL_COUNT) return fail(GAP_EINVAL, "unknown kernel %d", kernel);
    if (launches) *launches = g->launches[kernel];
    if (total_ms) *total_ms = g->total_ms[kernel];
    return GAP_OK;
}

gap_status gap_pcg_history(gap_grid_t g, int32_t capacity)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "gap_pcg_history");
    if (capacity < 0 || capacity > (1 << 24)) return fail(GAP_EINVAL, "capacity must lie in [0, 2^24]");
    if (g->hist) {
        HIPCHK(hipDeviceSynchronize());
        (void)hipFree(g->hist);
        g->hist = nullptr;
        g->hist_cap = 0;
    }
    if (capacity > 0) {
        gap_status s = dmalloc(&g->hist, 2 * (size_t)capacity);
        if (s != GAP_OK) return s;
        HIPCHK(hipMemset(g->hist, 0, 2 * (size_t)capacity * sizeof(double)));
        g->hist_cap = capacity;
    }
    return GAP_OK;
}

gap_status gap_get_pcg_history(gap_grid_t g, double* alpha, double* beta, int32_t cap, int32_t* count, void* stream)
{
    if (!g || !alpha || !beta || !count || cap < 0) return fail(GAP_EINVAL, "grid, alpha, beta and count must be non-NULL, cap >= 0");
    if (!g->hist) return fail(GAP_ESTATE, "PCG scalars are not being recorded (gap_pcg_history)");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(st));
    const int k = std::min(std::min(g->sc_host->iterations, g->hist_cap), (int)cap);
    *count = 0;
    if (k > 0) {
        std::vector<double> h(2 * (size_t)k);
        HIPCHK(hipMemcpyAsync(h.data(), g->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int j = 0; j < k; ++j) {
            alpha[j] = h[2 * j];
            beta[j] = j ? h[2 * j + 1] : 0.0;
        }
    }
    *count = k;
    return GAP_OK;
}

gap_status gap_get_pcg_config(gap_grid_t g, gap_pcg_config* cfg)
{
    if (!g || !cfg) return fail(GAP_EINVAL, "grid and cfg must be non-NULL");
    cfg->threads_a = g->shape_a.NT;
    cfg->cols_per_thread_a = g->shape_a.Q;
    cfg->wg_per_cu_a = g->wg_a;
    cfg->occupancy_a = g->occ[0];
    cfg->threads_b = g->shape_b.NT;
    cfg->cols_per_thread_b = g->shape_b.Q;
    cfg->wg_per_cu_b = g->wg_b;
    cfg->occupancy_b = std::min(g->occ[1], g->occ[2]);
    cfg->threads_f = g->shape_f.NT;
    cfg->cols_per_thread_f = g->shape_f.Q;
    cfg->wg_per_cu_f = g->wg_f;
    cfg->occupancy_f = g->occ_f;
    cfg->cols_per_lane_w = g->shape_w.Q;
    cfg->wg_per_cu_w = g->wg_w;
    cfg->occupancy_w = g->occ_w;
    int groups = 1;
    strip_layout(g->nt, g->shape_w.Q, 1, cfg->strips_w, groups);
    return GAP_OK;
}

namespace {

gap_status check_shape(gap_grid_t g, PcgShape sh)
{
    const int cols = sh.NT * sh.Q;
    if (!shape_known(sh) || cols < g->nt || cols >= 2 * g->nt + 64)
        return fail(GAP_EINVAL, "shape %d x %d does not fit a ring of %d cells", sh.NT, sh.Q, g->nt);
    if (pcg_lds_bytes(kPcgOne, cols) + 2048 > (size_t)g->lds_max)
        return fail(GAP_EINVAL, "shape %d x %d needs more LDS than a workgroup may use", sh.NT, sh.Q);
    return GAP_OK;
}

// One timed run of the tuner: average device us per launch of A and of B (two-launch
// iteration), or of the one-launch kernel in *us_a (*us_b = 0).
gap_status tune_run(gap_grid_t g, const gap_solver_opts* t, double* p, void* stream, double* us_a, double* us_b)
{
    for (int k = 0; k < GAP_KERNEL_COUNT; ++k) {
        g->launches[k] = 0;
        g->total_ms[k] = 0.0;
    }
    const int period = g->timing_period;
    g->timing = true;
    g->timing_period = 1;
    g->ev_tick = 0;
    gap_status s = solve_joint_pcg(g, t, p, nullptr, stream);
    g->timing = false;
    g->timing_period = period;
    if (s != GAP_OK && s != GAP_ENOCONV) return s;
    const int ka = t->iteration == GAP_ITERATION_STRIPS     ? GAP_KERNEL_PCG_STRIPS
                   : t->iteration == GAP_ITERATION_ONE_LAUNCH ? GAP_KERNEL_PCG_ONE
                                                               : GAP_KERNEL_PCG_A;
    const int kb = t->iteration == GAP_ITERATION_TWO_LAUNCH ? GAP_KERNEL_PCG_B : -1;
    if (!g->launches[ka] || (kb >= 0 && !g->launches[kb])) return fail(GAP_EDEVICE, "the tuning run recorded no launches");
    *us_a = 1e3 * g->total_ms[ka] / (double)g->launches[ka];
    *us_b = kb >= 0 ? 1e3 * g->total_ms[kb] / (double)g->launches[kb] : 0.0;
    return GAP_OK;
}

}  // namespace

gap_status gap_set_pcg_config(gap_grid_t g, const gap_pcg_config* cfg)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    GAP_NOT_IN_BATCH(g, "gap_set_pcg_config");
    PcgShape sa = g->rings_ok ? pcg_candidates(g->nt)[0] : PcgShape{}, sb = sa, sf = sa;
    int wa = 0, wb = 0, wf = 0, qw = kStripDefaultQ, ww = 0;
    if (cfg) {
        if (g->rings_ok) {
            sa.NT = cfg->threads_a;
            sa.Q = cfg->cols_per_thread_a;
            sb.NT = cfg->threads_b;
            sb.Q = cfg->cols_per_thread_b;
            sf.NT = cfg->threads_f;
            sf.Q = cfg->cols_per_thread_f;
            gap_status cs = check_shape(g, sa);
            if (cs == GAP_OK) cs = check_shape(g, sb);
            if (cs == GAP_OK) cs = check_shape(g, sf);
            if (cs != GAP_OK) return cs;
        }
        if (!strip_q_known(cfg->cols_per_lane_w))
            return fail(GAP_EINVAL, "cols_per_lane_w = %d outside [1, %d]", cfg->cols_per_lane_w, kStripMaxQ);
        const int w[4] = {cfg->wg_per_cu_a, cfg->wg_per_cu_b, cfg->wg_per_cu_f, cfg->wg_per_cu_w};
        for (int k = g->rings_ok ? 0 : 3; k < 4; ++k)
            if (w[k] < 1 || w[k] > 8) return fail(GAP_EINVAL, "wg_per_cu must lie in [1, 8]");
        wa = w[0];
        wb = w[1];
        wf = w[2];
        qw = cfg->cols_per_lane_w;
        ww = w[3];
    }
    hipError_t e = hipSuccess;
    if (g->rings_ok) {
        e = use_shape(g, sa, sb, wa, wb);
        if (e == hipSuccess) e = use_shape_f(g, sf, wf);
    }
    if (e == hipSuccess) e = use_shape_w(g, qw, ww);
    if (e != hipSuccess) return fail(GAP_EDEVICE, "preparing the PCG kernels: %s", hipGetErrorString(e));
    return GAP_OK;
}

gap_status gap_tune_pcg(gap_grid_t g, const gap_solver_opts* o, double* p, int32_t iterations, gap_pcg_config* best,
                        double* us_per_iteration, void* stream)
{
    if (!g || !o || !p) return fail(GAP_EINVAL, "grid, opts and p must be non-NULL");
    GAP_NOT_IN_BATCH(g, "gap_tune_pcg");
    if (iterations < 2 || iterations > 10000) return fail(GAP_EINVAL, "iterations must lie in [2, 10000]");
    gap_status vs = validate_opts(g, o);
    if (vs != GAP_OK) return vs;
    if (!g->assembled) return fail(GAP_ESTATE, "gap_tune_pcg before assemble_joint_system");
    // a fixed number of iterations, no stopping test, plain launches timed by events
    gap_solver_opts t = *o;
    t.eps = 1e-300;
    t.max_iter = iterations;
    t.check_every = iterations;
    t.graph = 0;
    t.warm_start = 0;
    t.strategy = GAP_STRATEGY_SYNC;
    const bool timing = g->timing;
    const PcgShape orig_a = g->shape_a, orig_b = g->shape_b, orig_f = g->shape_f, orig_w = g->shape_w;
    const int orig_wa = g->wg_a, orig_wb = g->wg_b, orig_wf = g->wg_f, orig_ww = g->wg_w;   // restored if tuning fails
    const bool strip = o->iteration == GAP_ITERATION_STRIPS;
    const bool one = o->iteration == GAP_ITERATION_ONE_LAUNCH;
    struct Pick {
        PcgShape sh;
        int wg = 0;
        double us = 0.0;
        bool have = false;
    } pa, pb, da, db;   // best and default, per kernel
    std::vector<PcgShape> cands;
    if (strip) {
        for (int q = 1; q <= kStripMaxQ; ++q) cands.push_back(PcgShape{kStripThreads, q});
    } else {
        cands = pcg_candidates(g->nt);
    }
    const PcgShape def = strip ? PcgShape{kStripThreads, kStripDefaultQ} : cands[0];
    gap_status result = GAP_OK;
    for (const PcgShape sh : cands) {
        if (result != GAP_OK) break;
        if (!strip && pcg_lds_bytes(one ? kPcgOne : kPcgB, sh.NT * sh.Q) + 2048 > (size_t)g->lds_max) continue;
        int occ[3];
        bool ok = true;
        if (strip) {
            ok = strip_q(sh.Q, o->neumann) == sh.Q && strip_prepare(sh.Q, o->neumann, &occ[0]) == hipSuccess;
            occ[1] = occ[2] = occ[0];
        } else if (one) {
            for (int k = 0; k < 2 && ok; ++k) ok = pcg_prepare(sh, k ? kPcgOneInit : kPcgOne, g->nt, &occ[k]) == hipSuccess;
            occ[0] = std::min(occ[0], occ[1]);
            occ[1] = occ[2] = occ[0];
        } else {
            for (int which = 0; which < 3 && ok; ++which) ok = pcg_prepare(sh, which, g->nt, &occ[which]) == hipSuccess;
        }
        if (!ok) continue;
        const int ob = std::min(occ[1], occ[2]);
        // A and B are timed in the same runs; wg_per_cu of A and of B advance together.  The
        // one-launch kernel is timed as "A".
        for (int w = 1; w <= std::max(occ[0], ob) && result == GAP_OK; ++w) {
            const int wa = std::min(w, occ[0]), wb = std::min(w, ob);
            const hipError_t pe = strip ? use_shape_w(g, sh.Q, wa) : one ? use_shape_f(g, sh, wa) : use_shape(g, sh, sh, wa, wb);
            if (pe != hipSuccess) {
                result = fail(GAP_EDEVICE, "preparing the PCG kernels");
                break;
            }
            double ua = 0.0, ub = 0.0, ta = 0.0, tb = 0.0;
            result = tune_run(g, &t, p, stream, &ua, &ub);                       // warm-up
            for (int rep = 0; rep < 2 && result == GAP_OK; ++rep) {
                result = tune_run(g, &t, p, stream, &ua, &ub);
                ta = rep ? std::min(ta, ua) : ua;
                tb = rep ? std::min(tb, ub) : ub;
            }
            if (result != GAP_OK) break;
            if (!pa.have || ta < pa.us) pa = {sh, wa, ta, true};
            if (!pb.have || tb < pb.us || one || strip) pb = {sh, wb, tb, true};
            const bool is_def = sh.NT == def.NT && sh.Q == def.Q;
            if (is_def && wa == occ[0]) da = {sh, wa, ta, true};
            if (is_def && wb == ob) db = {sh, wb, tb, true};
        }
    }
    g->timing = timing;
    if (result != GAP_OK || !pa.have || !pb.have) {
        if (g->rings_ok) {
            (void)use_shape(g, orig_a, orig_b, orig_wa, orig_wb);
            (void)use_shape_f(g, orig_f, orig_wf);
        }
        (void)use_shape_w(g, orig_w.Q, orig_ww);
        return result != GAP_OK ? result : fail(GAP_EDEVICE, "no kernel shape could be prepared");
    }
    // keep the default unless the best is at least 1 % faster (stable choice on near-ties)
    if (da.have && da.us <= 1.01 * pa.us) pa = da;
    if (db.have && db.us <= 1.01 * pb.us) pb = db;
    // the kernels of the other iteration kind keep their configuration
    hipError_t e = strip ? use_shape_w(g, pa.sh.Q, pa.wg)
                   : one ? use_shape_f(g, pa.sh, pa.wg) : use_shape(g, pa.sh, pb.sh, pa.wg, pb.wg);
    if (e != hipSuccess) return fail(GAP_EDEVICE, "preparing the PCG kernels: %s", hipGetErrorString(e));
    gap_pcg_config win{};
    gap_get_pcg_config(g, &win);
    if (best) *best = win;
    if (us_per_iteration) *us_per_iteration = pa.us + pb.us;
    return GAP_OK;
}

gap_status gap_tune_neumann(gap_grid_t g, const gap_solver_opts* o, double* p, int32_t max_order, int32_t* best,
                            double* seconds, void* stream)
{
    if (!g || !o || !p || !best) return fail(GAP_EINVAL, "grid, opts, p and best must be non-NULL");
    GAP_NOT_IN_BATCH(g, "gap_tune_neumann");
    if (max_order < 1 || max_order > kStripMaxNeumann)
        return fail(GAP_EINVAL, "max_order must lie in [1, %d]", kStripMaxNeumann);
    if (o->precond != GAP_PRECOND_ASSOR2 || o->iteration != GAP_ITERATION_STRIPS)
        return fail(GAP_EINVAL, "the Neumann order is tuned for precond = GAP_PRECOND_ASSOR2, iteration = GAP_ITERATION_STRIPS");
    if (!g->assembled) return fail(GAP_ESTATE, "gap_tune_neumann before assemble_joint_system");
    gap_solver_opts t = *o;
    t.warm_start = 0;
    gap_pcg_config cfgs[kStripMaxNeumann + 1];
    double secs[kStripMaxNeumann + 1] = {0.0};
    int pick = 0;
    for (int m = 1; m <= max_order; ++m) {
        t.neumann = m;
        gap_status vs = validate_opts(g, &t);
        if (vs != GAP_OK) return vs;
        // the strip kernel's configuration for this order, then one warm and one timed solve
        gap_status ts = gap_tune_pcg(g, &t, p, 20, &cfgs[m], nullptr, stream);
        if (ts != GAP_OK) return ts;
        ts = solve_joint_pcg(g, &t, p, nullptr, stream);
        if (ts != GAP_OK && ts != GAP_ENOCONV) return ts;
        const auto t0 = std::chrono::steady_clock::now();
        ts = solve_joint_pcg(g, &t, p, nullptr, stream);       // synchronizes the stream
        const auto t1 = std::chrono::steady_clock::now();
        if (ts != GAP_OK) return ts;
        secs[m] = std::chrono::duration<double>(t1 - t0).count();
        if (!pick || secs[m] < secs[pick]) pick = m;
    }
    gap_status cs = gap_set_pcg_config(g, &cfgs[pick]);
    if (cs != GAP_OK) return cs;
    *best = pick;
    if (seconds)
        for (int m = 1; m <= max_order; ++m) seconds[m - 1] = secs[m];
    return GAP_OK;
}

gap_status gap_read_system(gap_grid_t g, int32_t k, double* kx, double* kz, double* S, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    if (!g->assembled) return fail(GAP_ESTATE, "nothing assembled");
    if (k < 0 || k >= g->n_cond) return fail(GAP_EINVAL, "condition %d out of range", k);
    hipStream_t st = (hipStream_t)stream;
    const int o = g->cd.op[k];
    const size_t n = g->n, nt = g->nt;
    if (kx) HIPCHK(hipMemcpyAsync(kx, g->kx + o * n, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (kz) HIPCHK(hipMemcpyAsync(kz, g->kz + o * (n + nt), (n + nt) * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (S) HIPCHK(hipMemcpyAsync(S, g->S + k * n, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    return GAP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Batched execution of several joint systems (requests) of possibly different grids.

__global__ void k_gather_records(const PcgDev* __restrict__ reqs, int cap, PcgScalars* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < cap && reqs[s].sc) out[s] = *reqs[s].sc;
}

struct gap_batch_s {
    static constexpr int kCap = 128;                         // request slots (work entries hold 8 bits)
    struct Req {
        int id = 0, slot = 0;
        gap_grid_t g = nullptr;
        bool done = false;
        bool held = false;                                   // excluded from the launches until released
        bool scheduled = false;                              // in the launches of the current schedule
        long f_count = 0;                                    // one-launch kernel launches that included it
    };
    std::vector<Req> reqs;
    PcgDev *reqs_dev = nullptr, *reqs_host = nullptr;        // slot-indexed request records
    PcgScalars *rec_dev = nullptr, *rec_host = nullptr;      // slot-indexed copies of their device records
    int* work = nullptr;                                     // tables A then B
    size_t work_cap = 0;
    int blocks_a = 0, blocks_b = 0;
    bool dirty = true;
    int* init_work = nullptr;
    size_t init_cap = 0;
    int occ_a = 1, occ_b = 1, occ_f = 1, cus = 256;
    PcgShape shape = pcg_candidates(2048)[0];            // the shape of the largest ring
    PcgShape shape_w{kStripThreads, kStripDefaultQ};         // the strip kernel's shape
    int occ_w = 1;
    int mode = GAP_ITERATION_ONE_LAUNCH;                     // iteration kind of the requests (set by the first)
    int neumann = 1;                                         // their Neumann order (set by the first)
    int wg_target = 0;                                       // strip chunking target (workgroups per CU), 0: occupancy
    long launches = 0;                                       // one-launch kernel launches so far
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int exec_iters = 0, exec_blocks_a = 0, exec_blocks_b = 0, exec_par0 = 0, exec_pk = -1, exec_sync = 0;
    int pk = -1;                                             // preconditioner common to the scheduled requests, or -1
    int sync = 0;                                            // strips: every scheduled request streams enough bytes
    const int* exec_work = nullptr;
    int next_id = 1;
};

namespace {

constexpr int kBatchShape = 2048;   // batch launches use the kernel shape of the largest ring

void batch_release(gap_batch_t b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->reqs_dev) (void)hipFree(b->reqs_dev);
    if (b->reqs_host) (void)hipHostFree(b->reqs_host);
    if (b->rec_dev) (void)hipFree(b->rec_dev);
    if (b->rec_host) (void)hipHostFree(b->rec_host);
    if (b->work) (void)hipFree(b->work);
    if (b->init_work) (void)hipFree(b->init_work);
    delete b;
}

// Grows a schedule table to hold `need` entries, at least doubling it, so that a batch whose
// membership keeps changing reallocates (and synchronizes the device in hipFree) only a few
// times.
gap_status ensure_ints(int** p, size_t* cap, size_t need)
{
    if (need <= *cap) return GAP_OK;
    need = std::max(need, std::max<size_t>(2 * *cap, 4096));
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc((void**)p, need * sizeof(int)) != hipSuccess) {
        *p = nullptr;
        return fail(GAP_ENOMEM, "hipMalloc of a schedule table failed");
    }
    *cap = need;
    return GAP_OK;
}

}  // namespace

extern "C" {

gap_status gap_grid_bytes(const gap_geom* geom, int32_t max_cond, int64_t* bytes)
{
    if (!bytes) return fail(GAP_EINVAL, "bytes is NULL");
    gap_status st = validate_geom(geom);
    if (st != GAP_OK) return st;
    if (max_cond != 1 && max_cond != GAP_MAX_COND) return fail(GAP_EINVAL, "max_cond must be 1 or 9");
    const int64_t nt = geom->n_theta, nz = geom->n_axial, n = nt * nz;
    const int64_t max_op = max_cond == GAP_MAX_COND ? 5 : 1;
    const ChunkMap cm1 = make_chunks((int)nz, 1), cm9 = make_chunks((int)nz, GAP_MAX_COND);
    int64_t d = 4 * nt + 2 * n + (nz + 1) * nt;              // tables and texture samples
    d += max_op * n + max_op * (n + nt);                     // face conductances
    d += max_op * 2 * (n + nt);                              // and as pairs
    d += 7 * (int64_t)max_cond * n;                          // S, r (2), u (2), z (2)
    d += 10 * (int64_t)std::max(cm1.total, cm9.total);       // force partials
    int strips1 = 1, groups1 = 1;
    strip_layout((int)nt, 1, kStripMaxNeumann, strips1, groups1);
    d += 15 * (int64_t)max_cond * std::max<int64_t>(nz, groups1);   // PCG partials
    d += (int64_t)max_cond * n;                              // the caller's pressure field
    *bytes = d * (int64_t)sizeof(double) + 4096;
    return GAP_OK;
}

gap_status gap_batch_create(gap_batch_t* out)
{
    if (!out) return fail(GAP_EINVAL, "out is NULL");
    *out = nullptr;
    gap_batch_t b = new gap_batch_s;
    const int cap = gap_batch_s::kCap;
    if (hipMalloc((void**)&b->reqs_dev, cap * sizeof(PcgDev)) != hipSuccess ||
        hipHostMalloc((void**)&b->reqs_host, cap * sizeof(PcgDev), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&b->rec_dev, cap * sizeof(PcgScalars)) != hipSuccess ||
        hipHostMalloc((void**)&b->rec_host, cap * sizeof(PcgScalars), hipHostMallocDefault) != hipSuccess) {
        batch_release(b);
        return fail(GAP_ENOMEM, "allocating the batch records failed");
    }
    std::memset(b->reqs_host, 0, cap * sizeof(PcgDev));
    std::memset(b->rec_host, 0, cap * sizeof(PcgScalars));
    hipError_t e = hipMemcpy(b->reqs_dev, b->reqs_host, cap * sizeof(PcgDev), hipMemcpyHostToDevice);
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess && hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        b->cus = 256;
    if (e == hipSuccess) e = pcg_prepare(b->shape, 0, kBatchShape, &b->occ_a);
    int occ_b = 1, occ_i = 1;
    if (e == hipSuccess) e = pcg_prepare(b->shape, 1, kBatchShape, &occ_b);
    if (e == hipSuccess) e = pcg_prepare(b->shape, 2, kBatchShape, &occ_i);
    int occ_f = 1, occ_fi = 1;
    if (e == hipSuccess) e = pcg_prepare(b->shape, kPcgOne, kBatchShape, &occ_f);
    if (e == hipSuccess) e = pcg_prepare(b->shape, kPcgOneInit, kBatchShape, &occ_fi);
    if (e != hipSuccess) {
        batch_release(b);
        return fail(GAP_EDEVICE, "creating the batch: %s", hipGetErrorString(e));
    }
    if (e == hipSuccess) e = strip_prepare(b->shape_w.Q, 1, &b->occ_w);
    if (e != hipSuccess) {
        batch_release(b);
        return fail(GAP_EDEVICE, "creating the batch: %s", hipGetErrorString(e));
    }
    b->occ_b = std::min(occ_b, occ_i);
    b->occ_f = std::min(occ_f, occ_fi);
    *out = b;
    return GAP_OK;
}

gap_status gap_batch_destroy(gap_batch_t b)
{
    if (!b) return GAP_OK;
    (void)hipDeviceSynchronize();
    for (auto& r : b->reqs) r.g->batch = nullptr;        // the handles are free again
    batch_release(b);
    return GAP_OK;
}

gap_status gap_batch_add(gap_batch_t b, gap_grid_t g, const gap_solver_opts* o, double* p, int32_t* id, void* stream)
{
    if (!b || !g || !p || !id) return fail(GAP_EINVAL, "batch, grid, p and id must be non-NULL");
    gap_status vs = validate_opts(g, o);
    if (vs != GAP_OK) return vs;
    if (!g->assembled) return fail(GAP_ESTATE, "gap_batch_add needs an assembled grid");
    if (g->batch) return fail(GAP_EINVAL, "this grid is already in a batch");
    if (!b->reqs.empty() && o->iteration == b->mode && o->neumann != b->neumann)
        return fail(GAP_EINVAL, "the requests of a batch share one Neumann order (the batch runs order %d)", b->neumann);
    if (!b->reqs.empty() && o->iteration != b->mode)
        return fail(GAP_EINVAL, "the requests of a batch share one iteration kind (the batch runs %s launches)",
                    b->mode == GAP_ITERATION_STRIPS ? "strip" : b->mode == GAP_ITERATION_ONE_LAUNCH ? "one-launch"
                                                                                                 : "two-launch");
    const bool strip = o->iteration == GAP_ITERATION_STRIPS;
    const bool one = o->iteration != GAP_ITERATION_TWO_LAUNCH;
    int slot = -1;
    std::vector<bool> used(gap_batch_s::kCap, false);
    for (const auto& r : b->reqs) used[r.slot] = true;
    for (int s = 0; s < gap_batch_s::kCap && slot < 0; ++s)
        if (!used[s]) slot = s;
    if (slot < 0) return fail(GAP_EBUDGET, "all %d batch slots are in use", gap_batch_s::kCap);
    hipStream_t st = (hipStream_t)stream;
    gap_status ps = prepare_precond(g, o, st);
    if (ps != GAP_OK) return ps;

    PcgDev a{};
    a.kx = g->kx;
    a.kxz = g->kxz;
    a.kz = g->kz;
    a.minv = g->minv;
    a.S = g->S;
    a.p = p;
    for (int c = 0; c < GAP_MAXC; ++c) a.op[c] = g->cd.op[c];
    a.n_cond = g->n_cond;
    a.per_cond = o->scalars == GAP_SCALARS_PER_COND;
    a.async = o->strategy == GAP_STRATEGY_ASYNC;
    a.warm = o->warm_start ? 1 : 0;
    fill_pcg(g, a, o);
    // chunking depends only on the request and the batch kernel shape, so a request gets
    // the same reduction order (bitwise the same result) alone and in any mix
    a.n_strips = a.strip_groups = 1;
    if (strip) {
        int occ = 1;
        const int Qb = strip_q(b->shape_w.Q, o->neumann);
        const hipError_t oe = strip_prepare(Qb, o->neumann, &occ);
        if (oe != hipSuccess) return fail(GAP_EDEVICE, "preparing the strip kernel: %s", hipGetErrorString(oe));
        const int wg = b->wg_target > 0 ? std::min(b->wg_target, occ) : occ;
        strip_chunks(g->nz, g->nt, a.n_cond, Qb, o->neumann, wg * b->cus, a);
    } else if (one) {
        pcg_chunks(g->nz, g->nt, a.n_cond, b->occ_f * b->cus, a.chunks_b, a.rows_b);
        a.chunks_a = a.chunks_b;
        a.rows_a = a.rows_b;
    } else {
        pcg_chunks(g->nz, g->nt, a.n_cond, b->occ_a * b->cus, a.chunks_a, a.rows_a);
        pcg_chunks(g->nz, g->nt, a.n_cond, b->occ_b * b->cus, a.chunks_b, a.rows_b);
    }
    a.par_off = 0;                               // set when the request enters a schedule
    HIPCHK(hipStreamSynchronize(st));
    b->reqs_host[slot] = a;
    HIPCHK(hipMemcpyAsync(b->reqs_dev + slot, b->reqs_host + slot, sizeof(PcgDev), hipMemcpyHostToDevice, st));

    std::vector<std::vector<int>> gb;
    pcg_groups(slot, a.chunks_b, a.n_cond, a.op, gb, strip ? a.strip_groups : 1);
    const std::vector<int> tb = pcg_schedule(gb);
    gap_status es = ensure_ints(&b->init_work, &b->init_cap, tb.size());
    if (es != GAP_OK) return es;
    HIPCHK(hipMemcpyAsync(b->init_work, tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice, st));
    PcgShape sh_init = strip ? b->shape_w : b->shape;
    sh_init.M = o->neumann;
    if (strip) {
        sh_init.Q = strip_q(sh_init.Q, sh_init.M);
        sh_init.sync = strip_sync(sh_init.M, a) ? 1 : 0;
    }
    hipError_t le = launch_pcg(sh_init, strip ? kPcgStripInit : (one ? kPcgOneInit : kPcgInit), kBatchShape,
                               b->reqs_dev, b->init_work, (int)tb.size(), st);
    if (le != hipSuccess) return fail(GAP_EDEVICE, "launch of the initial residual kernel: %s", hipGetErrorString(le));
    HIPCHK(hipStreamSynchronize(st));

    gap_batch_s::Req r;
    r.id = b->next_id++;
    r.slot = slot;
    r.g = g;
    b->mode = o->iteration;
    b->neumann = o->neumann;
    g->batch = b;
    b->reqs.push_back(r);
    b->dirty = true;
    *id = r.id;
    return GAP_OK;
}

gap_status gap_batch_step(gap_batch_t b, int32_t iterations, int32_t use_graph, int32_t* n_done, void* stream)
{
    if (!b) return fail(GAP_EINVAL, "batch is NULL");
    if (iterations < 1) return fail(GAP_EINVAL, "iterations must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    const bool strip = b->mode == GAP_ITERATION_STRIPS;
    const bool one = b->mode != GAP_ITERATION_TWO_LAUNCH;
    const int one_which = strip ? kPcgStrip : (one ? kPcgOne : 0);
    if (b->dirty) {
        std::vector<std::vector<int>> ga, gb;
        b->pk = -2;                                  // the preconditioner common to the scheduled requests
        b->sync = 1;                                 // the synchronized march if every one qualifies
        for (auto& r : b->reqs) {
            r.scheduled = !(r.done || r.held);
            if (!r.scheduled) continue;
            PcgDev& a = b->reqs_host[r.slot];
            b->pk = (b->pk == -2 || b->pk == a.precond) ? a.precond : -1;
            if (!strip_sync(b->neumann, a)) b->sync = 0;
            if (!one) pcg_groups(r.slot, a.chunks_a, a.n_cond, a.op, ga);
            pcg_groups(r.slot, a.chunks_b, a.n_cond, a.op, gb, strip ? a.strip_groups : 1);
            if (one) {
                // the request's next iteration has the parity of its own launch count
                const int off = (int)((r.f_count ^ b->launches) & 1);
                if (a.par_off != off) {
                    a.par_off = off;
                    HIPCHK(hipMemcpyAsync(b->reqs_dev + r.slot, b->reqs_host + r.slot, sizeof(PcgDev),
                                          hipMemcpyHostToDevice, st));
                }
            }
        }
        const std::vector<int> ta = pcg_schedule(ga), tb = pcg_schedule(gb);
        gap_status es = ensure_ints(&b->work, &b->work_cap, ta.size() + tb.size() + 1);
        if (es != GAP_OK) return es;
        if (!ta.empty()) HIPCHK(hipMemcpyAsync(b->work, ta.data(), ta.size() * sizeof(int), hipMemcpyHostToDevice, st));
        if (!tb.empty())
            HIPCHK(hipMemcpyAsync(b->work + ta.size(), tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        b->blocks_a = (int)ta.size();
        b->blocks_b = (int)tb.size();
        b->dirty = false;
    }
    PcgShape sh_one = strip ? b->shape_w : b->shape;
    if (strip) {
        sh_one.pk = b->pk >= 0 ? b->pk : -1;
        sh_one.M = b->neumann;
        sh_one.Q = strip_q(sh_one.Q, sh_one.M);
        sh_one.sync = b->sync;
    }
    if ((one ? b->blocks_b : b->blocks_a) > 0) {
        const int* wa = b->work;
        const int* wb = b->work + b->blocks_a;
        const int par0 = one ? (int)(b->launches & 1) : 0;
        if (use_graph) {
            if (!b->exec || b->exec_iters != iterations || b->exec_blocks_a != b->blocks_a ||
                b->exec_blocks_b != b->blocks_b || b->exec_work != b->work || b->exec_par0 != par0 ||
                b->exec_pk != sh_one.pk || b->exec_sync != sh_one.sync) {
                if (b->exec) (void)hipGraphExecDestroy(b->exec);
                b->exec = nullptr;
                if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
                hipError_t ce = capture_block(b->cap_stream, iterations, b->shape, sh_one, kBatchShape, b->reqs_dev, wa,
                                              b->blocks_a, wb, b->blocks_b, &b->exec, one_which, par0);
                if (ce != hipSuccess) {
                    b->exec = nullptr;
                    return fail(GAP_EDEVICE, "capturing the batch block: %s", hipGetErrorString(ce));
                }
                b->exec_iters = iterations;
                b->exec_blocks_a = b->blocks_a;
                b->exec_blocks_b = b->blocks_b;
                b->exec_work = b->work;
                b->exec_par0 = par0;
                b->exec_pk = sh_one.pk;
                b->exec_sync = sh_one.sync;
            }
            HIPCHK(hipGraphLaunch(b->exec, st));
        } else {
            for (int it = 0; it < iterations; ++it) {
                hipError_t le;
                if (one) {
                    le = launch_pcg(sh_one, one_which, kBatchShape, b->reqs_dev, wb, b->blocks_b, st, (par0 + it) & 1);
                } else {
                    le = launch_pcg(b->shape, kPcgA, kBatchShape, b->reqs_dev, wa, b->blocks_a, st);
                    if (le == hipSuccess) le = launch_pcg(b->shape, kPcgB, kBatchShape, b->reqs_dev, wb, b->blocks_b, st);
                }
                if (le != hipSuccess) return fail(GAP_EDEVICE, "launch of a batch iteration: %s", hipGetErrorString(le));
            }
        }
        if (one) {
            b->launches += iterations;
            for (auto& r : b->reqs)
                if (r.scheduled) r.f_count += iterations;
        }
    }
    hipLaunchKernelGGL(k_gather_records, dim3(1), dim3(gap_batch_s::kCap), 0, st, (const PcgDev*)b->reqs_dev,
                       gap_batch_s::kCap, b->rec_dev);
    HIPLAUNCHCHK("k_gather_records");
    HIPCHK(hipMemcpyAsync(b->rec_host, b->rec_dev, gap_batch_s::kCap * sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int done = 0;
    for (auto& r : b->reqs) {
        if (!r.done && b->rec_host[r.slot].done) {
            r.done = true;
            b->dirty = true;
        }
        done += r.done ? 1 : 0;
    }
    if (n_done) *n_done = done;
    return GAP_OK;
}

gap_status gap_batch_set_target(gap_batch_t b, int32_t wg_per_cu)
{
    if (!b) return fail(GAP_EINVAL, "batch is NULL");
    if (wg_per_cu < 0 || wg_per_cu > 8) return fail(GAP_EINVAL, "wg_per_cu must lie in [0, 8]");
    b->wg_target = wg_per_cu;
    return GAP_OK;
}

gap_status gap_batch_hold(gap_batch_t b, int32_t id, int32_t hold)
{
    if (!b) return fail(GAP_EINVAL, "batch is NULL");
    for (auto& r : b->reqs)
        if (r.id == id) {
            if (r.held != (hold != 0)) {
                r.held = hold != 0;
                b->dirty = true;
            }
            return GAP_OK;
        }
    return fail(GAP_EINVAL, "no request %d in the batch", id);
}

gap_status gap_batch_poll(gap_batch_t b, int32_t* ids, int32_t cap, int32_t* count)
{
    if (!b || !count) return fail(GAP_EINVAL, "batch and count must be non-NULL");
    int k = 0;
    for (const auto& r : b->reqs)
        if (r.done) {
            if (ids && k < cap) ids[k] = r.id;
            ++k;
        }
    *count = k;
    return GAP_OK;
}

gap_status gap_batch_remove(gap_batch_t b, int32_t id, gap_solve_info* info, void* stream)
{
    if (!b) return fail(GAP_EINVAL, "batch is NULL");
    auto it = std::find_if(b->reqs.begin(), b->reqs.end(), [&](const gap_batch_s::Req& r) { return r.id == id; });
    if (it == b->reqs.end()) return fail(GAP_EINVAL, "no request %d in the batch", id);
    hipStream_t st = (hipStream_t)stream;
    const PcgScalars& h = b->rec_host[it->slot];
    gap_status result = GAP_OK;
    if (!it->done) result = fail(GAP_ENOCONV, "request %d removed before convergence", id);
    else if (h.status == -4) result = fail(GAP_ENONFINITE, "request %d: non-finite value", id);
    else if (h.status == -3) result = fail(GAP_ENOCONV, "request %d: no convergence after %d iterations", id, h.iterations);
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iterations = h.iterations;
        info->n_cond = b->reqs_host[it->slot].n_cond;
        info->rel_residual = h.rel;
        for (int c = 0; c < info->n_cond; ++c) info->rel_residual_cond[c] = h.rel_cond[c];
        info->true_rel_residual = -1.0;
        for (int c = 0; c < GAP_MAX_COND; ++c) info->true_rel_residual_cond[c] = -1.0;
        info->status = result;
    }
    // clear the slot so the record gather skips it
    HIPCHK(hipStreamSynchronize(st));
    std::memset(b->reqs_host + it->slot, 0, sizeof(PcgDev));
    HIPCHK(hipMemcpyAsync(b->reqs_dev + it->slot, b->reqs_host + it->slot, sizeof(PcgDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    it->g->batch = nullptr;
    b->reqs.erase(it);
    b->dirty = true;
    return GAP_OK;
}

}  // extern "C"
