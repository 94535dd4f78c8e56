// Host side of the gapsolve C ABI: handle management, validation, launches and the device-
// resident PCG loop.  See include/gapsolve.h for the contract of every entry point.
#include "gapsolve.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "gap_kernels.hpp"

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

constexpr int kTargetChunks = 2048;
constexpr int kMaxThetaCells = 4096;
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
    double *kx = nullptr, *kz = nullptr, *minv = nullptr;
    double *S = nullptr, *r = nullptr, *u0 = nullptr, *u1 = nullptr, *z = nullptr, *y = nullptr, *w = nullptr;
    double *partial = nullptr;
    ScalarsDev *sc = nullptr;
    ScalarsDev *sc_host = nullptr;                           // pinned
    int minv_kind = -1;
    double minv_omega = 0.0;
    // kernel timing (measurement support)
    bool timing = false;
    std::vector<hipEvent_t> ev;                              // pairs: start, stop
    std::vector<int> ev_kind;                                // kernel kind of each used pair
    int ev_used = 0;
    long long launches[GAP_KERNEL_COUNT] = {0};
    double total_ms[GAP_KERNEL_COUNT] = {0};

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
    double* bufs[] = {g->trig, g->tex, g->kx, g->kz, g->minv, g->S, g->r, g->u0, g->u1, g->z, g->y, g->w, g->partial};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    if (g->sc) (void)hipFree(g->sc);
    if (g->sc_host) (void)hipHostFree(g->sc_host);
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
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return fail(GAP_EDEVICE, "hipEventCreate: %s", hipGetErrorString(r));
        g->ev.push_back(e);
    }
    g->ev_kind.resize(pairs);
    g->ev_used = 0;
    return GAP_OK;
}

// Record the start (before) or stop (after) event of a timed launch.
inline void timing_mark(gap_grid_t g, int kind, bool start, hipStream_t st)
{
    if (!g->timing) return;
    if (start) {
        g->ev_kind[g->ev_used] = kind;
        (void)hipEventRecord(g->ev[2 * g->ev_used], st);
    } else {
        (void)hipEventRecord(g->ev[2 * g->ev_used + 1], st);
        ++g->ev_used;
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
    return GAP_OK;
}

gap_status create_gap_grid(const gap_geom* geom, const gap_dimples* dimples, int32_t max_cond, gap_grid_t* out)
{
    if (!out) return fail(GAP_EINVAL, "out is NULL");
    *out = nullptr;
    gap_status st = validate_geom(geom);
    if (st != GAP_OK) return st;
    if (max_cond != 1 && max_cond != GAP_MAX_COND) return fail(GAP_EINVAL, "max_cond must be 1 or 9");
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

    gap_grid_t g = new gap_grid_s;
    g->geom = *geom;
    g->nt = geom->n_theta;
    g->nz = geom->n_axial;
    g->n = (size_t)g->nt * g->nz;
    g->max_cond = max_cond;
    g->max_op = (max_cond == GAP_MAX_COND) ? 5 : 1;
    GeomDev& d = g->gd;
    d.R = geom->R;
    d.Rc = geom->R + geom->clearance;
    d.c2R = geom->clearance * (2.0 * geom->R + geom->clearance);
    d.L = geom->length;
    d.mu = geom->mu;
    d.U = geom->U;
    d.V = geom->V;
    d.p_in = geom->p_in;
    d.p_out = geom->p_out;
    d.dth = 2.0 * M_PI / g->nt;
    d.dz = geom->length / g->nz;
    d.dx = geom->R * d.dth;
    d.nt = g->nt;
    d.nz = g->nz;

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
    ALLOC(g->S, max_cond * n);
    ALLOC(g->r, max_cond * n);
    ALLOC(g->u0, max_cond * n);
    ALLOC(g->u1, max_cond * n);
    ALLOC(g->z, max_cond * n);
    ALLOC(g->y, max_cond * n);
    ALLOC(g->w, max_cond * n);
    ALLOC(g->partial, 4 * max_chunks);
#undef ALLOC
    if (hipMalloc((void**)&g->sc, sizeof(ScalarsDev)) != hipSuccess) {
        g->sc = nullptr;
        release(g);
        return fail(GAP_ENOMEM, "hipMalloc of the scalar block failed");
    }
    if (hipHostMalloc((void**)&g->sc_host, sizeof(ScalarsDev), hipHostMallocDefault) != hipSuccess) {
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
    hipError_t e = hipMemcpy(g->trig, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(g->tex, 0, (2 * n + (g->nz + 1) * nt) * sizeof(double));
    if (e == hipSuccess) e = hipMemset(g->sc, 0, sizeof(ScalarsDev));
    if (e != hipSuccess) {
        release(g);
        return fail(GAP_EDEVICE, "initialising tables: %s", hipGetErrorString(e));
    }
    if (count > 0) {
        double* dm = nullptr;
        if (dmalloc(&dm, 4 * (size_t)count) != GAP_OK) { release(g); return GAP_ENOMEM; }
        const double* src[4] = {dimples->theta, dimples->z, dimples->radius, dimples->depth};
        for (int k = 0; k < 4 && e == hipSuccess; ++k)
            e = hipMemcpy(dm + k * count, src[k], count * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            const TablesDev t = g->tables();
            hipLaunchKernelGGL(k_texture, dim3(count, 3), dim3(GAP_BLOCK), 0, 0, d, count, dm, dm + count,
                               dm + 2 * count, dm + 3 * count, (double*)t.tex_c, (double*)t.tex_e, (double*)t.tex_f);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipDeviceSynchronize();
        (void)hipFree(dm);
        if (e != hipSuccess) {
            release(g);
            return fail(GAP_EDEVICE, "texture evaluation: %s", hipGetErrorString(e));
        }
    }
    *out = g;
    return GAP_OK;
}

gap_status destroy_gap_grid(gap_grid_t g)
{
    if (!g) return GAP_OK;
    (void)hipDeviceSynchronize();
    release(g);
    return GAP_OK;
}

gap_status assemble_joint_system(gap_grid_t g, const double e[4], const double edot[4], const double delta[8],
                                 int32_t n_cond, void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
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
    if (!o) return fail(GAP_EINVAL, "opts is NULL");
    if (!p) return fail(GAP_EINVAL, "p is NULL");
    if (!g->assembled) return fail(GAP_ESTATE, "solve_joint_pcg before assemble_joint_system");
    if (!is_finite(o->omega) || !(o->omega > 0.0 && o->omega < 2.0)) return fail(GAP_EINVAL, "omega must lie in (0, 2)");
    if (!is_finite(o->eps) || !(o->eps > 0.0)) return fail(GAP_EINVAL, "eps must be > 0");
    if (o->max_iter < 1) return fail(GAP_EINVAL, "max_iter must be >= 1");
    if (o->precond < GAP_PRECOND_JACOBI || o->precond > GAP_PRECOND_ASSOR2) return fail(GAP_EINVAL, "unknown precond");
    if (o->precond == GAP_PRECOND_ASSOR2 && o->neumann != 1) return fail(GAP_EINVAL, "neumann must be 1");
    if (o->scalars != GAP_SCALARS_GLOBAL && o->scalars != GAP_SCALARS_PER_COND)
        return fail(GAP_EINVAL, "unknown scalars mode");
    if (o->check_every < 0) return fail(GAP_EINVAL, "check_every must be >= 0");
    const int check_every = o->check_every ? o->check_every : 32;
    hipStream_t st = (hipStream_t)stream;
    const GeomDev& gd = g->gd;
    const ChunkMap cm = g->cm;

    if (o->precond != GAP_PRECOND_ASSOR2 && (g->minv_kind != o->precond || g->minv_omega != o->omega)) {
        if (!g->minv) {
            gap_status s = dmalloc(&g->minv, g->max_op * g->n);
            if (s != GAP_OK) return s;
        }
        hipLaunchKernelGGL(k_diag_precond, dim3((unsigned)((g->n + GAP_BLOCK - 1) / GAP_BLOCK), g->n_op),
                           dim3(GAP_BLOCK), 0, st, gd, o->precond, o->omega, g->kx, g->kz, g->minv, g->n_op);
        HIPLAUNCHCHK("k_diag_precond");
        g->minv_kind = o->precond;
        g->minv_omega = o->omega;
    }

    PcgArgs a;
    a.kx = g->kx;
    a.kz = g->kz;
    a.minv = g->minv;
    a.S = g->S;
    a.p = p;
    a.r = g->r;
    a.u_in = g->u0;
    a.u_out = g->u1;
    a.z = g->z;
    a.y = g->y;
    a.w = g->w;
    a.partial = g->partial;
    a.sc = g->sc;
    a.omega = o->omega;
    a.precond = o->precond;
    const dim3 grid(cm.total), block(GAP_BLOCK);
    const int per_cond = o->scalars == GAP_SCALARS_PER_COND;

    hipLaunchKernelGGL(k_init, grid, block, 0, st, gd, g->cd, cm, a, o->warm_start ? 1 : 0);
    HIPLAUNCHCHK("k_init");
    if (o->precond == GAP_PRECOND_ASSOR2) {
        hipLaunchKernelGGL(k_assor_lower, grid, block, 0, st, gd, g->cd, cm, a, 0);
        hipLaunchKernelGGL(k_assor_upper, grid, block, 0, st, gd, g->cd, cm, a, 0, 2);
        HIPLAUNCHCHK("ASSOR (init)");
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), block, 0, st, cm, g->n_cond, (const double*)g->partial, g->sc, (int)FIN_INIT,
                       per_cond, o->eps, o->max_iter);
    HIPLAUNCHCHK("k_finalize (init)");

    const long max_blocks = o->max_iter / check_every + 2;
    for (long blk = 0; blk < max_blocks; ++blk) {
        HIPCHK(hipMemcpyAsync(g->sc_host, g->sc, sizeof(ScalarsDev), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (g->timing) {
            gap_status ts = timing_collect(g);
            if (ts != GAP_OK) return ts;
        }
        if (g->sc_host->done) break;
        if (g->timing) {
            gap_status ts = timing_reserve(g, 6 * check_every);
            if (ts != GAP_OK) return ts;
        }
        for (int it = 0; it < check_every; ++it) {
            timing_mark(g, GAP_KERNEL_SPMV_DOT, true, st);
            hipLaunchKernelGGL(k_spmv_dot, grid, block, 0, st, gd, g->cd, cm, a);
            timing_mark(g, GAP_KERNEL_SPMV_DOT, false, st);
            timing_mark(g, GAP_KERNEL_FINALIZE, true, st);
            hipLaunchKernelGGL(k_finalize, dim3(1), block, 0, st, cm, g->n_cond, (const double*)g->partial, g->sc,
                               (int)FIN_ALPHA, per_cond, o->eps, o->max_iter);
            timing_mark(g, GAP_KERNEL_FINALIZE, false, st);
            timing_mark(g, GAP_KERNEL_UPDATE, true, st);
            hipLaunchKernelGGL(k_update, grid, block, 0, st, gd, g->cd, cm, a);
            timing_mark(g, GAP_KERNEL_UPDATE, false, st);
            if (o->precond == GAP_PRECOND_ASSOR2) {
                timing_mark(g, GAP_KERNEL_ASSOR_LOWER, true, st);
                hipLaunchKernelGGL(k_assor_lower, grid, block, 0, st, gd, g->cd, cm, a, 1);
                timing_mark(g, GAP_KERNEL_ASSOR_LOWER, false, st);
                timing_mark(g, GAP_KERNEL_ASSOR_UPPER, true, st);
                hipLaunchKernelGGL(k_assor_upper, grid, block, 0, st, gd, g->cd, cm, a, 1, 1);
                timing_mark(g, GAP_KERNEL_ASSOR_UPPER, false, st);
            }
            timing_mark(g, GAP_KERNEL_FINALIZE, true, st);
            hipLaunchKernelGGL(k_finalize, dim3(1), block, 0, st, cm, g->n_cond, (const double*)g->partial, g->sc,
                               (int)FIN_BETA, per_cond, o->eps, o->max_iter);
            timing_mark(g, GAP_KERNEL_FINALIZE, false, st);
            HIPLAUNCHCHK("PCG iteration");
            std::swap(a.u_in, a.u_out);
        }
    }
    HIPCHK(hipMemcpyAsync(g->sc_host, g->sc, sizeof(ScalarsDev), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (g->timing) {
        gap_status ts = timing_collect(g);
        if (ts != GAP_OK) return ts;
    }
    const ScalarsDev& h = *g->sc_host;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iterations = h.iter;
        info->n_cond = g->n_cond;
        info->rel_residual = h.rel;
        for (int c = 0; c < g->n_cond; ++c) info->rel_residual_cond[c] = h.rel_cond[c];
    }
    gap_status result = GAP_OK;
    if (h.status == -4) result = fail(GAP_ENONFINITE, "non-finite value in the PCG reductions at iteration %d", h.iter);
    else if (h.status == -3 || !h.done) result = fail(GAP_ENOCONV, "no convergence after %d iterations (rel %.3e)", h.iter, h.rel);
    if (info) info->status = result;
    return result;
}

gap_status integrate_force_moment(gap_grid_t g, const double* p, int32_t cavitation, double p_cav, double* F,
                                  void* stream)
{
    if (!g) return fail(GAP_EINVAL, "grid is NULL");
    if (!p || !F) return fail(GAP_EINVAL, "p and F must be non-NULL");
    if (!g->assembled) return fail(GAP_ESTATE, "integrate_force_moment before assemble_joint_system");
    if (cavitation != GAP_CAVITATION_NONE && cavitation != GAP_CAVITATION_CLAMP)
        return fail(GAP_EINVAL, "unknown cavitation mode");
    if (!is_finite(p_cav)) return fail(GAP_EINVAL, "p_cav must be finite");
    hipStream_t st = (hipStream_t)stream;
    const ChunkMap cm = g->cm;
    hipLaunchKernelGGL(k_forces, dim3(cm.total), dim3(GAP_BLOCK), 0, st, g->gd, g->cd, cm, g->tables(), p, cavitation,
                       p_cav, g->partial);
    hipLaunchKernelGGL(k_forces_finalize, dim3(1), dim3(GAP_BLOCK), 0, st, cm, g->n_cond, g->gd.dx * g->gd.dz,
                       (const double*)g->partial, F);
    HIPLAUNCHCHK("force integration");
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
    if (enable) {
        for (int k = 0; k < GAP_KERNEL_COUNT; ++k) {
            g->launches[k] = 0;
            g->total_ms[k] = 0.0;
        }
    }
    g->timing = enable != 0;
    g->ev_used = 0;
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
