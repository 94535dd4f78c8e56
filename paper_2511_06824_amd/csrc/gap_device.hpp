// Device-side data structures and helpers shared by the gapsolve kernels (gfx950, FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GAP_MAXC 9
#define GAP_BLOCK 256

// Geometry as the kernels see it (derived quantities precomputed on the host).
struct GeomDev {
    double R, Rc, c2R;       // piston radius, bore radius, R_c^2 - R^2 computed as c (2R + c)
    double L, mu, U, V, p_in, p_out;
    double dth, dz, dx;      // cell sizes: dtheta, dz, dx = R dtheta
    int nt, nz;              // n_theta, n_axial
};

// State of every condition of the joint system (Eq 2.17-2.19).
struct CondDev {
    double e[GAP_MAXC][4];
    double ed[GAP_MAXC][4];
    int op[GAP_MAXC];        // operator (stencil) index used by each condition
    int n_cond, n_op;
};

// Read-only tables and texture samples of one grid.
struct TablesDev {
    const double *cos_c, *sin_c;   // at theta_i = (i + 1/2) dtheta       [nt]
    const double *cos_e, *sin_e;   // at the east face theta_i + dtheta/2 [nt]
    const double *tex_c;           // texture depth at cell centres        [n]
    const double *tex_e;           // at east faces                        [n]
    const double *tex_f;           // at axial faces z = f dz, f=0..nz     [(nz+1) nt]
};

// Film thickness of Eq 2.3 in cancellation-free form at (cos, sin) of the angle, axial
// position z, plus the texture depth.  e: (e1, e2) at z = 0, (e3, e4) at z = L.
__device__ __forceinline__ double film_h(const GeomDev& g, const double* e, double cs, double sn,
                                         double z, double tex)
{
    const double t = z / g.L;
    const double ex = e[0] + (e[2] - e[0]) * t;
    const double ey = e[1] + (e[3] - e[1]) * t;
    const double q = g.c2R - 2.0 * g.Rc * (ex * cs + ey * sn) + ex * ex + ey * ey;
    const double d = sqrt(g.R * g.R + q);
    return q / (d + g.R) + tex;
}

// Time derivative of the film through the eccentricity rates (texture is fixed).
__device__ __forceinline__ double film_rate(const GeomDev& g, const double* e, const double* ed,
                                            double cs, double sn, double z)
{
    const double t = z / g.L;
    const double ex = e[0] + (e[2] - e[0]) * t;
    const double ey = e[1] + (e[3] - e[1]) * t;
    const double exd = ed[0] + (ed[2] - ed[0]) * t;
    const double eyd = ed[1] + (ed[3] - ed[1]) * t;
    const double ax = g.Rc * cs - ex;
    const double ay = g.Rc * sn - ey;
    return -(ax * exd + ay * eyd) / sqrt(ax * ax + ay * ay);
}

// Sum of NV values over a 256-thread block, fixed reduction order (wave64 shuffles, then
// the 4 wave results in order).  The total is valid in thread 0 only.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double part[NV][GAP_BLOCK / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = part[k][0];
            for (int w = 1; w < GAP_BLOCK / 64; ++w) s += part[k][w];
            v[k] = s;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ bool finite_d(double x) { return x - x == 0.0; }

// A double that every lane of the wave holds alike, moved to scalar registers (values the
// workgroup derives from LDS are otherwise kept in vector registers, one copy per lane).
__device__ __forceinline__ double wave_uniform(double x)
{
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffull));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Global-memory views of generic pointers.  Kernels that read their buffer addresses from a
// record in device memory see generic pointers, for which the compiler emits flat loads and
// stores; those count against the LDS wait counter as well, so every wait for an LDS read
// also waits for all outstanding memory loads (including loads issued a row step ahead).
// Accesses through these views are global instructions, counted on the memory counter only.
#define GAP_AS1 __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GAP_AS1 T* as_global(T* p)
{
    return (GAP_AS1 T*)p;
}
