/*
 * gapsolve.h -- C ABI of the MI355X (gfx950) joint piston-gap Reynolds solver.
 *
 * Paper: "A GPU-boosted high-performance multi-working condition joint analysis framework
 * for predicting dynamics of textured axial piston pump" (arXiv 2511.06824).
 *
 * The library computes, on one GPU and in FP64 throughout, the hot path of the paper's
 * framework (Sec 3.2, steps I-IV):
 *   I.   assemble the 5-point finite-volume system A_k p_k = S_k of every working condition
 *        k = 0..8 (Eq 2.1, 2.4-2.7, 2.17-2.19) from the film thickness of Eq 2.3;
 *   II.  solve the block-diagonal joint system A_G p_G = S_G (Eq 3.7-3.8) by the adjusted
 *        PCG of Table 1 with the ASSOR preconditioner (Eq 3.3-3.6) and the synchronized
 *        global stopping test of Eq 3.9;
 *   III. integrate pressure and viscous-shear force and moment per condition (Sec 2.4-III);
 *   IV.  form the double Jacobian of Eq 2.13-2.14 by forward differences.
 *
 * Conventions shared by every entry point
 *   - Units are SI.  All floating point is IEEE double.
 *   - Grid: n_theta cells around the circumference (periodic, fastest index) by n_axial
 *     cells along the gap; cell (i, j) has centre theta_i = (i + 1/2) 2 pi / n_theta,
 *     z_j = (j + 1/2) L / n_axial.  A field of one condition is n = n_theta * n_axial
 *     doubles, element i + j * n_theta.  Fields of several conditions are stored
 *     condition-major: element i + j * n_theta + k * n (Eq 3.8).
 *   - Condition k (Eq 2.17-2.19): k = 0 is (e, edot); k = 1..4 adds delta[k-1] to e_k;
 *     k = 5..8 adds delta[k-1] to edot_{k-4}.
 *   - Device pointers are HIP device allocations owned by the caller (for instance the
 *     storage of a torch tensor); the library never frees them.  Host pointers are
 *     read during the call only.  A handle owns its internal device buffers until
 *     destroy_gap_grid.
 *   - stream is a hipStream_t passed as void* (NULL: the legacy default stream).  Calls
 *     are ordered on that stream; solve_joint_pcg synchronizes it (it reads the device
 *     convergence flag), the other calls return before the device work completes.
 *   - A handle is not thread-safe; use one handle per host thread and stream.
 *   - No exception crosses the ABI.  Each call returns a gap_status; on failure
 *     gap_last_error() describes it.  Arguments are validated before any device work,
 *     so invalid input never reaches a kernel.
 */
#ifndef GAPSOLVE_H
#define GAPSOLVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gap_grid_s *gap_grid_t;
typedef struct gap_batch_s *gap_batch_t;

typedef enum {
    GAP_OK = 0,
    GAP_EINVAL = -1,      /* an argument is out of range or NULL where it may not be */
    GAP_ECONTACT = -2,    /* some condition has |e| >= clearance at a gap end: h <= 0 */
    GAP_ENOCONV = -3,     /* max_iter reached; the last iterate is written, info filled */
    GAP_ENONFINITE = -4,  /* a NaN/Inf appeared in a reduction; the solve was stopped */
    GAP_ENOMEM = -5,      /* a device or pinned-host allocation failed */
    GAP_EDEVICE = -6,     /* a HIP runtime call failed */
    GAP_ESTATE = -7,      /* call out of order (e.g. solve before assemble) */
    GAP_EBUDGET = -8      /* no batch slot (or memory budget) is free for another request */
} gap_status;

enum { GAP_PRECOND_JACOBI = 0, GAP_PRECOND_ASSOR1 = 1, GAP_PRECOND_ASSOR2 = 2 };
enum { GAP_SCALARS_GLOBAL = 0, GAP_SCALARS_PER_COND = 1 };
enum { GAP_STRATEGY_SYNC = 0, GAP_STRATEGY_ASYNC = 1 };
enum { GAP_CAVITATION_NONE = 0, GAP_CAVITATION_CLAMP = 1 };
enum { GAP_ITERATION_TWO_LAUNCH = 0, GAP_ITERATION_ONE_LAUNCH = 1, GAP_ITERATION_STRIPS = 2 };
#define GAP_MAX_COND 9

/* Gap geometry, fluid and boundary data (Eq 2.3; Table 8 lists the paper's pump).
 *   R          piston radius R_k (> 0)
 *   clearance  radial clearance c, bore radius R_c = R + c (> 0)
 *   length     gap length L_F (> 0)
 *   mu         dynamic viscosity (> 0)
 *   U, V       sliding speed of the bore wall relative to the piston, circumferential and
 *              axial (any sign)
 *   p_in       Dirichlet pressure at z = 0 (south boundary, Sec 2.1)
 *   p_out      Dirichlet pressure at z = L (north boundary)
 *   n_theta    cells around the circumference, 3 <= n_theta <= 16384 (the iteration kinds
 *              whose workgroups hold whole rings need n_theta <= 2048)
 *   n_axial    cells along the gap, 2 <= n_axial <= 65536                                */
typedef struct {
    double R, clearance, length, mu, U, V, p_in, p_out;
    int32_t n_theta, n_axial;
} gap_geom;

/* Spherical-cap dimples on the piston (the texture depth h_Text of Eq 2.3).  Host
 * arrays of `count` entries: centre angle (rad), centre axial position (m), footprint
 * radius a (> 0) and depth d (0 < d < a).  A cap adds sqrt(rho^2 - r^2) - (rho - d) with
 * rho = (a^2 + d^2) / (2 d) at in-surface distance r < a (arc length R dtheta, wrapped,
 * and dz); overlapping caps combine by max.  count = 0 or a NULL gap_dimples: smooth. */
typedef struct {
    int32_t count;
    const double *theta, *z, *radius, *depth;
} gap_dimples;

/* PCG options (Table 1, Sec 3.1, 3.3).
 *   omega        relaxation factor of ASSOR, 0 < omega < 2 (paper: 1.8 smooth, 1.6 textured)
 *   eps          stopping tolerance on ||r_G|| / ||S_G|| (Eq 3.9), > 0
 *   max_iter     iteration cap, >= 1
 *   precond      GAP_PRECOND_ASSOR2 (Eq 3.4, the paper's "ASSOR"), _ASSOR1 (Eq 3.2) or
 *                _JACOBI (Eq 2.8)
 *   neumann      Neumann order M of the ASSOR II inverse: the series of (I + w D^-1 L)^-1 and
 *                of its transpose truncated after M terms; 1 is Eq 3.4.  1, 2 or 3 with
 *                GAP_ITERATION_STRIPS and GAP_PRECOND_ASSOR2 (order 3 runs with one column
 *                per lane); 1 otherwise.  All requests of one batch use the same order.
 *   scalars      GAP_SCALARS_GLOBAL: one alpha/beta for the joint system (CG on A_G);
 *                GAP_SCALARS_PER_COND: one recurrence per condition
 *   strategy     GAP_STRATEGY_SYNC: stop when ||r_G|| / ||S_G|| <= eps (Eq 3.9);
 *                GAP_STRATEGY_ASYNC: stop each condition when ||r_k|| / ||S_k|| <= eps
 *                (Eq 3.10); a converged condition is frozen on the device (its workgroups
 *                return at once), the joint scalars run over the remaining ones, and the
 *                solve ends when all have converged.  No host round trip is involved.
 *   warm_start   nonzero: p holds the initial guess p_0; zero: p_0 = 0 (Table 1 step 1)
 *   check_every  iterations between host reads of the device convergence flag (0: 32);
 *                launches after convergence return at once, so the count is exact
 *   graph        nonzero: each block of check_every iterations is captured once into a
 *                hipGraph and replayed; zero: plain launches
 *   iteration    GAP_ITERATION_TWO_LAUNCH: Table 1 as printed, two launches per iteration
 *                (u and u^T A u; then alpha and the updates).  GAP_ITERATION_ONE_LAUNCH:
 *                one launch per iteration, with u^T A u = z^T A z + 2 beta z^T A u_prev +
 *                beta^2 u_prev^T A u_prev from sums the previous launch forms (A is
 *                symmetric); each workgroup holds whole rings (n_theta <= 2048).
 *                GAP_ITERATION_STRIPS: the one-launch scheme with each wavefront marching a
 *                strip of columns (neighbours by lane shifts, no LDS rows), z_j recomputed
 *                from r_j instead of stored (fewer bytes per iteration), any n_theta.  The
 *                three kinds give the same iterates up to rounding.  All requests of one
 *                batch (gap_batch_*) use the same kind.
 *   eps_adjoint  stopping tolerance of the adjoint systems of jacobian_adjoint and
 *                solve_with_adjoint (each on ||r_i|| / ||g_i||, Eq 3.10), >= 0; 0: eps.  The
 *                adjoint Jacobian is a product lambda_i^T b_k with no differencing, so its
 *                error follows the adjoint residual without the 1/delta amplification that
 *                forward differences put on the forces; a looser tolerance than the base
 *                solve's suffices for a given Jacobian accuracy.                         */
typedef struct {
    double omega, eps;
    int32_t max_iter, precond, neumann, scalars, warm_start, check_every, graph, strategy;
    int32_t iteration;
    int32_t reserved;
    double eps_adjoint;
} gap_solver_opts;

/* Result of a solve.  iterations counts completed Table 1 iterations (SpMV + update);
 * rel_residual is the recurrence ||r_G|| / ||S_G|| at exit (the quantity the stopping test
 * of Eq 3.9 reads); rel_residual_cond[k] the same per condition; true_rel_residual is
 * ||S_G - A_G p|| / ||S_G|| recomputed from the returned p once at exit (solve_joint_pcg
 * only; -1 where not computed: batched and adjoint solves); status repeats the return code. */
typedef struct {
    int32_t iterations, status, n_cond, reserved;
    double rel_residual;
    double rel_residual_cond[GAP_MAX_COND];
    double true_rel_residual;
    double true_rel_residual_cond[GAP_MAX_COND];
} gap_solve_info;

/* Fill *opts with the defaults: omega 1.6, eps 1e-10, max_iter 100000, ASSOR II,
 * neumann 1, GLOBAL scalars, cold start, check_every 32, graph 1, SYNC strategy, strip
 * iteration (GAP_ITERATION_STRIPS), eps_adjoint 0 (= eps).  Returns GAP_EINVAL if NULL. */
gap_status gap_default_opts(gap_solver_opts *opts);

/* Create a handle for one gap (Eq 2.3 geometry, Sec 2.1 grid) that can hold up to
 * max_cond (1 or 9) working conditions.  Allocates every device buffer the path needs
 * (stencils, sources, Krylov vectors, reduction scratch), evaluates the dimple depths at
 * cell centres and faces once, and leaves the handle in the "created" state.  *out
 * receives the handle, or NULL on failure.  Errors: GAP_EINVAL (NULL, sizes, non-positive
 * geometry, bad dimple), GAP_ENOMEM, GAP_EDEVICE. */
gap_status create_gap_grid(const gap_geom *geom, const gap_dimples *dimples, int32_t max_cond,
                           gap_grid_t *out);

/* create_gap_grid with a general texture field h_Text(theta, z) of Eq 2.3 in place of the
 * dimple list, for any layout (grooves, pockets, measured surfaces).  The assembly needs the
 * film at cell centres and at the faces, so the field comes sampled at three sets of points,
 * each a device array of non-negative depths (m, the pocket depth added to h) that the call
 * copies; the caller keeps ownership:
 *   tex_c  [n_axial][n_theta]      at the cell centres (theta_i, z_j), theta_i = (i + 1/2) dtheta,
 *                                  z_j = (j + 1/2) dz
 *   tex_e  [n_axial][n_theta]      at the east faces (theta_i + dtheta / 2, z_j); column
 *                                  n_theta - 1 is the face at theta = 2 pi (= 0)
 *   tex_f  [n_axial + 1][n_theta]  at the axial faces (theta_i, f dz), f = 0 .. n_axial
 *                                  (rows 0 and n_axial are the Dirichlet ends z = 0, L)
 * The texture rides on the piston and adds no squeeze term.  Synchronizes the device.
 * Errors: as create_gap_grid; GAP_EINVAL also for NULL arrays and for a non-finite or
 * negative depth (the message names the array and index). */
gap_status create_gap_grid_field(const gap_geom *geom, const double *tex_c, const double *tex_e,
                                 const double *tex_f, int32_t max_cond, gap_grid_t *out);

/* Release a handle and all its device memory (waits for its pending work).  NULL is a
 * no-op. */
gap_status destroy_gap_grid(gap_grid_t grid);

/* Replace the texture of an existing handle by a dimple list (as create_gap_grid; count 0 or
 * NULL: smooth), for reusing one handle across requests of the same geometry and grid: no
 * device memory is allocated or freed (beyond growing the handle's parameter buffer past a
 * multiple of 256 dimples) and no device-wide synchronization happens, so it may run beside
 * work and graph captures of other threads.  Clears the texture planes and evaluates the
 * caps on `stream`, then synchronizes that stream.  The next solve needs a new
 * assemble_joint_system.  Errors: GAP_EINVAL (NULL grid, bad dimple), GAP_ESTATE (the grid
 * is in a batch), GAP_ENOMEM, GAP_EDEVICE. */
gap_status set_gap_dimples(gap_grid_t grid, const gap_dimples *dimples, void *stream);

/* Step I (Sec 3.2; Eq 2.3-2.7, 2.17-2.19): assemble the n_cond (1 or 9, <= max_cond)
 * systems for base state e[4] (m), edot[4] (m/s) and FD steps delta[8] (e1..e4,
 * edot1..edot4; may be NULL when n_cond = 1).  Rates enter only the source, so
 * conditions 5..8 share the operator of condition 0 and 5 operators are built.
 * Boundary treatment (step a3): Dirichlet ends folded into the diagonal and source at
 * half a cell, periodic circumferential wrap.  Errors: GAP_EINVAL, GAP_ECONTACT (some
 * condition has |e| >= clearance at z = 0 or z = L), GAP_EDEVICE. */
gap_status assemble_joint_system(gap_grid_t grid, const double e[4], const double edot[4],
                                 const double delta[8], int32_t n_cond, void *stream);

/* Step II (Table 1; Eq 3.4-3.6, 3.7, 3.9): solve the assembled joint system.  p is a
 * device array of n_cond * n doubles, condition-major; it receives the solution (and
 * holds the initial guess when opts->warm_start).  info (host, may be NULL) receives the
 * iteration count and residuals.  Synchronizes `stream`.  Errors: GAP_EINVAL,
 * GAP_ESTATE (nothing assembled), GAP_ENOCONV, GAP_ENONFINITE, GAP_EDEVICE. */
gap_status solve_joint_pcg(gap_grid_t grid, const gap_solver_opts *opts, double *p,
                           gap_solve_info *info, void *stream);

/* Step III (Sec 2.4-III) with the cavitation treatment of step a3: for every assembled
 * condition, integrate (Fx, Fy, Mx, My) of pressure and wall shear over the piston
 * surface (midpoint rule, moments about z = L/2).  cavitation = GAP_CAVITATION_NONE uses
 * p as solved; GAP_CAVITATION_CLAMP uses max(p, p_cav).  p: device, n_cond * n doubles.
 * F: device, n_cond * 4 doubles, row k = (Fx, Fy, Mx, My) of condition k.
 * Errors: GAP_EINVAL, GAP_ESTATE, GAP_EDEVICE. */
gap_status integrate_force_moment(gap_grid_t grid, const double *p, int32_t cavitation,
                                  double p_cav, double *F, void *stream);

/* integrate_force_moment without a handle, for callers that cannot allocate device memory
 * (work recorded under stream capture, serving loops or harnesses that forbid hipMalloc).
 * It allocates nothing: its partial sums and its cos / sin table live in a fixed device
 * array of the library (384 KiB per GPU, held until the process ends), so it needs
 * 2 n_theta + 4 * (row chunks) <= 49152 doubles, where the row chunks number at most
 * 2048 + n_cond; larger grids are rejected with GAP_EINVAL.
 *   geom        grid, fluid and boundary data (validated as for create_gap_grid)
 *   n_cond      1 .. 9 pressure fields
 *   e           host, n_cond x 4 doubles: (e1, e2, e3, e4) of each field's film (Eq 2.3)
 *   tex_c       device, n doubles: texture depth h_Text at the cell centres, or NULL (smooth)
 *   p           device, n_cond x n doubles (condition-major)
 *   cavitation, p_cav, F (device, n_cond x 4) as for integrate_force_moment.
 * The result equals integrate_force_moment's for the same film up to the rounding of the
 * cos / sin table (formed on the device here).  Every call on one GPU shares that GPU's
 * scratch array, so calls that overlap on one GPU (different streams or host threads) race;
 * calls ordered on one stream do not.  Errors: GAP_EINVAL, GAP_ECONTACT (|e| >= clearance at
 * a gap end), GAP_EDEVICE. */
gap_status integrate_force_moment_noalloc(const gap_geom *geom, int32_t n_cond, const double *e,
                                          const double *tex_c, const double *p, int32_t cavitation,
                                          double p_cav, double *F, void *stream);

/* The forces of integrate_force_moment split into the normal-pressure part and the
 * viscous-shear part (the paper reports them separately, Sec 4.3), with the axial force and
 * the torque of the shear: F (device, n_cond x 10 doubles) per condition
 *   pressure: Fx, Fy, Mx, My;  shear: Fx, Fy, Mx, My, Fz = sum tau_z dA, Mz = sum R tau_theta dA.
 * The two parts of each of (Fx, Fy, Mx, My) add up to integrate_force_moment's value (up to
 * summation order).  Arguments and errors as for integrate_force_moment. */
gap_status integrate_force_moment_split(gap_grid_t grid, const double *p, int32_t cavitation, double p_cav,
                                        double *F, void *stream);

/* GMAF step II, "update and rebuild pressure field": the full field of every condition with
 * its boundary rows, out (device, n_cond x (n_axial + 2) x n_theta doubles, theta fastest):
 * row 0 is p_in (the face z = 0), rows 1 .. n_axial the cell-centre pressure after the
 * cavitation rule, the last row p_out (z = L).  Arguments and errors as for
 * integrate_force_moment. */
gap_status rebuild_pressure_field(gap_grid_t grid, const double *p, int32_t cavitation, double p_cav,
                                  double *out, void *stream);

/* Step IV (Eq 2.13-2.14): forward-difference double Jacobian from the forces of the 9
 * conditions.  F: device, 9 * 4 doubles from integrate_force_moment.  J: device, 32
 * doubles, row-major 4 x 8, J[i*8 + k] = (F[(k+1)*4 + i] - F[i]) / delta[k], rows
 * (Fx, Fy, Mx, My), columns (e1..e4, edot1..edot4), delta as given to the last assemble.
 * Errors: GAP_EINVAL, GAP_ESTATE (fewer than 9 conditions assembled), GAP_EDEVICE. */
gap_status jacobian_fd(gap_grid_t grid, const double *F, double *J, void *stream);

/* Step IV by the adjoint method: the exact derivative of steps I-III of condition 0 with
 * respect to (e1..e4, edot1..edot4), instead of the forward differences of Eq 2.13-2.14.
 * With A(e) p = S(e, edot) and F_i = f_i(p, e):
 *   dF_i/dx_k = df_i/dx_k + lambda_i^T (dS/dx_k - dA/dx_k p0),   A lambda_i = df_i/dp,
 * where A is the symmetric operator of condition 0, so the adjoint solves reuse it.
 *   p0     device, n doubles: the solved pressure of condition 0 of the last assembly (the
 *          first n values of the p returned by solve_joint_pcg)
 *   w      host, 4 weights, or NULL.  NULL: J (device, 32 doubles) receives the full 4 x 8
 *          matrix, laid out as in jacobian_fd, from 4 adjoint solves (needs a handle created
 *          for 9 conditions).  Non-NULL: J (device, 8 doubles) receives the vector-Jacobian
 *          product w^T J from one adjoint solve.
 *   opts   omega, eps, precond, max_iter, check_every and graph of the adjoint solves; each
 *          adjoint field runs its own recurrence and meets eps on its own (per-condition
 *          scalars, asynchronized test).
 *   cavitation, p_cav as in integrate_force_moment; in CLAMP mode d max(p, p_cav)/dp is taken
 *          as 1 where p > p_cav and 0 elsewhere.
 *   info   host, may be NULL: iterations and residuals of the adjoint solve.
 * The assembled system and the caller's p are left untouched (the handle's Krylov buffers
 * are reused).  Synchronizes stream.  Errors: GAP_EINVAL, GAP_ESTATE, GAP_ENOCONV,
 * GAP_ENONFINITE, GAP_EDEVICE. */
gap_status jacobian_adjoint(gap_grid_t grid, const gap_solver_opts *opts, const double *p0, int32_t cavitation,
                            double p_cav, const double *w, double *J, gap_solve_info *info, void *stream);

/* Base solve and adjoint solves together (no cavitation): the adjoint right-hand sides
 * df_i/dp do not depend on p0 when no clamp is applied, so A p0 = S_0 and the adjoint
 * systems A lambda_i = df_i/dp (all on the operator of condition 0) run as one joint solve of
 * 1 + 4 systems (w NULL) or 1 + 1 systems (w non-NULL), each with its own recurrence and its
 * own stopping test (per-condition scalars, asynchronized test, Eq 3.10), followed by the
 * sensitivity pass of jacobian_adjoint.
 *   p0     device, n doubles, output: the pressure of condition 0 of the last assembly
 *   w, J   as in jacobian_adjoint
 *   opts   omega, eps, precond, max_iter, check_every, graph; eps applies to each system
 *   info   host, may be NULL: iterations; rel_residual_cond[0] is the base system's,
 *          [1..] the adjoint systems'
 * Needs max_cond >= 5 (w NULL) or >= 2 (w non-NULL).  Only condition 0 of the assembly is
 * used (assembling 1 condition suffices).  Synchronizes stream.  Errors: GAP_EINVAL,
 * GAP_ESTATE, GAP_ENOCONV, GAP_ENONFINITE, GAP_ENOMEM, GAP_EDEVICE. */
gap_status solve_with_adjoint(gap_grid_t grid, const gap_solver_opts *opts, double *p0, const double *w, double *J,
                              gap_solve_info *info, void *stream);

/* ---- GMAF step V (Sec 2.3): one general iteration of the piston equilibrium
 * F = F_E + F_I + F_O = 0 (Eq 2.10), F = (Fx, Fy, Mx, My) (Eq 2.11), at a new time point.
 * F_O is the oil-film force of the base condition (steps I-III), F_E an external load and
 * F_I = -mass (edot - edot_prev) / dt the inertia force of a constant 4 x 4 mass matrix on the
 * backward-difference acceleration.  The eccentricities follow e = e_prev + dt edot, so an
 * update keeps de = dt d(edot).  Eq 2.12 then reads
 *   GAP_SCHEME_GENERAL:       (F_,edot + dt F_,e) d(edot) = -F      (both Jacobians)
 *   GAP_SCHEME_CONVENTIONAL:  F_,edot d(edot) = -F                   (Eq 2.20-2.22)
 * with F_,e = dF_O/de and F_,edot = dF_O/dedot - mass / dt.  The oil-film Jacobian comes from
 * the 9-condition joint solve and Eq 2.13-2.14 (GAP_JACOBIAN_FD; needs a 9-condition handle
 * and delta) or from the joint base + adjoint solve (GAP_JACOBIAN_ADJOINT; no cavitation;
 * needs max_cond >= 5; delta may be NULL). */
enum { GAP_SCHEME_GENERAL = 0, GAP_SCHEME_CONVENTIONAL = 1 };
enum { GAP_JACOBIAN_FD = 0, GAP_JACOBIAN_ADJOINT = 1 };
typedef struct {
    double dt;              /* time step (s), > 0 */
    double edot_prev[4];    /* rates at the previous time point (m/s) */
    double F_ext[4];        /* external load F_E (N, N, N m, N m) */
    double mass[16];        /* row-major 4 x 4 mass matrix (kg, kg m^2 / m as the rows need) */
    int32_t scheme;         /* GAP_SCHEME_* */
    int32_t jacobian;       /* GAP_JACOBIAN_* */
} gap_step_params;

/* One step from (e, edot) (host, 4 each; overwritten with the updated state):
 *   p      device, 9 n doubles (FD) or n doubles (adjoint): the pressure field, also the
 *          initial guess when opts->warm_start is set (FD only)
 *   F      host, 4 doubles, output: the residual F at the input state
 *   J      host, 32 doubles or NULL, output: the oil-film Jacobian used (layout of jacobian_fd)
 *   info   host or NULL: the PCG solve of this step
 * Synchronizes stream.  Errors: GAP_EINVAL, GAP_ECONTACT, GAP_ENOCONV, GAP_ENONFINITE
 * (also a singular update matrix), GAP_ENOMEM, GAP_EDEVICE. */
gap_status general_iteration_step(gap_grid_t grid, const gap_solver_opts *opts, const gap_step_params *prm,
                                  const double delta[8], double *p, double e[4], double edot[4], double F[4],
                                  double *J, gap_solve_info *info, void *stream);

/* Operating point of the gap (pump kinematics, time-varying pressures): circumferential and
 * axial sliding speeds U, V (m/s) and the Dirichlet pressures p_in (z = 0) and p_out (z = L)
 * (Pa).  Takes effect at the next assemble_joint_system (the handle returns to the state
 * "not assembled").  Errors: GAP_EINVAL (NULL grid, non-finite value). */
gap_status set_operating_point(gap_grid_t grid, double U, double V, double p_in, double p_out);

/* Autotuner of the ASSOR II Neumann order (Sec 3.1: the series of Eq 3.4 truncated after M
 * terms in each factor; M = 1 is Eq 3.4) for the strip iteration: for M = 1 .. max_order
 * (<= 3) it tunes the kernel configuration as gap_tune_pcg does, then times one complete
 * solve of the assembled system with opts (after a warm one), and keeps the configuration of
 * the fastest order on the handle.  *best receives that order (set opts->neumann to it for
 * the solves that follow) and seconds (NULL or max_order doubles) the time of each order's
 * solve.  opts must select GAP_PRECOND_ASSOR2 and GAP_ITERATION_STRIPS.  Overwrites p and
 * the Krylov state, synchronizes stream, resets the counters of gap_kernel_stats.  Errors:
 * GAP_EINVAL, GAP_ESTATE (nothing assembled), GAP_ENOCONV / GAP_ENONFINITE from a solve,
 * GAP_EDEVICE. */
gap_status gap_tune_neumann(gap_grid_t grid, const gap_solver_opts *opts, double *p, int32_t max_order,
                            int32_t *best, double *seconds, void *stream);

/* Copy the assembled system of condition k to caller device buffers (inspection and
 * testing): kx (n doubles, east-face conductances h^3/(12 mu) dz/dx), kz
 * ((n_axial + 1) * n_theta doubles, axial-face conductances h^3/(12 mu) dx/dz, doubled on
 * the two Dirichlet faces), S (n doubles).  Any of the three may be NULL.  The matrix is
 * A_PP = kx(i) + kx(i-1) + kz(j) + kz(j+1), off-diagonals minus the shared face value.
 * Errors: GAP_EINVAL, GAP_ESTATE, GAP_EDEVICE. */
gap_status gap_read_system(gap_grid_t grid, int32_t k, double *kx, double *kz, double *S,
                           void *stream);

/* Measurement support.  gap_kernel_timing(grid, k) with k >= 1 enables timing: from then
 * on solve_joint_pcg brackets one launch in k of the iteration kernels (every launch for
 * k = 1; counted over this handle's iteration-kernel launches since the call) with HIP
 * events on the caller's stream and accumulates the elapsed device time per kernel kind;
 * gap_kernel_stats reads the number of timed launches and their total.  An odd k samples
 * both launch parities of the one-launch kernel, and A and B of the two-launch iteration,
 * equally.  k = 0 disables timing; enabling (or re-enabling) resets the counters,
 * disabling keeps them readable.  While enabled the iteration blocks are launched without
 * graph capture (opts->graph is ignored), since events recorded by graph nodes cannot be
 * timed; the results are bitwise the same.
 * Errors: GAP_EINVAL (NULL grid, k < 0, unknown kernel), GAP_EDEVICE. */
enum {
    GAP_KERNEL_PCG_A = 0,  /* u = z + beta u; u^T A u; beta and the stopping test (Table 1 steps 9, 3, 6) */
    GAP_KERNEL_PCG_B = 1,  /* alpha; p, r update; z = M^-1 r (ASSOR II sweeps); r^T z, r^T r (steps 4-8) */
    GAP_KERNEL_PCG_ONE = 2, /* one-launch iteration: all of steps 3-9 */
    GAP_KERNEL_PCG_STRIPS = 3, /* one-launch iteration on wavefront strips, z recomputed */
    GAP_KERNEL_COUNT = 4
};
gap_status gap_kernel_timing(gap_grid_t grid, int32_t enable);
gap_status gap_kernel_stats(gap_grid_t grid, int32_t kernel, int64_t *launches, double *total_ms);

/* Measurement support: record the PCG scalars of every iteration of the following solves of
 * this handle (Table 1 steps 3 and 9): alpha_j and beta_{j-1}, the beta that formed u_j (0 at
 * j = 0), for iterations j < capacity.  With GLOBAL scalars they are the joint recurrence's;
 * with PER_COND, condition 0's.  They define the Lanczos tridiagonal of the preconditioned
 * operator, whose extreme eigenvalues estimate the condition number that bounds the
 * attainable accuracy.  Device memory: 16 B per recorded iteration, held by the handle.
 * capacity 0 stops recording and frees the buffer.  Errors: GAP_EINVAL (NULL grid,
 * capacity outside [0, 2^24]), GAP_ESTATE (grid in a batch), GAP_ENOMEM, GAP_EDEVICE. */
gap_status gap_pcg_history(gap_grid_t grid, int32_t capacity);

/* Copy the scalars recorded during the last solve of this handle (solve_joint_pcg or a solve
 * inside jacobian_adjoint, solve_with_adjoint, general_iteration_step) to host arrays of cap
 * doubles: alpha[j], beta[j] for j < *count = min(that solve's iterations, capacity, cap).
 * Synchronizes stream.  Errors: GAP_EINVAL (NULL argument, cap < 0), GAP_ESTATE (not
 * recording), GAP_EDEVICE. */
gap_status gap_get_pcg_history(gap_grid_t grid, double *alpha, double *beta, int32_t cap, int32_t *count,
                               void *stream);

/* ---- Launch configuration of the PCG iteration kernels (tuning; no effect on the method).
 * A workgroup of `threads` threads owns whole rings of one condition (thread t handles the
 * columns t, t + threads, ...; threads * cols_per_thread >= n_theta) and marches over a
 * chunk of rows; the rows of every condition are cut into chunks so that one launch places
 * wg_per_cu x (compute units) workgroups.  The A kernel (steps 9, 3 of Table 1), the B
 * kernels (steps 4-8, and the initial residual) and the one-launch kernel (F: all steps, and
 * its initial residual) are configured separately.  occupancy_*
 * report how many workgroups of the kernel fit on one CU with its shape (output only).
 * Results depend on the configuration only through the summation order of the reductions. */
typedef struct {
    int32_t threads_a;          /* A: 64, 128, 256, 512 or 1024 */
    int32_t cols_per_thread_a;  /* A: 1, 2 or 4 */
    int32_t wg_per_cu_a;        /* A: row chunking target, >= 1 */
    int32_t occupancy_a;        /* output: A workgroups that fit on one CU */
    int32_t threads_b;          /* B: as for A */
    int32_t cols_per_thread_b;
    int32_t wg_per_cu_b;
    int32_t occupancy_b;        /* output */
    int32_t threads_f;          /* F: as for A */
    int32_t cols_per_thread_f;
    int32_t wg_per_cu_f;
    int32_t occupancy_f;        /* output */
    int32_t cols_per_lane_w;    /* W (strip iteration): ring columns per lane, 1; a
                                   wavefront's strip spans 64 columns and owns all but
                                   4M + 2 on either side (M the Neumann order) */
    int32_t wg_per_cu_w;        /* W: row chunking target, >= 1 */
    int32_t occupancy_w;        /* output: W workgroups (4 wavefronts each) that fit on one CU */
    int32_t strips_w;           /* output: strips per ring */
} gap_pcg_config;

/* Read the configuration the next solve_joint_pcg of this handle uses.
 * Errors: GAP_EINVAL (NULL argument). */
gap_status gap_get_pcg_config(gap_grid_t grid, gap_pcg_config *cfg);

/* Select a configuration (cfg NULL: the default, the first candidate shape for n_theta with
 * as many workgroups per CU as fit, for every kernel).  Accepted shapes: threads x
 * cols_per_thread one of 64x1, 128x1, 128x2, 256x1, 256x2, 256x4, 512x1, 512x2, 512x4,
 * 1024x1, 1024x2 with n_theta <= threads * cols_per_thread < 2 n_theta + 64; wg_per_cu in
 * [1, 8].  Errors: GAP_EINVAL (unsupported shape or range), GAP_EDEVICE. */
gap_status gap_set_pcg_config(gap_grid_t grid, const gap_pcg_config *cfg);

/* Autotuner: time `iterations` PCG iterations of the assembled system (options of opts, run
 * from p = 0 without a stopping test) for every candidate shape of n_theta and every
 * wg_per_cu up to that shape's occupancy, with HIP events around each kernel launch; keep,
 * for each kernel of the iteration kind opts->iteration selects (A and B, or F), the fastest
 * configuration (the default unless another is at least 1 % faster), and return the whole
 * configuration in best (may be NULL) with the device time per iteration of the chosen
 * kernels in us (may be NULL).  Overwrites p (caller device memory, n_cond * n
 * doubles) and the handle's Krylov state; call solve_joint_pcg afterwards.  Stream-ordered on
 * stream, synchronizes it; resets the counters of gap_kernel_stats.  Errors: GAP_EINVAL (NULL
 * grid/opts/p, iterations outside [2, 10000]), GAP_ESTATE (nothing assembled), GAP_EDEVICE. */
gap_status gap_tune_pcg(gap_grid_t grid, const gap_solver_opts *opts, double *p, int32_t iterations,
                        gap_pcg_config *best, double *us_per_iteration, void *stream);

/* Device bytes a handle of this geometry holds (create_gap_grid with max_cond) plus the
 * caller's pressure field of max_cond * n doubles: the figure an admission controller
 * compares against its HBM budget.  The adjoint buffers (allocated on the first
 * jacobian_adjoint) are not included.  Errors: GAP_EINVAL. */
gap_status gap_grid_bytes(const gap_geom *geom, int32_t max_cond, int64_t *bytes);

/* ---- Batched execution (serving): several joint systems, possibly of different grids,
 * advance together, one launch per PCG kernel per iteration over all active requests.
 * Each request keeps its own scalars, stopping test and Krylov state on the device (in its
 * grid handle), so requests can join and leave between steps.  The work split of a request
 * depends only on its own grid and condition count, so its result is bitwise the same alone
 * and in any mix.  All calls of one batch must use the same stream; not thread-safe. */

/* Create an empty batch.  Errors: GAP_EINVAL, GAP_ENOMEM, GAP_EDEVICE. */
gap_status gap_batch_create(gap_batch_t *out);

/* Workgroups per CU the strip kernel's row chunking of the requests added from now on targets
 * (wg_per_cu >= 1; 0 restores the default, as many as fit).  A batch that targets fewer than
 * fit leaves room on every CU for the launches of another batch on another stream, so two
 * batches (say one for large and one for small requests) overlap on the device.  Results
 * depend on the target only through the summation order.  Errors: GAP_EINVAL. */
gap_status gap_batch_set_target(gap_batch_t batch, int32_t wg_per_cu);

/* Destroy a batch (the grid handles of its requests are not touched).  NULL is a no-op. */
gap_status gap_batch_destroy(gap_batch_t batch);

/* Add a request: `grid` must be assembled (its conditions form the joint system), p is its
 * device solution array (n_cond * n doubles; the initial guess if opts->warm_start), opts as
 * for solve_joint_pcg (check_every and graph are ignored here).  Computes the initial
 * residual on `stream` and returns the request id in *id.  The grid lends its Krylov
 * buffers and device record to the batch: until gap_batch_remove, assembling, solving,
 * tuning, re-configuring or destroying it returns GAP_ESTATE, and p and opts must stay
 * unchanged.  A grid is in at most one batch (GAP_EINVAL otherwise).  The first request
 * of an empty batch fixes its iteration kind (opts->iteration); a request asking for the
 * other kind returns GAP_EINVAL.  Errors: GAP_EINVAL, GAP_ESTATE, GAP_EBUDGET (all 128 slots
 * in use), GAP_ENOMEM, GAP_EDEVICE. */
gap_status gap_batch_add(gap_batch_t batch, gap_grid_t grid, const gap_solver_opts *opts, double *p, int32_t *id,
                         void *stream);

/* Run `iterations` PCG iterations of every active request (use_graph nonzero: the block of
 * launches is captured once into a hipGraph and replayed while the set of requests is
 * unchanged), then read every request's device record.  *n_done (may be NULL) receives the
 * number of requests that have finished (converged or stopped).  Synchronizes stream.
 * Errors: GAP_EINVAL, GAP_EDEVICE. */
gap_status gap_batch_step(gap_batch_t batch, int32_t iterations, int32_t use_graph, int32_t *n_done, void *stream);

/* Hold (hold != 0) or release a request: a held request keeps its Krylov state and device
 * record but is left out of the launches of gap_batch_step until released, so a scheduler
 * can choose which requests advance in each step.  Errors: GAP_EINVAL (unknown id). */
gap_status gap_batch_hold(gap_batch_t batch, int32_t id, int32_t hold);

/* Ids of the finished requests (as of the last step): up to cap ids into ids (may be NULL),
 * the total count into *count.  Errors: GAP_EINVAL. */
gap_status gap_batch_poll(gap_batch_t batch, int32_t *ids, int32_t cap, int32_t *count);

/* Remove a request (finished, or cancelled before that) and fill info (host, may be NULL)
 * with its iterations and residuals.  Returns GAP_OK for a converged request, GAP_ENOCONV
 * for one removed early or stopped at max_iter, GAP_ENONFINITE.  Its p holds the last
 * iterate.  Errors: GAP_EINVAL (unknown id), GAP_EDEVICE. */
gap_status gap_batch_remove(gap_batch_t batch, int32_t id, gap_solve_info *info, void *stream);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char *gap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GAPSOLVE_H */
