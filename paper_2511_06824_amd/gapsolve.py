"""ctypes binding of the gapsolve C ABI (include/gapsolve.h), same names as the C entry points.

Argument marshalling only: every step of the solve runs in the HIP library.  Device
buffers are passed as integer addresses (for instance ``tensor.data_ptr()`` of a torch
CUDA tensor) and streams as the integer value of a hipStream_t (``None`` or 0: the
default stream).  Every non-OK status raises ``GapError`` carrying the library's message.
If the library has not been built, importing this module succeeds but the first call
raises ``GapLibraryMissing``: there is no fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libgapsolve.so")

GAP_OK = 0
GAP_EINVAL = -1
GAP_ECONTACT = -2
GAP_ENOCONV = -3
GAP_ENONFINITE = -4
GAP_ENOMEM = -5
GAP_EDEVICE = -6
GAP_ESTATE = -7
GAP_EBUDGET = -8
STATUS_NAMES = {0: "GAP_OK", -1: "GAP_EINVAL", -2: "GAP_ECONTACT", -3: "GAP_ENOCONV",
                -4: "GAP_ENONFINITE", -5: "GAP_ENOMEM", -6: "GAP_EDEVICE", -7: "GAP_ESTATE",
                -8: "GAP_EBUDGET"}

GAP_PRECOND_JACOBI, GAP_PRECOND_ASSOR1, GAP_PRECOND_ASSOR2 = 0, 1, 2
GAP_SCALARS_GLOBAL, GAP_SCALARS_PER_COND = 0, 1
GAP_STRATEGY_SYNC, GAP_STRATEGY_ASYNC = 0, 1
GAP_CAVITATION_NONE, GAP_CAVITATION_CLAMP = 0, 1
GAP_MAX_COND = 9
GAP_ITERATION_TWO_LAUNCH, GAP_ITERATION_ONE_LAUNCH, GAP_ITERATION_STRIPS = 0, 1, 2
GAP_KERNEL_PCG_A, GAP_KERNEL_PCG_B, GAP_KERNEL_PCG_ONE, GAP_KERNEL_PCG_STRIPS = 0, 1, 2, 3
GAP_KERNEL_COUNT = 4
KERNEL_NAMES = ["k_pcg_a", "k_pcg_b", "k_pcg_f", "k_pcg_w"]


class gap_geom(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("clearance", ctypes.c_double), ("length", ctypes.c_double),
                ("mu", ctypes.c_double), ("U", ctypes.c_double), ("V", ctypes.c_double),
                ("p_in", ctypes.c_double), ("p_out", ctypes.c_double),
                ("n_theta", ctypes.c_int32), ("n_axial", ctypes.c_int32)]


class gap_dimples(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("theta", ctypes.POINTER(ctypes.c_double)),
                ("z", ctypes.POINTER(ctypes.c_double)), ("radius", ctypes.POINTER(ctypes.c_double)),
                ("depth", ctypes.POINTER(ctypes.c_double))]


class gap_solver_opts(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("eps", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("neumann", ctypes.c_int32), ("scalars", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("check_every", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("strategy", ctypes.c_int32), ("iteration", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eps_adjoint", ctypes.c_double)]


class gap_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32), ("n_cond", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("rel_residual_cond", ctypes.c_double * GAP_MAX_COND),
                ("true_rel_residual", ctypes.c_double),
                ("true_rel_residual_cond", ctypes.c_double * GAP_MAX_COND)]


class gap_pcg_config(ctypes.Structure):
    _fields_ = [("threads_a", ctypes.c_int32), ("cols_per_thread_a", ctypes.c_int32),
                ("wg_per_cu_a", ctypes.c_int32), ("occupancy_a", ctypes.c_int32),
                ("threads_b", ctypes.c_int32), ("cols_per_thread_b", ctypes.c_int32),
                ("wg_per_cu_b", ctypes.c_int32), ("occupancy_b", ctypes.c_int32),
                ("threads_f", ctypes.c_int32), ("cols_per_thread_f", ctypes.c_int32),
                ("wg_per_cu_f", ctypes.c_int32), ("occupancy_f", ctypes.c_int32),
                ("cols_per_lane_w", ctypes.c_int32), ("wg_per_cu_w", ctypes.c_int32),
                ("occupancy_w", ctypes.c_int32), ("strips_w", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class gap_step_params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("edot_prev", ctypes.c_double * 4), ("F_ext", ctypes.c_double * 4),
                ("mass", ctypes.c_double * 16), ("scheme", ctypes.c_int32), ("jacobian", ctypes.c_int32)]


GAP_SCHEME_GENERAL, GAP_SCHEME_CONVENTIONAL = 0, 1
GAP_JACOBIAN_FD, GAP_JACOBIAN_ADJOINT = 0, 1


class GapLibraryMissing(RuntimeError):
    pass


class GapError(RuntimeError):
    def __init__(self, status, message, info=None):
        self.status = status
        self.info = info
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


_lib = None
_P = ctypes.c_void_p
_D8 = ctypes.POINTER(ctypes.c_double)

_SIGNATURES = {
    "gap_default_opts": [ctypes.POINTER(gap_solver_opts)],
    "create_gap_grid": [ctypes.POINTER(gap_geom), ctypes.POINTER(gap_dimples), ctypes.c_int32,
                        ctypes.POINTER(_P)],
    "create_gap_grid_field": [ctypes.POINTER(gap_geom), _P, _P, _P, ctypes.c_int32, ctypes.POINTER(_P)],
    "destroy_gap_grid": [_P],
    "set_gap_dimples": [_P, ctypes.POINTER(gap_dimples), _P],
    "assemble_joint_system": [_P, _D8, _D8, _D8, ctypes.c_int32, _P],
    "solve_joint_pcg": [_P, ctypes.POINTER(gap_solver_opts), _P, ctypes.POINTER(gap_solve_info), _P],
    "integrate_force_moment": [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P],
    "integrate_force_moment_split": [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P],
    "integrate_force_moment_noalloc": [ctypes.POINTER(gap_geom), ctypes.c_int32, _D8, _P, _P, ctypes.c_int32,
                                       ctypes.c_double, _P, _P],
    "rebuild_pressure_field": [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P],
    "jacobian_fd": [_P, _P, _P, _P],
    "gap_read_system": [_P, ctypes.c_int32, _P, _P, _P, _P],
    "jacobian_adjoint": [_P, ctypes.POINTER(gap_solver_opts), _P, ctypes.c_int32, ctypes.c_double, _D8, _P,
                         ctypes.POINTER(gap_solve_info), _P],
    "solve_with_adjoint": [_P, ctypes.POINTER(gap_solver_opts), _P, _D8, _P, ctypes.POINTER(gap_solve_info), _P],
    "general_iteration_step": [_P, ctypes.POINTER(gap_solver_opts), ctypes.POINTER(gap_step_params), _D8, _P, _D8, _D8,
                               _D8, _D8, ctypes.POINTER(gap_solve_info), _P],
    "set_operating_point": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "gap_grid_bytes": [ctypes.POINTER(gap_geom), ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)],
    "gap_batch_create": [ctypes.POINTER(_P)],
    "gap_batch_destroy": [_P],
    "gap_batch_add": [_P, _P, ctypes.POINTER(gap_solver_opts), _P, ctypes.POINTER(ctypes.c_int32), _P],
    "gap_batch_step": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _P],
    "gap_batch_poll": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "gap_batch_hold": [_P, ctypes.c_int32, ctypes.c_int32],
    "gap_batch_set_target": [_P, ctypes.c_int32],
    "gap_batch_remove": [_P, ctypes.c_int32, ctypes.POINTER(gap_solve_info), _P],
    "gap_kernel_timing": [_P, ctypes.c_int32],
    "gap_get_pcg_config": [_P, ctypes.POINTER(gap_pcg_config)],
    "gap_set_pcg_config": [_P, ctypes.POINTER(gap_pcg_config)],
    "gap_tune_pcg": [_P, ctypes.POINTER(gap_solver_opts), _P, ctypes.c_int32, ctypes.POINTER(gap_pcg_config),
                     ctypes.POINTER(ctypes.c_double), _P],
    "gap_kernel_stats": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "gap_tune_neumann": [_P, ctypes.POINTER(gap_solver_opts), _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                         _D8, _P],
    "gap_pcg_history": [_P, ctypes.c_int32],
    "gap_get_pcg_history": [_P, _D8, _D8, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _P],
}


def library_path():
    return LIB_PATH


def load():
    """Load the HIP library (once).  Raises GapLibraryMissing if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GapLibraryMissing(
                f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.gap_last_error.argtypes = []
        lib.gap_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def gap_last_error():
    return load().gap_last_error().decode()


def _check(status, info=None):
    if status != GAP_OK:
        raise GapError(status, gap_last_error(), info)


def _darr(values, count):
    if values is None:
        return None
    vals = [float(v) for v in values]
    if len(vals) != count:
        raise ValueError(f"expected {count} values, got {len(vals)}")
    return (ctypes.c_double * count)(*vals)


def _stream(stream):
    return ctypes.c_void_p(int(stream) if stream else 0)


def gap_default_opts():
    o = gap_solver_opts()
    _check(load().gap_default_opts(ctypes.byref(o)))
    return o


def make_geom(R, clearance, length, mu, U, V, p_in, p_out, n_theta, n_axial):
    return gap_geom(float(R), float(clearance), float(length), float(mu), float(U), float(V),
                    float(p_in), float(p_out), int(n_theta), int(n_axial))


def make_dimples(theta, z, radius, depth):
    """gap_dimples over host copies; the returned object keeps its arrays alive."""
    count = len(theta)
    d = gap_dimples()
    d.count = count
    d._keep = [(ctypes.c_double * max(count, 1))(*[float(v) for v in arr]) for arr in (theta, z, radius, depth)]
    d.theta, d.z, d.radius, d.depth = [ctypes.cast(a, _D8) for a in d._keep]
    return d


def create_gap_grid(geom, dimples, max_cond):
    h = ctypes.c_void_p()
    _check(load().create_gap_grid(ctypes.byref(geom), ctypes.byref(dimples) if dimples is not None else None,
                                  int(max_cond), ctypes.byref(h)))
    return h


def create_gap_grid_field(geom, tex_c_ptr, tex_e_ptr, tex_f_ptr, max_cond):
    h = ctypes.c_void_p()
    _check(load().create_gap_grid_field(ctypes.byref(geom), ctypes.c_void_p(int(tex_c_ptr)),
                                        ctypes.c_void_p(int(tex_e_ptr)), ctypes.c_void_p(int(tex_f_ptr)),
                                        int(max_cond), ctypes.byref(h)))
    return h


def destroy_gap_grid(handle):
    _check(load().destroy_gap_grid(handle))


def set_gap_dimples(handle, dimples, stream=None):
    _check(load().set_gap_dimples(handle, ctypes.byref(dimples) if dimples is not None else None, _stream(stream)))


def assemble_joint_system(handle, e, edot, delta, n_cond, stream=None):
    _check(load().assemble_joint_system(handle, _darr(e, 4), _darr(edot, 4), _darr(delta, 8), int(n_cond),
                                        _stream(stream)))


def solve_joint_pcg(handle, opts, p_ptr, stream=None, raise_on_error=True):
    """Returns (status, gap_solve_info); raises GapError on failure unless told not to."""
    info = gap_solve_info()
    st = load().solve_joint_pcg(handle, ctypes.byref(opts), ctypes.c_void_p(int(p_ptr)), ctypes.byref(info),
                                _stream(stream))
    if raise_on_error:
        _check(st, info)
    return st, info


def integrate_force_moment(handle, p_ptr, cavitation, p_cav, F_ptr, stream=None):
    _check(load().integrate_force_moment(handle, ctypes.c_void_p(int(p_ptr)), int(cavitation), float(p_cav),
                                         ctypes.c_void_p(int(F_ptr)), _stream(stream)))


def integrate_force_moment_split(handle, p_ptr, cavitation, p_cav, F_ptr, stream=None):
    _check(load().integrate_force_moment_split(handle, ctypes.c_void_p(int(p_ptr)), int(cavitation), float(p_cav),
                                               ctypes.c_void_p(int(F_ptr)), _stream(stream)))


def integrate_force_moment_noalloc(geom, e, tex_c_ptr, p_ptr, cavitation, p_cav, F_ptr, stream=None):
    """e: n_cond rows of (e1, e2, e3, e4); tex_c_ptr: device address or None (smooth)."""
    rows = [list(map(float, row)) for row in e]
    flat = [v for row in rows for v in row]
    _check(load().integrate_force_moment_noalloc(ctypes.byref(geom), len(rows), _darr(flat, 4 * len(rows)),
                                                 ctypes.c_void_p(int(tex_c_ptr) if tex_c_ptr else 0),
                                                 ctypes.c_void_p(int(p_ptr)), int(cavitation), float(p_cav),
                                                 ctypes.c_void_p(int(F_ptr)), _stream(stream)))


def rebuild_pressure_field(handle, p_ptr, cavitation, p_cav, out_ptr, stream=None):
    _check(load().rebuild_pressure_field(handle, ctypes.c_void_p(int(p_ptr)), int(cavitation), float(p_cav),
                                         ctypes.c_void_p(int(out_ptr)), _stream(stream)))


def jacobian_fd(handle, F_ptr, J_ptr, stream=None):
    _check(load().jacobian_fd(handle, ctypes.c_void_p(int(F_ptr)), ctypes.c_void_p(int(J_ptr)), _stream(stream)))


def jacobian_adjoint(handle, opts, p0_ptr, cavitation, p_cav, w, J_ptr, stream=None):
    """Adjoint Jacobian (w None: 4 x 8 into J) or vector-Jacobian product (w: 4 weights,
    8 values into J).  Returns the gap_solve_info of the adjoint solve."""
    info = gap_solve_info()
    _check(load().jacobian_adjoint(handle, ctypes.byref(opts), ctypes.c_void_p(int(p0_ptr)), int(cavitation),
                                   float(p_cav), _darr(w, 4), ctypes.c_void_p(int(J_ptr)), ctypes.byref(info),
                                   _stream(stream)), info)
    return info


def solve_with_adjoint(handle, opts, p0_ptr, w, J_ptr, stream=None):
    """Base solve of condition 0 and its adjoint solves as one joint solve (no cavitation);
    p0 (n values) and J (4 x 8, or 8 with weights w) are written.  Returns gap_solve_info."""
    info = gap_solve_info()
    _check(load().solve_with_adjoint(handle, ctypes.byref(opts), ctypes.c_void_p(int(p0_ptr)), _darr(w, 4),
                                     ctypes.c_void_p(int(J_ptr)), ctypes.byref(info), _stream(stream)), info)
    return info


def general_iteration_step(handle, opts, prm, delta, p_ptr, e, edot, stream=None):
    """One general iteration (GMAF step V).  e, edot: 4 values each (not modified).
    Returns (e_new, edot_new, residual F at the input state, oil-film J (4 x 8), info)."""
    e_arr = (ctypes.c_double * 4)(*[float(x) for x in e])
    ed_arr = (ctypes.c_double * 4)(*[float(x) for x in edot])
    F = (ctypes.c_double * 4)()
    J = (ctypes.c_double * 32)()
    info = gap_solve_info()
    _check(load().general_iteration_step(handle, ctypes.byref(opts), ctypes.byref(prm), _darr(delta, 8),
                                         ctypes.c_void_p(int(p_ptr)), e_arr, ed_arr, F, J, ctypes.byref(info),
                                         _stream(stream)), info)
    return list(e_arr), list(ed_arr), list(F), [list(J[8 * i:8 * i + 8]) for i in range(4)], info


def set_operating_point(handle, U, V, p_in, p_out):
    _check(load().set_operating_point(handle, float(U), float(V), float(p_in), float(p_out)))


def gap_read_system(handle, k, kx_ptr, kz_ptr, S_ptr, stream=None):
    _check(load().gap_read_system(handle, int(k), ctypes.c_void_p(int(kx_ptr or 0)),
                                  ctypes.c_void_p(int(kz_ptr or 0)), ctypes.c_void_p(int(S_ptr or 0)),
                                  _stream(stream)))


def gap_kernel_timing(handle, enable):
    _check(load().gap_kernel_timing(handle, int(enable)))


def gap_kernel_stats(handle, kernel):
    """(launches, total device milliseconds) of one iteration kernel kind."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(load().gap_kernel_stats(handle, int(kernel), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def gap_pcg_history(handle, capacity):
    """Record alpha_j and beta_{j-1} of the next solves' iterations j < capacity (0: stop)."""
    _check(load().gap_pcg_history(handle, int(capacity)))


def gap_get_pcg_history(handle, cap, stream=None):
    """(alpha, beta) of the last solve as numpy arrays: alpha[j] = alpha_j, beta[j] = beta_{j-1}
    (the beta that formed u_j; beta[0] = 0)."""
    import numpy as np
    a = (ctypes.c_double * max(int(cap), 1))()
    b = (ctypes.c_double * max(int(cap), 1))()
    n = ctypes.c_int32(0)
    _check(load().gap_get_pcg_history(handle, a, b, int(cap), ctypes.byref(n), _stream(stream)))
    return np.array(a[: n.value]), np.array(b[: n.value])


def gap_get_pcg_config(handle):
    cfg = gap_pcg_config()
    _check(load().gap_get_pcg_config(handle, ctypes.byref(cfg)))
    return cfg


def gap_set_pcg_config(handle, cfg=None):
    """cfg: a gap_pcg_config, or None for the default configuration."""
    _check(load().gap_set_pcg_config(handle, ctypes.byref(cfg) if cfg is not None else None))


def gap_tune_pcg(handle, opts, p_ptr, iterations, stream=None):
    """Autotune the PCG kernel configuration; returns (gap_pcg_config, us per iteration).
    Overwrites the device field at p_ptr."""
    cfg = gap_pcg_config()
    us = ctypes.c_double(0.0)
    _check(load().gap_tune_pcg(handle, ctypes.byref(opts), ctypes.c_void_p(int(p_ptr)), int(iterations),
                               ctypes.byref(cfg), ctypes.byref(us), _stream(stream)))
    return cfg, us.value


def gap_grid_bytes(geom, max_cond):
    b = ctypes.c_int64(0)
    _check(load().gap_grid_bytes(ctypes.byref(geom), int(max_cond), ctypes.byref(b)))
    return b.value


def gap_batch_create():
    h = ctypes.c_void_p()
    _check(load().gap_batch_create(ctypes.byref(h)))
    return h


def gap_batch_destroy(batch):
    _check(load().gap_batch_destroy(batch))


def gap_batch_add(batch, grid, opts, p_ptr, stream=None):
    rid = ctypes.c_int32(0)
    _check(load().gap_batch_add(batch, grid, ctypes.byref(opts), ctypes.c_void_p(int(p_ptr)), ctypes.byref(rid),
                                _stream(stream)))
    return rid.value


def gap_batch_step(batch, iterations, use_graph=True, stream=None):
    nd = ctypes.c_int32(0)
    _check(load().gap_batch_step(batch, int(iterations), int(bool(use_graph)), ctypes.byref(nd), _stream(stream)))
    return nd.value


def gap_batch_set_target(batch, wg_per_cu):
    _check(load().gap_batch_set_target(batch, int(wg_per_cu)))


def gap_batch_hold(batch, bid, hold):
    _check(load().gap_batch_hold(batch, int(bid), int(bool(hold))))


def gap_batch_poll(batch, cap=128):
    ids = (ctypes.c_int32 * cap)()
    count = ctypes.c_int32(0)
    _check(load().gap_batch_poll(batch, ids, int(cap), ctypes.byref(count)))
    return [ids[k] for k in range(min(count.value, cap))]


def gap_batch_remove(batch, rid, stream=None, raise_on_error=True):
    """Returns (status, gap_solve_info)."""
    info = gap_solve_info()
    st = load().gap_batch_remove(batch, int(rid), ctypes.byref(info), _stream(stream))
    if raise_on_error:
        _check(st, info)
    return st, info


def gap_tune_neumann(handle, opts, p_ptr, max_order=3, stream=None):
    """Returns (best Neumann order, [seconds per solve of orders 1 .. max_order])."""
    best = ctypes.c_int32()
    secs = (ctypes.c_double * int(max_order))()
    _check(load().gap_tune_neumann(handle, ctypes.byref(opts), ctypes.c_void_p(int(p_ptr)), int(max_order),
                                   ctypes.byref(best), secs, _stream(stream)))
    return best.value, list(secs)
