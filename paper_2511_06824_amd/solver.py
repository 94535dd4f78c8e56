"""Torch-facing wrapper of the gapsolve C ABI: device buffers and streams come from torch,
every step of the path runs in the HIP library (``gapsolve``)."""

import torch

from . import gapsolve as G


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class JointGapSolver:
    """One gap geometry (+ dimples) on one GPU, holding up to `max_cond` conditions.

    Owns the library handle and the caller-side buffers: p (n_cond x n), F (n_cond x 4),
    J (4 x 8), all float64 on `device`."""

    def __init__(self, R, clearance, length, mu, U, V, p_in, p_out, n_theta, n_axial,
                 dimples=None, max_cond=9, device="cuda:0", texture=None):
        if not torch.cuda.is_available():
            raise RuntimeError("JointGapSolver needs a HIP GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self.n_theta, self.n_axial = int(n_theta), int(n_axial)
        self.n = self.n_theta * self.n_axial
        self.max_cond = int(max_cond)
        self.geom = G.make_geom(R, clearance, length, mu, U, V, p_in, p_out, n_theta, n_axial)
        dm = None
        if dimples is not None and len(dimples[0]) > 0:
            dm = G.make_dimples(*dimples)
        with torch.cuda.device(self.device):
            if texture is not None:
                # a sampled texture field: (centres, east faces, axial faces), see create_gap_grid_field
                if dm is not None:
                    raise ValueError("give either dimples or a texture field, not both")
                shapes = [(self.n_axial, self.n_theta), (self.n_axial, self.n_theta),
                          (self.n_axial + 1, self.n_theta)]
                planes = [torch.as_tensor(t, dtype=torch.float64).to(self.device).contiguous() for t in texture]
                for t, shp in zip(planes, shapes):
                    if tuple(t.shape) != shp:
                        raise ValueError(f"texture plane of shape {tuple(t.shape)}, expected {shp}")
                torch.cuda.synchronize(self.device)     # the library copies the planes on its own stream
                self.handle = G.create_gap_grid_field(self.geom, planes[0].data_ptr(), planes[1].data_ptr(),
                                                      planes[2].data_ptr(), self.max_cond)
            else:
                self.handle = G.create_gap_grid(self.geom, dm, self.max_cond)
        self.p = torch.zeros(self.max_cond * self.n, dtype=torch.float64, device=self.device)
        self.F = torch.zeros(self.max_cond * 4, dtype=torch.float64, device=self.device)
        self.J = torch.zeros(32, dtype=torch.float64, device=self.device)
        self.J_adj = torch.zeros(32, dtype=torch.float64, device=self.device)
        self.n_cond = 0

    @staticmethod
    def device_bytes(n_theta, n_axial, max_cond=9, **geom):
        """Device bytes one solver of this grid holds (library buffers + its pressure field)."""
        d = dict(R=0.01, clearance=2e-5, length=0.04, mu=0.04, U=0.0, V=0.0, p_in=0.0, p_out=0.0)
        d.update(geom)
        g = G.make_geom(d["R"], d["clearance"], d["length"], d["mu"], d["U"], d["V"], d["p_in"], d["p_out"],
                        n_theta, n_axial)
        return G.gap_grid_bytes(g, max_cond) + (max_cond * 4 + 64) * 8

    @classmethod
    def from_case(cls, case, max_cond=9, device="cuda:0"):
        dimples = None
        if case.n_dimples:
            dimples = (case.dimple_theta, case.dimple_z, case.dimple_radius, case.dimple_depth)
        return cls(case.R, case.c, case.L, case.mu, case.U, case.V, case.p_in, case.p_out,
                   case.n_theta, case.n_axial, dimples=dimples, max_cond=max_cond, device=device)

    @staticmethod
    def geometry_key(case):
        """What a handle is built for, apart from its texture: grid and geometry."""
        return (case.n_theta, case.n_axial, case.R, case.c, case.L, case.mu, case.U, case.V, case.p_in, case.p_out)

    def set_dimples(self, dimples=None):
        """Replace the texture by a dimple list (theta, z, radius, depth), or make the gap smooth
        (None): reuses this handle for another request of the same geometry without allocating
        device memory.  The next solve needs a new assemble."""
        dm = G.make_dimples(*dimples) if dimples is not None and len(dimples[0]) > 0 else None
        G.set_gap_dimples(self.handle, dm, _stream(self.device))
        self.n_cond = 0

    @staticmethod
    def case_dimples(case):
        if not case.n_dimples:
            return None
        return (case.dimple_theta, case.dimple_z, case.dimple_radius, case.dimple_depth)

    def close(self):
        if getattr(self, "handle", None) is not None:
            G.destroy_gap_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the four steps -------------------------------------------------------------
    def assemble(self, e, edot, delta=None, n_cond=9):
        G.assemble_joint_system(self.handle, e, edot, delta, n_cond, _stream(self.device))
        self.n_cond = int(n_cond)

    @staticmethod
    def options(omega=1.6, eps=1e-10, max_iter=100000, precond=G.GAP_PRECOND_ASSOR2, scalars=G.GAP_SCALARS_GLOBAL,
                warm_start=False, check_every=0, neumann=1, graph=True, strategy=G.GAP_STRATEGY_SYNC,
                iteration=G.GAP_ITERATION_STRIPS, eps_adjoint=0.0):
        o = G.gap_default_opts()
        o.omega, o.eps, o.max_iter = float(omega), float(eps), int(max_iter)
        o.eps_adjoint = float(eps_adjoint)
        o.precond, o.scalars, o.neumann = int(precond), int(scalars), int(neumann)
        o.warm_start, o.check_every, o.graph = int(bool(warm_start)), int(check_every), int(bool(graph))
        o.strategy, o.iteration = int(strategy), int(iteration)
        return o

    def solve(self, opts=None, raise_on_error=True, **kw):
        """Returns (p view of shape (n_cond, n_axial, n_theta), gap_solve_info)."""
        opts = opts if opts is not None else self.options(**kw)
        st, info = G.solve_joint_pcg(self.handle, opts, self.p.data_ptr(), _stream(self.device), raise_on_error)
        return self.pressure(), info

    def set_operating_point(self, U, V, p_in, p_out):
        """Sliding speeds and end pressures for the next assembly (pump kinematics)."""
        G.set_operating_point(self.handle, U, V, p_in, p_out)
        self.geom.U, self.geom.V, self.geom.p_in, self.geom.p_out = float(U), float(V), float(p_in), float(p_out)

    def general_iteration_step(self, e, edot, delta, dt, edot_prev, F_ext, mass, opts=None,
                               scheme=G.GAP_SCHEME_GENERAL, jacobian=G.GAP_JACOBIAN_FD):
        """One general iteration of the piston equilibrium (GMAF step V); returns
        (e_new, edot_new, residual F, oil-film Jacobian, gap_solve_info)."""
        from .dynamics import step_params
        opts = opts if opts is not None else self.options()
        prm = step_params(dt, edot_prev, F_ext, mass, scheme, jacobian)
        return G.general_iteration_step(self.handle, opts, prm, delta, self.p.data_ptr(), e, edot,
                                        _stream(self.device))

    def tune(self, opts=None, iterations=20, **kw):
        """Autotune the PCG kernel shape and row chunking on the assembled system; the choice
        stays on the handle.  Overwrites the pressure field.  Returns (config dict, us per
        iteration)."""
        opts = opts or self.options(**kw)
        cfg, us = G.gap_tune_pcg(self.handle, opts, self.p.data_ptr(), iterations, _stream(self.device))
        return cfg.as_dict(), us

    def tune_neumann(self, opts=None, max_order=3, **kw):
        """Pick the ASSOR II Neumann order by time to solution (each order with its own tuned
        strip configuration, which stays on the handle for the winner).  Overwrites the pressure
        field.  Returns (order, [seconds per solve of orders 1 .. max_order]); pass the order as
        `neumann` to the solves that follow."""
        opts = opts or self.options(**kw)
        return G.gap_tune_neumann(self.handle, opts, self.p.data_ptr(), max_order, _stream(self.device))

    @property
    def pcg_config(self):
        return G.gap_get_pcg_config(self.handle).as_dict()

    def set_pcg_config(self, threads=None, cols_per_thread=None, wg_per_cu_a=None, wg_per_cu_b=None,
                       threads_b=None, cols_per_thread_b=None, threads_f=None, cols_per_thread_f=None,
                       wg_per_cu_f=None):
        """Select the PCG kernel configuration: shape (threads x columns per thread) of A, of B
        when threads_b / cols_per_thread_b are given (else the same as A) and of the one-launch
        kernel F when threads_f / cols_per_thread_f are given (else the same as B); F's row
        chunking follows wg_per_cu_f, else wg_per_cu_b.  No arguments: the default."""
        if threads is None:
            G.gap_set_pcg_config(self.handle, None)
            return self.pcg_config
        cur = G.gap_get_pcg_config(self.handle)
        cfg = G.gap_pcg_config()
        cfg.threads_a, cfg.cols_per_thread_a = int(threads), int(cols_per_thread)
        cfg.threads_b = int(threads if threads_b is None else threads_b)
        cfg.cols_per_thread_b = int(cols_per_thread if cols_per_thread_b is None else cols_per_thread_b)
        cfg.threads_f = int(cfg.threads_b if threads_f is None else threads_f)
        cfg.cols_per_thread_f = int(cfg.cols_per_thread_b if cols_per_thread_f is None else cols_per_thread_f)
        cfg.wg_per_cu_a = cur.wg_per_cu_a if wg_per_cu_a is None else int(wg_per_cu_a)
        cfg.wg_per_cu_b = cur.wg_per_cu_b if wg_per_cu_b is None else int(wg_per_cu_b)
        cfg.wg_per_cu_f = (cfg.wg_per_cu_b if wg_per_cu_b is not None else cur.wg_per_cu_f) \
            if wg_per_cu_f is None else int(wg_per_cu_f)
        cfg.cols_per_lane_w, cfg.wg_per_cu_w = cur.cols_per_lane_w, cur.wg_per_cu_w
        G.gap_set_pcg_config(self.handle, cfg)
        return self.pcg_config

    def set_strip_config(self, cols_per_lane, wg_per_cu):
        """Select the strip kernel's columns per lane and row-chunking target; the other
        kernels keep their configuration."""
        cfg = G.gap_get_pcg_config(self.handle)
        cfg.cols_per_lane_w, cfg.wg_per_cu_w = int(cols_per_lane), int(wg_per_cu)
        G.gap_set_pcg_config(self.handle, cfg)
        return self.pcg_config

    def pressure(self):
        return self.p[: self.n_cond * self.n].view(self.n_cond, self.n_axial, self.n_theta)

    def integrate(self, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0, p=None):
        src = self.p if p is None else p
        G.integrate_force_moment(self.handle, src.data_ptr(), cavitation, p_cav, self.F.data_ptr(),
                                 _stream(self.device))
        return self.F[: self.n_cond * 4].view(self.n_cond, 4)

    def integrate_split(self, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0, p=None):
        """Forces split per condition: (n_cond, 10) = pressure (Fx, Fy, Mx, My), shear (Fx, Fy, Mx,
        My, Fz, Mz)."""
        src = self.p if p is None else p
        out = torch.empty(self.n_cond * 10, dtype=torch.float64, device=self.device)
        G.integrate_force_moment_split(self.handle, src.data_ptr(), cavitation, p_cav, out.data_ptr(),
                                       _stream(self.device))
        return out.view(self.n_cond, 10)

    def full_pressure(self, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0, p=None):
        """The pressure of every condition with its two boundary rows: (n_cond, n_axial + 2, n_theta)."""
        src = self.p if p is None else p
        out = torch.empty(self.n_cond * (self.n_axial + 2) * self.n_theta, dtype=torch.float64, device=self.device)
        G.rebuild_pressure_field(self.handle, src.data_ptr(), cavitation, p_cav, out.data_ptr(), _stream(self.device))
        return out.view(self.n_cond, self.n_axial + 2, self.n_theta)

    def jacobian_fd(self):
        G.jacobian_fd(self.handle, self.F.data_ptr(), self.J.data_ptr(), _stream(self.device))
        return self.J.view(4, 8)

    def jacobian_adjoint(self, opts=None, p0=None, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0, w=None, **kw):
        """Adjoint derivative of the condition-0 forces: the 4 x 8 Jacobian (w None) or the
        8-vector w^T J (w: 4 weights).  p0 defaults to the solved pressure of condition 0.
        Returns (tensor, gap_solve_info of the adjoint solve)."""
        opts = opts if opts is not None else self.options(**kw)
        src = self.p if p0 is None else p0
        info = G.jacobian_adjoint(self.handle, opts, src.data_ptr(), cavitation, p_cav, w, self.J_adj.data_ptr(),
                                  _stream(self.device))
        out = self.J_adj[:8].clone() if w is not None else self.J_adj.view(4, 8).clone()
        return out, info

    def solve_with_adjoint(self, opts=None, w=None, **kw):
        """Solve condition 0 of the assembly together with its adjoint systems (no cavitation):
        returns (pressure of condition 0, 4 x 8 Jacobian or w^T J, gap_solve_info).  The
        pressure lands in the first block of the handle's field."""
        opts = opts if opts is not None else self.options(**kw)
        info = G.solve_with_adjoint(self.handle, opts, self.p.data_ptr(), w, self.J_adj.data_ptr(),
                                    _stream(self.device))
        out = self.J_adj[:8].clone() if w is not None else self.J_adj.view(4, 8).clone()
        return self.p[:self.n].view(self.n_axial, self.n_theta), out, info

    def read_system(self, k):
        kx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        kz = torch.empty(self.n + self.n_theta, dtype=torch.float64, device=self.device)
        S = torch.empty(self.n, dtype=torch.float64, device=self.device)
        G.gap_read_system(self.handle, k, kx.data_ptr(), kz.data_ptr(), S.data_ptr(), _stream(self.device))
        return (kx.view(self.n_axial, self.n_theta), kz.view(self.n_axial + 1, self.n_theta),
                S.view(self.n_axial, self.n_theta))

    def step(self, e, edot, delta, opts, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0):
        """One pass of the hot path: assemble 9 conditions, joint PCG, forces, FD Jacobian."""
        self.assemble(e, edot, delta, 9)
        _, info = self.solve(opts)
        F = self.integrate(cavitation, p_cav)
        J = self.jacobian_fd()
        return F, J, info
