"""Seeded synthetic inputs for the piston-gap workloads.

This module only draws inputs and fixes workload parameters; it holds none of the
solver's arithmetic.  Both the CPU oracle side (tests) and the GPU side (tests, bench,
smoke) take their inputs from here.

Workloads (all FP64, SI units):

* smooth gap:  radius 10 mm, length 40 mm, clearance 20 um, viscosity 0.04 Pa s,
  2000 rpm (U = omega R = 2.0944 m/s), no axial sliding, Dirichlet 10 MPa / 0.1 MPa.
  Draws from numpy.random.default_rng(seed): e_1..e_4 ~ U(-0.5 c, 0.5 c), then
  edot_1..edot_4 ~ U(-1e-3, 1e-3) m/s.
* finite-difference steps: 1e-3 of each variable's scale, scale(e) = c,
  scale(edot) = 1e-3 m/s.
* regular dimples: 20 (circumferential) x 8 (axial) spherical caps of footprint radius
  0.5 mm over the middle 60 % of the length, centres theta = (k + 1/2) 2 pi / 20,
  z = 0.2 L + (m + 1/2) 0.6 L / 8; depths U(5, 15) um from default_rng(seed + 1000),
  drawn as an (8, 20) array, m-major.
* random dimples: count U{0..200}, centres uniform in theta and in z in [0.2 L, 0.8 L],
  same footprint radius, depth U(5, 15) um.
* pocket arrays (a texture that is not made of caps, passed as a sampled field): 60
  pockets around the circumference by 10 ("short") or 20 ("long") rows along the gap,
  20 um deep, flat-bottomed with half-cosine edge ramps so that the depth is continuous;
  the rows start 2 mm from the inlet end at a 1 mm pitch, a pocket spans half of each
  pitch in both directions.
"""

from dataclasses import dataclass, field

import numpy as np

RADIUS = 10e-3
LENGTH = 40e-3
CLEARANCE = 20e-6
VISCOSITY = 0.04
RPM = 2000.0
P_IN = 10e6
P_OUT = 0.1e6
DIMPLE_RADIUS = 0.5e-3
RATE_SCALE = 1e-3


@dataclass
class GapCase:
    """One joint-solve input: geometry, base state, FD steps and texture."""
    n_theta: int
    n_axial: int
    R: float = RADIUS
    c: float = CLEARANCE
    L: float = LENGTH
    mu: float = VISCOSITY
    U: float = 2.0 * np.pi * RPM / 60.0 * RADIUS
    V: float = 0.0
    p_in: float = P_IN
    p_out: float = P_OUT
    e: np.ndarray = field(default_factory=lambda: np.zeros(4))
    edot: np.ndarray = field(default_factory=lambda: np.zeros(4))
    delta: np.ndarray = field(default_factory=lambda: np.concatenate(
        [np.full(4, 1e-3 * CLEARANCE), np.full(4, 1e-3 * RATE_SCALE)]))
    dimple_theta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    dimple_z: np.ndarray = field(default_factory=lambda: np.zeros(0))
    dimple_radius: np.ndarray = field(default_factory=lambda: np.zeros(0))
    dimple_depth: np.ndarray = field(default_factory=lambda: np.zeros(0))
    omega: float = 1.6
    eps: float = 1e-10
    label: str = ""

    @property
    def n(self):
        return self.n_theta * self.n_axial

    @property
    def n_dimples(self):
        return int(self.dimple_theta.size)


def draw_state(seed, clearance=CLEARANCE):
    rng = np.random.default_rng(seed)
    e = rng.uniform(-0.5 * clearance, 0.5 * clearance, 4)
    edot = rng.uniform(-RATE_SCALE, RATE_SCALE, 4)
    return e, edot


def smooth_case(n_theta, n_axial, seed, **kw):
    e, edot = draw_state(seed)
    kw.setdefault("omega", 1.8)
    return GapCase(n_theta=n_theta, n_axial=n_axial, e=e, edot=edot,
                   label=f"smooth {n_theta}x{n_axial} seed {seed}", **kw)


def regular_dimples(seed, L=LENGTH, n_circ=20, n_ax=8):
    rng = np.random.default_rng(seed + 1000)
    depth = rng.uniform(5e-6, 15e-6, size=(n_ax, n_circ))
    k = np.arange(n_circ)
    m = np.arange(n_ax)
    th = (k + 0.5) * 2.0 * np.pi / n_circ
    zc = 0.2 * L + (m + 0.5) * 0.6 * L / n_ax
    TH, Z = np.meshgrid(th, zc)
    return TH.ravel(), Z.ravel(), np.full(TH.size, DIMPLE_RADIUS), depth.ravel()


def random_dimples(rng, L=LENGTH, max_count=200):
    count = int(rng.integers(0, max_count + 1))
    th = rng.uniform(0.0, 2.0 * np.pi, count)
    zc = rng.uniform(0.2 * L, 0.8 * L, count)
    depth = rng.uniform(5e-6, 15e-6, count)
    return th, zc, np.full(count, DIMPLE_RADIUS), depth


def _plateau(x, half, ramp):
    """1 for |x| <= half - ramp, 0 for |x| >= half, a half-cosine in between."""
    a = np.abs(x)
    t = np.clip((a - (half - ramp)) / ramp, 0.0, 1.0)
    return 0.5 * (1.0 + np.cos(np.pi * t))


def pocket_texture(kind="short", depth=20e-6, n_circ=60, L=LENGTH):
    """Depth function h_text(theta, z) of a pocket array ("short": 60 x 10 pockets,
    "long": 60 x 20), see the module docstring.  Returns a callable of numpy arrays."""
    n_ax = {"short": 10, "long": 20}[kind]
    pitch_t = 2.0 * np.pi / n_circ
    pitch_z = 1e-3
    z0 = 2e-3
    half_t, half_z = 0.25 * pitch_t, 0.25 * pitch_z
    ramp_t, ramp_z = 0.3 * half_t, 0.3 * half_z

    def tex(theta, z):
        theta, z = np.broadcast_arrays(np.asarray(theta, dtype=float), np.asarray(z, dtype=float))
        # offset from the nearest pocket centre, in theta (centres at (k + 1/2) pitch,
        # periodic) and in z (within the rows)
        dt = np.mod(theta, pitch_t) - 0.5 * pitch_t
        m = np.clip(np.floor((z - z0) / pitch_z), 0, n_ax - 1)
        dz = z - (z0 + (m + 0.5) * pitch_z)
        return depth * _plateau(dt, half_t, ramp_t) * _plateau(dz, half_z, ramp_z)

    return tex


def texture_samples(tex, n_theta, n_axial, L=LENGTH):
    """The depth function sampled where the assembly needs the film: cell centres
    [n_axial, n_theta], east faces [n_axial, n_theta] and axial faces [n_axial + 1, n_theta]."""
    dth, dz = 2.0 * np.pi / n_theta, L / n_axial
    i = np.arange(n_theta)
    th_c, th_e = (i + 0.5) * dth, (i + 1.0) * dth
    z_c = (np.arange(n_axial) + 0.5) * dz
    z_f = np.arange(n_axial + 1) * dz
    return (tex(th_c[None, :], z_c[:, None]), tex(th_e[None, :], z_c[:, None]),
            tex(th_c[None, :], z_f[:, None]))


def textured_case(n_theta, n_axial, seed, **kw):
    e, edot = draw_state(seed)
    th, zc, a, d = regular_dimples(seed)
    kw.setdefault("omega", 1.6)
    return GapCase(n_theta=n_theta, n_axial=n_axial, e=e, edot=edot, dimple_theta=th,
                   dimple_z=zc, dimple_radius=a, dimple_depth=d,
                   label=f"textured {n_theta}x{n_axial} seed {seed}", **kw)


SERVE_SIZES = [(128, 64), (256, 128), (512, 256), (1024, 512), (2048, 1024)]


def served_request(rng, seed):
    """One request of the served stream: size class, smooth or random dimples (50/50)."""
    nt, nz = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
    e, edot = draw_state(seed)
    if rng.uniform() < 0.5:
        th, zc, a, d = random_dimples(rng)
        return GapCase(n_theta=nt, n_axial=nz, e=e, edot=edot, dimple_theta=th, dimple_z=zc,
                       dimple_radius=a, dimple_depth=d, omega=1.6,
                       label=f"served dimpled {nt}x{nz} seed {seed}")
    return GapCase(n_theta=nt, n_axial=nz, e=e, edot=edot, omega=1.6,
                   label=f"served smooth {nt}x{nz} seed {seed}")


def poisson_arrivals(rng, rate, count):
    """Arrival times (s) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, count))


# Named workloads with their sizes.
WORKLOADS = {
    "smooth_64x32": dict(n_theta=64, n_axial=32, kind="smooth", n_cond=1),
    "joint_smooth_512x256": dict(n_theta=512, n_axial=256, kind="smooth", n_cond=9),
    "joint_textured_2048x1024": dict(n_theta=2048, n_axial=1024, kind="textured", n_cond=9),
    "adjoint_textured_1024x512": dict(n_theta=1024, n_axial=512, kind="textured", n_cond=9),
}


def make_case(name, seed=0, **kw):
    w = WORKLOADS[name]
    f = smooth_case if w["kind"] == "smooth" else textured_case
    return f(w["n_theta"], w["n_axial"], seed, **kw)


def projection_weights(n, count=4, seed=7000):
    """Seeded standard-normal weight vectors (count, n) for random projections w . p of a
    pressure field: a check of the whole field against stored values without storing it."""
    return np.stack([np.random.default_rng(seed + m).standard_normal(n) for m in range(count)])


def golden_sample_index(n_theta, n_axial, col_stride=32, row_stride=16):
    """Rows and columns of the stored pressure sample: every row_stride-th ring and every
    col_stride-th column, plus the last ring (outlet end) and the last column (wrap)."""
    rows = np.unique(np.concatenate([np.arange(0, n_axial, row_stride), [n_axial - 1]]))
    cols = np.unique(np.concatenate([np.arange(0, n_theta, col_stride), [n_theta - 1]]))
    return rows, cols
