"""A general texture field through create_gap_grid_field (Eq 2.3's h_Text sampled at the cell
centres, east faces and axial faces) against the oracle evaluating the same depth function
at its own points.  The layouts are the pocket arrays of the paper's Sec 4.4 (60 x 10
"short" and 60 x 20 "long" rectangular pockets, 20 um deep), which no list of spherical caps
describes.  Bars: assembly entries 1e-12 relative (the source 1e-11 of its largest entry),
pressure 1e-9, forces 1e-8 per pair, the FD Jacobian 1e-5 per block."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_06824_amd import gapsolve as G  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402

P_TOL, F_TOL, J_TOL = 1e-9, 1e-8, 1e-5


def log(msg):
    print(msg, flush=True)


def field_solver(case, tex, max_cond=9):
    planes = synth.texture_samples(tex, case.n_theta, case.n_axial, case.L)
    return JointGapSolver(case.R, case.c, case.L, case.mu, case.U, case.V, case.p_in, case.p_out,
                          case.n_theta, case.n_axial, max_cond=max_cond, texture=planes)


def rel_pair(F, ref):
    return max(np.linalg.norm(F[:2] - ref[:2]) / np.linalg.norm(ref[:2]),
               np.linalg.norm(F[2:4] - ref[2:4]) / np.linalg.norm(ref[2:4]))


@pytest.mark.parametrize("kind,shape", [("short", (240, 160)), ("long", (300, 200)), ("long", (61, 37))],
                         ids=["short_240x160", "long_300x200", "long_61x37"])
def test_pocket_texture_field_against_oracle(kind, shape):
    case = synth.smooth_case(*shape, 5, omega=1.6)
    tex = synth.pocket_texture(kind)
    log(f"case: {kind} pockets on {shape[0]}x{shape[1]}, seed 5, 9 conditions, texture field")
    gap = gap_of(case)
    s = field_solver(case, tex)
    s.assemble(case.e, case.edot, case.delta, 9)
    # assembly: face conductances and source of every distinct operator / condition
    conds = oracle.conditions(case.e, case.edot, case.delta)
    for k in (0, 1, 5):
        kx, kz, S = [t.cpu().numpy() for t in s.read_system(k)]
        kx_r, kz_r = oracle.face_conductances(gap, conds[k][0], tex)
        S_r = oracle.source(gap, *conds[k], tex)
        # the oracle forms R_c^2 - R^2 literally (about 3e-14 of cancellation, amplified where
        # the film is thinnest); the kernel uses c (2 R + c)
        assert np.max(np.abs(kx - kx_r) / np.abs(kx_r)) < 1e-12
        assert np.max(np.abs(kz - kz_r) / np.abs(kz_r)) < 1e-12
        assert np.max(np.abs(S - S_r)) < 1e-11 * np.max(np.abs(S_r))
    p, info = s.solve(s.options(omega=1.6, eps=1e-13))
    F = s.integrate().cpu().numpy()
    J = s.jacobian_fd().cpu().numpy()
    p = p.reshape(9, -1).cpu().numpy()
    F_ref = np.zeros((9, 4))
    worst_p = 0.0
    for k, (ek, edk) in enumerate(conds):
        F_ref[k], p_ref = oracle.condition_forces(gap, ek, edk, tex)
        worst_p = max(worst_p, np.linalg.norm(p[k] - p_ref) / np.linalg.norm(p_ref))
        assert rel_pair(F[k], F_ref[k]) <= F_TOL
    J_ref = oracle.jacobian_fd(F_ref, case.delta)
    blocks = [J[0:2, 0:4], J[0:2, 4:8], J[2:4, 0:4], J[2:4, 4:8]]
    blocks_ref = [J_ref[0:2, 0:4], J_ref[0:2, 4:8], J_ref[2:4, 0:4], J_ref[2:4, 4:8]]
    e_j = max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(blocks, blocks_ref))
    log(f"  iterations {info.iterations}, pressure {worst_p:.2e}, jacobian {e_j:.2e}")
    assert worst_p <= P_TOL
    assert e_j <= J_TOL
    s.close()


def test_texture_field_of_zeros_equals_the_smooth_grid():
    """A field of zeros and the dimple-free create give the same system, bitwise."""
    case = synth.smooth_case(128, 64, 2)
    log(f"case: {case.label}, zero texture field against no dimples")
    a = field_solver(case, lambda th, z: np.zeros(np.broadcast(th, z).shape))
    b = JointGapSolver.from_case(case, max_cond=9)
    for s in (a, b):
        s.assemble(case.e, case.edot, case.delta, 9)
    for k in (0, 3, 7):
        for x, y in zip(a.read_system(k), b.read_system(k)):
            assert torch.equal(x, y)
    a.close()
    b.close()


def test_texture_field_rejects_bad_depths():
    case = synth.smooth_case(32, 16, 0)
    tc, te, tf = synth.texture_samples(synth.pocket_texture("short"), 32, 16)
    for plane, name in ((0, "tex_c"), (1, "tex_e"), (2, "tex_f")):
        for bad in (-1e-6, float("nan")):
            planes = [tc.copy(), te.copy(), tf.copy()]
            planes[plane][3, 5] = bad
            log(f"case: 32x16, {name}[3, 5] = {bad}")
            with pytest.raises(G.GapError) as ei:
                JointGapSolver(case.R, case.c, case.L, case.mu, case.U, case.V, case.p_in, case.p_out,
                               32, 16, texture=planes)
            assert ei.value.status == G.GAP_EINVAL and name in str(ei.value)
    lib = G.load()
    h = G.ctypes.c_void_p()
    assert lib.create_gap_grid_field(G.ctypes.byref(G.make_geom(case.R, case.c, case.L, case.mu, case.U, case.V,
                                                                case.p_in, case.p_out, 32, 16)),
                                     None, None, None, 9, G.ctypes.byref(h)) == G.GAP_EINVAL
