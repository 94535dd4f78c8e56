"""integrate_force_moment_noalloc (the handle-free force integration whose partial sums live
in the library's fixed device scratch array) against integrate_force_moment on the same
pressure fields, called through the C ABI twice in a row, the second time on a smaller grid
with fewer conditions, so the scratch array holds the first call's partials when the second
one starts.  Bar: forces and moments within 1e-8 per (Fx, Fy) and (Mx, My) pair, the force
bar of the parity tests; the two paths differ only in the rounding of the cos / sin table."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_06824_amd import gapsolve as G  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402

F_TOL = 1e-8


def log(msg):
    print(msg, flush=True)


def rel_pair(F, ref):
    return max(np.linalg.norm(F[:2] - ref[:2]) / np.linalg.norm(ref[:2]),
               np.linalg.norm(F[2:4] - ref[2:4]) / np.linalg.norm(ref[2:4]))


def condition_eccentricities(e, delta, n_cond):
    """(e1..e4) of conditions 0 .. n_cond - 1 (Eq 2.17-2.19: the rate conditions keep e)."""
    rows = []
    for k in range(n_cond):
        ek = np.array(e, dtype=float)
        if 1 <= k <= 4:
            ek[k - 1] += delta[k - 1]
        rows.append(ek)
    return np.array(rows)


def run_pair(case, n_cond, cavitation, texture):
    """(noalloc forces, handle forces) on the handle's solved pressure."""
    planes = None
    if texture is not None:
        planes = synth.texture_samples(texture, case.n_theta, case.n_axial, case.L)
        s = JointGapSolver(case.R, case.c, case.L, case.mu, case.U, case.V, case.p_in, case.p_out,
                           case.n_theta, case.n_axial, max_cond=9, texture=planes)
    else:
        s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, n_cond)
    p, info = s.solve(s.options(omega=case.omega, eps=1e-12))
    stream = torch.cuda.current_stream().cuda_stream
    F_ref = torch.zeros(n_cond * 4, dtype=torch.float64, device="cuda:0")
    G.integrate_force_moment(s.handle, s.p.data_ptr(), cavitation, 0.0, F_ref.data_ptr(), stream)
    tex_c = None
    if planes is not None:
        tex_c = torch.as_tensor(planes[0], dtype=torch.float64).to("cuda:0").contiguous()
    F = torch.full((n_cond * 4,), float("nan"), dtype=torch.float64, device="cuda:0")
    E = condition_eccentricities(case.e, case.delta, n_cond)
    G.integrate_force_moment_noalloc(s.geom, E, tex_c.data_ptr() if tex_c is not None else None,
                                     s.p.data_ptr(), cavitation, 0.0, F.data_ptr(), stream)
    torch.cuda.synchronize()
    out = F.view(n_cond, 4).cpu().numpy(), F_ref.view(n_cond, 4).cpu().numpy()
    log(f"  {info.iterations} iterations")
    s.close()
    return out


def test_noalloc_forces_match_the_handle_twice_in_a_row():
    big = synth.smooth_case(256, 128, 4, omega=1.6)
    log("case: short pockets on 256x128, seed 4, 9 conditions, no cavitation (first call)")
    F, F_ref = run_pair(big, 9, G.GAP_CAVITATION_NONE, synth.pocket_texture("short"))
    errs = [rel_pair(F[k], F_ref[k]) for k in range(9)]
    log(f"  worst pair error {max(errs):.2e}")
    assert np.all(np.isfinite(F)) and max(errs) <= F_TOL

    small = synth.smooth_case(64, 32, 1)
    log("case: smooth 64x32, seed 1, 1 condition, clamp cavitation (second call, smaller)")
    F2, F2_ref = run_pair(small, 1, G.GAP_CAVITATION_CLAMP, None)
    err2 = rel_pair(F2[0], F2_ref[0])
    log(f"  pair error {err2:.2e}")
    assert np.all(np.isfinite(F2)) and err2 <= F_TOL


def test_noalloc_rejects_bad_arguments():
    case = synth.smooth_case(64, 32, 0)
    geom = G.make_geom(case.R, case.c, case.L, case.mu, case.U, case.V, case.p_in, case.p_out, 64, 32)
    p = torch.zeros(64 * 32, dtype=torch.float64, device="cuda:0")
    F = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    log("case: 64x32, noalloc argument checks")
    with pytest.raises(G.GapError) as ei:
        G.integrate_force_moment_noalloc(geom, [[0.0, 0.0, case.c, 0.0]], None, p.data_ptr(),
                                         G.GAP_CAVITATION_NONE, 0.0, F.data_ptr())
    assert ei.value.status == G.GAP_ECONTACT
    with pytest.raises(G.GapError) as ei:
        G.integrate_force_moment_noalloc(geom, [[0.0] * 4] * 10, None, p.data_ptr(),
                                         G.GAP_CAVITATION_NONE, 0.0, F.data_ptr())
    assert ei.value.status == G.GAP_EINVAL
    with pytest.raises(G.GapError) as ei:
        G.integrate_force_moment_noalloc(geom, [[0.0] * 4], None, p.data_ptr(), 7, 0.0, F.data_ptr())
    assert ei.value.status == G.GAP_EINVAL
