"""GPU edge cases through the C ABI: closed-form degenerate solutions, the largest axial size,
an empty batch."""

import numpy as np
import pytest

import oracle
import synth
from conftest import gap_of, texture_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_06824_amd import gapsolve as G  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402


def log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("ecc,U", [((0.0, 0.0, 0.0, 0.0), 2.0), ((6e-6, -3e-6, 6e-6, -3e-6), 0.0)],
                         ids=["concentric", "parallel-offset"])
def test_linear_axial_profile_closed_form(ecc, U):
    """A film independent of z without wedge or squeeze: the discrete solution is exactly
    p = p_in + (p_out - p_in) z / L (cell centres, Dirichlet faces half a cell away)."""
    case = synth.smooth_case(96, 40, 0)
    log(f"case: linear axial profile, e = {ecc}, U = {U}")
    s = JointGapSolver(case.R, case.c, case.L, case.mu, U, 0.0, case.p_in, case.p_out, 96, 40, max_cond=1)
    s.assemble(np.array(ecc), np.zeros(4), None, 1)
    p, info = s.solve(omega=1.8, eps=1e-13)
    p = p.reshape(40, 96).cpu().numpy()
    s.close()
    z = (np.arange(40) + 0.5) * case.L / 40
    exact = case.p_in + (case.p_out - case.p_in) * z / case.L
    err = np.max(np.abs(p - exact[:, None])) / case.p_in
    log(f"  iterations {info.iterations}, max error {err:.1e} of p_in")
    assert err <= 1e-9


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                          G.GAP_ITERATION_STRIPS],
                         ids=["two_launch", "one_launch", "strips"])
def test_largest_axial_size_follows_the_oracle_recurrence(iteration):
    """n_axial = 65536 (the largest accepted) on a 16-cell ring, one condition: 100 iterations of
    the GPU recurrence against 100 iterations of the oracle's Table 1 PCG with ASSOR II."""
    nt, nz = 16, 65536
    case = synth.smooth_case(nt, nz, 1)
    log(f"case: {case.label}, 100 PCG iterations against the oracle, iteration kind {iteration}")
    gap = gap_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot)
    M = oracle.assor2_precond(A, 1.8)
    p_ref, it_ref, hist = oracle.pcg(A, S, M, 1e-300, 100)
    s = JointGapSolver.from_case(case, max_cond=1)
    s.assemble(case.e, case.edot, None, 1)
    p, info = s.solve(omega=1.8, eps=1e-300, max_iter=100, raise_on_error=False, iteration=iteration)
    p = p.reshape(-1).cpu().numpy()
    kx, kz, Sg = [t.cpu().numpy() for t in s.read_system(0)]
    s.close()
    assert info.status == G.GAP_ENOCONV and info.iterations == 100 == it_ref
    perr = np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref)
    rerr = abs(info.rel_residual - hist[-1]) / hist[-1]
    true_rel = np.linalg.norm(Sg.ravel() - oracle.stencil_matrix(gap, kx, kz) @ p) / np.linalg.norm(Sg)
    log(f"  pressure {perr:.1e}, recurrence residual {info.rel_residual:.3e} vs {hist[-1]:.3e}, true {true_rel:.3e}")
    assert perr <= 1e-8 and rerr <= 1e-6
    assert abs(true_rel - info.rel_residual) <= 1e-6 * info.rel_residual
    np.testing.assert_allclose(Sg.ravel(), S, rtol=1e-11, atol=1e-11 * np.max(np.abs(S)))


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                          G.GAP_ITERATION_STRIPS],
                         ids=["two_launch", "one_launch", "strips"])
@pytest.mark.parametrize("scalars,strategy,eps,max_iter", [
    ("global", "sync", 1e-300, 7), ("global", "sync", 1e-300, 8),
    ("per_cond", "async", 3e-3, 1000), ("global", "async", 3e-3, 1000)],
    ids=["cap_odd", "cap_even", "per_cond_async", "global_async"])
def test_pressure_is_whole_after_a_stop_at_either_parity(scalars, strategy, eps, max_iter, iteration):
    """p after the solve stops at an odd or an even iteration: by the iteration cap, or by
    conditions frozen one by one under the asynchronized test (Eq 3.10).  The one-launch kernel
    moves p on odd iterations only, so a stop after an even iteration has a term left to
    settle.  The perturbations are large enough that the nine conditions freeze at iterations
    of both parities (31 to 42 at eps 3e-3), and the stops come early, where the last
    update of p is far above the 1e-8 bound."""
    case = synth.textured_case(64, 32, 5)
    delta = np.array([0.2 * case.c * f for f in (1.0, -1.0, 0.5, -0.7)] + [3e-2, -2e-2, 1e-2, 4e-2])
    log(f"case: {case.label}, {scalars} scalars, {strategy}, eps {eps}, max_iter {max_iter}, "
        f"iteration kind {iteration}")
    gap, tex = gap_of(case), texture_of(case)
    blocks_, rhs = [], []
    for ek, edk in oracle.conditions(case.e, case.edot, delta):
        A, S = oracle.assemble(gap, ek, edk, tex)
        blocks_.append(A)
        rhs.append(S)
    M = [oracle.assor2_precond(A, 1.6) for A in blocks_]
    p_ref, it_ref, _ = oracle.pcg_blocks(blocks_, rhs, M, eps, max_iter, scalars, strategy)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, delta, 9)
    p, info = s.solve(omega=1.6, eps=eps, max_iter=max_iter, raise_on_error=False,
                      scalars=G.GAP_SCALARS_PER_COND if scalars == "per_cond" else G.GAP_SCALARS_GLOBAL,
                      strategy=G.GAP_STRATEGY_ASYNC if strategy == "async" else G.GAP_STRATEGY_SYNC,
                      iteration=iteration)
    p = p.reshape(9, -1).cpu().numpy()
    s.close()
    errs = [np.linalg.norm(p[k] - p_ref[k]) / np.linalg.norm(p_ref[k]) for k in range(9)]
    log(f"  iterations {info.iterations} (oracle {it_ref}), worst pressure error {max(errs):.1e}")
    if strategy == "sync":
        assert info.status == G.GAP_ENOCONV and info.iterations == max_iter == it_ref
    else:
        assert info.status == G.GAP_OK and abs(info.iterations - it_ref) <= 1
    assert max(errs) <= 1e-8, errs


def test_ring_wider_than_2048_cells_needs_strips_and_matches_the_exact_solution():
    """n_theta = 2304: more columns than a whole-ring workgroup holds.  The strip iteration cuts
    each ring into 20 strips; against the oracle's banded-Cholesky solution at eps 1e-13 the
    pressure meets 1e-9 and the forces 1e-8 per pair; the whole-ring kinds refuse the grid."""
    case = synth.textured_case(2304, 6, 7)
    log(f"case: {case.label}, 9 conditions, strips on a ring of 2304 cells")
    gap, tex = gap_of(case), texture_of(case)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    for it in (G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH):
        with pytest.raises(G.GapError) as ei:
            s.solve(omega=1.6, eps=1e-10, iteration=it)
        assert ei.value.status == G.GAP_EINVAL and "STRIPS" in str(ei.value)
    cfg = s.pcg_config
    assert cfg["cols_per_lane_w"] == 1 and cfg["strips_w"] == -(-2304 // (64 - 12))   # 52 owned columns each
    p, info = s.solve(omega=1.6, eps=1e-13, iteration=G.GAP_ITERATION_STRIPS)
    F = s.integrate().cpu().numpy()
    p = p.reshape(9, -1).cpu().numpy()
    conds = oracle.conditions(case.e, case.edot, case.delta)
    for k in (0, 1, 5):
        F_ref, p_ref = oracle.condition_forces(gap, *conds[k], tex)
        perr = np.linalg.norm(p[k] - p_ref) / np.linalg.norm(p_ref)
        ferr = max(np.linalg.norm(F[k, :2] - F_ref[:2]) / np.linalg.norm(F_ref[:2]),
                   np.linalg.norm(F[k, 2:] - F_ref[2:]) / np.linalg.norm(F_ref[2:]))
        log(f"  condition {k}: {info.iterations} iterations, pressure {perr:.1e}, forces {ferr:.1e}")
        assert perr <= 1e-9 and ferr <= 1e-8
    s.close()


def test_widest_ring_follows_the_oracle_pcg():
    """n_theta = 16384, the largest ring: 100 strip iterations against the oracle's Table 1 PCG
    on the same system (the exact solve is out of reach at this bandwidth)."""
    case = synth.textured_case(16384, 3, 8)
    log(f"case: {case.label}, 1 condition, 100 strip iterations")
    gap, tex = gap_of(case), texture_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot, tex)
    p_ref, it_ref, hist = oracle.pcg(A, S, oracle.assor2_precond(A, 1.6), 1e-300, 100)
    s = JointGapSolver.from_case(case, max_cond=1)
    s.assemble(case.e, case.edot, None, 1)
    p, info = s.solve(omega=1.6, eps=1e-300, max_iter=100, raise_on_error=False,
                      iteration=G.GAP_ITERATION_STRIPS)
    p = p.reshape(-1).cpu().numpy()
    s.close()
    perr = np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref)
    log(f"  pressure {perr:.1e}, recurrence residual {info.rel_residual:.3e} vs {hist[-1]:.3e}")
    assert info.status == G.GAP_ENOCONV and info.iterations == 100 == it_ref
    assert perr <= 1e-8 and abs(info.rel_residual - hist[-1]) <= 1e-6 * hist[-1]


def test_empty_batch_steps_and_polls():
    log("case: empty batch")
    b = G.gap_batch_create()
    stream = torch.cuda.current_stream().cuda_stream
    for use_graph in (True, False):
        G.gap_batch_step(b, 4, use_graph, stream)
    assert G.gap_batch_poll(b) == []
    G.gap_batch_destroy(b)


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                          G.GAP_ITERATION_STRIPS],
                         ids=["two_launch", "one_launch", "strips"])
def test_non_finite_warm_start_reports_enonfinite_and_the_handle_recovers(iteration):
    """A warm-start field holding a NaN: r_0 = S - A p_0 is NaN near that cell, so the first
    reduction is not finite.  The solve stops with GAP_ENONFINITE (NaN arithmetic only, every
    kernel runs its bounded loops), and a cold solve on the same handle afterwards gives the
    same pressure, bit for bit, as the one before."""
    case = synth.smooth_case(64, 32, 3)
    log(f"case: {case.label}, NaN in the warm start, iteration kind {iteration}")
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    p0, info0 = s.solve(omega=1.8, eps=1e-12, iteration=iteration)
    p0 = p0.clone()
    s.p[5 * s.n + 1234] = float("nan")
    _, info = s.solve(omega=1.8, eps=1e-12, warm_start=True, raise_on_error=False, iteration=iteration)
    log(f"  status {info.status} after {info.iterations} iterations: {G.gap_last_error()}")
    assert info.status == G.GAP_ENONFINITE
    assert "non-finite" in G.gap_last_error()
    s.p.fill_(float("nan"))
    with pytest.raises(G.GapError) as ei:
        s.solve(omega=1.8, eps=1e-12, warm_start=True, iteration=iteration)
    assert ei.value.status == G.GAP_ENONFINITE
    p1, info1 = s.solve(omega=1.8, eps=1e-12, iteration=iteration)
    assert info1.status == G.GAP_OK and info1.iterations == info0.iterations
    assert torch.equal(p1, p0)
    s.close()
