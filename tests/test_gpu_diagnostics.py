"""The PCG scalars recorded on the device (gap_pcg_history) define the Lanczos tridiagonal of
the preconditioned operator; its extreme eigenvalues against the oracle's dense spectrum of
M^{-1} A (ASSOR II, Eq 3.4), per condition and over the joint block-diagonal system."""

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
from paper_2511_06824_amd.diagnostics import condition_estimate  # noqa: E402
from paper_2511_06824_amd.solver import JointGapSolver  # noqa: E402


def log(msg):
    print(msg, flush=True)


def oracle_spectrum(case, n_cond, omega):
    """(lambda_min, lambda_max) of M_k^{-1} A_k over the conditions (the joint operator is
    block diagonal, so its spectrum is the union)."""
    gap, tex = gap_of(case), texture_of(case)
    lo, hi = np.inf, -np.inf
    for ek, edk in oracle.conditions(case.e, case.edot, case.delta)[:n_cond]:
        A, _ = oracle.assemble(gap, ek, edk, tex)
        Minv = oracle.assor2_explicit(A, omega)
        lam = np.linalg.eigvals(Minv @ A.toarray()).real
        lo, hi = min(lo, lam.min()), max(hi, lam.max())
    return lo, hi


@pytest.mark.parametrize("iteration", [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                          G.GAP_ITERATION_STRIPS],
                         ids=["two_launch", "one_launch", "strips"])
@pytest.mark.parametrize("n_cond", [1, 9])
def test_lanczos_extremes_match_the_oracle_spectrum(n_cond, iteration):
    case = synth.textured_case(24, 16, 4)
    log(f"case: {case.label} x{n_cond}, iteration kind {iteration}, Lanczos extremes")
    lo_ref, hi_ref = oracle_spectrum(case, n_cond, 1.6)
    s = JointGapSolver.from_case(case, max_cond=9 if n_cond == 9 else 1)
    s.assemble(case.e, case.edot, case.delta if n_cond == 9 else None, n_cond)
    # a fixed 200 iterations: the extreme eigenvalues of the 9 blocks lie within 5e-5 of each
    # other, and the Ritz values separate them to 1e-6 only after about 150 iterations
    G.gap_pcg_history(s.handle, 4096)
    _, info = s.solve(omega=1.6, eps=1e-300, max_iter=200, raise_on_error=False, iteration=iteration)
    alpha, beta = G.gap_get_pcg_history(s.handle, 4096)
    G.gap_pcg_history(s.handle, 0)
    s.close()
    assert info.iterations == 200 and len(alpha) == 200 and beta[0] == 0.0
    lo, hi, kappa = condition_estimate(alpha, beta)
    log(f"  {info.iterations} iterations: lambda {lo:.6e} .. {hi:.6e} (oracle {lo_ref:.6e} .. {hi_ref:.6e}), "
        f"kappa {kappa:.3e}")
    assert abs(hi - hi_ref) <= 1e-6 * hi_ref
    assert abs(lo - lo_ref) <= 1e-6 * lo_ref


def test_history_needs_recording_and_respects_capacity():
    case = synth.smooth_case(64, 32, 1)
    log(f"case: {case.label}, history capacity")
    s = JointGapSolver.from_case(case, max_cond=1)
    s.assemble(case.e, case.edot, None, 1)
    with pytest.raises(G.GapError) as ei:
        G.gap_get_pcg_history(s.handle, 8)
    assert ei.value.status == G.GAP_ESTATE
    G.gap_pcg_history(s.handle, 10)
    _, info = s.solve(omega=1.8, eps=1e-10)
    a, b = G.gap_get_pcg_history(s.handle, 64)
    assert info.iterations > 10 and len(a) == 10 and np.all(a > 0) and np.all(b[1:] > 0)
    a4, _ = G.gap_get_pcg_history(s.handle, 4)
    assert np.array_equal(a4, a[:4])
    with pytest.raises(G.GapError) as ei:
        G.gap_pcg_history(s.handle, -1)
    assert ei.value.status == G.GAP_EINVAL
    G.gap_pcg_history(s.handle, 0)
    s.close()
