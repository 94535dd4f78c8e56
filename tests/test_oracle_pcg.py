"""Pins for the oracle's preconditioners and PCG (paper Table 1, Eq 2.8, 3.2-3.6, 3.9)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from conftest import gap_of, texture_of


def random_spd(n, seed):
    """Random symmetric M-matrix (graph Laplacian of a random graph + positive diagonal)."""
    rng = np.random.default_rng(seed)
    W = np.triu(rng.uniform(0, 1, (n, n)) * (rng.uniform(0, 1, (n, n)) < 0.5), 1)
    W = W + W.T
    A = np.diag(W.sum(1) + rng.uniform(0.1, 1.0, n)) - W
    return sp.csr_matrix(A)


@pytest.mark.parametrize("n,seed", [(6, 0), (9, 1), (12, 2)])
@pytest.mark.parametrize("omega", [0.4, 1.0, 1.6, 1.8])
def test_two_step_assor2_equals_explicit_eq_3_4(n, seed, omega):
    A = random_spd(n, seed)
    Minv = oracle.assor2_explicit(A, omega)
    apply = oracle.assor2_precond(A, omega)
    I = np.eye(n)
    two_step = np.column_stack([apply(I[:, k]) for k in range(n)])
    assert np.max(np.abs(two_step - Minv)) <= 1e-13 * np.max(np.abs(Minv))


@pytest.mark.parametrize("omega", [0.3, 1.0, 1.6, 1.9])
def test_assor2_inverse_is_spd(omega):
    A = random_spd(10, 7)
    Minv = oracle.assor2_explicit(A, omega)
    assert np.max(np.abs(Minv - Minv.T)) <= 1e-14 * np.max(np.abs(Minv))
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0


def test_neumann_series_to_full_length_is_exact_ssor_inverse():
    """D^{-1}L is strictly lower triangular (nilpotent): keeping n-1 Neumann terms inverts
    (D + wL) exactly, so the apply must equal the exact inverse of M of Eq 3.3."""
    n, omega = 8, 1.3
    A = random_spd(n, 3)
    Ad = np.asarray(A.todense())
    D = np.diag(np.diag(Ad))
    L = np.tril(Ad, -1)
    M = (D + omega * L) @ np.linalg.inv(D) @ (D + omega * L).T / (omega * (2 - omega))
    apply = oracle.assor2_precond(A, omega, neumann=n - 1)
    I = np.eye(n)
    got = np.column_stack([apply(I[:, k]) for k in range(n)])
    assert np.max(np.abs(got - np.linalg.inv(M))) <= 1e-12 * np.max(np.abs(got))


@pytest.mark.parametrize("omega", [0.5, 1.2, 1.8])
def test_assor1_is_diagonal_of_eq_3_2(omega):
    A = random_spd(11, 4)
    Ad = np.asarray(A.todense())
    D = np.diag(np.diag(Ad))
    L = np.tril(Ad, -1)
    prod = (D + omega * L) @ np.linalg.inv(D) @ (D + omega * L).T
    r = np.random.default_rng(0).normal(size=11)
    assert np.allclose(oracle.assor1_precond(A, omega)(r), omega * (2 - omega) * r / np.diag(prod),
                       rtol=1e-14, atol=0)


def test_wrap_entries_split_between_l_and_lt():
    """Natural order: the east wrap of the last ring column is below the diagonal."""
    case = synth.smooth_case(8, 3, 0)
    gap = gap_of(case)
    A, _ = oracle.assemble(gap, case.e, case.edot)
    from oracle.pcg import split
    D, L = split(A)
    nt = gap.n_theta
    g_last = 1 * nt + nt - 1       # (i = nt-1, j = 1)
    g_first = 1 * nt               # (i = 0, j = 1)
    assert L[g_last, g_first] != 0 and L[g_first, g_last] == 0


def test_unpreconditioned_table1_matches_textbook_cg():
    case = synth.smooth_case(64, 32, 1)
    gap = gap_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot)
    p, it, hist = oracle.pcg(A, S, lambda r: r.copy(), 1e-8, 100000)
    count = [0]

    def cb(xk):
        count[0] += 1

    ref, info = spla.cg(A, S, rtol=1e-8, atol=0.0, maxiter=100000, callback=cb)
    assert info == 0
    assert abs(it - count[0]) <= 1
    assert np.linalg.norm(p - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("seed", range(3))
def test_pcg_reaches_exact_solution_and_assor_halves_iterations(seed):
    case = synth.textured_case(128, 64, seed)
    gap = gap_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot, texture_of(case))
    exact = oracle.solve_band(A, S, gap.n_theta)
    pj, itj, _ = oracle.pcg(A, S, oracle.jacobi_precond(A), 1e-12, 100000)
    pa, ita, hist = oracle.pcg(A, S, oracle.assor2_precond(A, 1.6), 1e-12, 100000)
    for q in (pj, pa):
        assert np.linalg.norm(q - exact) / np.linalg.norm(exact) < 1e-9
    assert 0.35 < ita / itj < 0.7          # paper Table 2: 1709 / 3308 = 0.52
    assert hist[-1] <= 1e-12 < hist[-2]


def test_joint_system_global_scalars_solves_every_block():
    case = synth.smooth_case(64, 32, 2)
    gap = gap_of(case)
    AG, SG = oracle.assemble_joint(gap, case.e, case.edot, case.delta)
    pG, it, hist = oracle.pcg(AG, SG, oracle.assor2_precond(AG, 1.8), 1e-13, 100000)
    n = gap.n_theta * gap.n_axial
    assert np.linalg.norm(SG - AG @ pG) / np.linalg.norm(SG) < 1e-12
    for k, (ek, edk) in enumerate(oracle.conditions(case.e, case.edot, case.delta)):
        A, S = oracle.assemble(gap, ek, edk)
        exact = oracle.solve_band(A, S, gap.n_theta)
        assert np.linalg.norm(pG[k * n:(k + 1) * n] - exact) / np.linalg.norm(exact) < 1e-10
    # synchronized test (Eq 3.9) on the joint vector equals the recurrence norm at exit
    assert hist[-1] <= 1e-13


def test_zero_iterations_for_exact_start():
    case = synth.smooth_case(16, 8, 0)
    gap = gap_of(case)
    A, S = oracle.assemble(gap, case.e, case.edot)
    exact = oracle.solve_band(A, S, gap.n_theta)
    _, it, _ = oracle.pcg(A, S, oracle.jacobi_precond(A), 1e-10, 100, p0=exact)
    assert it == 0


def _blocks(case):
    gap = gap_of(case)
    tex = texture_of(case)
    blocks, rhs = [], []
    for ek, edk in oracle.conditions(case.e, case.edot, case.delta):
        A, S = oracle.assemble(gap, ek, edk, tex)
        blocks.append(A)
        rhs.append(S)
    return blocks, rhs


def test_block_pcg_global_sync_equals_pcg_on_joint_matrix():
    case = synth.textured_case(48, 24, 1)
    blocks, rhs = _blocks(case)
    M = [oracle.assor2_precond(A, 1.6) for A in blocks]
    pb, itb, hb = oracle.pcg_blocks(blocks, rhs, M, 1e-10, 10000, "global", "sync")
    AG = sp.block_diag(blocks, format="csr")
    pG, itG, hG = oracle.pcg(AG, np.concatenate(rhs), oracle.assor2_precond(AG, 1.6), 1e-10, 10000)
    assert itb == itG
    assert np.allclose(hb, hG, rtol=1e-8, atol=0)
    assert np.linalg.norm(np.concatenate(pb) - pG) <= 1e-12 * np.linalg.norm(pG)


def test_block_pcg_per_cond_async_equals_solo_solves():
    """Independent recurrences stopped by their own test are exactly the solo solves."""
    case = synth.textured_case(48, 24, 2)
    blocks, rhs = _blocks(case)
    M = [oracle.assor2_precond(A, 1.6) for A in blocks]
    pb, itb, _ = oracle.pcg_blocks(blocks, rhs, M, 1e-10, 10000, "per_cond", "async")
    its = []
    for k, (A, S) in enumerate(zip(blocks, rhs)):
        ps, it, _ = oracle.pcg(A, S, M[k], 1e-10, 10000)
        its.append(it)
        assert np.array_equal(ps, pb[k])
    assert itb == max(its)


def test_block_pcg_variants_reach_the_solution():
    case = synth.smooth_case(40, 20, 3)
    blocks, rhs = _blocks(case)
    M = [oracle.assor2_precond(A, 1.8) for A in blocks]
    exact = [oracle.solve_band(A, S, 40) for A, S in zip(blocks, rhs)]
    for sc in ("global", "per_cond"):
        for st in ("sync", "async"):
            pb, it, _ = oracle.pcg_blocks(blocks, rhs, M, 1e-12, 10000, sc, st)
            for k in range(len(blocks)):
                assert np.linalg.norm(pb[k] - exact[k]) <= 1e-9 * np.linalg.norm(exact[k]), (sc, st, k)
