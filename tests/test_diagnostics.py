"""The Lanczos condition estimate from PCG scalars (host logic): on SPD matrices with known
spectra, scalars of a plain CG written here give the extreme eigenvalues."""

import numpy as np
import pytest

from paper_2511_06824_amd.diagnostics import condition_estimate, lanczos_tridiagonal


def cg_scalars(A, b, Minv, iters):
    """Preconditioned CG; alpha[j] and beta[j] = beta_{j-1} (beta[0] = 0)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv @ r
    u = z.copy()
    d = r @ z
    alpha, beta = [], [0.0]
    for _ in range(iters):
        v = A @ u
        a = d / (u @ v)
        alpha.append(a)
        x += a * u
        r -= a * v
        z = Minv @ r
        dn = r @ z
        beta.append(dn / d)
        u = z + (dn / d) * u
        d = dn
    return np.array(alpha), np.array(beta[:-1])


@pytest.mark.parametrize("seed", range(3))
def test_extremes_of_a_known_spectrum(seed):
    rng = np.random.default_rng(seed)
    n = 60
    lam = np.sort(rng.uniform(1.0, 500.0, n))
    lam[0], lam[-1] = 0.5, 900.0
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(lam) @ Q.T
    b = rng.normal(size=n)
    alpha, beta = cg_scalars(A, b, np.eye(n), 45)
    lo, hi, kappa = condition_estimate(alpha, beta)
    assert abs(hi - 900.0) <= 1e-6 * 900.0
    assert abs(lo - 0.5) <= 1e-6 * 0.5
    assert abs(kappa - 1800.0) <= 1e-5 * 1800.0


def test_preconditioned_spectrum():
    """With a preconditioner the estimate is the spectrum of M^{-1} A."""
    rng = np.random.default_rng(5)
    n = 40
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    Minv = np.diag(1.0 / np.diag(A))
    alpha, beta = cg_scalars(A, rng.normal(size=n), Minv, n)
    lam = np.linalg.eigvals(Minv @ A).real
    lo, hi, _ = condition_estimate(alpha, beta)
    assert abs(hi - lam.max()) <= 1e-8 * lam.max() and abs(lo - lam.min()) <= 1e-8 * lam.min()


def test_tridiagonal_matches_the_lanczos_relation():
    alpha = np.array([0.5, 0.25, 0.2])
    beta = np.array([0.0, 0.3, 0.1])
    d, e = lanczos_tridiagonal(alpha, beta)
    assert np.allclose(d, [2.0, 4.0 + 0.3 / 0.5, 5.0 + 0.1 / 0.25])
    assert np.allclose(e, [np.sqrt(0.3) / 0.5, np.sqrt(0.1) / 0.25])
