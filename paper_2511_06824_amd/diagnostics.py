"""Spectral diagnostics of a PCG solve from its recorded scalars (measurement support).

PCG is the Lanczos process on the preconditioned operator M^{-1} A in the M-inner product.
Its scalars alpha_j (Table 1 step 3) and beta_j (step 9) give the Lanczos tridiagonal

    T[j, j]     = 1 / alpha_j + beta_{j-1} / alpha_{j-1}        (the second term absent at j = 0)
    T[j, j + 1] = sqrt(beta_j) / alpha_j,

whose extreme eigenvalues converge to those of M^{-1} A.  Their ratio estimates the condition
number kappa, and kappa times the unit roundoff bounds the relative accuracy a FP64 solve can
reach.  The scalars come from the device (gap_pcg_history / gap_get_pcg_history); only this
small eigenproblem runs on the host.
"""

import numpy as np


def lanczos_tridiagonal(alpha, beta):
    """(diagonal, off-diagonal) of T from alpha[j] = alpha_j and beta[j] = beta_{j-1} (the
    beta that formed u_j, beta[0] = 0), as gap_get_pcg_history returns them."""
    alpha = np.asarray(alpha, dtype=float)
    beta = np.asarray(beta, dtype=float)
    k = alpha.size
    d = 1.0 / alpha
    d[1:] += beta[1:] / alpha[:-1]
    e = np.sqrt(beta[1:k]) / alpha[: k - 1]
    return d, e


def condition_estimate(alpha, beta):
    """(lambda_min, lambda_max, kappa) of the preconditioned operator from the Lanczos
    tridiagonal of the recorded scalars."""
    from scipy.linalg import eigvalsh_tridiagonal
    d, e = lanczos_tridiagonal(alpha, beta)
    if d.size == 1:
        return d[0], d[0], 1.0
    lo = eigvalsh_tridiagonal(d, e, select="i", select_range=(0, 0))[0]
    hi = eigvalsh_tridiagonal(d, e, select="i", select_range=(d.size - 1, d.size - 1))[0]
    return float(lo), float(hi), float(hi / lo)
