"""Oracle: the adjusted PCG of Table 1 and its preconditioners (paper Sec 2.2, 3.1, 3.3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A = L + D + L^T with L the strict lower triangle in the natural order (theta fastest),
so the periodic east-wrap entry of the last column of each ring lies in L and the
west-wrap entry of the first column lies in L^T.

* Jacobi (Eq 2.8): M = D.
* ASSOR I (Eq 3.2): diagonal M^{-1}_ii = w (2 - w) / {(D + w L) D^{-1} (D + w L)^T}_ii.
* ASSOR II (Eq 3.3-3.6): M = (D + w L) D^{-1} (D + w L)^T / (w (2 - w)); its inverse is
  approximated by truncating the Neumann series of (I + w D^{-1} L)^{-1} after the linear
  term (Eq 3.4), and applied in the two steps of Eq 3.5-3.6:
      v = (I - w D^{-1} L) D^{-1} r,     z = (2 - w) w (I - w D^{-1} L^T) v.
  ``neumann`` > 1 keeps further terms of the same series in both factors.
* PCG (Table 1), with the initial residual read as r0 = S - A p0 (the printed sign of
  step 2 would make the iteration ascend), the stopping test of step 6 applied to the
  recurrence residual, ||r|| / ||S|| <= eps, which on the joint block-diagonal system is
  the synchronized criterion of Eq 3.9.
"""

import numpy as np
import scipy.sparse as sp


def split(A):
    A = sp.csr_matrix(A)
    return A.diagonal(), sp.tril(A, k=-1, format="csr")


def jacobi_precond(A):
    D, _ = split(A)
    return lambda r: r / D


def assor1_diagonal(A, omega):
    """Diagonal of (D + wL) D^{-1} (D + wL)^T = D_ii + w^2 sum_k L_ik^2 / D_kk."""
    D, L = split(A)
    return D + omega * omega * (L.multiply(L) @ (1.0 / D))


def assor1_precond(A, omega):
    d = assor1_diagonal(A, omega)
    return lambda r: omega * (2.0 - omega) * r / d


def assor2_precond(A, omega, neumann=1):
    """z = M^{-1} r for ASSOR II via the two steps of Eq 3.5-3.6 (Neumann order `neumann`)."""
    D, L = split(A)
    LT = sp.csr_matrix(L.T)

    def apply(r):
        y = r / D
        v, t = y.copy(), y.copy()
        for _ in range(neumann):
            t = -omega * (L @ t) / D
            v = v + t
        z, t = v.copy(), v.copy()
        for _ in range(neumann):
            t = -omega * (LT @ t) / D
            z = z + t
        return omega * (2.0 - omega) * z

    return apply


def assor2_explicit(A, omega):
    """Dense matrix of Eq 3.4: (2-w) w D^{-1} (I - w L^T D^{-1}) D (I - w D^{-1} L) D^{-1}."""
    A = np.asarray(sp.csr_matrix(A).todense())
    D = np.diag(np.diag(A))
    Dinv = np.diag(1.0 / np.diag(A))
    L = np.tril(A, k=-1)
    I = np.eye(A.shape[0])
    return (2.0 - omega) * omega * Dinv @ (I - omega * L.T @ Dinv) @ D @ (I - omega * Dinv @ L) @ Dinv


def pcg(A, S, precond, eps, max_iter, p0=None):
    """Table 1.  Returns (p, iterations, history of ||r_j|| / ||S||)."""
    A = sp.csr_matrix(A)
    S = np.asarray(S, dtype=float)
    p = np.zeros_like(S) if p0 is None else np.array(p0, dtype=float)
    s_norm = np.linalg.norm(S)
    r = S - A @ p
    hist = [np.linalg.norm(r) / s_norm]
    if hist[-1] <= eps:
        return p, 0, hist
    z = precond(r)
    u = z.copy()
    d = r @ z
    it = 0
    while it < max_iter:
        v = A @ u
        alpha = d / (u @ v)
        p = p + alpha * u
        r = r - alpha * v
        it += 1
        hist.append(np.linalg.norm(r) / s_norm)
        if hist[-1] <= eps:
            break
        z = precond(r)
        d_new = r @ z
        beta = d_new / d
        d = d_new
        u = z + beta * u
    return p, it, hist


def pcg_blocks(blocks, rhs, preconds, eps, max_iter, scalars="global", strategy="sync"):
    """Table 1 on the joint system of Eq 3.7 kept as a list of blocks, with the variants of
    Sec 3.3: scalars "global" (one alpha, beta over all blocks: CG on A_G) or "per_cond"
    (one recurrence per block); strategy "sync" (stop when ||r_G|| / ||S_G|| <= eps, Eq 3.9)
    or "async" (a block stops when ||r_k|| / ||S_k|| <= eps, Eq 3.10, and is frozen; the
    global scalars then run over the remaining blocks).
    Returns (list of p_k, iterations, history of ||r_G|| / ||S_G||)."""
    K = len(blocks)
    A = [sp.csr_matrix(b) for b in blocks]
    S = [np.asarray(s, dtype=float) for s in rhs]
    p = [np.zeros_like(s) for s in S]
    r = [s.copy() for s in S]
    s_norm2 = [s @ s for s in S]
    z = [preconds[k](r[k]) for k in range(K)]
    u = [zk.copy() for zk in z]
    d = [r[k] @ z[k] for k in range(K)]

    def rel_all():
        return np.sqrt(sum(rk @ rk for rk in r) / sum(s_norm2))

    def rel_k(k):
        return np.sqrt((r[k] @ r[k]) / s_norm2[k])

    def active_set():
        if strategy == "sync":
            return list(range(K))
        return [k for k in range(K) if rel_k(k) > eps]

    hist = [rel_all()]
    it = 0
    act = active_set()
    done = (rel_all() <= eps) if strategy == "sync" else not act
    while not done and it < max_iter:
        v = {k: A[k] @ u[k] for k in act}
        uv = {k: u[k] @ v[k] for k in act}
        if scalars == "global":
            alpha = {k: sum(d[m] for m in act) / sum(uv[m] for m in act) for k in act}
        else:
            alpha = {k: d[k] / uv[k] for k in act}
        for k in act:
            p[k] = p[k] + alpha[k] * u[k]
            r[k] = r[k] - alpha[k] * v[k]
        it += 1
        hist.append(rel_all())
        new_act = active_set()
        done = (hist[-1] <= eps) if strategy == "sync" else not new_act
        if done:
            break
        for k in new_act:
            z[k] = preconds[k](r[k])
        d_new = {k: r[k] @ z[k] for k in new_act}
        if scalars == "global":
            beta = {k: sum(d_new[m] for m in new_act) / sum(d[m] for m in new_act) for k in new_act}
        else:
            beta = {k: d_new[k] / d[k] for k in new_act}
        for k in new_act:
            d[k] = d_new[k]
            u[k] = z[k] + beta[k] * u[k]
        act = new_act
    return p, it, hist
