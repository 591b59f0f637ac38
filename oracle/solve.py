"""Linear solvers for K phi = g.

Oracle (test infrastructure): see the package docstring.

Paper, Sec. 3.3 and Sec. 5: the dense non-symmetric system may be solved
directly (LU / Gaussian elimination) or by GMRES; the examples use GMRES with
relative tolerance 1e-8.  Reading: x0 = 0, no restart, modified Gram-Schmidt
Arnoldi with Givens rotations, stop when ||g - K phi|| <= tol ||g||.  With a
preconditioner M ~ K^{-1} it is applied on the right, so the monitored residual
is the unpreconditioned one.
"""

import numpy as np
import scipy.linalg


def lu_solve(K, g):
    return scipy.linalg.lu_solve(scipy.linalg.lu_factor(K), g)


def gmres(apply_K, g, tol=1e-8, max_iter=None, apply_M=None):
    """Returns (phi, iterations, residual history)."""
    g = np.asarray(g, dtype=complex)
    n = g.size
    m = n if max_iter is None else max_iter
    beta = np.linalg.norm(g)
    if beta == 0.0:
        return np.zeros(n, dtype=complex), 0, [0.0]
    M = (lambda v: v) if apply_M is None else apply_M
    V = np.zeros((m + 1, n), dtype=complex)
    H = np.zeros((m + 1, m), dtype=complex)
    cs = np.zeros(m, dtype=complex)
    sn = np.zeros(m, dtype=complex)
    e1 = np.zeros(m + 1, dtype=complex)
    e1[0] = beta
    V[0] = g / beta
    hist = [1.0]
    j_done = 0
    for j in range(m):
        w = apply_K(M(V[j]))
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] != 0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            a, b = H[i, j], H[i + 1, j]
            H[i, j] = np.conj(cs[i]) * a + np.conj(sn[i]) * b
            H[i + 1, j] = -sn[i] * a + cs[i] * b
        a, b = H[j, j], H[j + 1, j]
        r = np.hypot(abs(a), abs(b))
        cs[j] = a / r if r else 1.0
        sn[j] = b / r if r else 0.0
        H[j, j] = np.conj(cs[j]) * a + np.conj(sn[j]) * b
        H[j + 1, j] = 0.0
        e1[j + 1] = -sn[j] * e1[j]
        e1[j] = np.conj(cs[j]) * e1[j]
        j_done = j + 1
        hist.append(abs(e1[j + 1]) / beta)
        if hist[-1] <= tol or H[j, j] == 0:
            break
    y = scipy.linalg.solve_triangular(H[:j_done, :j_done], e1[:j_done])
    phi = M(V[:j_done].T @ y)
    return phi, j_done, hist
