"""Plain unrestarted GMRES (oracle; test infrastructure only).

The paper solves the equilibrium system with unrestarted GMRES at a relative
tolerance (Section 5, Section 5.2).  Orthogonalisation, initial guess and norm
are not stated; this oracle takes x0 = 0, the relative 2-norm residual and
modified Gram-Schmidt, with Givens rotations for the small least-squares
problem.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, rhs, tol=1e-8, maxit=500):
    """Return (x, iterations, residual history)."""
    rhs = np.asarray(rhs, dtype=np.float64).ravel()
    beta = np.linalg.norm(rhs)
    if beta == 0.0:
        return np.zeros_like(rhs), 0, [0.0]
    n = rhs.size
    V = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    gvec = np.zeros(maxit + 1)
    gvec[0] = beta
    V[0] = rhs / beta
    hist = [1.0]
    k = 0
    for k in range(maxit):
        w = matvec(V[k])
        for i in range(k + 1):
            H[i, k] = np.dot(V[i], w)
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        for i in range(k):
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        r = np.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / r, H[k + 1, k] / r
        H[k, k] = r
        H[k + 1, k] = 0.0
        gvec[k + 1] = -sn[k] * gvec[k]
        gvec[k] = cs[k] * gvec[k]
        hist.append(abs(gvec[k + 1]) / beta)
        if hist[-1] <= tol:
            k += 1
            break
    else:
        k = maxit
    y = np.linalg.solve(np.triu(H[:k, :k]), gvec[:k])
    return V[:k].T @ y, k, hist
