"""Discrete adjoint of the FD solve w.r.t. the cellwise coefficient (oracle).

The paper has no adjoint; this is the plain definition.  For the residual
``F(u, kappa) = A(kappa) u + A_IB(kappa) g - f = 0`` and a loss ``L(u)``:

    A^T lambda = dL/du,        dL/dkappa = - lambda^T dF/dkappa .

With the edge coefficient equal to the mean of the ``2^(d-1)`` cells sharing
the edge, only the diffusion part depends on kappa, and

    dL/dkappa_c = - 1/(2^(d-1) h^2) * sum_{edges (p,q) of cell c}
                    (lambda_p - lambda_q) (u_p - u_q)

with ``lambda = 0`` and ``u = g`` on the boundary nodes.  The transposed
system is solved with a sparse LU (``trans='T'``).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse.linalg as spla

from . import fd


def sensor_loss(u, sensors, data):
    r = u.ravel()[sensors] - data
    return 0.5 * float(r @ r)


def sensor_loss_grad(u, sensors, data, N):
    gbar = np.zeros(N)
    np.add.at(gbar, sensors, u.ravel()[sensors] - data)
    return gbar


def solve_transposed(prob, gbar):
    A, _ = fd.assemble(prob)
    return spla.splu(A.tocsc()).solve(np.asarray(gbar, dtype=np.float64).ravel(), trans="T")


def cell_gradient(prob, u, lam):
    """dL/dkappa on the (n+1)^d cells from the state ``u`` and adjoint ``lam``."""
    d, n, h = prob.dim, prob.n, prob.h
    U = np.zeros((n + 2,) * d) if prob.g is None else np.array(prob.g, dtype=np.float64)
    inner = tuple(slice(1, n + 1) for _ in range(d))
    U[inner] = np.asarray(u).reshape((n,) * d)
    L = np.zeros((n + 2,) * d)
    L[inner] = np.asarray(lam).reshape((n,) * d)
    grad = np.zeros((n + 1,) * d)
    for axis in range(d):
        others = [a for a in range(d) if a != axis]
        for shifts in itertools.product((0, 1), repeat=len(others)):
            # edge from node (c + off) to (c + off + e_axis), off_axis = 0
            lo = [slice(0, n + 1)] * d
            hi = [slice(0, n + 1)] * d
            for a, s in zip(others, shifts):
                lo[a] = slice(s, s + n + 1)
                hi[a] = slice(s, s + n + 1)
            hi[axis] = slice(1, n + 2)
            lo, hi = tuple(lo), tuple(hi)
            grad += (L[lo] - L[hi]) * (U[lo] - U[hi])
    return -grad / (2 ** (d - 1) * h * h)


def gradient(prob, u, gbar):
    lam = solve_transposed(prob, gbar)
    return cell_gradient(prob, u, lam), lam
