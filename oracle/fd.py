"""Finite-difference model problem (oracle; test infrastructure only).

Discretisation of ``-div(kappa grad u) + b . grad u + c u = f`` with Dirichlet
data ``g`` (the model problem of eq. ``basic``, discretised with the 5-point /
7-point stencil of Section 2.1 and Section 5.2).  For a variable cellwise
coefficient the paper gives no stencil; the reading used here is: the
coefficient on a grid edge is the mean of the ``2^(d-1)`` cells that share the
edge, and convection uses centred differences.  With ``kappa = 1, b = 0,
c = 0`` this is exactly the textbook Laplacian stencil.

Node ``p`` (interior) gives the row
    (A u)_p = sum_axis sum_{q = p +- e_axis} kappa_pq (u_p - u_q) / h^2
              + sum_axis b_axis (u_{p+e} - u_{p-e}) / (2h) + c_p u_p .
Boundary neighbours carry ``g`` and are moved to the right-hand side.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def edge_coefficient(prob, axis):
    """Coefficient on every edge ``p -> p + e_axis``.

    Returned array has extent ``n+1`` along ``axis`` (edge index ``p_axis`` in
    ``0..n``) and ``n`` along the other axes (node index ``1..n``).  It is the
    mean of the cells ``c`` with ``c_axis = p_axis`` and ``c_b in {p_b-1, p_b}``.
    """
    d, n = prob.dim, prob.n
    shape = tuple(n + 1 if a == axis else n for a in range(d))
    if prob.kappa is None:
        return np.ones(shape)
    kap = np.asarray(prob.kappa, dtype=np.float64)
    acc = np.zeros(shape)
    others = [a for a in range(d) if a != axis]
    for shifts in itertools.product((0, 1), repeat=len(others)):
        sl = [slice(None)] * d
        for a, s in zip(others, shifts):
            # node index p_b = 1..n  ->  cell index p_b - 1 + s  in 0..n
            sl[a] = slice(s, s + n)
        acc += kap[tuple(sl)]
    return acc / (2 ** len(others))


def node_index(n, dim):
    """Flat C-order index of interior nodes, padded with -1 on the boundary."""
    idx = -np.ones((n + 2,) * dim, dtype=np.int64)
    inner = tuple(slice(1, n + 1) for _ in range(dim))
    idx[inner] = np.arange(n ** dim).reshape((n,) * dim)
    return idx


def assemble(prob):
    """Sparse interior matrix ``A`` (CSR, N x N) and the full node-box map.

    Returns ``(A, Bcoef)`` where ``Bcoef`` is a list of (row, box_flat_index,
    value) triples for couplings to boundary nodes, used by :func:`rhs`.
    """
    d, n, h = prob.dim, prob.n, prob.h
    idx = node_index(n, d)
    inner = tuple(slice(1, n + 1) for _ in range(d))
    rows_p = idx[inner].ravel()
    diag = np.zeros(n ** d)
    if prob.c is not None:
        diag += np.asarray(prob.c, dtype=np.float64).ravel()
    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    box_flat = np.arange((n + 2) ** d).reshape((n + 2,) * d)
    for axis in range(d):
        K = edge_coefficient(prob, axis) / (h * h)
        bconv = prob.bvec[axis] / (2.0 * h)
        for sgn in (+1, -1):
            # neighbour q = p + sgn e_axis; edge index is p_axis (sgn=+1) or p_axis-1
            sl_edge = [slice(None)] * d
            sl_edge[axis] = slice(1, n + 1) if sgn > 0 else slice(0, n)
            kq = K[tuple(sl_edge)].ravel()
            diag += kq
            off = -kq + sgn * bconv
            sl_q = list(inner)
            sl_q[axis] = slice(1 + sgn, n + 1 + sgn)
            q_idx = idx[tuple(sl_q)].ravel()
            q_box = box_flat[tuple(sl_q)].ravel()
            inside = q_idx >= 0
            rows.append(rows_p[inside]); cols.append(q_idx[inside]); vals.append(off[inside])
            brow.append(rows_p[~inside]); bcol.append(q_box[~inside]); bval.append(off[~inside])
    rows.append(rows_p); cols.append(rows_p); vals.append(diag)
    N = n ** d
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sum_duplicates()
    return A, (np.concatenate(brow), np.concatenate(bcol), np.concatenate(bval))


def rhs(prob, A_and_b=None, f=None, g=None):
    """Right-hand side ``b = f - A_{I,boundary} g`` on interior nodes (flat)."""
    if A_and_b is None:
        A_and_b = assemble(prob)
    _, (brow, bcol, bval) = A_and_b
    n, d = prob.n, prob.dim
    f = prob.f if f is None else f
    g = prob.g if g is None else g
    b = np.zeros(n ** d) if f is None else np.asarray(f, dtype=np.float64).ravel().copy()
    if g is not None:
        gf = np.asarray(g, dtype=np.float64).ravel()
        np.add.at(b, brow, -bval * gf[bcol])
    return b


def apply(prob, u_interior, g=None):
    """Stencil action on the full node box: returns (A_full u~)_p for interior p,
    with u~ = u on interior nodes and g on the boundary (b = f means residual 0)."""
    A, (brow, bcol, bval) = assemble(prob)
    out = A @ np.asarray(u_interior, dtype=np.float64).ravel()
    g = prob.g if g is None else g
    if g is not None:
        gf = np.asarray(g, dtype=np.float64).ravel()
        np.add.at(out, brow, bval * gf[bcol])
    return out


def solve_global(prob, ordering="COLAMD"):
    """Plain global sparse direct solve of ``A u = b`` (reference solution).
    ``ordering`` is SuperLU's fill-reducing column permutation; it changes
    the cost, not the system (``MMD_AT_PLUS_A`` is the faster one for the
    large 2D grids)."""
    import scipy.sparse.linalg as spla
    Ab = assemble(prob)
    b = rhs(prob, Ab)
    return spla.splu(Ab[0].tocsc(), permc_spec=ordering).solve(b)


def solve_global_cg(prob, rtol=1e-14, maxiter=50000):
    """Global reference by conjugate gradients with the diagonal as
    preconditioner, for symmetric positive definite FD operators (no
    convection, c >= 0): the 3D workload, whose sparse LU is impractical at
    full size.  Stops at ||b - A u||_2 <= rtol ||b||_2."""
    import scipy.sparse.linalg as spla
    Ab = assemble(prob)
    A = Ab[0].tocsr()
    b = rhs(prob, Ab)
    d = A.diagonal()
    precond = spla.LinearOperator(A.shape, matvec=lambda x: x / d)
    u, info = spla.cg(A, b, rtol=rtol, atol=0.0, maxiter=maxiter, M=precond)
    if info != 0:
        raise RuntimeError(f"CG did not reach rtol={rtol} in {maxiter} iterations")
    return u

