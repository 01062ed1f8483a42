"""Overlapping solution-transfer DD, written out plainly (oracle; tests only).

Follows Section 2 of the paper:

* double slab ``Psi_j`` (j = 1..N_ds) = the node planes strictly between
  interfaces ``Gamma_{j-1}`` and ``Gamma_{j+1}``; its central interface
  ``C_j`` is ``Gamma_j`` (Section 2.5, local / global assembly);
* solution-transfer block, eq. ``defS``:
      S_{j,j'} = - R_{C_j} A_j(I_j,I_j)^{-1} A_j(I_j, J_{j,j'}),
  computed here exactly as written, with a sparse LU of ``A_j(I_j,I_j)``
  taken from the global FD matrix and dense right-hand sides;
* equivalent load, eq. ``equilib1``: the trace on ``Gamma_j`` of the local
  solve with the global load (and physical boundary data) and zero data on
  ``Gamma_{j+-1}``;
* equilibrium system, eq. ``modelS``:
      u_j - S_{j,j-1} u_{j-1} - S_{j,j+1} u_{j+1} = hhat_j ;
  interfaces next to the physical boundary have a single block;
* volume recovery: each single slab solved with the interface traces as
  Dirichlet data.

Everything is float64 and deliberately unblocked.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fd


def plane_nodes(prob, i):
    """Flat interior-node indices of node plane ``i`` (1-based along x)."""
    M = prob.M
    return np.arange((i - 1) * M, i * M)


def planes_nodes(prob, i0, i1):
    """Nodes of planes ``i0..i1`` inclusive."""
    M = prob.M
    return np.arange((i0 - 1) * M, i1 * M)


class DDOracle:
    """Holds the global FD matrix and evaluates the method's objects."""

    def __init__(self, prob):
        self.prob = prob
        self.Ab = fd.assemble(prob)
        self.A = self.Ab[0].tocsr()
        self._lu = {}

    # -- local problems ----------------------------------------------------
    def double_slab(self, j):
        """Interior node set I_j of Psi_j and the local offset of C_j."""
        p = self.prob
        I = planes_nodes(p, (j - 1) * p.m + 1, (j + 1) * p.m - 1)
        centre = np.arange((p.m - 1) * p.M, p.m * p.M)
        return I, centre

    def _local_lu(self, j):
        if j not in self._lu:
            I, _ = self.double_slab(j)
            self._lu[j] = spla.splu(self.A[I][:, I].tocsc())
        return self._lu[j]

    def transfer_block(self, j, jp):
        """S_{j,jp} for jp = j-1 or j+1 (1-based interfaces), eq. defS."""
        p = self.prob
        if abs(jp - j) != 1 or not (1 <= jp <= p.n_ds):
            raise ValueError("jp must be an interior neighbour interface")
        I, centre = self.double_slab(j)
        J = plane_nodes(p, jp * p.m)
        AIJ = self.A[I][:, J].toarray()
        X = self._local_lu(j).solve(AIJ)
        return -X[centre, :]

    def transfer_columns(self, j, jp, cols, rtol=1e-14):
        """Columns ``cols`` of S_{j,jp} (eq. defS) for symmetric positive
        definite operators, each by conjugate gradients (diagonal
        preconditioner) on the double slab instead of a sparse LU: the route
        for the 3D workload, whose double-slab LU takes minutes."""
        p = self.prob
        if abs(jp - j) != 1 or not (1 <= jp <= p.n_ds):
            raise ValueError("jp must be an interior neighbour interface")
        I, centre = self.double_slab(j)
        J = plane_nodes(p, jp * p.m)
        AII = self.A[I][:, I].tocsr()
        AIJ = self.A[I][:, J].tocsc()
        d = AII.diagonal()
        precond = spla.LinearOperator(AII.shape, matvec=lambda x: x / d)
        out = np.zeros((p.M, len(cols)))
        for k, c in enumerate(cols):
            rhs = AIJ[:, int(c)].toarray().ravel()
            x, info = spla.cg(AII, rhs, rtol=rtol, atol=0.0, maxiter=20000, M=precond)
            if info != 0:
                raise RuntimeError("CG did not converge on the double slab")
            out[:, k] = -x[centre]
        return out

    def sample(self, j, jp, X, transpose=False):
        """Algorithm 1's sampling step through the local factorisation:
        Y = S_{j,jp} X = -R_{C_j} A_j(I,I)^{-1} A_j(I,J_{j,jp}) X, or with
        transpose Z = S_{j,jp}^T X = -A_j(I,J_{j,jp})^T A_j(I,I)^{-T} R_{C_j}^T X
        (the transposed local solve of the same LU), never forming S."""
        p = self.prob
        if abs(jp - j) != 1 or not (1 <= jp <= p.n_ds):
            raise ValueError("jp must be an interior neighbour interface")
        I, centre = self.double_slab(j)
        J = plane_nodes(p, jp * p.m)
        AIJ = self.A[I][:, J]
        lu = self._local_lu(j)
        X = np.asarray(X, dtype=np.float64)
        if not transpose:
            return -lu.solve(np.asarray(AIJ @ X))[centre]
        R = np.zeros((len(I), X.shape[1]))
        R[centre] = X
        return -np.asarray(AIJ.T @ lu.solve(R, trans="T"))

    def all_blocks(self):
        """Dict {(j, jp): S_{j,jp}} over all interior neighbour pairs."""
        out = {}
        for j in range(1, self.prob.n_ds + 1):
            for jp in (j - 1, j + 1):
                if 1 <= jp <= self.prob.n_ds:
                    out[(j, jp)] = self.transfer_block(j, jp)
        return out

    def rhs(self, f=None, g=None):
        return fd.rhs(self.prob, self.Ab, f=f, g=g)

    def loads(self, b):
        """Equivalent loads hhat_j (eq. equilib1) for the interior RHS ``b``."""
        p = self.prob
        out = np.zeros((p.n_ds, p.M))
        for j in range(1, p.n_ds + 1):
            I, centre = self.double_slab(j)
            out[j - 1] = self._local_lu(j).solve(b[I])[centre]
        return out

    # -- interface system --------------------------------------------------
    def assemble_S(self, blocks=None):
        """Dense equilibrium matrix S = I - K (eq. modelS), N_ds*M square."""
        p = self.prob
        blocks = self.all_blocks() if blocks is None else blocks
        M = p.M
        S = np.eye(p.n_ds * M)
        for (j, jp), B in blocks.items():
            S[(j - 1) * M:j * M, (jp - 1) * M:jp * M] -= B
        return S

    def interface_solve(self, hhat, S=None):
        """Dense LU solve of the equilibrium system."""
        S = self.assemble_S() if S is None else S
        return np.linalg.solve(S, hhat.ravel()).reshape(hhat.shape)

    def reconstruct(self, b, u_gamma):
        """Interior solution from interface traces (single-slab solves)."""
        p = self.prob
        u = np.zeros(p.N)
        for j in range(1, p.n_ds + 1):
            u[plane_nodes(p, j * p.m)] = u_gamma[j - 1]
        for s in range(p.n_slabs):
            lo, hi = s * p.m + 1, (s + 1) * p.m - 1
            I = planes_nodes(p, lo, hi)
            r = b[I].copy()
            for j in (s, s + 1):
                if 1 <= j <= p.n_ds:
                    J = plane_nodes(p, j * p.m)
                    r -= self.A[I][:, J] @ u_gamma[j - 1]
            u[I] = spla.spsolve(self.A[I][:, I].tocsc(), r)
        return u

    def solve(self, b=None):
        """Full DD pipeline: blocks, loads, interface solve, volume."""
        b = self.rhs() if b is None else b
        hh = self.loads(b)
        ug = self.interface_solve(hh)
        return ug, self.reconstruct(b, ug)

    def interface_trace(self, u):
        """Restriction of a volume vector to the interfaces, (N_ds, M)."""
        p = self.prob
        return np.stack([u[plane_nodes(p, j * p.m)] for j in range(1, p.n_ds + 1)])

    # -- Schur form (Section 2.1, eq. efewin) -- used only as a check -------
    def schur_T(self):
        """Dense interface Schur complement T = A_JJ - A_JI A_II^{-1} A_IJ."""
        p = self.prob
        J = np.concatenate([plane_nodes(p, j * p.m) for j in range(1, p.n_ds + 1)])
        mask = np.ones(p.N, bool)
        mask[J] = False
        I = np.nonzero(mask)[0]
        A = self.A.toarray()
        AII = A[np.ix_(I, I)]
        T = A[np.ix_(J, J)] - A[np.ix_(J, I)] @ sla.solve(AII, A[np.ix_(I, J)])
        return T
