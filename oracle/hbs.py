"""HBS compression of a transfer block from two-sided random samples (oracle;
test infrastructure only).

Section 2.4 and Algorithm 1 of the paper: a block S_{j,j'} (N x N) is
compressed into the Hierarchically Block Separable form with rank k on a
cluster tree shared by rows and columns, from s = alpha k + q samples
    Y = S Omega,   Z = S^T Psi,     Omega, Psi ~ N(0,1)^{N x s},
alpha = 3, q = 10; memory and matrix-vector cost are O(kN).  The paper takes
the compression from its reference [fastHBS] without detail; this oracle
writes out the single-pass black-box construction of the public literature
(Levitt and Martinsson, randomized compression of HBS matrices from
Y = A Omega and Z = A^* Psi alone), level by level from the leaves:

for every node tau of the current level, with its rows Om, Ps, Y, Z of the
current (reduced) sketches (n_tau x s; at the leaves the rows I_tau of the
original ones):
  1. Yh = Y Om^+ and Zh = Z Ps^+ (right pseudo-inverses; Om has full row rank
     since n_tau < s).  Yh is A(tau, tau) up to the part of the other columns
     that Om's row space sees;
  2. W_Y = Y - Yh Om = Y (I - Om^+ Om) removes the diagonal block: its
     columns are random combinations of the columns of A(tau, tau^c), whose
     range is what U_tau must span (likewise W_Z for V_tau);
  3. U_tau, V_tau: orthonormal bases of the leading k columns of the
     Householder QR with column pivoting of W_Y and W_Z (k = rank, at most
     n_tau);
  4. D_tau = A(tau,tau) - U U^T A(tau,tau) V V^T, from the sketches:
     D = Yh + U U^T (Zh^T - Yh) - U (U^T Zh^T V) V^T;
  5. reduced sketches of the next level: Om' = V^T Om, Ps' = U^T Ps,
     Y' = U^T (Y - D Om), Z' = V^T (Z - D^T Ps); a parent's rows are its
     children's stacked.
At the root, D_root = Y Om^+ (the remaining 2k x 2k block).  The HBS form
is then A ~ D^(L) + U^(L) (D^(L-1) + U^(L-1) ( ... D^(0) ... ) V^(L-1)^T) V^(L)^T
with block-diagonal D^(l), U^(l), V^(l) per level.  When every block
A(tau, tau^c) has rank <= k the construction is exact (up to rounding).

Cluster trees: ``kd_tree`` splits every node at every level (so all leaves
share one depth) until no node holds more than ``leaf`` points: index
ranges at the midpoint for 2D interfaces (lines), and for 3D interfaces the
n x n grid rectangles alternately along y and z (the longer side first),
giving a permutation to cluster order.

Everything is float64; the sample generator is the caller's.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class Tree:
    """levels[l] = list of nodes at depth l (0 = root); a node is
    (lo, hi, children) over the cluster order; perm[c] = natural index of
    cluster position c."""

    def __init__(self, levels, perm):
        self.levels = levels
        self.perm = np.asarray(perm, dtype=np.int64)

    @property
    def depth(self):
        return len(self.levels) - 1


def kd_tree(M, leaf, grid_n=None):
    """Uniform-depth binary cluster tree.  grid_n=None: an index line of M
    points split at the midpoint (lo + ceil((hi - lo) / 2)).  grid_n=n
    (M = n^2, natural index y n + z): rectangles split at the midpoint of
    their longer side (y on ties)."""
    if grid_n is None:
        levels = [[(0, M)]]
        while max(b - a for a, b in levels[-1]) > leaf:
            nxt = []
            for a, b in levels[-1]:
                mid = a + (b - a + 1) // 2
                nxt += [(a, mid), (mid, b)]
            levels.append(nxt)
        depth = len(levels) - 1
        out = [[(a, b, [2 * i, 2 * i + 1] if d < depth else []) for i, (a, b) in enumerate(lev)]
               for d, lev in enumerate(levels)]
        return Tree(out, np.arange(M))
    n = grid_n
    assert M == n * n
    # rectangles (y0, y1, z0, z1) per level
    rl = [[(0, n, 0, n)]]
    while max((y1 - y0) * (z1 - z0) for y0, y1, z0, z1 in rl[-1]) > leaf:
        nxt = []
        for y0, y1, z0, z1 in rl[-1]:
            if (y1 - y0) >= (z1 - z0):
                ym = y0 + (y1 - y0 + 1) // 2
                nxt += [(y0, ym, z0, z1), (ym, y1, z0, z1)]
            else:
                zm = z0 + (z1 - z0 + 1) // 2
                nxt += [(y0, y1, z0, zm), (y0, y1, zm, z1)]
        rl.append(nxt)
    depth = len(rl) - 1
    perm = []
    for y0, y1, z0, z1 in rl[-1]:
        for y in range(y0, y1):
            for z in range(z0, z1):
                perm.append(y * n + z)
    # ranges: leaves in order; a parent spans its two children
    counts = [[(y1 - y0) * (z1 - z0) for y0, y1, z0, z1 in lev] for lev in rl]
    levels = []
    for d in range(depth + 1):
        starts = np.concatenate([[0], np.cumsum(counts[d])])
        levels.append([(int(starts[i]), int(starts[i + 1]),
                        [2 * i, 2 * i + 1] if d < depth else []) for i in range(len(rl[d]))])
    return Tree(levels, perm)


def cpqr_basis(W, k):
    """Orthonormal basis (n x k) of the first k columns chosen by Householder
    QR with column pivoting of W (LAPACK geqp3)."""
    n = W.shape[0]
    k = min(k, n, W.shape[1])
    Q, _, _ = sla.qr(W, mode="economic", pivoting=True)
    return Q[:, :k]


def right_pinv_apply(X, Om):
    """X Om^+ with Om^+ = Om^T (Om Om^T)^{-1} (Om: n x s, full row rank)."""
    G = Om @ Om.T
    return sla.solve(G, (X @ Om.T).T, assume_a="pos").T


def compress(Omega, Psi, Y, Z, k, tree):
    """HBS form of A from Y = A Omega, Z = A^T Psi (rows in natural order).
    Returns a dict with per-level lists of (U, V, D) (leaf level first:
    'levels'[0] is the leaf level) and 'root' (D at the root), plus the tree."""
    perm = tree.perm
    Om = [Omega[perm][a:b] for a, b, _ in tree.levels[-1]]
    Ps = [Psi[perm][a:b] for a, b, _ in tree.levels[-1]]
    Ys = [Y[perm][a:b] for a, b, _ in tree.levels[-1]]
    Zs = [Z[perm][a:b] for a, b, _ in tree.levels[-1]]
    out = []
    for d in range(tree.depth, 0, -1):
        lev = []
        nOm, nPs, nY, nZ = [], [], [], []
        for t in range(len(tree.levels[d])):
            om, ps, y, z = Om[t], Ps[t], Ys[t], Zs[t]
            n, s = om.shape
            if n + min(k, n) > s:
                raise ValueError(f"{s} samples cannot separate a node of {n} points from a "
                                 f"rank-{min(k, n)} far field (need s >= n + k)")
            Yh = right_pinv_apply(y, om)
            Zh = right_pinv_apply(z, ps)
            U = cpqr_basis(y - Yh @ om, k)
            V = cpqr_basis(z - Zh @ ps, k)
            D = Yh + U @ (U.T @ (Zh.T - Yh)) - U @ ((U.T @ Zh.T @ V) @ V.T)
            lev.append((U, V, D))
            nOm.append(V.T @ om)
            nPs.append(U.T @ ps)
            nY.append(U.T @ (y - D @ om))
            nZ.append(V.T @ (z - D.T @ ps))
        out.append(lev)
        parents = tree.levels[d - 1]
        Om = [np.vstack([nOm[c] for c in kids]) for _, _, kids in parents]
        Ps = [np.vstack([nPs[c] for c in kids]) for _, _, kids in parents]
        Ys = [np.vstack([nY[c] for c in kids]) for _, _, kids in parents]
        Zs = [np.vstack([nZ[c] for c in kids]) for _, _, kids in parents]
    root = right_pinv_apply(Ys[0], Om[0])
    return {"levels": out, "root": root, "tree": tree}


def apply(H, x, transpose=False):
    """y = A_H x (or A_H^T x) by the upward / downward passes of the HBS form."""
    tree = H["tree"]
    perm = tree.perm
    xc = np.asarray(x, dtype=np.float64)[perm]
    levs = H["levels"]  # leaf level first
    L = tree.depth
    if L == 0:
        Dr = H["root"].T if transpose else H["root"]
        y = np.empty_like(xc)
        y[perm] = Dr @ xc
        return y
    # upward: xh[d][t] for the nodes of depth d (d = L .. 1)
    xh = {}
    cur = [xc[a:b] for a, b, _ in tree.levels[L]]
    for i, d in enumerate(range(L, 0, -1)):
        U_or_V = [(V if not transpose else U) for U, V, _ in levs[i]]
        xh[d] = [B.T @ v for B, v in zip(U_or_V, cur)]
        cur = [np.concatenate([xh[d][c] for c in kids]) for _, _, kids in tree.levels[d - 1]]
    # downward
    Dr = H["root"].T if transpose else H["root"]
    yr = Dr @ cur[0]
    # split the root's output to its children (depth 1)
    yh = {}
    sizes = [v.size for v in xh[1]]
    yh[1] = np.split(yr, np.cumsum(sizes)[:-1])
    for i, d in enumerate(range(1, L)):
        lev = levs[L - d]
        nxt = []
        for t, (a, b, kids) in enumerate(tree.levels[d]):
            U, V, D = lev[t]
            B = V if transpose else U
            Dd = D.T if transpose else D
            xin = np.concatenate([xh[d + 1][c] for c in kids])
            v = B @ yh[d][t] + Dd @ xin
            parts = np.split(v, np.cumsum([xh[d + 1][c].size for c in kids])[:-1])
            nxt += parts
        yh[d + 1] = nxt
    yc = np.empty_like(xc)
    for t, (a, b, _) in enumerate(tree.levels[L]):
        U, V, D = levs[0][t]
        B = V if transpose else U
        Dd = D.T if transpose else D
        yc[a:b] = B @ yh[L][t] + Dd @ xc[a:b]
    y = np.empty_like(yc)
    y[perm] = yc
    return y


def to_dense(H, N):
    """The dense matrix of an HBS form (column by column: tests only)."""
    A = np.zeros((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = apply(H, e)
        e[j] = 0.0
    return A


def storage(H):
    """Number of stored entries (U, V, D of every node and the root)."""
    n = H["root"].size
    for lev in H["levels"]:
        for U, V, D in lev:
            n += U.size + V.size + D.size
    return n
