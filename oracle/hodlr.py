"""Weak-admissibility hierarchical low-rank reference (oracle; tests only).

Section 2.4: a dense transfer block is split along a cluster tree shared by
source and target interface; every interaction between two distinct children
of a tree node is stored at low rank, the leaf diagonal blocks stay dense
(weak admissibility, the paper's Figure on admissibility: only the closest
cluster pair is dense).  The paper compresses with HBS; this oracle uses the
plain HODLR form of the same partition, with the optimal rank of each
admissible block from a truncated SVD (Eckart-Young):
keep singular values ``sigma_i > tol * ||S||_2``.

Cluster trees:
* ``binary_tree(M, leaf)`` -- index ranges split at the midpoint (2D
  interfaces are lines);
* ``quad_tree(n, leaf)`` -- the n x n interface grid split into four
  quadrants at the midpoints (3D interfaces are planes); clusters are lists
  of flat (y, z) C-order indices.
"""
from __future__ import annotations

import numpy as np


class Node:
    def __init__(self, idx, children=()):
        self.idx = np.asarray(idx, dtype=np.int64)
        self.children = list(children)


def binary_tree(M, leaf):
    def build(lo, hi):
        if hi - lo <= leaf:
            return Node(np.arange(lo, hi))
        mid = lo + (hi - lo + 1) // 2
        return Node(np.arange(lo, hi), [build(lo, mid), build(mid, hi)])
    return build(0, M)


def quad_tree(n, leaf):
    def build(y0, y1, z0, z1):
        yy, zz = np.meshgrid(np.arange(y0, y1), np.arange(z0, z1), indexing="ij")
        idx = (yy * n + zz).ravel()
        if idx.size <= leaf or (y1 - y0 < 2 and z1 - z0 < 2):
            return Node(idx)
        ym = y0 + (y1 - y0 + 1) // 2
        zm = z0 + (z1 - z0 + 1) // 2
        kids = [build(a, b, c, d) for (a, b) in ((y0, ym), (ym, y1))
                for (c, d) in ((z0, zm), (zm, z1)) if b > a and d > c]
        return Node(idx, kids)
    return build(0, n, 0, n)


def blocks(tree):
    """Yield ('lr', rows, cols) for admissible pairs and ('dense', rows, rows)."""
    stack = [tree]
    while stack:
        nd = stack.pop()
        if not nd.children:
            yield ("dense", nd.idx, nd.idx)
            continue
        for a in nd.children:
            for b in nd.children:
                if a is not b:
                    yield ("lr", a.idx, b.idx)
        stack.extend(nd.children)


def compress(S, tree, tol):
    """Optimal-rank HODLR of S: list of (kind, rows, cols, data)."""
    norm2 = np.linalg.norm(S, 2)
    out = []
    for kind, r, c in blocks(tree):
        B = S[np.ix_(r, c)]
        if kind == "dense":
            out.append((kind, r, c, B.copy()))
            continue
        U, s, Vt = np.linalg.svd(B, full_matrices=False)
        k = int(np.sum(s > tol * norm2))
        out.append(("lr", r, c, (U[:, :k] * s[:k], Vt[:k])))
    return out


def ranks(H):
    return [d[0].shape[1] for kind, _, _, d in H if kind == "lr"]


def apply(H, x, M):
    y = np.zeros(M)
    for kind, r, c, d in H:
        if kind == "dense":
            y[r] += d @ x[c]
        else:
            y[r] += d[0] @ (d[1] @ x[c])
    return y


def to_dense(H, M):
    S = np.zeros((M, M))
    for kind, r, c, d in H:
        S[np.ix_(r, c)] = d if kind == "dense" else d[0] @ d[1]
    return S
