"""Pins of the oracle's sampled HBS construction (Section 2.4, Algorithm 1).

* exact recovery: a matrix built with exact HBS structure of rank k on the
  cluster tree (random bases and diagonal blocks at every level) is
  reproduced to rounding from s = 3k + 10 two-sided samples, on the line
  tree of 2D interfaces and the grid tree of 3D ones; a wrong sign, a dropped
  transpose or an exchanged basis in the construction breaks this;
* the transposed product is the transpose of the product (dense, brute force);
* the sampling step (local solves, forward and transposed) against the
  closed-form Poisson transfer block (separation of variables);
* the closed-form 2D Poisson block is compressed to rounding at k = 32
  (every off-diagonal block of it has numerical rank below that);
* too few samples for a node are refused.
"""
import numpy as np
import pytest

from problems import Problem
from oracle import dd, hbs
from tests.test_oracle_pins import dst_transfer


def random_hbs(tree, k, rng):
    """An exactly rank-structured matrix in the oracle's HBS layout."""
    L = tree.depth
    levs = []
    sizes = [b - a for a, b, _ in tree.levels[L]]
    for d in range(L, 0, -1):
        lev, nsz = [], []
        for n in sizes:
            r = min(k, n)
            U = np.linalg.qr(rng.standard_normal((n, r)))[0]
            V = np.linalg.qr(rng.standard_normal((n, r)))[0]
            lev.append((U, V, rng.standard_normal((n, n))))
            nsz.append(r)
        levs.append(lev)
        sizes = [sum(nsz[c] for c in kids) for _, _, kids in tree.levels[d - 1]]
    return {"levels": levs, "root": rng.standard_normal((sizes[0], sizes[0])), "tree": tree}


def dense_by_levels(H, N):
    """The same matrix assembled from the telescoping formula directly
    (block-diagonal D, U, V per level; no use of hbs.apply)."""
    tree = H["tree"]
    L = tree.depth
    A = H["root"]
    for i, d in enumerate(range(1, L + 1)):
        lev = H["levels"][L - d]
        Ub = np.zeros((sum(U.shape[0] for U, _, _ in lev), sum(U.shape[1] for U, _, _ in lev)))
        Vb = np.zeros_like(Ub)
        Db = np.zeros((Ub.shape[0], Ub.shape[0]))
        r = c = 0
        for U, V, D in lev:
            Ub[r:r + U.shape[0], c:c + U.shape[1]] = U
            Vb[r:r + V.shape[0], c:c + V.shape[1]] = V
            Db[r:r + D.shape[0], r:r + D.shape[0]] = D
            r += U.shape[0]
            c += U.shape[1]
        A = Db + Ub @ A @ Vb.T
    out = np.empty_like(A)
    p = tree.perm
    out[np.ix_(p, p)] = A
    return out


@pytest.mark.parametrize("M,k,grid", [(300, 12, None), (1000, 20, None), (225, 10, 15),
                                      (961, 16, 31)])
def test_exact_recovery_of_rank_structured_matrix(M, k, grid):
    rng = np.random.default_rng(M + k)
    tree = hbs.kd_tree(M, 2 * k, grid)
    A = dense_by_levels(random_hbs(tree, k, rng), M)
    s = 3 * k + 10
    Om, Ps = rng.standard_normal((M, s)), rng.standard_normal((M, s))
    H = hbs.compress(Om, Ps, A @ Om, A.T @ Ps, k, tree)
    A2 = hbs.to_dense(H, M)
    assert np.abs(A2 - A).max() <= 1e-12 * np.abs(A).max()
    x = rng.standard_normal(M)
    assert np.abs(hbs.apply(H, x, transpose=True) - A2.T @ x).max() <= 1e-12 * np.abs(A2).max() * M
    # O(kN) storage, against N^2 dense
    assert hbs.storage(H) < 0.5 * M * M


def test_trees_are_uniform_and_cover():
    for M, leaf, grid in [(2047, 128, None), (16129, 128, 127), (961, 64, 31), (127, 128, None)]:
        t = hbs.kd_tree(M, leaf, grid)
        assert sorted(t.perm.tolist()) == list(range(M))
        for d, lev in enumerate(t.levels):
            assert lev[0][0] == 0 and lev[-1][1] == M
            assert all(lev[i][1] == lev[i + 1][0] for i in range(len(lev) - 1))
            assert len(lev) == 2 ** d
        assert max(b - a for a, b, _ in t.levels[-1]) <= leaf


@pytest.mark.parametrize("dim,n,ns", [(2, 63, 4), (3, 15, 4)])
def test_sampling_step_matches_closed_form(dim, n, ns):
    p = Problem(dim, n, ns)
    o = dd.DDOracle(p)
    S = dst_transfer(n, p.m, dim)  # every block of the Poisson problem
    X = np.random.default_rng(3).standard_normal((p.M, 9))
    for j, jp in ((1, 2), (2, 1), (2, 3)):
        assert np.abs(o.sample(j, jp, X) - S @ X).max() <= 1e-12
        assert np.abs(o.sample(j, jp, X, transpose=True) - S.T @ X).max() <= 1e-12


def test_poisson_block_compressed_to_rounding():
    n, m, k = 255, 16, 32
    S = dst_transfer(n, m, 2)
    rng = np.random.default_rng(7)
    s = 3 * k + 10
    Om, Ps = rng.standard_normal((n, s)), rng.standard_normal((n, s))
    H = hbs.compress(Om, Ps, S @ Om, S.T @ Ps, k, hbs.kd_tree(n, 2 * k))
    err = np.linalg.norm(hbs.to_dense(H, n) - S, 2) / np.linalg.norm(S, 2)
    assert err <= 1e-12


def test_too_few_samples_refused():
    rng = np.random.default_rng(1)
    M, k = 200, 10
    tree = hbs.kd_tree(M, 50)  # leaves of 50 > s - k = 30
    A = rng.standard_normal((M, M))
    Om, Ps = rng.standard_normal((M, 40)), rng.standard_normal((M, 40))
    with pytest.raises(ValueError):
        hbs.compress(Om, Ps, A @ Om, A.T @ Ps, k, tree)
