"""Pins of the oracle's sparse approximation of A11 and its ILU(0)
(oracle/ilu.py) against what the definitions fix:
  * ILU(0) with a full pattern is exact LU without pivoting (L U = A);
  * on any pattern, (L U)_ij = A_ij at every pattern position (the defining
    property of ILU(0)), while an update outside the pattern would break it;
  * a tridiagonal matrix has no fill: ILU(0) is its exact LU and the
    triangular solves solve A z = r;
  * a block-diagonal pattern gives the exact block inverse;
  * the colouring is proper and greedy (no lower colour was free);
  * the selection keeps exactly the entries whose key reaches the k-th
    largest, at least k of them, all keys kept >= all dropped;
  * the near field of the 256 x 256 fault (leaf 64, eta 2) has the 8,836
    inadmissible leaf pairs of the partition (a count derived by hand from
    the admissibility rule) and is symmetric.
"""
import numpy as np
import pytest

import oracle
from oracle import ilu
from workloads import rect_grid, square_fault

YOUNG, NU = 30e9, 0.25


def _dd_matrix(n, density, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    A += np.diag(np.abs(A).sum(axis=1) + 1.0)
    return A


def test_full_pattern_is_exact_lu():
    A = _dd_matrix(30, 1.0, 1)
    order = np.arange(30)
    F = ilu.ilu0(A, np.ones_like(A, dtype=bool), order)
    L = np.tril(F, -1) + np.eye(30)
    U = np.triu(F)
    assert np.abs(L @ U - A).max() <= 1e-12 * np.abs(A).max()


def test_lu_product_matches_a_on_the_pattern():
    n = 45
    A = _dd_matrix(n, 0.25, 2)
    pat = (A != 0) | np.eye(n, dtype=bool)
    rng = np.random.default_rng(3)
    order = rng.permutation(n)
    F = ilu.ilu0(A, pat, order)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    LU = L @ U
    Ap, Sp = A[np.ix_(order, order)], pat[np.ix_(order, order)]
    assert np.abs(LU[Sp] - Ap[Sp]).max() <= 1e-12 * np.abs(A).max()
    # there is fill outside the pattern (this is an incomplete factorisation)
    assert np.abs(LU[~Sp]).max() > 1e-3
    # a factorisation that also updated positions outside the pattern is
    # exact LU, which differs from ILU(0) on the pattern
    Fx = ilu.ilu0(A, np.ones_like(pat), order)
    assert np.abs(np.where(Sp, Fx, 0) - F).max() > 1e-6


def test_tridiagonal_has_no_fill_and_solves_exactly():
    n = 40
    rng = np.random.default_rng(4)
    A = np.diag(rng.random(n) + 3.0) + np.diag(rng.standard_normal(n - 1), 1) + np.diag(rng.standard_normal(n - 1), -1)
    pat = A != 0
    order = np.arange(n)
    F = ilu.ilu0(A, pat, order)
    r = rng.standard_normal((2, n))
    z = ilu.ilu0_apply(F, order, r)
    assert np.abs(z @ A.T - r).max() <= 1e-12 * np.abs(r).max()


def test_block_diagonal_pattern_gives_the_block_inverse():
    n = 10
    rng = np.random.default_rng(5)
    blocks = [rng.standard_normal((3, 3)) + 4 * np.eye(3) for _ in range(n)]
    A = np.zeros((3 * n, 3 * n))
    for e, b in enumerate(blocks):
        A[3 * e:3 * e + 3, 3 * e:3 * e + 3] = b
    E = np.zeros_like(A)
    keep = np.zeros_like(A, dtype=bool)
    At, pat = ilu.tilde_a11(E, keep, -np.array(blocks), None)
    assert np.array_equal(At, A)
    col = ilu.greedy_colouring(pat)
    assert np.all(col == 0)
    order = ilu.dof_order(col)
    F = ilu.ilu0(At, pat, order)
    r = rng.standard_normal((3, 3 * n))
    z = ilu.ilu0_apply(F, order, r)
    assert np.abs(z - np.linalg.solve(A, r.T).T).max() <= 1e-13 * np.abs(z).max()


def test_colouring_is_proper_and_greedy():
    rng = np.random.default_rng(6)
    n = 60
    G = rng.random((n, n)) < 0.08
    pat = np.kron(G, np.ones((3, 3), bool)) | np.eye(3 * n, dtype=bool)
    col = ilu.greedy_colouring(pat)
    S = G | G.T
    np.fill_diagonal(S, False)
    assert not np.any(S & (col[:, None] == col[None, :]))
    for e in range(n):
        lower = set(col[np.flatnonzero(S[e, :e])])
        assert all(c in lower for c in range(col[e]))
    order = ilu.dof_order(col)
    assert np.all(np.diff(col[order[::3] // 3]) >= 0)


def test_selection_keeps_the_largest_keys():
    m = rect_grid(9, 7, 1.0, 0.8)
    E = oracle.dense(m, YOUNG, NU)
    near = ilu.near_field_mask(m.ne, ilu.near_field_blocks(m, 16, 2.0))
    for p in (0.01, 0.1, 1.0):
        keep, kth, k = ilu.select_near_field(E, near, p)
        keys = ilu.magnitude_key(E)
        assert keep.sum() >= k and not np.any(keep & ~near)
        assert keys[keep].min() == kth
        dropped = near & ~keep
        if dropped.any():
            assert keys[dropped].max() < kth
    keep, _, _ = ilu.select_near_field(E, near, 1.0)
    assert np.array_equal(keep, near)
    # every self block's diagonal is among the largest entries
    keep, _, _ = ilu.select_near_field(E, near, 0.01)
    assert all(keep[i, i] for i in range(3 * m.ne))


def test_near_field_of_the_primary_fault():
    blocks = ilu.near_field_blocks(square_fault(256), 64, 2.0)
    assert len(blocks) == 8836
    assert all(len(t) == 64 and len(s) == 64 for t, s in blocks)
    pairs = {(int(t.min()), int(s.min())) for t, s in blocks}
    assert all((b, a) in pairs for a, b in pairs)
