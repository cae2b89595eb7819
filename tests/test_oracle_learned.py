"""Pins of the learned-preconditioner oracle (oracle/learned.py).

Each pin checks the oracle against something other than itself:
  * the hand-written gradient against central finite differences of the
    loss (a dropped term, a wrong ReLU mask or a transposed layer fails);
  * the sum over pairs against the dense matrix built block by block
    (swapping element and neighbour fails);
  * block-diagonal systems, where block-Jacobi is the exact inverse, give a
    zero loss with a zero network; the same for systems block-diagonal over
    groups of elements with the group inverse as a dense base;
  * a dense base equal to the 3x3 blocks reproduces the block form, and the
    gradient with a general dense base matches central differences;
  * features of a flat square grid, whose values follow from geometry
    (offset one cell along s1 or s2, unit distance, aligned frames);
  * invariance of the dimensionless features under a rigid motion plus a
    uniform scaling of mesh and stiffness (a feature measured in the wrong
    frame or with the wrong length scale fails).
"""
import numpy as np
import pytest

import oracle
import oracle.learned as OL
import workloads as W


def _random_problem(ne=9, K=4, H=4, ns=3, seed=0):
    rng = np.random.default_rng(seed)
    cent = rng.standard_normal((ne, 3))
    pe, pf = OL.knn_bruteforce(cent, K)
    F = np.zeros((len(pe), 32))
    F[:, :20] = rng.standard_normal((len(pe), 20))
    scale = rng.uniform(0.5, 1.5, len(pe))
    Bb = rng.standard_normal((ne, 3, 3)) * 0.3 + np.eye(3)
    Bs = rng.standard_normal((ns, 3 * ne))
    Xs = rng.standard_normal((ns, 3 * ne))
    theta = rng.standard_normal(OL.n_params(H)) * 0.4
    return theta, H, F, scale, pe, pf, Bb, Bs, Xs


def test_gradient_matches_central_differences():
    theta, H, F, scale, pe, pf, Bb, Bs, Xs = _random_problem()
    L, g = OL.loss_grad(theta, H, F, scale, pe, pf, Bb, Bs, Xs)
    assert L == pytest.approx(OL.loss(theta, H, F, scale, pe, pf, Bb, Bs, Xs), rel=1e-14)
    eps = 1e-6
    fd = np.empty_like(g)
    for i in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd[i] = (OL.loss(tp, H, F, scale, pe, pf, Bb, Bs, Xs) - OL.loss(tm, H, F, scale, pe, pf, Bb, Bs, Xs)) / (
            2 * eps)
    # truncation O(eps^2) and cancellation O(1e-16 L / eps) are both far below this
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
    # every layer receives gradient (none is silently dropped)
    sizes = [32 * H, H, H * H, H, H * 9, 9]
    o = 0
    for n in sizes:
        assert np.any(g[o:o + n] != 0.0)
        o += n


def test_pair_sum_matches_dense_matrix():
    theta, H, F, scale, pe, pf, Bb, Bs, Xs = _random_problem(seed=1)
    Wb = OL.blocks(theta, H, F, scale)
    M = OL.dense_preconditioner(Bb, pe, pf, Wb, len(Bb))
    Z = OL.apply(Bb, pe, pf, Wb, Bs)
    np.testing.assert_allclose(Z, Bs @ M.T, rtol=0, atol=1e-12 * np.abs(Z).max())


def test_dense_base_matches_block_base_and_central_differences():
    """A dense M_base (the leaf block-Jacobi form) in place of the 3x3 blocks:
    the block-diagonal matrix of the blocks reproduces the block form
    exactly, and for a general dense base the gradient still matches
    central differences of the loss."""
    theta, H, F, scale, pe, pf, Bb, Bs, Xs = _random_problem(seed=3)
    ne = len(Bb)
    Mb = np.zeros((3 * ne, 3 * ne))
    for e in range(ne):
        Mb[3 * e:3 * e + 3, 3 * e:3 * e + 3] = Bb[e]
    Wb = OL.blocks(theta, H, F, scale)
    np.testing.assert_allclose(OL.apply(Mb, pe, pf, Wb, Bs), OL.apply(Bb, pe, pf, Wb, Bs), rtol=0, atol=1e-13)
    L1, g1 = OL.loss_grad(theta, H, F, scale, pe, pf, Bb, Bs, Xs)
    L2, g2 = OL.loss_grad(theta, H, F, scale, pe, pf, Mb, Bs, Xs)
    assert L2 == pytest.approx(L1, rel=1e-13) and np.allclose(g2, g1, rtol=0, atol=1e-12 * np.abs(g1).max())
    rng = np.random.default_rng(4)
    Md = rng.standard_normal((3 * ne, 3 * ne)) * 0.2 + np.eye(3 * ne)
    L, g = OL.loss_grad(theta, H, F, scale, pe, pf, Md, Bs, Xs)
    eps = 1e-6
    fd = np.empty_like(g)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd[i] = (OL.loss(tp, H, F, scale, pe, pf, Md, Bs, Xs) - OL.loss(tm, H, F, scale, pe, pf, Md, Bs, Xs)) / (
            2 * eps)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
    # the dense preconditioner carries the dense base plus the pair blocks
    M = OL.dense_preconditioner(Md, pe, pf, Wb, ne)
    np.testing.assert_allclose(OL.apply(Md, pe, pf, Wb, Bs), Bs @ M.T, rtol=0, atol=1e-12 * np.abs(Bs @ M.T).max())


def test_leaf_block_system_with_leaf_base_zero_network_is_exact():
    """A system block-diagonal over groups of elements ("leaves"): the
    inverse of the group blocks as M_base is exact, so a zero network gives a
    zero loss, while the 3x3 block base does not."""
    rng = np.random.default_rng(5)
    ne, groups = 8, [[0, 1, 2], [3, 4], [5, 6, 7]]
    A = np.zeros((3 * ne, 3 * ne))
    for g in groups:
        d = (3 * np.asarray(g)[:, None] + np.arange(3)).ravel()
        A[np.ix_(d, d)] = rng.standard_normal((len(d), len(d))) + 6 * np.eye(len(d))
    Mleaf = np.zeros_like(A)
    for g in groups:
        d = (3 * np.asarray(g)[:, None] + np.arange(3)).ravel()
        Mleaf[np.ix_(d, d)] = np.linalg.inv(A[np.ix_(d, d)])
    X = rng.standard_normal((4, 3 * ne))
    Bs = X @ A.T
    H = 4
    pe, pf = OL.knn_bruteforce(rng.standard_normal((ne, 3)), 3)
    F = rng.standard_normal((len(pe), 32))
    assert OL.loss(np.zeros(OL.n_params(H)), H, F, np.ones(len(pe)), pe, pf, Mleaf, Bs, X) < 1e-26
    assert OL.loss(np.zeros(OL.n_params(H)), H, F, np.ones(len(pe)), pe, pf, OL.block_jacobi(A, ne), Bs, X) > 1e-6


def test_block_diagonal_system_zero_network_is_exact():
    rng = np.random.default_rng(2)
    ne = 7
    A = np.zeros((3 * ne, 3 * ne))
    for e in range(ne):
        A[3 * e:3 * e + 3, 3 * e:3 * e + 3] = rng.standard_normal((3, 3)) + 4 * np.eye(3)
    Bb = OL.block_jacobi(A, ne)
    X = rng.standard_normal((4, 3 * ne))
    Bs = X @ A.T
    H = 4
    pe, pf = OL.knn_bruteforce(rng.standard_normal((ne, 3)), 3)
    F = rng.standard_normal((len(pe), 32))
    assert OL.loss(np.zeros(OL.n_params(H)), H, F, np.ones(len(pe)), pe, pf, Bb, Bs, X) < 1e-28
    # a nonzero network whose pairs are all switched off (inactive) changes nothing
    theta = rng.standard_normal(OL.n_params(H))
    assert OL.loss(theta, H, F, np.zeros(len(pe)), pe, pf, Bb, Bs, X) < 1e-28
    # and with them switched on it does
    assert OL.loss(theta, H, F, np.ones(len(pe)), pe, pf, Bb, Bs, X) > 1e-6


def test_square_grid_features_from_geometry():
    h = 2.0
    m = W.rect_grid(5, 5, h=h)
    cent, frame, area = oracle.frames(m)
    pe, pf = OL.knn_bruteforce(cent, 5)
    e = 12  # the centre cell (i, j) = (2, 2)
    nb = list(pf[pe == e])
    assert nb[0] == e and sorted(nb[1:]) == [7, 11, 13, 17] and nb[1:] == [7, 11, 13, 17]
    young, nu = 30e9, 0.25
    Ep = young / (1 - nu * nu)
    D = np.zeros((m.ne, 3, 3))
    D[:] = np.diag([1.0, 2.0, 3.0]) * Ep / h
    D[:, 0, 2] = -0.6 * Ep / h
    F, scale = OL.features(cent, frame, area, D, None, [np.arange(m.ne)], pe, pf, young, nu)
    rows = {int(f): F[p] for p, f in enumerate(pf) if pe[p] == e}
    expect_offset = {13: (1, 0), 11: (-1, 0), 17: (0, 1), 7: (0, -1), 12: (0, 0)}
    for f, (dx, dy) in expect_offset.items():
        r = rows[f]
        np.testing.assert_allclose(r[0:4], [dx, dy, 0, np.hypot(dx, dy)], atol=1e-14)
        np.testing.assert_allclose(r[4:7], [1, 1, 1], atol=1e-14)
        np.testing.assert_allclose(r[7:13], [1, 2, 3, 1, 2, 3], rtol=1e-14)
        np.testing.assert_allclose(r[13:16], [-0.6, -0.6, 0.0], rtol=1e-14, atol=1e-15)
        assert r[16] == pytest.approx(1.0) and r[17] == (1.0 if f == e else 0.0)
        np.testing.assert_allclose(r[18:20], [3.0, 1.5], rtol=1e-14)
        assert np.all(r[20:] == 0)
    np.testing.assert_allclose(scale, h / Ep, rtol=1e-15)
    # inactive elements switch their pairs off, and leave the patch means
    active = np.ones(m.ne, bool)
    active[13] = False
    D2 = D.copy()
    D2[13] = np.diag([50.0, 50.0, 50.0]) * Ep / h
    F2, scale2 = OL.features(cent, frame, area, D2, active, [np.arange(m.ne)], pe, pf, young, nu)
    assert all(scale2[p] == 0 for p in range(len(pe)) if pe[p] == 13 or pf[p] == 13)
    assert all(scale2[p] > 0 for p in range(len(pe)) if pe[p] != 13 and pf[p] != 13)
    np.testing.assert_allclose(F2[:, 18:20], F[:, 18:20], rtol=1e-14)


def test_features_invariant_under_rigid_motion_and_scaling():
    rng = np.random.default_rng(5)
    base = W.rect_tri_mesh(8.0, 6.0, 4, 3, (0.0, 0.0, 0.0), np.eye(3), "a")
    xyz = base.xyz + rng.normal(0, 0.2, base.xyz.shape)
    m = W.Mesh(xyz, base.conn, "jittered", {})
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    lam = 3.7
    m2 = W.Mesh(lam * xyz @ Q.T + np.array([5.0, -2.0, 7.0]), base.conn, "moved", {})
    young, nu = 20e9, 0.3
    D = rng.standard_normal((m.ne, 3, 3)) * 1e10
    c1, f1, a1 = oracle.frames(m)
    c2, f2, a2 = oracle.frames(m2)
    pe, pf = OL.knn_bruteforce(c1, 6)
    pe2, pf2 = OL.knn_bruteforce(c2, 6)
    assert np.array_equal(pe, pe2) and np.array_equal(pf, pf2)
    groups = [np.arange(0, 12), np.arange(12, m.ne)]
    F1, s1 = OL.features(c1, f1, a1, D, None, groups, pe, pf, young, nu)
    F2, s2 = OL.features(c2, f2, a2, D / lam, None, groups, pe, pf, young, nu)
    np.testing.assert_allclose(F2, F1, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(s2, lam * s1, rtol=1e-12)
