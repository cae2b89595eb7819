"""GPU tests of the learned correction of the block preconditioner.

Against the CPU FP64 oracle (oracle/learned.py), on a two-part jittered
triangle mesh of 56 elements (one cluster-tree leaf, so the patch of every
element is the whole mesh, and no two centroid distances tie):
  * pairs: bit-exact against brute-force K-nearest search;
  * features: within one FP32 rounding of the oracle's FP64 values;
  * loss and gradient of the library's own backward kernels: the network
    runs in FP32, so the bar is derived from FP32 rounding through three
    layers of width <= 64: |dL| <= 1e-5 L, ||dg|| <= 1e-4 ||g||;
  * M^-1 R: the W blocks are stored in FP32, so <= 1e-6 per column;
    linearity of M^-1 to FP64 rounding.
The same with the leaf block-Jacobi inverse as the base (oracle: the dense
leaf inverse), and its fallback.  Then, on the HF x fault mesh at h = 4 m:
training is deterministic, lowers the loss, and the trained correction
needs fewer GMRES iterations than block-Jacobi on held-out tangent states;
the correction trained on the leaf blocks against the leaf blocks alone, in
iterations and time; and the fallback to block-Jacobi.
"""
import time

import numpy as np
import pytest

import oracle
import oracle.learned as OL
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25
H, K = 32, 8


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available(), "GPU tests need a device"
    return hm


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _two_part_mesh(seed=11):
    rng = np.random.default_rng(seed)
    a = W.rect_tri_mesh(8.0, 6.0, 4, 3, (0.0, 0.0, 0.0), np.eye(3), "a")
    ax = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(1.1), np.sin(1.1)], [0.0, -np.sin(1.1), np.cos(1.1)]])
    b = W.rect_tri_mesh(7.0, 7.0, 4, 4, (1.0, 0.5, 4.0), ax, "b")
    xyz = np.concatenate([a.xyz, b.xyz])
    xyz = xyz + rng.normal(0.0, 0.12, xyz.shape)
    conn = np.concatenate([a.conn, b.conn + a.nv])
    return W.Mesh(xyz, conn, "two_parts", {"parts": [(0, a.ne), (a.ne, b.ne)]})


@pytest.fixture(scope="module")
def tiny():
    hm = _hm()
    m = _two_part_mesh()
    assert m.ne <= 64
    D = W.tangent_state(m, 10, injection=(0.0, 0.0, 2.0), rmax=7.0)
    active = np.ones(m.ne, bool)
    active[[3, 40]] = False
    E = oracle.dense(m, YOUNG, NU)
    A = oracle.tangent_dense(E, D, active)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64)
    op.set_tangent(cuda(D), cuda(active.astype(np.uint8), torch.uint8))
    cent, frame, area = oracle.frames(m)
    pe, pf = OL.knn_bruteforce(cent, K)
    F, scale = OL.features(cent, frame, area, D, active, [np.arange(m.ne)], pe, pf, YOUNG, NU)
    Bb = OL.block_jacobi(A, m.ne)
    return dict(m=m, D=D, active=active, A=A, op=op, cent=cent, pe=pe, pf=pf, F=F, scale=scale, Bb=Bb)


def _theta(hm, seed=3):
    """Seeded parameters with an output layer of full size (the library's
    own initialisation scales it by 0.01)."""
    rng = np.random.default_rng(seed)
    n = OL.n_params(H)
    th = rng.uniform(-1, 1, n) * 0.25
    return th.astype(np.float32)


def test_pairs_and_features_match_oracle(tiny):
    hm = _hm()
    d2 = np.sum((tiny["cent"][:, None] - tiny["cent"][None]) ** 2, -1)
    srt = np.sort(d2, axis=1)
    # no ties among the K + 1 nearest, so the pair list is unique
    assert np.min(np.diff(srt[:, :K + 1], axis=1)) > 1e-9 * np.max(srt)
    pe, pf, feat, scale = hm.learned_features(tiny["op"], K)
    assert np.array_equal(pe, tiny["pe"]) and np.array_equal(pf, tiny["pf"])
    np.testing.assert_allclose(feat.astype(np.float64), tiny["F"], rtol=2.0 ** -23, atol=1e-12)
    np.testing.assert_allclose(scale, tiny["scale"], rtol=1e-14, atol=0)
    assert np.all(feat[:, 20:] == 0)


def test_loss_and_gradient_match_oracle(tiny):
    hm = _hm()
    net = hm.Learned(hidden=H, neighbors=K, seed=1)
    th = _theta(hm)
    net.set_params(th)
    assert np.array_equal(net.get_params(), th)
    rng = np.random.default_rng(21)
    X = rng.standard_normal((4, 3 * tiny["m"].ne))
    B = X @ tiny["A"].T
    L, g = net.loss_grad(tiny["op"], cuda(B), cuda(X))
    F32 = tiny["F"].astype(np.float32).astype(np.float64)  # the network input the device sees
    Lo, go = OL.loss_grad(th.astype(np.float64), H, F32, tiny["scale"], tiny["pe"], tiny["pf"], tiny["Bb"], B, X)
    assert abs(L - Lo) <= 1e-5 * Lo
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    assert np.max(np.abs(g - go)) <= 1e-3 * np.max(np.abs(go))
    # parameters untouched by a gradient evaluation
    assert np.array_equal(net.get_params(), th)


def test_preconditioner_apply_matches_oracle_and_is_linear(tiny):
    hm = _hm()
    net = hm.Learned(hidden=H, neighbors=K, seed=1)
    th = _theta(hm)
    net.set_params(th)
    net.attach(tiny["op"])
    rng = np.random.default_rng(22)
    n = 3 * tiny["m"].ne
    R = rng.standard_normal((3, n))
    Z = tiny["op"].precond_apply(cuda(R), hm.HM_PC_LEARNED).cpu().numpy()
    F32 = tiny["F"].astype(np.float32).astype(np.float64)
    Wb = OL.blocks(th.astype(np.float64), H, F32, tiny["scale"])
    Zo = OL.apply(tiny["Bb"], tiny["pe"], tiny["pf"], Wb, R)
    # active rows scale like h / G; inactive rows pass R through: compare them apart
    act = np.repeat(tiny["active"], 3)
    for c in range(3):
        assert np.linalg.norm(Z[c, act] - Zo[c, act]) <= 1e-6 * np.linalg.norm(Zo[c, act])
    # the correction is not negligible here (the test would pass vacuously otherwise)
    Zbj = OL.apply(tiny["Bb"], tiny["pe"], tiny["pf"], 0 * Wb, R)
    assert np.linalg.norm(Zo[:, act] - Zbj[:, act]) > 1e-2 * np.linalg.norm(Zo[:, act])
    # inactive rows pass through unchanged
    for e in np.flatnonzero(~tiny["active"]):
        np.testing.assert_array_equal(Z[:, 3 * e:3 * e + 3], R[:, 3 * e:3 * e + 3])
    # linearity
    a, b = 0.7, -2.5
    Zab = tiny["op"].precond_apply(cuda(a * R[0:1] + b * R[1:2]), hm.HM_PC_LEARNED).cpu().numpy()[0]
    assert np.linalg.norm(Zab - (a * Z[0] + b * Z[1])) <= 1e-13 * np.linalg.norm(Zab)
    # the plain block-Jacobi path
    Zb = tiny["op"].precond_apply(cuda(R), hm.HM_PC_BLOCK3).cpu().numpy()
    np.testing.assert_allclose(Zb[:, act], Zbj[:, act], rtol=1e-12, atol=1e-12 * np.abs(Zbj[:, act]).max())
    np.testing.assert_array_equal(Zb[:, ~act], R[:, ~act])


def test_fallback_to_block_jacobi(tiny):
    hm = _hm()
    op = tiny["op"]
    n = 3 * tiny["m"].ne
    rng = np.random.default_rng(23)
    b = rng.standard_normal((2, n))
    x_ref = oracle.solve_dense(tiny["A"], b)
    hm.learned_detach(op)
    x, rep = op.solve(cuda(b), precond=hm.HM_PC_LEARNED, restart=30, rtol=1e-10)
    assert rep["fallback"] == hm.HM_FALLBACK_NOT_ATTACHED and rep["precond_used"] == hm.HM_PC_BLOCK3
    assert rep["converged"] == 1
    # a correction poisoned with NaN: detected, solved again with block-Jacobi
    net = hm.Learned(hidden=H, neighbors=K, seed=2)
    th = net.get_params()
    th[-9:] = np.nan
    net.set_params(th)
    net.attach(op)
    x, rep = op.solve(cuda(b), precond=hm.HM_PC_LEARNED, restart=30, rtol=1e-10)
    assert rep["fallback"] == hm.HM_FALLBACK_NONFINITE and rep["precond_used"] == hm.HM_PC_BLOCK3
    assert rep["converged"] == 1 and rep["rel_residual"] <= 1e-10
    xc = x.cpu().numpy()
    for c in range(2):
        assert np.linalg.norm(xc[c] - x_ref[c]) <= 1e-6 * np.linalg.norm(x_ref[c])
    # an iteration budget too small for either attempt
    net.set_params(_theta(hm))
    net.attach(op)
    x, rep = op.solve(cuda(b), precond=hm.HM_PC_LEARNED, restart=30, rtol=1e-10, max_iter=2,
                      raise_on_notconv=False)
    assert rep["fallback"] == hm.HM_FALLBACK_NOT_CONVERGED and rep["converged"] == 0
    assert rep["discarded_iterations"] == 2
    with pytest.raises(hm.HMError):
        hm.learned_detach(op)
        op.precond_apply(cuda(b), hm.HM_PC_LEARNED)


def test_leaf_base_loss_gradient_apply_and_fallback(tiny):
    """The correction added to the leaf block-Jacobi inverse (four leaves of
    at most 16 elements) instead of the 3x3 blocks: loss and gradient, and
    M^-1 R, against the oracle with the dense leaf inverse as its base; a
    poisoned correction falls back to the leaf blocks."""
    from test_host_logic import _py_plan

    hm = _hm()
    m, A = tiny["m"], tiny["A"]
    leaf = 16
    nodes, _, _ = _py_plan(m, leaf, 2.0)
    leaves = [np.asarray(nd[0]) for nd in nodes if nd[2] is None]
    assert len(leaves) >= 4
    Mleaf = np.zeros_like(A)
    for idx in leaves:
        d = (3 * idx[:, None] + np.arange(3)).ravel()
        Mleaf[np.ix_(d, d)] = np.linalg.inv(A[np.ix_(d, d)])
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=leaf)
    op.set_tangent(cuda(tiny["D"]), cuda(tiny["active"].astype(np.uint8), torch.uint8))
    _, frame, area = oracle.frames(m)
    F, scale = OL.features(tiny["cent"], frame, area, tiny["D"], tiny["active"], leaves, tiny["pe"], tiny["pf"],
                           YOUNG, NU)
    F32 = F.astype(np.float32).astype(np.float64)
    net = hm.Learned(hidden=H, neighbors=K, seed=1)
    net.set_base(hm.HM_PC_LEAF)
    th = _theta(hm)
    net.set_params(th)
    rng = np.random.default_rng(24)
    n = 3 * m.ne
    X = rng.standard_normal((4, n))
    B = X @ A.T
    L, g = net.loss_grad(op, cuda(B), cuda(X))
    Lo, go = OL.loss_grad(th.astype(np.float64), H, F32, scale, tiny["pe"], tiny["pf"], Mleaf, B, X)
    assert abs(L - Lo) <= 1e-5 * Lo
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    net.attach(op)
    R = rng.standard_normal((3, n))
    Z = op.precond_apply(cuda(R), hm.HM_PC_LEARNED).cpu().numpy()
    Wb = OL.blocks(th.astype(np.float64), H, F32, scale)
    Zo = OL.apply(Mleaf, tiny["pe"], tiny["pf"], Wb, R)
    act = np.repeat(tiny["active"], 3)
    for c in range(3):
        assert np.linalg.norm(Z[c, act] - Zo[c, act]) <= 1e-6 * np.linalg.norm(Zo[c, act])
        assert np.allclose(Z[c, ~act], R[c, ~act], rtol=1e-13, atol=0)
    # the leaf base differs from the 3x3 base here (the test is not vacuous)
    Zb3 = OL.apply(tiny["Bb"], tiny["pe"], tiny["pf"], Wb, R)
    assert np.linalg.norm(Zo[:, act] - Zb3[:, act]) > 1e-2 * np.linalg.norm(Zo[:, act])
    # a poisoned correction: solved again with the leaf blocks
    th_bad = th.copy()
    th_bad[-9:] = np.nan
    net.set_params(th_bad)
    net.attach(op)
    b = rng.standard_normal((2, n))
    x, rep = op.solve(cuda(b), precond=hm.HM_PC_LEARNED, restart=30, rtol=1e-10)
    assert rep["fallback"] == hm.HM_FALLBACK_NONFINITE and rep["precond_used"] == hm.HM_PC_LEAF
    x_ref = oracle.solve_dense(A, b)
    xc = x.cpu().numpy()
    for c in range(2):
        assert np.linalg.norm(xc[c] - x_ref[c]) <= 1e-6 * np.linalg.norm(x_ref[c])
    with pytest.raises(hm.HMError):
        net.set_base(hm.HM_PC_JACOBI)


# ------------------------------------------------------------ training
@pytest.fixture(scope="module")
def hf():
    hm = _hm()
    m = W.hf_fault_mesh(h=4.0)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU)
    data = []
    for k in range(16):
        op.set_tangent(cuda(W.tangent_state(m, k)))
        X = cuda(W.rhs_columns(m.ndof, 16, 7000 + 16 * k))
        B = op.apply(X, tangent=True)
        data.append((B, X))
    return m, op, data


def _train(hm, m, op, data, epochs, seed=5):
    net = hm.Learned(hidden=64, neighbors=K, seed=seed)
    hist = []
    for _ in range(epochs):
        for k in range(16):
            op.set_tangent(cuda(W.tangent_state(m, k)))
            B, X = data[k]
            hist.extend(net.train(op, B, X, steps=8, batch=8, lr=1e-3))
    return net, np.array(hist)


def test_training_is_deterministic_and_lowers_the_loss(hf):
    hm = _hm()
    m, op, data = hf
    n1, h1 = _train(hm, m, op, data, 1)
    n2, h2 = _train(hm, m, op, data, 1)
    assert np.array_equal(n1.get_params(), n2.get_params())
    assert np.array_equal(h1, h2)
    assert np.all(np.isfinite(h1))
    assert np.mean(h1[-16:]) < 0.8 * np.mean(h1[:16])


def test_trained_correction_reduces_gmres_iterations_on_held_out_states(hf):
    hm = _hm()
    m, op, data = hf
    net, hist = _train(hm, m, op, data, 8)
    its_bj, its_l = [], []
    for k in range(16, 20):
        op.set_tangent(cuda(W.tangent_state(m, k)))
        net.attach(op)
        b = cuda(W.tangent_rhs(m, 4, 9000 + k))
        _, r0 = op.solve(b, precond=hm.HM_PC_BLOCK3, restart=50, rtol=1e-8)
        _, r1 = op.solve(b, precond=hm.HM_PC_LEARNED, restart=50, rtol=1e-8)
        assert r0["converged"] == 1 and r1["converged"] == 1
        assert r1["fallback"] == hm.HM_FALLBACK_NONE and r1["precond_used"] == hm.HM_PC_LEARNED
        assert r1["rel_residual"] <= 1e-8
        its_bj.append(r0["iterations"])
        its_l.append(r1["iterations"])
    print("block-Jacobi", its_bj, "learned", its_l, "final loss", hist[-16:].mean())
    assert sum(its_l) <= 0.8 * sum(its_bj)


def _timed_solve(op, b, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, rep = op.solve(b, **kw)
    torch.cuda.synchronize()
    return x, rep, time.perf_counter() - t0


def test_correction_on_leaf_blocks_against_leaf_blocks_alone(hf):
    """The strongest plain preconditioner built here is the leaf
    block-Jacobi inverse; the correction trained on top of it is compared
    with it alone on the held-out states, in iterations and time.  The gain
    is small (a few per cent of the iterations on the injection states; in
    the precision form the extra apply can cost more than it saves), so the
    bar is that the correction converges without a fallback and does not
    need more iterations than its base."""
    hm = _hm()
    m, op, data = hf
    net = hm.Learned(hidden=64, neighbors=K, seed=5)
    net.set_base(hm.HM_PC_LEAF)
    for _ in range(8):
        for k in range(16):
            op.set_tangent(cuda(W.tangent_state(m, k)))
            B, X = data[k]
            net.train(op, B, X, steps=8, batch=8, lr=1e-3)
    its_leaf, its_l, t_leaf, t_l = [], [], 0.0, 0.0
    for k in range(16, 20):
        op.set_tangent(cuda(W.tangent_state(m, k)))
        net.attach(op)
        b = cuda(W.tangent_rhs(m, 4, 9000 + k))
        x0, r0, s0 = _timed_solve(op, b, precond=hm.HM_PC_LEAF, restart=50, rtol=1e-8)
        x1, r1, s1 = _timed_solve(op, b, precond=hm.HM_PC_LEARNED, restart=50, rtol=1e-8)
        assert r0["converged"] == 1 and r1["converged"] == 1
        assert r1["fallback"] == hm.HM_FALLBACK_NONE and r1["precond_used"] == hm.HM_PC_LEARNED
        assert r1["rel_residual"] <= 1e-8
        # both solve the same system
        assert torch.linalg.norm(x1 - x0) <= 1e-6 * torch.linalg.norm(x0)
        its_leaf.append(r0["iterations"])
        its_l.append(r1["iterations"])
        t_leaf += s0
        t_l += s1
    print(f"leaf block-Jacobi {its_leaf} {t_leaf:.3f} s, learned on leaf {its_l} {t_l:.3f} s")
    assert sum(its_l) <= sum(its_leaf)


def test_full_size_sampled_apply_matches_oracle():
    """The learned correction at the HF x fault size (199,880 triangles,
    16 neighbours, 64 hidden units, as timed): at sampled elements whose 16
    nearest elements are unique (a clear gap to the 17th), the pairs, the
    features and M^-1 R match the oracle, which finds the neighbours by
    brute force over all elements, takes the base block from the exact
    self coefficient and sums the correction over the pairs.  The tangent
    state has D_e h_e / E' constant, so the patch means (features 18-19)
    are the same for any grouping of the elements."""
    hm = _hm()
    Hf, Kf = 64, 16
    m = W.hf_fault_mesh()
    cent, frame, area = oracle.frames(m)
    h = np.sqrt(area)
    Ep = YOUNG / (1 - NU * NU)
    Mfix = np.array([[1.0, 0.0, 0.2], [0.0, 0.8, 0.0], [0.3, 0.0, 2.0]])
    D = (0.5 * Ep / h)[:, None, None] * Mfix
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6)
    op.set_tangent(cuda(D))
    rng = np.random.default_rng(3)
    th = (rng.uniform(-1, 1, OL.n_params(Hf)) * 0.25).astype(np.float32)
    net = hm.Learned(hidden=Hf, neighbors=Kf, seed=1)
    net.set_params(th)
    net.attach(op)
    R = np.random.default_rng(31).standard_normal((2, m.ndof))
    Z = op.precond_apply(cuda(R), hm.HM_PC_LEARNED).cpu().numpy()
    pe_g, pf_g, feat_g, scale_g = hm.learned_features(op, Kf)
    # sampled elements with a unique neighbour set, nearest by brute force
    # (twelve on the hydraulic fracture, twelve on the fault)
    sample, nbrs = [], []
    srng = np.random.default_rng(32)
    for lo, n in m.meta["parts"]:
        got = 0
        for e in lo + srng.choice(n, 300, replace=False):
            d2 = np.sum((cent - cent[e]) ** 2, axis=1)
            order = np.lexsort((np.arange(m.ne), d2))
            if d2[order[Kf]] - d2[order[Kf - 1]] > 1e-9 * d2[order[Kf]]:
                sample.append(int(e))
                nbrs.append(order[:Kf])
                got += 1
            if got == 12:
                break
    assert len(sample) == 24
    pe = np.repeat(np.array(sample, np.int64), Kf)
    pf = np.concatenate(nbrs).astype(np.int64)
    for e, nb in zip(sample, nbrs):
        assert sorted(pf_g[pe_g == e].tolist()) == sorted(nb.tolist()), e
    F, scale = OL.features(cent, frame, area, D, None, [np.arange(m.ne)], pe, pf, YOUNG, NU)
    gidx = {(int(a), int(b)): i for i, (a, b) in
            enumerate(zip(pe_g[np.isin(pe_g, sample)], pf_g[np.isin(pe_g, sample)]))}
    sel = np.flatnonzero(np.isin(pe_g, sample))
    rows_g = sel[[gidx[(int(a), int(b))] for a, b in zip(pe, pf)]]
    np.testing.assert_allclose(feat_g[rows_g].astype(np.float64), F, rtol=2.0 ** -22, atol=1e-12)
    np.testing.assert_allclose(scale_g[rows_g], scale, rtol=1e-14, atol=0)
    # M^-1 R on the sampled elements: the oracle's apply over the elements involved
    U = np.unique(np.concatenate([pe, pf]))
    loc = {int(u): i for i, u in enumerate(U)}
    Bb = np.zeros((len(U), 3, 3))
    for e in sample:
        Eee = oracle.blocks(m, YOUNG, NU, [e], [e], method=1)[0, 0]
        Bb[loc[e]] = np.linalg.inv(Eee - D[e])
    Wb = OL.blocks(th.astype(np.float64), Hf, F.astype(np.float32).astype(np.float64), scale)
    dof = (3 * U[:, None] + np.arange(3)).ravel()
    Zo = OL.apply(Bb, np.array([loc[int(a)] for a in pe]), np.array([loc[int(b)] for b in pf]), Wb, R[:, dof])
    Zb = OL.apply(Bb, np.array([loc[int(a)] for a in pe]), np.array([loc[int(b)] for b in pf]), 0 * Wb, R[:, dof])
    rows_o = (3 * np.array([loc[e] for e in sample])[:, None] + np.arange(3)).ravel()
    rows_z = (3 * np.array(sample)[:, None] + np.arange(3)).ravel()
    for c in range(2):
        err = np.linalg.norm(Z[c, rows_z] - Zo[c, rows_o]) / np.linalg.norm(Zo[c, rows_o])
        corr = np.linalg.norm(Zo[c, rows_o] - Zb[c, rows_o]) / np.linalg.norm(Zo[c, rows_o])
        print(f"column {c}: sampled error {err:.2e}, correction share {corr:.2e}", flush=True)
        assert err <= 1e-6 and corr > 1e-2
    # a learned-form solve at this size (a fresh network: the library's own
    # initialisation), judged by the exact operator: b - (E x - D x) on 64
    # sampled rows, exact rows by the oracle's Peach-Koehler quadrature
    net2 = hm.Learned(hidden=Hf, neighbors=Kf, seed=2)
    net2.attach(op)
    b = np.random.default_rng(33).standard_normal((1, m.ndof)) * 1e6
    x, rep = op.solve(cuda(b), precond=hm.HM_PC_LEARNED, restart=50, rtol=1e-8, max_iter=2000)
    assert rep["converged"] and rep["fallback"] == hm.HM_FALLBACK_NONE
    assert rep["precond_used"] == hm.HM_PC_LEARNED and rep["rel_residual"] <= 1e-8
    xh = x.cpu().numpy()
    rows = np.sort(np.random.default_rng(34).choice(m.ne, 64, replace=False))
    dof = (3 * rows[:, None] + np.arange(3)).ravel()
    Ax = oracle.rows_matvec(m, YOUNG, NU, rows, xh, method=1)[0] - np.einsum(
        "eab,eb->ea", D[rows], xh[0].reshape(-1, 3)[rows]).ravel()
    r_exact = np.linalg.norm(b[0, dof] - Ax) / np.linalg.norm(b[0, dof])
    print(f"learned-form solve: {rep['iterations']} its; exact residual on 64 rows {r_exact:.2e}", flush=True)
    assert r_exact <= 1e-5
