"""GPU ILU(0) preconditioner of the sparse approximation of A11 (HM_PC_ILU)
against the CPU oracle (oracle/ilu.py: its own partition, selection,
colouring and textbook ILU(0) on the dense matrix).

On a jittered two-part triangle mesh (non-coplanar parts, no two near-field
magnitudes within 1e-9 of the threshold, so the kept set cannot depend on
rounding) with a tangent D and inactive elements:
  * the factors' entry count and colour count equal the oracle's exactly;
  * M^-1 R equals the oracle's triangular solves (bar 1e-10 per column: the
    factors are FP64, the coefficients agree to ~1e-13);
  * two set-ups give bit-identical results; a new tangent (the kept
    structure with new values) and a new active mask (a new structure)
    match the oracle again;
  * GMRES with it reaches the dense-LU solution of the exact tangent system
    (ACA 1e-10: bar 1e-8) in fewer iterations than point Jacobi;
  * a fraction outside (0, 1] is rejected (0 selects the default 1 %).
"""
import numpy as np
import pytest

import oracle
from oracle import ilu as OI
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25
LEAF = 16


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available()
    return hm


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _mesh(seed=21):
    rng = np.random.default_rng(seed)
    a = W.rect_tri_mesh(16.0, 10.0, 12, 8, (0.0, 0.0, 0.0), np.eye(3), "a")
    ax = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(1.2), np.sin(1.2)], [0.0, -np.sin(1.2), np.cos(1.2)]])
    b = W.rect_tri_mesh(12.0, 9.0, 9, 7, (2.0, 1.0, 3.0), ax, "b")
    xyz = np.concatenate([a.xyz, b.xyz])
    xyz = xyz + rng.normal(0.0, 0.08, xyz.shape)
    conn = np.concatenate([a.conn, b.conn + a.nv])
    return W.Mesh(xyz, conn, "two_parts", {"parts": [(0, a.ne), (a.ne, b.ne)]})


@pytest.fixture(scope="module")
def case():
    m = _mesh()
    E = oracle.dense(m, YOUNG, NU)
    rng = np.random.default_rng(22)
    D = np.zeros((m.ne, 3, 3))
    D[:, [0, 1, 2], [0, 1, 2]] = 1e9 * (0.5 + rng.random((m.ne, 3)))
    D[:, 0, 2] = 2e8 * rng.standard_normal(m.ne)        # a Coulomb-like off-diagonal coupling
    active = np.ones(m.ne, bool)
    active[[5, 77, 200]] = False
    near = OI.near_field_mask(m.ne, OI.near_field_blocks(m, LEAF, 2.0))
    return dict(m=m, E=E, D=D, active=active, near=near)


def _oracle_precond(c, p):
    keep, kth, k = OI.select_near_field(c["E"], c["near"], p)
    # no near-field magnitude close to the cut: the kept set cannot hinge on rounding
    mags = np.abs(c["E"][c["near"]])
    tval = np.abs(c["E"][keep]).min()
    below = mags[mags < tval]
    assert below.size == 0 or below.max() < tval * (1 - 1e-9), "choose another seed: near tie at the threshold"
    A, pat = OI.tilde_a11(c["E"], keep, c["D"], c["active"])
    col = OI.greedy_colouring(pat)
    order = OI.dof_order(col)
    F = OI.ilu0(A, pat, order)
    return F, order, int(pat.sum()), int(col.max()) + 1


@pytest.mark.parametrize("p", [0.01, 0.05])
def test_ilu_matches_the_oracle(case, p):
    hm = _hm()
    m = case["m"]
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=LEAF, eta=2.0, aca_tol=1e-10)
    op.set_tangent(cuda(case["D"]), cuda(case["active"].astype(np.uint8), torch.uint8))
    F, order, nnz, ncol = _oracle_precond(case, p)
    b = cuda(W.rhs_columns(m.ndof, 1, 23))
    _, rep = op.solve(b, precond=hm.HM_PC_ILU, ilu_fraction=p, rtol=1e-10, restart=60, max_iter=600)
    assert rep["precond_nnz"] == nnz and rep["precond_colors"] == ncol, (rep["precond_nnz"], nnz)
    R = W.rhs_columns(m.ndof, 5, 24)
    Z = op.precond_apply(cuda(R), hm.HM_PC_ILU).cpu().numpy()     # the factors of the last fraction
    Zo = OI.ilu0_apply(F, order, R)
    act = case["active"].repeat(3)
    # inactive elements: identity rows, exactly; active ones within the bar
    assert np.array_equal(Z[:, ~act], R[:, ~act])
    err = max(np.linalg.norm(Z[c, act] - Zo[c, act]) / np.linalg.norm(Zo[c, act]) for c in range(5))
    print(f"p = {p}: {nnz} entries, {ncol} colours, M^-1 R error {err:.2e}", flush=True)
    assert err <= 1e-10
    # a second set-up (new tangent object, same values) repeats it bit for bit
    op.set_tangent(cuda(case["D"]), cuda(case["active"].astype(np.uint8), torch.uint8))
    _, _ = op.solve(b, precond=hm.HM_PC_ILU, ilu_fraction=p, rtol=1e-10, restart=60, max_iter=600)
    Z2 = op.precond_apply(cuda(R), hm.HM_PC_ILU).cpu().numpy()
    assert np.array_equal(Z, Z2)
    # a new tangent (other D, same mask: the kept structure, new values),
    # then a new mask (the structure is formed again)
    D2 = case["D"] * 1.7
    D2[:, 2, 0] = 3e8
    act2 = case["active"].copy()
    act2[[9, 140]] = False
    for D_, act_ in ((D2, case["active"]), (D2, act2)):
        op.set_tangent(cuda(D_), cuda(act_.astype(np.uint8), torch.uint8))
        _, _ = op.solve(b, precond=hm.HM_PC_ILU, ilu_fraction=p, rtol=1e-10, restart=60, max_iter=600)
        Zn = op.precond_apply(cuda(R), hm.HM_PC_ILU).cpu().numpy()
        Fn, on, _, _ = _oracle_precond(dict(case, D=D_, active=act_), p)
        Zon = OI.ilu0_apply(Fn, on, R)
        a3 = act_.repeat(3)
        assert np.array_equal(Zn[:, ~a3], R[:, ~a3])
        errn = max(np.linalg.norm(Zn[c, a3] - Zon[c, a3]) / np.linalg.norm(Zon[c, a3]) for c in range(5))
        assert errn <= 1e-10, errn


def test_ilu_gmres_reaches_the_dense_solution(case):
    hm = _hm()
    m = case["m"]
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=LEAF, eta=2.0, aca_tol=1e-10)
    op.set_tangent(cuda(case["D"]), cuda(case["active"].astype(np.uint8), torch.uint8))
    A = oracle.tangent_dense(case["E"], case["D"], case["active"])
    B = W.rhs_columns(m.ndof, 3, 25) * case["active"].repeat(3)[None, :]
    X_ref = oracle.solve_dense(A, B)
    its = {}
    for name, pc in (("jacobi", hm.HM_PC_JACOBI), ("ilu", hm.HM_PC_ILU)):
        X, rep = op.solve(cuda(B), precond=pc, rtol=1e-10, restart=80, max_iter=2000)
        err = max(np.linalg.norm(X.cpu().numpy()[c] - X_ref[c]) / np.linalg.norm(X_ref[c]) for c in range(3))
        assert rep["converged"] and err <= 1e-8, (name, err)
        its[name] = rep["iterations"]
    print("GMRES iterations", its, flush=True)
    assert its["ilu"] < its["jacobi"]
    for bad in (-0.5, 1.5):
        with pytest.raises(hm.HMError) as ei:
            op.solve(cuda(B), precond=hm.HM_PC_ILU, ilu_fraction=bad)
        assert ei.value.status == hm.HM_EINVAL
