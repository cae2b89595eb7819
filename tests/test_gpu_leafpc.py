"""GPU parity of the leaf block-Jacobi preconditioner (HM_PC_LEAF).

M is the block diagonal of A11 over the cluster-tree leaves.  The oracle
builds A11 densely (exact coefficients, D on active elements, identity
rows and columns on inactive ones), takes each leaf's diagonal block (leaf
membership from the independent Python construction of the cluster tree)
and inverts it with LAPACK.  The library forms the same inverses by its own
Gauss-Jordan elimination; the two agree to FP64 rounding (relative 1e-11
on M^-1 R, the blocks' condition numbers are small).  A solve with it
converges to the dense LU solution in fewer iterations than with the 3x3
block-Jacobi preconditioner.
"""
import numpy as np
import pytest

import oracle
from test_host_logic import _py_plan
from workloads import penny_active_mask, rect_grid, rhs_columns, square_fault

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available(), "GPU tests need a device"
    return hm


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def leaf_inverse(m, A, leaf):
    """Block-diagonal inverse of A over the leaves (original element order)."""
    nodes, _, _ = _py_plan(m, leaf, 2.0)
    Minv = np.zeros_like(A)
    for idx, _, children in nodes:
        if children is not None:
            continue
        d = (3 * np.asarray(idx)[:, None] + np.arange(3)).ravel()
        Minv[np.ix_(d, d)] = np.linalg.inv(A[np.ix_(d, d)])
    return Minv


def random_tangent(m, seed, frac_active=0.7):
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(m.ne, 3, 3))
    D = 2e9 * (np.einsum("nij,nkj->nik", Q, Q) + np.eye(3)) + 1e8 * rng.normal(size=(m.ne, 3, 3))
    mask = (rng.random(m.ne) < frac_active).astype(np.uint8)
    return D, mask


def colerr(Y, R):
    return max(np.linalg.norm(Y[c] - R[c]) / np.linalg.norm(R[c]) for c in range(R.shape[0]))


@pytest.mark.parametrize("nx,ny,leaf", [(16, 16, 64), (23, 7, 5), (14, 9, 16), (3, 1, 64)],
                         ids=["full_leaves_192dof", "ragged_small", "mid", "single_leaf"])
def test_leaf_inverse_matches_lapack(nx, ny, leaf):
    hm = _hm()
    m = rect_grid(nx, ny, 1.0)
    E = oracle.dense(m, YOUNG, NU)
    R = rhs_columns(m.ndof, 5, 5100)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=leaf)
    # plain operator: M = blocks of E
    Z = op.precond_apply(cuda(R), precond=hm.HM_PC_LEAF).cpu().numpy()
    assert colerr(Z, R @ leaf_inverse(m, E, leaf).T) <= 1e-11
    # tangent with D and a mask; a new tangent replaces the cached inverses
    for seed in (1, 2):
        D, mask = random_tangent(m, 5200 + seed)
        op.set_tangent(cuda(D), cuda(mask, torch.uint8))
        Z = op.precond_apply(cuda(R), precond=hm.HM_PC_LEAF).cpu().numpy()
        A = oracle.tangent_dense(E, D, mask)
        assert colerr(Z, R @ leaf_inverse(m, A, leaf).T) <= 1e-11, seed
        inactive = np.repeat(mask == 0, 3)
        assert np.array_equal(Z[:, inactive], R[:, inactive])   # identity on inactive elements


def test_leaf_preconditioned_penny_solve():
    hm = _hm()
    m = square_fault(32)
    E = oracle.dense(m, YOUNG, NU)
    act = penny_active_mask(m)
    b = np.zeros((m.ne, 3))
    b[act.astype(bool), 2] = -1e6
    b = b.ravel()
    x_ref = oracle.solve_dense(oracle.tangent_dense(E, None, act), b)[0]
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, aca_tol=1e-10)
    op.set_tangent(None, cuda(act, torch.uint8))
    its = {}
    for pc in (hm.HM_PC_BLOCK3, hm.HM_PC_LEAF):
        x, rep = op.solve(cuda(b), rtol=1e-10, restart=50, max_iter=400, precond=pc)
        err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
        print(f"precond {pc}: its {rep['iterations']} relres {rep['rel_residual']:.2e} err vs LU {err:.2e}")
        assert rep["converged"] and rep["precond_used"] == pc and err <= 1e-8
        its[pc] = rep["iterations"]
    assert its[hm.HM_PC_LEAF] < its[hm.HM_PC_BLOCK3]


def test_singular_leaf_block_is_reported():
    hm = _hm()
    # one-element leaves: D equal to an element's own coefficient block makes
    # that leaf's block zero
    m = rect_grid(4, 3, 1.0)
    E = oracle.dense(m, YOUNG, NU)
    D = np.zeros((m.ne, 3, 3))
    D[5] = E[15:18, 15:18]
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=1)
    op.set_tangent(cuda(D), None)
    with pytest.raises(hm.HMError) as e:
        op.precond_apply(cuda(rhs_columns(m.ndof, 1, 5300)), precond=hm.HM_PC_LEAF)
    assert e.value.status == hm.HM_EINVAL
    # the other preconditioners are unaffected, and a regular tangent recovers
    op.set_tangent(cuda(0.5 * D), None)
    Z = op.precond_apply(cuda(rhs_columns(m.ndof, 1, 5300)), precond=hm.HM_PC_LEAF)
    assert torch.isfinite(Z).all()
