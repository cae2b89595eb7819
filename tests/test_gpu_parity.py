"""GPU parity: the HIP library against the CPU FP64 oracle.

Error metric for products (per right-hand side column c):
    err_c = ||Y_gpu[c] - Y_ref[c]||_2 / ||Y_ref[c]||_2, reported as max over c.
Bars (stated in each test):
  * exact coefficients (FP64): per element pair, max |dE| <= 1e-10 max |E_ij|;
  * FP64 H-matrix at ACA tolerance 1e-6 against the exact operator: <= 1e-6;
  * FP32 near and far field, FP32 accumulation: <= 1e-5 (measured ~1e-6);
  * FP32 near, BF16 far (hi/lo split in-vector), FP32 accumulation: <= 5e-3;
  * GMRES solution vs dense LU of the exact system: <= 1e-6 at ACA 1e-6 and
    <= 1e-8 at ACA 1e-10 (the gap is bounded by cond(A) x ACA error).
"""
import numpy as np
import pytest

import oracle
from workloads import (Mesh, disk_mesh, penny_active_mask, rect_grid, rhs_columns, square_fault)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available(), "GPU tests need a device"
    return hm


def colerr(Y, R):
    Y = np.atleast_2d(Y)
    R = np.atleast_2d(R)
    return max(np.linalg.norm(Y[c] - R[c]) / np.linalg.norm(R[c]) for c in range(R.shape[0]))


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


# ---------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def c1():
    m = square_fault(32)
    return m, oracle.dense(m, YOUNG, NU), rhs_columns(m.ndof, 8, 1001)


@pytest.fixture(scope="module")
def two_disks():
    """Two non-coplanar triangulated disks (non-uniform leaves, coupled n/s)."""
    a = disk_mesh(6.0, 8, center=(0, 0, 0))
    ax = np.array([[1.0, 0, 0], [0, np.cos(0.7), np.sin(0.7)], [0, -np.sin(0.7), np.cos(0.7)]])
    b = disk_mesh(5.0, 7, center=(3.0, 1.0, 9.0), axes=ax, spin=0.3)
    xyz = np.concatenate([a.xyz, b.xyz])
    conn = np.concatenate([a.conn, b.conn + a.nv])
    m = Mesh(xyz, conn, "two_disks")
    return m, oracle.dense(m, YOUNG, NU, method=1)


# ---------------------------------------------------------------- coefficients
def test_kernel_block_rectangles_vs_oracle(c1):
    hm = _hm()
    m, E, _ = c1
    M = hm.Mesh.from_workload(m)
    rng = np.random.default_rng(0)
    rows = np.concatenate([[0, 31, 528, 1023], rng.choice(m.ne, 60, replace=False)])
    cols = np.arange(m.ne)
    got = M.kernel_block(YOUNG, NU, rows, cols).cpu().numpy()
    ref = oracle.blocks(m, YOUNG, NU, rows, cols)
    scale = np.abs(ref).max(axis=(2, 3), keepdims=True)
    assert np.all(np.abs(got - ref) <= 1e-10 * scale)


def test_kernel_block_triangles_non_coplanar_vs_pk_quadrature(two_disks):
    hm = _hm()
    m, E = two_disks
    M = hm.Mesh.from_workload(m)
    rows = np.arange(0, m.ne, 7)
    cols = np.arange(m.ne)
    got = M.kernel_block(YOUNG, NU, rows, cols).cpu().numpy()
    ref = E.reshape(m.ne, 3, m.ne, 3).transpose(0, 2, 1, 3)[rows]
    scale = np.abs(ref).max(axis=(2, 3), keepdims=True)
    assert np.all(np.abs(got - ref) <= 1e-10 * scale)


def test_kernel_block_rejects_bad_moduli(c1):
    hm = _hm()
    M = hm.Mesh.from_workload(c1[0])
    for young, nu in ((-1.0, 0.25), (30e9, 0.5), (30e9, -1.0)):
        with pytest.raises(hm.HMError) as e:
            M.kernel_block(young, nu, [0], [0])
        assert e.value.status == hm.HM_EINVAL


# ---------------------------------------------------------------- H-matvec
def test_apply_f64_matches_exact_operator(c1):
    hm = _hm()
    m, E, X = c1
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, eta=2.0, aca_tol=1e-6)
    Y = op.apply(cuda(X)).cpu().numpy()
    err = colerr(Y, oracle.matvec(E, X))
    st = op.stats()
    print(f"C1 FP64 H-matvec rel err {err:.3e}; ranks {st['min_rank']}..{st['max_rank']}")
    assert err <= 1e-6
    assert st["n_dense_blocks"] == 340 and st["n_lowrank_blocks"] == 192


def test_apply_all_dense_is_exact_to_rounding(c1):
    hm = _hm()
    m, E, X = c1
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, eta=1e-9)
    assert op.stats()["n_lowrank_blocks"] == 0
    Y = op.apply(cuda(X)).cpu().numpy()
    assert colerr(Y, oracle.matvec(E, X)) <= 1e-13


@pytest.mark.parametrize("near,far,bar", [(1, 1, 1e-5), (1, 2, 5e-3), (1, 3, 5e-3)],
                         ids=["fp32", "fp32_bf16", "fp32_bf16_single"])
def test_apply_low_precision_forms(c1, near, far, bar):
    hm = _hm()
    m, E, X = c1
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=near, far_prec=far,
                     keep_f64_reference=1)
    ref = oracle.matvec(E, X)
    err = colerr(op.apply(cuda(X)).cpu().numpy(), ref)
    err64 = colerr(op.apply(cuda(X), reference=True).cpu().numpy(), ref)
    print(f"C1 near={near} far={far}: rel err {err:.3e} (FP64 reference copy {err64:.3e})")
    assert err <= bar and err64 <= 1e-6


def test_apply_ragged_triangles_non_coplanar(two_disks):
    hm = _hm()
    m, E = two_disks
    X = rhs_columns(m.ndof, 5, 77)
    for leaf, tol, bar in ((16, 1e-6, 1e-6), (24, 1e-9, 1e-9)):
        op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=leaf, aca_tol=tol)
        st = op.stats()
        assert st["n_lowrank_blocks"] > 0
        err = colerr(op.apply(cuda(X)).cpu().numpy(), oracle.matvec(E, X))
        print(f"two disks leaf {leaf} tol {tol}: rel err {err:.3e}")
        assert err <= bar


@pytest.mark.parametrize("stack_rows,items,window", [(1, 8, 8), (-1, 8, 3), (64, 1, 2), (-1, 1, 1), (17, 3, 6)],
                         ids=["unstacked", "one_stack_per_cluster", "stacked_partials", "tall_partials", "odd"])
def test_apply_product_layouts_match_oracle(c1, two_disks, stack_rows, items, window):
    # stacked V^T panels (any row cap), phase-A runs split into partial
    # slots and phase-B windows of 1 to 8 row tiles change only the
    # summation order: every layout meets the FP64 bar
    # on the coplanar grid and on the coupled (three-component) disks
    hm = _hm()
    m, E, X = c1
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, aca_tol=1e-6, stack_rows=stack_rows,
                     phase_a_items=items, phase_b_window=window)
    st = op.stats()
    err = colerr(op.apply(cuda(X)).cpu().numpy(), oracle.matvec(E, X))
    print(f"C1 stack_rows {stack_rows} items {items}: {st['phase_a_stacks']} stacks, {st['phase_a_tasks']} tasks, "
          f"{st['phase_a_partial_bytes']} partial bytes, rel err {err:.3e}")
    assert err <= 1e-6
    if stack_rows == 1:      # one factorisation per stack: the shear and normal parts of each coplanar block
        assert st["phase_a_stacks"] >= st["n_lowrank_blocks"]
    elif stack_rows in (-1, 64):
        assert st["phase_a_stacks"] < st["n_lowrank_blocks"]
    if items == 1:
        assert st["phase_a_partial_bytes"] > 0
    md, Ed = two_disks
    Xd = rhs_columns(md.ndof, 5, 78)
    opd = hm.Operator(hm.Mesh.from_workload(md), YOUNG, NU, leaf_size=16, aca_tol=1e-9, stack_rows=stack_rows,
                      phase_a_items=items, phase_b_window=window, near_prec=hm.HM_F32, far_prec=hm.HM_BF16,
                      keep_f64_reference=1)
    ref = oracle.matvec(Ed, Xd)
    e64 = colerr(opd.apply(cuda(Xd), reference=True).cpu().numpy(), ref)
    ebf = colerr(opd.apply(cuda(Xd)).cpu().numpy(), ref)
    print(f"two disks stack_rows {stack_rows} items {items}: FP64 {e64:.3e}, BF16 far {ebf:.3e}")
    assert e64 <= 1e-9 and ebf <= 5e-3


def test_apply_column_independence_and_determinism(c1):
    hm = _hm()
    m, E, X = c1
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=1, far_prec=1)
    X16 = rhs_columns(m.ndof, 16, 5)
    Y16 = op.apply(cuda(X16)).cpu().numpy()
    again = op.apply(cuda(X16)).cpu().numpy()
    assert np.array_equal(Y16, again)                       # run-to-run bitwise
    for cols in ([0], [3, 4, 5], list(range(9))):
        Yc = op.apply(cuda(X16[cols])).cpu().numpy()
        assert np.array_equal(Yc, Y16[cols])                 # other columns do not leak


def test_apply_strided_and_bad_arguments(c1):
    hm = _hm()
    m, E, X = c1
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32)
    big = torch.zeros((3, m.ndof + 17), dtype=torch.float64, device="cuda")
    big[:, :m.ndof] = cuda(X[:3])
    Y = op.apply(big[:, :m.ndof]).cpu().numpy()
    assert colerr(Y, oracle.matvec(E, X[:3])) <= 1e-6
    with pytest.raises(hm.HMError):
        op.apply(torch.zeros((17, m.ndof), dtype=torch.float64, device="cuda"))
    with pytest.raises(hm.HMError):
        op.apply(torch.zeros((2, m.ndof - 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(hm.HMError) as e:
        hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, near_prec=0, far_prec=2)
    assert e.value.status == hm.HM_EUNSUPPORTED
    op32 = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=1, far_prec=1)
    with pytest.raises(hm.HMError) as e:
        op32.apply(cuda(X[:1]), reference=True)            # no FP64 copy was kept
    assert e.value.status == hm.HM_EINVAL


def test_tangent_apply_with_D_and_mask(c1):
    hm = _hm()
    m, E, X = c1
    rng = np.random.default_rng(9)
    Q = rng.normal(size=(m.ne, 3, 3))
    D = 2e9 * (np.einsum("nij,nkj->nik", Q, Q) + np.eye(3))
    mask = (rng.random(m.ne) < 0.7).astype(np.uint8)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32)
    op.set_tangent(cuda(D), cuda(mask, torch.uint8))
    Y = op.apply(cuda(X), tangent=True).cpu().numpy()
    A = oracle.tangent_dense(E, D, mask)
    assert colerr(Y, oracle.matvec(A, X)) <= 1e-6
    inactive = np.repeat(mask == 0, 3)
    assert np.array_equal(Y[:, inactive], X[:, inactive])   # identity rows exactly


# ---------------------------------------------------------------- solves
def _penny_system(m):
    act = penny_active_mask(m)
    b = np.zeros((m.ne, 3))
    b[act.astype(bool), 2] = -1e6
    return act, b.ravel()


@pytest.mark.parametrize("aca_tol,bar", [(1e-6, 1e-6), (1e-10, 1e-8)])
def test_penny_gmres_matches_dense_lu(c1, aca_tol, bar):
    hm = _hm()
    m, E, _ = c1
    act, b = _penny_system(m)
    x_ref = oracle.solve_dense(oracle.tangent_dense(E, None, act), b)[0]
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, aca_tol=aca_tol)
    op.set_tangent(None, cuda(act, torch.uint8))
    x, rep = op.solve(cuda(b), rtol=1e-12, restart=50, max_iter=400)
    x = x.cpu().numpy()
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    print(f"penny aca {aca_tol}: its {rep['iterations']} relres {rep['rel_residual']:.2e} err vs LU {err:.2e}")
    assert rep["converged"] and err <= bar
    hist = np.array(rep["history"])
    assert np.all(np.diff(hist) <= 1e-12 * hist[0] + 1e-300)   # GMRES residual never increases


def test_refinement_mixed_precision_reaches_1e8(c1):
    hm = _hm()
    m, E, _ = c1
    act, b = _penny_system(m)
    x_ref = oracle.solve_dense(oracle.tangent_dense(E, None, act), b)[0]
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=1, far_prec=2,
                     keep_f64_reference=1)
    op.set_tangent(None, cuda(act, torch.uint8))
    x, rep = op.solve(cuda(b), rtol=1e-8, refine=1, inner_rtol=1e-3, max_iter=400)
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    print(f"mixed+refine: sweeps {rep['refinements']} its {rep['iterations']} relres {rep['rel_residual']:.2e} err {err:.2e}")
    assert rep["converged"] and rep["rel_residual"] <= 1e-8 and err <= 1e-6


def test_solve_batched_columns_ragged_grid():
    hm = _hm()
    # six right-hand sides advance in lock-step; each must converge on its own
    m = rect_grid(20, 11, 1.0)
    E = oracle.dense(m, YOUNG, NU)
    B = rhs_columns(m.ndof, 6, 300)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=16, aca_tol=1e-10)
    X, rep = op.solve(cuda(B), rtol=1e-10, restart=30, max_iter=600)
    X_ref = oracle.solve_dense(E, B)
    assert rep["converged"] and colerr(X.cpu().numpy(), X_ref) <= 1e-7


# ---------------------------------------------------------------- full size
def test_primary_configuration_sampled_rows():
    """256 x 256 squares, leaf 64, eta 2, ACA 1e-6, 16 right-hand sides: the
    launch configuration of the benchmark; exact rows sampled by the oracle."""
    hm = _hm()
    m = square_fault(256)
    X = rhs_columns(m.ndof, 16, 2001)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, aca_tol=1e-6, near_prec=1, far_prec=1,
                     keep_f64_reference=1)
    rng = np.random.default_rng(2)
    rows = np.unique(np.concatenate([[0, 255, 32640, 65535], rng.choice(m.ne, 124, replace=False)]))
    dof = (3 * rows[:, None] + np.arange(3)).ravel()
    ref = oracle.rows_matvec(m, YOUNG, NU, rows, X)
    Xd = cuda(X)
    y32 = op.apply(Xd).cpu().numpy()[:, dof]
    y64 = op.apply(Xd, reference=True).cpu().numpy()[:, dof]
    e32, e64 = colerr(y32, ref), colerr(y64, ref)
    st = op.stats()
    print(f"256x256: FP64 {e64:.3e} FP32 {e32:.3e}; ranks {st['min_rank']}..{st['max_rank']} mean {st['mean_rank']:.1f};"
          f" build {st['build_ms']:.0f} ms (coef {st['coef_ms']:.0f}, aca {st['aca_ms']:.0f}, pack {st['pack_ms']:.0f})")
    assert e64 <= 1e-6 and e32 <= 1e-5
