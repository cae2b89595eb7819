"""hm_operator_apply_noalloc (the product with its workspace in the
library's fixed device array) against hm_operator_apply, called through the
C ABI: two calls in a row, the second on a smaller operator with fewer
columns, each bit for bit equal to the allocating entry point (the same
kernels, task lists and summation order run in both); the tangent and
accumulate flags; the FP64 reference copy; and an operator whose workspace
exceeds the array is rejected before anything runs."""
import ctypes

import numpy as np
import pytest

from workloads import rect_grid, rhs_columns, square_fault

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available()
    return hm


def _raw_noalloc(hm, op, X, Y, flags=0):
    """Direct C-ABI call (no binding helper in between)."""
    f = hm.lib().hm_operator_apply_noalloc
    return f(op._h, X.shape[0], ctypes.c_void_p(X.data_ptr()), X.stride(0), ctypes.c_void_p(Y.data_ptr()),
             Y.stride(0), flags, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_allocating_apply_two_calls():
    hm = _hm()
    big = square_fault(96)
    small = rect_grid(37, 19, 1.0, 0.8)
    op_big = hm.Operator(hm.Mesh.from_workload(big), YOUNG, NU, leaf_size=64, near_prec=hm.HM_F32,
                         far_prec=hm.HM_BF16, keep_f64_reference=1)
    op_small = hm.Operator(hm.Mesh.from_workload(small), YOUNG, NU, leaf_size=32)
    assert op_small.stats()["apply_workspace_bytes"] < op_big.stats()["apply_workspace_bytes"]
    # first call: the larger operator, 16 columns
    Xb = torch.as_tensor(rhs_columns(big.ndof, 16, 71), device="cuda")
    Yb = torch.full_like(Xb, float("nan"))
    assert _raw_noalloc(hm, op_big, Xb, Yb) == hm.HM_OK
    torch.cuda.synchronize()
    assert torch.equal(Yb, op_big.apply(Xb))
    # second call: a smaller operator and fewer columns; the array still
    # holds the first call's contents
    Xs = torch.as_tensor(rhs_columns(small.ndof, 5, 72), device="cuda")
    Ys = torch.full_like(Xs, float("nan"))
    assert _raw_noalloc(hm, op_small, Xs, Ys) == hm.HM_OK
    torch.cuda.synchronize()
    assert torch.equal(Ys, op_small.apply(Xs))
    # the FP64 reference copy, then the mixed form again
    Yr = torch.empty_like(Xb)
    assert _raw_noalloc(hm, op_big, Xb, Yr, hm.HM_APPLY_REFERENCE) == hm.HM_OK
    assert torch.equal(Yr, op_big.apply(Xb, reference=True))
    Yb2 = torch.empty_like(Xb)
    assert _raw_noalloc(hm, op_big, Xb, Yb2) == hm.HM_OK
    torch.cuda.synchronize()
    assert torch.equal(Yb2, Yb)


def test_noalloc_tangent_accumulate_and_limits():
    hm = _hm()
    m = rect_grid(30, 22, 1.0)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32)
    rng = np.random.default_rng(73)
    D = torch.as_tensor(rng.standard_normal((m.ne, 3, 3)) * 1e9, device="cuda")
    mask = torch.as_tensor((rng.random(m.ne) > 0.2).astype(np.uint8), device="cuda")
    op.set_tangent(D, mask)
    X = torch.as_tensor(rhs_columns(m.ndof, 3, 74), device="cuda")
    Y0 = torch.as_tensor(rhs_columns(m.ndof, 3, 75), device="cuda")
    Ya = Y0.clone()
    Yb = Y0.clone()
    op.apply(X, Ya, tangent=True, accumulate=True)
    op.apply_noalloc(X, Yb, tangent=True, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(Ya, Yb)
    # no reference copy, bad flags, too many columns: errors, nothing written
    Yc = torch.full_like(X, 7.0)
    for flags in (64, 128):
        assert _raw_noalloc(hm, op, X, Yc, flags) == hm.HM_EINVAL
    X17 = torch.zeros(17, m.ndof, dtype=torch.float64, device="cuda")
    assert _raw_noalloc(hm, op, X17, torch.zeros_like(X17)) == hm.HM_EINVAL
    torch.cuda.synchronize()
    assert bool((Yc == 7.0).all())


def test_noalloc_rejects_a_workspace_beyond_the_array():
    hm = _hm()
    limit = 256 << 20
    # the 256 x 256 fault in FP64 needs more product workspace than the array
    m = square_fault(256)
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64)
    need = op.stats()["apply_workspace_bytes"]
    print(f"256x256 FP64 product workspace {need / 2**20:.1f} MiB (array {limit / 2**20:.0f} MiB)", flush=True)
    X = torch.zeros(1, m.ndof, dtype=torch.float64, device="cuda")
    Y = torch.full_like(X, 3.0)
    st = _raw_noalloc(hm, op, X, Y)
    if need > limit:
        assert st == hm.HM_EINVAL and "scratch" in hm.lib().hm_last_error().decode()
        torch.cuda.synchronize()
        assert bool((Y == 3.0).all())
    else:
        assert st == hm.HM_OK
        torch.cuda.synchronize()
        assert torch.equal(Y, op.apply(X))
