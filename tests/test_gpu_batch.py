"""GPU parity of the batched form: many independent planar faults (seeded
sizes, aspect ratios and orientations) applied by merged launches captured
as one HIP graph.

* each operator's columns from the batch equal its own single product bit
  for bit (same kernels, same task lists, fixed summation order);
* every operator matches the oracle's exact dense product (FP64 form bar
  1e-6, FP32 form 1e-5, FP32 near + BF16 far form 5e-3; ACA 1e-6);
* graph replays interleaved with eager products and new vector pointers
  give the same result every time.
"""
import numpy as np
import pytest

import oracle
from workloads import batched_faults, rhs_columns

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YOUNG, NU = 30e9, 0.25


def _hm():
    import paper_2605_14397_amd as hm

    assert torch.cuda.is_available()
    return hm


def colerr(Y, R):
    return max(np.linalg.norm(Y[c] - R[c]) / np.linalg.norm(R[c]) for c in range(R.shape[0]))


@pytest.fixture(scope="module")
def small_faults():
    # same generator as the 64-mesh workload, small element counts
    return batched_faults(n_meshes=7, seed=4001, nmin=300, nmax=1500)


@pytest.mark.parametrize("near,far,bar", [(0, 0, 1e-6), (1, 1, 1e-5), (1, 2, 5e-3)], ids=["fp64", "fp32", "mixed"])
def test_batch_equals_single_products_and_oracle(small_faults, near, far, bar):
    hm = _hm()
    ops = [hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=near, far_prec=far)
           for m in small_faults]
    batch = hm.Batch(ops, use_graph=True, autotune=True)
    info = batch.info()
    assert info["n_ops"] == len(ops) and info["leaves_per_task_a"] in info["tune_candidates"]
    assert info["phase_b_window"] in info["tune_b_candidates"] and min(info["tune_b_ms"]) > 0
    nrhs = 5
    Xs = [torch.as_tensor(rhs_columns(m.ndof, nrhs, 4101 + k), device="cuda") for k, m in enumerate(small_faults)]
    Ys = [torch.empty_like(x) for x in Xs]
    batch.apply(Xs, Ys)
    torch.cuda.synchronize()
    for k, (m, op) in enumerate(zip(small_faults, ops)):
        single = op.apply(Xs[k]).cpu().numpy()
        got = Ys[k].cpu().numpy()
        assert np.array_equal(got, single), k
        err = colerr(got, oracle.matvec(oracle.dense(m, YOUNG, NU), Xs[k].cpu().numpy()))
        assert err <= bar, (k, err)


def test_graph_replays_with_eager_work_and_new_pointers(small_faults):
    hm = _hm()
    ops = [hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=1, far_prec=1)
           for m in small_faults[:4]]
    batch = hm.Batch(ops, use_graph=True, autotune=False)
    Xs = [torch.as_tensor(rhs_columns(op.ndof, 16, 77 + k), device="cuda") for k, op in enumerate(ops)]
    ref = [op.apply(x).clone() for op, x in zip(ops, Xs)]
    for rep in range(4):
        Ys = [torch.full_like(x, float("nan")) for x in Xs]    # fresh pointers every replay
        batch.apply(Xs, Ys)
        torch.cuda.synchronize()
        for y, r in zip(Ys, ref):
            assert torch.equal(y, r), rep
        # eager work between replays
        _ = [op.apply(x) for op, x in zip(ops, Xs)]
        torch.cuda.synchronize()
    # fewer columns: a new graph for the new width
    Xs2 = [x[:3].contiguous() for x in Xs]
    Ys2 = [torch.empty_like(x) for x in Xs2]
    batch.apply(Xs2, Ys2)
    torch.cuda.synchronize()
    for y, r in zip(Ys2, ref):
        assert torch.equal(y, r[:3])


def test_batch_rejects_mixed_precision_forms(small_faults):
    hm = _hm()
    a = hm.Operator(hm.Mesh.from_workload(small_faults[0]), YOUNG, NU, leaf_size=32)
    b = hm.Operator(hm.Mesh.from_workload(small_faults[1]), YOUNG, NU, leaf_size=32, near_prec=1, far_prec=1)
    with pytest.raises(hm.HMError) as e:
        hm.Batch([a, b])
    assert e.value.status == hm.HM_EUNSUPPORTED


def test_full_size_batch_sampled_rows():
    """The timed batched configuration (64 faults, 2k-40k elements, FP32,
    leaf 64, eta 2, ACA 1e-6, graph-captured, autotuned, 16 columns): the
    largest, the smallest and four seeded meshes equal their own single
    products bit for bit and match 32 exact rows each from the oracle
    (FP32 bar 1e-5); a second graph replay repeats the first bit for bit;
    all 64 meshes match the exact Toeplitz product at every row (1e-5)."""
    hm = _hm()
    meshes = batched_faults(n_meshes=64, seed=4001)
    ops = [hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6,
                       near_prec=hm.HM_F32, far_prec=hm.HM_F32) for m in meshes]
    batch = hm.Batch(ops, use_graph=True, autotune=True)
    Xs = [torch.as_tensor(rhs_columns(m.ndof, 16, 4101 + 100 * k), device="cuda") for k, m in enumerate(meshes)]
    Ys = [torch.empty_like(x) for x in Xs]
    batch.apply(Xs, Ys)
    first = [y.cpu().numpy() for y in Ys]
    batch.apply(Xs, Ys)
    torch.cuda.synchronize()
    sizes = np.array([m.ne for m in meshes])
    rng = np.random.default_rng(4202)
    picks = [int(np.argmax(sizes)), int(np.argmin(sizes))] + rng.choice(64, 4, replace=False).tolist()
    for k in picks:
        got = Ys[k].cpu().numpy()
        assert np.array_equal(got, first[k]), k
        assert np.array_equal(got, ops[k].apply(Xs[k]).cpu().numpy()), k
        rows = np.sort(rng.choice(meshes[k].ne, 32, replace=False))
        dof = (3 * rows[:, None] + np.arange(3)).ravel()
        ref = oracle.rows_matvec(meshes[k], YOUNG, NU, rows, Xs[k][:4].cpu().numpy())
        err = colerr(got[:4, dof], ref)
        print(f"mesh {k} ({meshes[k].ne} elements): sampled FP32 error {err:.2e}", flush=True)
        assert err <= 1e-5, (k, err)
    assert all(np.array_equal(Ys[k].cpu().numpy(), first[k]) for k in range(64))
    # every row of every mesh: each fault is a uniform grid of unit squares
    # in one plane and frame, so its exact operator is the oracle's Toeplitz
    # sum (FFT route), in the mesh's own frame whatever its orientation
    worst = 0.0
    for k, m in enumerate(meshes):
        nx, ny = m.meta["nx"], m.meta["ny"]
        ref = oracle.grid_matvec_fft(oracle.grid_table(YOUNG, NU, nx, ny), nx, ny, Xs[k].cpu().numpy())
        err = colerr(first[k], ref)
        worst = max(worst, err)
        assert err <= 1e-5, (k, err)
    print(f"64 meshes, every row: worst FP32 per-column error {worst:.2e}", flush=True)


def test_batches_with_few_tasks_and_empty_phases():
    """Queue-driven launches with fewer tasks than XCD ranges or resident
    workgroups: a batch of one all-dense operator (no phase-A task), one of
    a single small operator and one mixing both, each replayed twice, equal
    bit for bit to the operators' own products."""
    from workloads import square_fault

    hm = _hm()
    meshes = [square_fault(4), square_fault(24), square_fault(10)]
    ops = [hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=32, near_prec=1, far_prec=1) for m in meshes]
    assert ops[0].stats()["phase_a_tasks"] == 0 and ops[1].stats()["phase_a_tasks"] > 0
    for sel in ([0], [1], [0, 1, 2]):
        batch = hm.Batch([ops[k] for k in sel], use_graph=True, autotune=False)
        for nrhs in (1, 16):
            Xs = [torch.as_tensor(rhs_columns(meshes[k].ndof, nrhs, 4300 + k), device="cuda") for k in sel]
            singles = [ops[k].apply(x).cpu().numpy() for k, x in zip(sel, Xs)]
            for _ in range(2):
                Ys = [torch.full_like(x, float("nan")) for x in Xs]
                batch.apply(Xs, Ys)
                torch.cuda.synchronize()
                for j in range(len(sel)):
                    assert np.array_equal(Ys[j].cpu().numpy(), singles[j]), (sel, nrhs, j)
        del batch
