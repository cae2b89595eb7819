"""Host-side logic of the library and its C boundary (no GPU needed).

* the shared library loads and exports every function include/hmdd.h declares;
* mesh validation errors and the element-frame convention;
* the cluster/block tree against an independent Python construction of the
  same rules (median bisection, vertex-box admissibility), and the
  partition property: every (receiver, source) element pair is covered by
  exactly one block.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2605_14397_amd as hm
from workloads import disk_mesh, rect_grid, square_fault

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "hmdd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = hm.lib()
    declared = _declared_functions()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(hm.EXPORTS) == declared
    assert L.hm_version().decode().startswith("hmdd")


def test_abi_check_accepts_the_mirrors_and_names_a_mismatch():
    import ctypes
    L = hm.lib()            # loading already ran the check with the binding's mirrors
    mirrors = (hm.PlanInfo, hm.BuildOpts, hm.OpStats, hm.BatchOpts, hm.BatchInfo, hm.SolveOpts, hm.SolveReport,
               hm.InterfaceMaterial, hm.NewtonOpts, hm.NewtonReport, hm.FlowParams, hm.CoupledOpts,
               hm.CoupledReport, hm.TimestepOpts)
    sizes = [ctypes.sizeof(m) for m in mirrors]
    arr = (ctypes.c_size_t * len(sizes))(*sizes)
    assert L.hm_abi_check(len(sizes), arr) == hm.HM_OK
    arr[6] -= 8             # a report struct from an older header
    assert L.hm_abi_check(len(sizes), arr) == hm.HM_EINVAL
    assert "hm_solve_report" in L.hm_last_error().decode()
    assert L.hm_abi_check(len(sizes) - 1, arr) == hm.HM_EINVAL
    assert L.hm_abi_check(len(sizes), None) == hm.HM_EINVAL


def test_mesh_validation_errors():
    tri = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], float)
    with pytest.raises(hm.HMError) as e:
        hm.Mesh(tri, np.array([[0, 1, 2]]))
    assert e.value.status == hm.HM_EBADMESH
    quad = np.array([[0, 0, 0], [1, 0, 0], [1.2, 1, 0], [0, 1, 0]], float)
    with pytest.raises(hm.HMError) as e:
        hm.Mesh(quad, np.array([[0, 1, 2, 3]]))
    assert e.value.status == hm.HM_EBADMESH
    warped = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0.01], [0, 1, 0]], float)
    with pytest.raises(hm.HMError) as e:
        hm.Mesh(warped, np.array([[0, 1, 2, 3]]))
    assert e.value.status == hm.HM_EBADMESH
    with pytest.raises(hm.HMError) as e:
        hm.Mesh(tri, np.array([[0, 1, 5]]))
    assert e.value.status == hm.HM_EINVAL
    with pytest.raises(hm.HMError) as e:
        hm.Mesh(tri, np.zeros((1, 2), dtype=np.int64))
    assert e.value.status == hm.HM_EINVAL


def test_error_message_is_thread_local_and_cleared():
    with pytest.raises(hm.HMError):
        hm.Mesh(np.zeros((3, 3)), np.array([[0, 1, 2]]))
    assert "degenerate" in hm.lib().hm_last_error().decode()
    hm.Mesh(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float), np.array([[0, 1, 2]]))
    assert hm.lib().hm_last_error().decode() == ""


@pytest.mark.parametrize("make", [lambda: square_fault(8), lambda: disk_mesh(5.0, 6),
                                  lambda: rect_grid(5, 3, 0.7, 1.3, axes=np.array([[0, 0.6, 0.8], [1, 0, 0], [0, 0.8, -0.6]]))],
                         ids=["square", "disk", "tilted_rect"])
def test_frames_follow_the_stated_convention(make):
    m = make()
    c, f, a = hm.Mesh.from_workload(m).frames()
    c2, f2, a2 = oracle.frames(m)
    assert np.allclose(c, c2, atol=1e-14) and np.allclose(f, f2, atol=1e-14) and np.allclose(a, a2, rtol=1e-14)
    assert np.allclose(np.einsum("nij,nkj->nik", f, f), np.eye(3), atol=1e-14)   # orthonormal rows
    assert np.allclose(np.linalg.det(f), 1.0)                                     # right-handed


# ---------------------------------------------------------------- planner
def _py_plan(m, leaf, eta):
    """Independent construction of the same cluster and block trees."""
    cent = m.vertex_means()
    v = m.xyz[m.conn]
    vmin, vmax = v.min(axis=1), v.max(axis=1)
    nodes = []

    def build(idx):
        nid = len(nodes)
        nodes.append(None)
        box = (vmin[idx].min(0), vmax[idx].max(0))
        if len(idx) > leaf:
            ext = cent[idx].max(0) - cent[idx].min(0)
            ax = int(np.argmax(ext))
            order = np.lexsort((idx, cent[idx, ax]))
            idx = idx[order]
            h = len(idx) // 2
            a = build(idx[:h])
            b = build(idx[h:])
            nodes[nid] = (idx, box, (a, b))
        else:
            nodes[nid] = (np.sort(idx) if False else idx, box, None)
        return nid

    build(np.arange(m.ne))

    def diam(b):
        return np.linalg.norm(b[1] - b[0])

    def dist(a, b):
        g = np.maximum(0, np.maximum(a[0] - b[1], b[0] - a[1]))
        return np.linalg.norm(g)

    dense, lr = [], []

    def blocks(t, s):
        bt, bs = nodes[t][1], nodes[s][1]
        d = dist(bt, bs)
        if d > 0 and min(diam(bt), diam(bs)) <= eta * d:
            lr.append((t, s))
            return
        ct, cs = nodes[t][2], nodes[s][2]
        if ct is None and cs is None:
            dense.append((t, s))
        elif ct is None:
            blocks(t, cs[0]); blocks(t, cs[1])
        elif cs is None:
            blocks(ct[0], s); blocks(ct[1], s)
        else:
            for i in ct:
                for j in cs:
                    blocks(i, j)

    blocks(0, 0)
    return nodes, dense, lr


@pytest.mark.parametrize("make,leaf", [(lambda: square_fault(16), 8), (lambda: disk_mesh(10.0, 9), 16),
                                       (lambda: rect_grid(23, 7, 1.0), 5)], ids=["square16", "disk", "ragged_rect"])
def test_plan_matches_independent_construction(make, leaf):
    m = make()
    info, perm = hm.Mesh.from_workload(m).plan(leaf, 2.0, want_perm=True)
    nodes, dense, lr = _py_plan(m, leaf, 2.0)
    leaves = [n for n in nodes if n[2] is None]
    assert info["n_leaves"] == len(leaves)
    assert info["n_dense_blocks"] == len(dense)
    assert info["n_lowrank_blocks"] == len(lr)
    assert info["dense_entries"] == sum(9 * len(nodes[t][0]) * len(nodes[s][0]) for t, s in dense)
    assert info["lowrank_sum_mn"] == sum(len(nodes[t][0]) + len(nodes[s][0]) for t, s in lr)
    assert np.array_equal(np.sort(perm), np.arange(m.ne))
    assert np.array_equal(perm, np.concatenate([n[0] for n in leaves]))
    assert info["max_leaf"] <= leaf
    # partition: every element pair lies in exactly one block
    cover = np.zeros((m.ne, m.ne), dtype=np.int32)
    for t, s in dense + lr:
        cover[np.ix_(nodes[t][0], nodes[s][0])] += 1
    assert np.all(cover == 1)


def test_plan_counts_primary_configuration():
    # 256 x 256 squares, leaf 64, eta 2: 1,024 leaves of 8 x 8 elements
    info = hm.Mesh.from_workload(square_fault(256)).plan(64, 2.0)
    assert info["n_leaves"] == 1024 and info["max_leaf"] == info["min_leaf"] == 64 and info["depth"] == 10
    assert info["n_dense_blocks"] == 8836
    assert info["dense_entries"] == 8836 * 192 * 192
    assert info["n_lowrank_blocks"] == 26652
    assert info["lowrank_by_level"][3] == 8 and info["lowrank_by_level"][10] == 19500


def test_plan_rejects_bad_options():
    M = hm.Mesh.from_workload(square_fault(4))
    with pytest.raises(hm.HMError):
        M.plan(65, 2.0)
    with pytest.raises(hm.HMError):
        M.plan(16, -1.0)


def test_structs_match_c_layout(tmp_path):
    """Every struct the binding passes by pointer has the size and field
    offsets that a C compiler gives the declarations in include/hmdd.h."""
    import subprocess

    pairs = [("hm_solve_report", hm.SolveReport), ("hm_solve_opts", hm.SolveOpts),
             ("hm_build_opts", hm.BuildOpts), ("hm_op_stats", hm.OpStats), ("hm_batch_opts", hm.BatchOpts),
             ("hm_batch_info", hm.BatchInfo), ("hm_plan_info", hm.PlanInfo),
             ("hm_interface_material", hm.InterfaceMaterial), ("hm_newton_opts", hm.NewtonOpts),
             ("hm_newton_report", hm.NewtonReport), ("hm_timestep_opts", hm.TimestepOpts),
             ("hm_flow_params", hm.FlowParams), ("hm_coupled_opts", hm.CoupledOpts),
             ("hm_coupled_report", hm.CoupledReport)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hmdd.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in pairs:
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_timestep_controller_follows_the_printed_formula():
    """The step-size controller (paper Sec. 3.4) on the host: its fixed point,
    the exponents of each factor, the growth cap and the bounds."""
    eps = 1e-3
    fl = np.sqrt(np.finfo(np.float64).eps)
    nxt = lambda *a, **k: hm.timestep_next(*a, eps_tol=eps, n_target=6, growth_max=10.0, **k)
    e_fix = eps - fl      # e + sqrt(machine epsilon) = eps
    assert nxt(2.0, 2.0, e_fix, e_fix, 6) == pytest.approx(2.0, rel=1e-14)
    e_half = 0.5 * eps - fl
    assert nxt(2.0, 2.0, e_half, e_fix, 6) == pytest.approx(2.0 * 2 ** 0.25, rel=1e-13)
    assert nxt(2.0, 2.0, e_fix, e_half, 6) == pytest.approx(2.0 * 2 ** 0.25, rel=1e-13)
    assert nxt(2.0, 1.0, e_fix, e_fix, 6) == pytest.approx(2.0 * 2 ** -0.25, rel=1e-13)
    assert nxt(2.0, 2.0, e_fix, e_fix, 12) == pytest.approx(2.0 * 2 ** (-1 / 3), rel=1e-13)
    # first step: no previous step, no previous error
    assert nxt(2.0, 0.0, e_fix, 0.0, 6) == pytest.approx(2.0, rel=1e-14)
    # growth cap and bounds
    assert hm.timestep_next(1.0, 1.0, 0.0, 0.0, 1, eps_tol=eps, growth_max=1.2) == pytest.approx(1.2)
    assert hm.timestep_next(1.0, 1.0, 10.0, 0.0, 50, dt_min=0.5) == 0.5
    assert hm.timestep_next(1.0, 1.0, 0.0, 0.0, 1, growth_max=100.0, dt_max=3.0) == 3.0
    with pytest.raises(hm.HMError, match="unknown"):
        hm.timestep_next(1.0, 1.0, 1e-3, 1e-3, 6, eps=1e-3)
    with pytest.raises(hm.HMError):
        hm.timestep_next(0.0, 1.0, 1e-3, 1e-3, 6)
    with pytest.raises(hm.HMError):
        hm.timestep_next(1.0, 1.0, 1e-3, 1e-3, 0)


def test_interface_inputs_are_seeded_and_consistent():
    """The seeded interface states: reproducible, every regime drawn, the
    internal variables at or above the current inelastic DD (they are
    maxima over the history), materials inside the library's bounds."""
    from workloads.interface import injection_path, injection_pressure, interface_materials, interface_states

    mats = interface_materials()
    assert (mats[:, 6] >= mats[:, 2] * mats[:, 7]).all() and (mats[:, 0] > 0).all() and (mats[:, 1] > 0).all()
    a, b = interface_states(500, 11, mats), interface_states(500, 11, mats)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    st = a
    assert st["dd"].shape == (500, 3) and st["mat_id"].dtype == np.int32
    assert set(np.unique(st["mat_id"])) == {0, 1, 2}
    assert (st["chi"][:, 0] >= np.hypot(st["dp"][:, 0], st["dp"][:, 1]) * (1 - 1e-15)).all()
    assert (st["chi"][:, 1] >= np.linalg.norm(st["dp"], axis=1) * (1 - 1e-15)).all()
    m = square_fault(12)
    p = injection_path(m, 5)
    assert len(p["dd"]) == 5 and p["t"].shape == (m.ne, 3)
    assert np.array_equal(injection_pressure(m, -1, 5), np.zeros(m.ne))
    assert (injection_pressure(m, 4, 5) >= injection_pressure(m, 3, 5)).all()


def test_unknown_options_are_rejected():
    """A misspelt option name raises instead of being silently ignored."""
    with pytest.raises(hm.HMError, match="unknown build option"):
        hm.build_opts(leafsize=32)
    with pytest.raises(hm.HMError, match="unknown solve option"):
        hm.solve_opts(precon=hm.HM_PC_LEAF)
    assert hm.solve_opts(precond=hm.HM_PC_LEAF).precond == hm.HM_PC_LEAF


def test_scale_update_matches_the_oracle():
    """The scale update of Sec. 3.3.2 on the host against the oracle's
    restatement, on seeded inputs spanning both clips and the open range."""
    from oracle import timestep as OT

    rng = np.random.default_rng(77)
    for _ in range(200):
        old = 10 ** rng.uniform(-6, 6)
        new = old * 10 ** rng.uniform(-1, 1)
        a, lo, hi = rng.uniform(0, 1), rng.uniform(0.5, 1.0), rng.uniform(1.0, 2.0)
        assert hm.scale_update(old, new, a, lo, hi) == pytest.approx(OT.scale_update(old, new, a, lo, hi), rel=1e-15)
    for bad in ((0.0, 1.0, 0.5, 0.8, 1.2), (1.0, -1.0, 0.5, 0.8, 1.2), (1.0, 1.0, 1.5, 0.8, 1.2),
                (1.0, 1.0, 0.5, 1.1, 1.2), (1.0, 1.0, 0.5, 0.8, 0.9)):
        with pytest.raises(hm.HMError):
            hm.scale_update(*bad)
