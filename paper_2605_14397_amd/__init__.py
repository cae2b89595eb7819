"""Python binding of libhmdd (H-matrix DD-BEM operator for MI355X / gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and streams.  The functions keep
the C names (hm_mesh_create, hm_operator_apply, ...); the classes Mesh and
Operator are thin owners of the opaque handles.  If the library is not
built, or no gfx950 device is present, calls raise HMError: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmdd.so")

HM_OK, HM_EINVAL, HM_ENOMEM, HM_EDEVICE, HM_EBADMESH, HM_EUNSUPPORTED, HM_ENOTCONV, HM_EINTERNAL = (
    0, -1, -2, -3, -4, -5, -6, -7)
HM_F64, HM_F32, HM_BF16, HM_BF16_1 = 0, 1, 2, 3
HM_APPLY_REFERENCE, HM_APPLY_TANGENT, HM_APPLY_ACCUMULATE = 1, 2, 4
HM_PC_NONE, HM_PC_JACOBI, HM_PC_BLOCK3, HM_PC_LEARNED, HM_PC_LEAF, HM_PC_ILU = 0, 1, 2, 3, 4, 5
HM_FALLBACK_NONE, HM_FALLBACK_NOT_ATTACHED, HM_FALLBACK_NONFINITE, HM_FALLBACK_NOT_CONVERGED = 0, 1, 2, 3
HM_IF_ELASTIC, HM_IF_SHEAR, HM_IF_TENSILE, HM_IF_CORNER, HM_IF_OPEN, HM_IF_BAD_MATERIAL = 0, 1, 2, 3, 4, -1

_STATUS = {0: "HM_OK", -1: "HM_EINVAL", -2: "HM_ENOMEM", -3: "HM_EDEVICE", -4: "HM_EBADMESH",
           -5: "HM_EUNSUPPORTED", -6: "HM_ENOTCONV", -7: "HM_EINTERNAL"}

# symbols declared in include/hmdd.h
EXPORTS = [
    "hm_last_error", "hm_version", "hm_abi_check", "hm_mesh_create", "hm_mesh_destroy", "hm_mesh_num_elements",
    "hm_mesh_frames", "hm_plan_summary", "hm_kernel_block", "hm_build_opts_default",
    "hm_operator_build", "hm_op_destroy", "hm_operator_stats", "hm_operator_apply", "hm_operator_apply_timed",
    "hm_operator_apply_noalloc",
    "hm_tangent_set",
    "hm_solve_opts_default", "hm_solve", "hm_batch_opts_default", "hm_batch_create", "hm_batch_apply",
    "hm_batch_get_info", "hm_batch_destroy",
    "hm_learned_create", "hm_learned_destroy", "hm_learned_set_base", "hm_learned_num_params",
    "hm_learned_get_params",
    "hm_learned_set_params", "hm_learned_features", "hm_learned_loss_grad", "hm_learned_train",
    "hm_learned_attach", "hm_learned_detach", "hm_precond_apply", "hm_interface_update",
    "hm_newton_opts_default", "hm_newton_step", "hm_timestep_opts_default", "hm_timestep_next",
    "hm_lte_estimate", "hm_flow_create", "hm_flow_destroy", "hm_flow_num_nodes", "hm_flow_nnz",
    "hm_flow_matrices", "hm_coupled_opts_default", "hm_coupled_step", "hm_scale_update",
]
HM_PERM_CUBIC, HM_PERM_CONSTANT = 0, 1


class HMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int), ("eta", ctypes.c_double), ("aca_tol", ctypes.c_double),
                ("max_rank", ctypes.c_int), ("near_prec", ctypes.c_int), ("far_prec", ctypes.c_int),
                ("keep_f64_reference", ctypes.c_int), ("recompress", ctypes.c_int), ("stack_rows", ctypes.c_int),
                ("phase_a_items", ctypes.c_int), ("phase_b_window", ctypes.c_int)]


class OpStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_elements", "n_dof", "n_leaves", "n_dense_blocks", "n_lowrank_blocks", "dense_entries",
        "lowrank_entries", "self_f64_entries", "bytes_near", "bytes_far", "bytes_self", "bytes_reference")] + [
        ("min_rank", ctypes.c_int), ("max_rank", ctypes.c_int), ("mean_rank", ctypes.c_double),
        ("near_prec", ctypes.c_int), ("far_prec", ctypes.c_int), ("build_ms", ctypes.c_double),
        ("coef_ms", ctypes.c_double), ("aca_ms", ctypes.c_double), ("pack_ms", ctypes.c_double),
        ("max_dense_bytes_per_leaf", ctypes.c_int64), ("bytes_far_u", ctypes.c_int64),
        ("bytes_far_v", ctypes.c_int64), ("rank_sum", ctypes.c_int64), ("rank_sum_aca", ctypes.c_int64),
        ("recompress_ms", ctypes.c_double), ("apply_workspace_bytes", ctypes.c_int64),
        ("lowrank_entries_u", ctypes.c_int64), ("dense_entries_stored", ctypes.c_int64),
        ("phase_a_tasks", ctypes.c_int64), ("phase_b_tasks", ctypes.c_int64), ("phase_a_stacks", ctypes.c_int64),
        ("phase_a_partial_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double),
                ("precond", ctypes.c_int), ("refine", ctypes.c_int), ("inner_rtol", ctypes.c_double),
                ("max_refine", ctypes.c_int), ("ilu_fraction", ctypes.c_double)]


class NewtonOpts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("lin", SolveOpts), ("forcing", ctypes.c_int)]


class TimestepOpts(ctypes.Structure):
    _fields_ = [("eps_tol", ctypes.c_double), ("n_target", ctypes.c_int), ("growth_max", ctypes.c_double),
                ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double)]


class NewtonReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("n_history", ctypes.c_int),
                ("residual", ctypes.c_double * 64), ("gmres_iterations", ctypes.c_int * 64),
                ("modes", ctypes.c_int64 * 5), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {"iterations": self.iterations, "converged": bool(self.converged),
                "residual": list(self.residual[:self.n_history]),
                "gmres_iterations": list(self.gmres_iterations[:self.iterations]), "modes": list(self.modes),
                "ms": self.ms}


class SolveReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("refinements", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double), ("n_history", ctypes.c_int),
                ("history", ctypes.c_double * 1024), ("precond_used", ctypes.c_int), ("fallback", ctypes.c_int),
                ("discarded_iterations", ctypes.c_int), ("precond_setup_ms", ctypes.c_double),
                ("precond_nnz", ctypes.c_int64), ("precond_colors", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history"}
        d["history"] = list(self.history[:self.n_history])
        return d


class BatchOpts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int), ("autotune", ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_ops", ctypes.c_int), ("total_elements", ctypes.c_int64), ("use_graph", ctypes.c_int),
                ("leaves_per_task_a", ctypes.c_int), ("tune_candidates", ctypes.c_int * 5),
                ("tune_ms", ctypes.c_double * 5), ("bytes_operators", ctypes.c_int64),
                ("phase_b_window", ctypes.c_int), ("tune_b_candidates", ctypes.c_int * 3),
                ("tune_b_ms", ctypes.c_double * 3)]


class FlowParams(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("mu", ctypes.c_double), ("perm_law", ctypes.c_int), ("k0", ctypes.c_double)]


class CoupledOpts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("scales", ctypes.c_double * 4), ("outer_restart", ctypes.c_int), ("outer_max_iter", ctypes.c_int),
                ("outer_rtol", ctypes.c_double), ("inner", SolveOpts), ("schur", ctypes.c_int),
                ("schur_rtol", ctypes.c_double), ("schur_max_iter", ctypes.c_int)]


class CoupledReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("n_history", ctypes.c_int),
                ("residual", ctypes.c_double * 64), ("residual_mech", ctypes.c_double * 64),
                ("residual_flow", ctypes.c_double * 64), ("outer_iterations", ctypes.c_int * 64),
                ("inner_iterations", ctypes.c_int * 64), ("modes", ctypes.c_int64 * 5), ("ms", ctypes.c_double),
                ("schur_iterations", ctypes.c_int * 64)]

    def as_dict(self):
        n, k = self.n_history, self.iterations
        return {"iterations": k, "converged": bool(self.converged), "residual": list(self.residual[:n]),
                "residual_mech": list(self.residual_mech[:n]), "residual_flow": list(self.residual_flow[:n]),
                "outer_iterations": list(self.outer_iterations[:k]), "inner_iterations": list(self.inner_iterations[:k]),
                "schur_iterations": list(self.schur_iterations[:k]),
                "modes": list(self.modes), "ms": self.ms}


class InterfaceMaterial(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "k_s", "k_n", "f_peak", "f_res", "psi_peak", "d_c", "c_peak", "sigma_peak", "w_c")]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_leaves", "n_dense_blocks", "n_lowrank_blocks", "dense_entries", "lowrank_sum_mn", "max_leaf",
        "min_leaf")] + [("depth", ctypes.c_int), ("lowrank_by_level", ctypes.c_int64 * 64)]


_lib = None


def lib():
    """Load libhmdd.so (raises HMError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HMError(HM_EDEVICE, f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I, D, U = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint
        sig = {
            "hm_last_error": ([], ctypes.c_char_p),
            "hm_version": ([], ctypes.c_char_p),
            "hm_abi_check": ([I, P], I),
            "hm_mesh_create": ([I, I64, P, I64, P, ctypes.POINTER(P)], I),
            "hm_mesh_destroy": ([P], None),
            "hm_mesh_num_elements": ([P], I64),
            "hm_mesh_frames": ([P, P, P, P], I),
            "hm_plan_summary": ([P, I, D, ctypes.POINTER(PlanInfo), P], I),
            "hm_kernel_block": ([P, D, D, I64, P, I64, P, P, P], I),
            "hm_build_opts_default": ([ctypes.POINTER(BuildOpts)], None),
            "hm_operator_build": ([P, D, D, ctypes.POINTER(BuildOpts), P, ctypes.POINTER(P)], I),
            "hm_op_destroy": ([P], None),
            "hm_operator_stats": ([P, ctypes.POINTER(OpStats)], I),
            "hm_operator_apply": ([P, I, P, I64, P, I64, U, P], I),
            "hm_operator_apply_timed": ([P, I, P, I64, P, I64, U, P, P], I),
            "hm_operator_apply_noalloc": ([P, I, P, I64, P, I64, U, P], I),
            "hm_tangent_set": ([P, P, P, P], I),
            "hm_solve_opts_default": ([ctypes.POINTER(SolveOpts)], None),
            "hm_solve": ([P, ctypes.POINTER(SolveOpts), I, P, I64, P, I64, ctypes.POINTER(SolveReport), P], I),
            "hm_batch_opts_default": ([ctypes.POINTER(BatchOpts)], None),
            "hm_batch_create": ([I, ctypes.POINTER(P), ctypes.POINTER(BatchOpts), P, ctypes.POINTER(P)], I),
            "hm_batch_apply": ([P, I, ctypes.POINTER(P), P, ctypes.POINTER(P), P, P], I),
            "hm_batch_get_info": ([P, ctypes.POINTER(BatchInfo)], I),
            "hm_batch_destroy": ([P], None),
            "hm_learned_create": ([I, I, ctypes.c_uint64, ctypes.POINTER(P)], I),
            "hm_learned_destroy": ([P], None),
            "hm_learned_set_base": ([P, I], I),
            "hm_learned_num_params": ([P, ctypes.POINTER(I64)], I),
            "hm_learned_get_params": ([P, P, I64], I),
            "hm_learned_set_params": ([P, P, I64], I),
            "hm_learned_features": ([P, I, I64, ctypes.POINTER(I64), P, P, P, P, P], I),
            "hm_learned_loss_grad": ([P, P, I, P, I64, P, I64, ctypes.POINTER(D), P, P], I),
            "hm_learned_train": ([P, P, I, P, I64, P, I64, I, I, D, P, P], I),
            "hm_learned_attach": ([P, P, P], I),
            "hm_learned_detach": ([P], None),
            "hm_precond_apply": ([P, I, I, P, I64, P, I64, P], I),
            "hm_interface_update": ([I, P, I64, P, P, P, P, P, P, P, P, P, P, P, P, P], I),
            "hm_newton_opts_default": ([ctypes.POINTER(NewtonOpts)], None),
            "hm_timestep_opts_default": ([ctypes.POINTER(TimestepOpts)], None),
            "hm_timestep_next": ([ctypes.POINTER(TimestepOpts), D, D, D, D, I, ctypes.POINTER(D)], I),
            "hm_lte_estimate": ([I64, P, D, P, D, P, ctypes.POINTER(D), P], I),
            "hm_newton_step": ([P, I, P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.POINTER(NewtonOpts),
                                ctypes.POINTER(NewtonReport), P], I),
            "hm_flow_create": ([P, ctypes.POINTER(FlowParams), P, ctypes.POINTER(P)], I),
            "hm_flow_destroy": ([P], None),
            "hm_flow_num_nodes": ([P], I64),
            "hm_flow_nnz": ([P], I64),
            "hm_flow_matrices": ([P, P, P, P, P, P, P], I),
            "hm_coupled_opts_default": ([ctypes.POINTER(CoupledOpts)], None),
            "hm_coupled_step": ([P, P, I, P, P, P, P, P, P, P, P, P, P, P, P, P, D, P, P, P, P, P,
                                 ctypes.POINTER(CoupledOpts), ctypes.POINTER(CoupledReport), P], I),
            "hm_scale_update": ([D, D, D, D, D, ctypes.POINTER(D)], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        # the ctypes mirrors below must have the header's layout, else the
        # library would write past the end of a report
        mirrors = (PlanInfo, BuildOpts, OpStats, BatchOpts, BatchInfo, SolveOpts, SolveReport, InterfaceMaterial,
                   NewtonOpts, NewtonReport, FlowParams, CoupledOpts, CoupledReport, TimestepOpts)
        sizes = (ctypes.c_size_t * len(mirrors))(*[ctypes.sizeof(m) for m in mirrors])
        if L.hm_abi_check(len(mirrors), sizes) != HM_OK:
            raise HMError(HM_EINVAL, "binding and library disagree: " + L.hm_last_error().decode())
        _lib = L
    return _lib


def _check(status: int):
    if status != HM_OK:
        raise HMError(status, lib().hm_last_error().decode())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ld(t):
    """Leading dimension of a [rows, n] block of vectors (rows contiguous)."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise HMError(HM_EINVAL, "expected a 2-D tensor with contiguous rows")
    return t.shape[1] if t.shape[0] == 1 else t.stride(0)


def _shape(t, shape, name):
    """Raise HMError unless tensor t has exactly the given shape (checked
    before anything is launched: the C ABI cannot see buffer sizes)."""
    if tuple(t.shape) != tuple(shape):
        raise HMError(HM_EINVAL, f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


def _vecs(t, n, name, rows=None):
    """A [rows, n] block of vectors (rows contiguous) with n = 3N."""
    if t.dim() != 2 or t.shape[1] != n or (rows is not None and t.shape[0] != rows):
        want = f"[{rows if rows is not None else 'nrhs'}, {n}]"
        raise HMError(HM_EINVAL, f"{name}: expected shape {want}, got {tuple(t.shape)}")


def _dev_ptr(t, dtype):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype):
        raise HMError(HM_EINVAL, f"expected a CUDA tensor of {dtype}")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- handles
class Mesh:
    """Owner of an hm_mesh handle (host-side geometry)."""

    def __init__(self, xyz, conn):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int64)
        h = ctypes.c_void_p()
        _check(lib().hm_mesh_create(conn.shape[1], xyz.shape[0], xyz.ctypes.data, conn.shape[0], conn.ctypes.data,
                                    ctypes.byref(h)))
        self._h = h
        self.ne = conn.shape[0]
        self.ndof = 3 * self.ne

    @classmethod
    def from_workload(cls, m):
        return cls(m.xyz, m.conn)

    def frames(self):
        cent = np.empty((self.ne, 3))
        fr = np.empty((self.ne, 3, 3))
        area = np.empty(self.ne)
        _check(lib().hm_mesh_frames(self._h, cent.ctypes.data, fr.ctypes.data, area.ctypes.data))
        return cent, fr, area

    def plan(self, leaf_size=64, eta=2.0, want_perm=False):
        info = PlanInfo()
        perm = np.empty(self.ne, dtype=np.int64) if want_perm else None
        _check(lib().hm_plan_summary(self._h, leaf_size, eta, ctypes.byref(info),
                                     perm.ctypes.data if want_perm else None))
        d = {k: getattr(info, k) for k, _ in PlanInfo._fields_ if k != "lowrank_by_level"}
        d["lowrank_by_level"] = {lv: int(info.lowrank_by_level[lv]) for lv in range(64) if info.lowrank_by_level[lv]}
        return (d, perm) if want_perm else d

    def kernel_block(self, young, nu, rows, cols, stream=None):
        """Exact FP64 blocks E[rows, cols] computed on the GPU: [nr, nc, 3, 3] tensor."""
        import torch

        rows = torch.as_tensor(rows, dtype=torch.int64, device="cuda").contiguous()
        cols = torch.as_tensor(cols, dtype=torch.int64, device="cuda").contiguous()
        out = torch.empty((rows.numel(), cols.numel(), 3, 3), dtype=torch.float64, device="cuda")
        _check(lib().hm_kernel_block(self._h, young, nu, rows.numel(), _dev_ptr(rows, torch.int64), cols.numel(),
                                     _dev_ptr(cols, torch.int64), _dev_ptr(out, torch.float64), _stream(stream)))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_mesh_destroy(self._h)
            self._h = None


def _set_fields(o, kw, what):
    """Set struct fields by name; an unknown name is an error, not a new
    Python attribute that the library would never see."""
    names = [f for f, _ in type(o)._fields_]
    for k, v in kw.items():
        if k not in names:
            raise HMError(HM_EINVAL, f"unknown {what} option {k!r}")
        setattr(o, k, v)
    return o


def build_opts(**kw) -> BuildOpts:
    o = BuildOpts()
    lib().hm_build_opts_default(ctypes.byref(o))
    return _set_fields(o, kw, "build")


def solve_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().hm_solve_opts_default(ctypes.byref(o))
    return _set_fields(o, kw, "solve")


class Operator:
    """Owner of an hm_op handle: the H-matrix of E for a mesh and moduli."""

    def __init__(self, mesh: Mesh, young: float, nu: float, stream=None, **opts):
        self.mesh = mesh
        self.ne = mesh.ne
        self.ndof = mesh.ndof
        h = ctypes.c_void_p()
        o = build_opts(**opts)
        _check(lib().hm_operator_build(mesh._h, young, nu, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self._h = h

    def stats(self) -> dict:
        st = OpStats()
        _check(lib().hm_operator_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def apply(self, X, Y=None, reference=False, tangent=False, accumulate=False, stream=None):
        """Y = E X (or A11 X; Y += ... with accumulate) for X a CUDA float64
        tensor [nrhs, 3N] or [3N]."""
        import torch

        squeeze = X.dim() == 1
        X2 = X.reshape(1, -1) if squeeze else X
        if Y is None:
            if accumulate:
                raise ValueError("accumulate needs Y")
            Y = torch.empty_like(X2)
        elif squeeze:
            Y = Y.reshape(1, -1)
        _vecs(X2, self.ndof, "X")
        _vecs(Y, self.ndof, "Y", X2.shape[0])
        flags = ((HM_APPLY_REFERENCE if reference else 0) | (HM_APPLY_TANGENT if tangent else 0)
                 | (HM_APPLY_ACCUMULATE if accumulate else 0))
        _check(lib().hm_operator_apply(self._h, X2.shape[0], _dev_ptr(X2, torch.float64), _ld(X2),
                                       _dev_ptr(Y, torch.float64), _ld(Y), flags, _stream(stream)))
        return Y.reshape(-1) if squeeze else Y

    def apply_noalloc(self, X, Y, reference=False, tangent=False, accumulate=False, stream=None):
        """apply() through hm_operator_apply_noalloc (workspace in the
        library's fixed device array; Y must be given)."""
        import torch

        _vecs(X, self.ndof, "X")
        _vecs(Y, self.ndof, "Y", X.shape[0])
        flags = ((HM_APPLY_REFERENCE if reference else 0) | (HM_APPLY_TANGENT if tangent else 0)
                 | (HM_APPLY_ACCUMULATE if accumulate else 0))
        _check(lib().hm_operator_apply_noalloc(self._h, X.shape[0], _dev_ptr(X, torch.float64), _ld(X),
                                               _dev_ptr(Y, torch.float64), _ld(Y), flags, _stream(stream)))
        return Y

    STAGES = ("gather", "phaseA", "reduceT", "phaseB", "scatter")

    def apply_timed(self, X, Y, reference=False, tangent=False, stream=None):
        """apply() with per-stage durations (ms) from HIP events on the stream."""
        import torch

        _vecs(X, self.ndof, "X")
        _vecs(Y, self.ndof, "Y", X.shape[0])
        flags = (HM_APPLY_REFERENCE if reference else 0) | (HM_APPLY_TANGENT if tangent else 0)
        ms = (ctypes.c_double * 5)()
        _check(lib().hm_operator_apply_timed(self._h, X.shape[0], _dev_ptr(X, torch.float64), _ld(X),
                                             _dev_ptr(Y, torch.float64), _ld(Y), flags, _stream(stream), ms))
        return dict(zip(self.STAGES, list(ms)))

    def set_tangent(self, D=None, mask=None, stream=None):
        """A11 = E - D on active elements (D: CUDA float64 [N,3,3]; mask: CUDA uint8 [N])."""
        import torch

        Dc = D.contiguous() if D is not None else None
        Mc = mask.contiguous() if mask is not None else None
        if Dc is not None and Dc.numel() != 9 * self.ne:
            raise HMError(HM_EINVAL, f"D: expected {self.ne} x 3 x 3 entries, got {tuple(D.shape)}")
        if Mc is not None and Mc.numel() != self.ne:
            raise HMError(HM_EINVAL, f"mask: expected {self.ne} entries, got {tuple(mask.shape)}")
        dp = _dev_ptr(Dc, torch.float64) if Dc is not None else None
        mp = _dev_ptr(Mc, torch.uint8) if Mc is not None else None
        _check(lib().hm_tangent_set(self._h, dp, mp, _stream(stream)))
        del Dc, Mc  # the library copied them (the call synchronises the stream)

    def solve(self, B, stream=None, raise_on_notconv=True, **opts):
        """Solve A11 X = B (B: CUDA float64 [nrhs, 3N]); returns (X, report dict)."""
        import torch

        squeeze = B.dim() == 1
        B2 = (B.reshape(1, -1) if squeeze else B).contiguous()
        _vecs(B2, self.ndof, "B")
        X = torch.empty_like(B2)
        o = solve_opts(**opts)
        rep = SolveReport()
        st = lib().hm_solve(self._h, ctypes.byref(o), B2.shape[0], _dev_ptr(B2, torch.float64), _ld(B2),
                            _dev_ptr(X, torch.float64), _ld(X), ctypes.byref(rep), _stream(stream))
        if st != HM_OK and (st != HM_ENOTCONV or raise_on_notconv):
            _check(st)
        return (X.reshape(-1) if squeeze else X), rep.as_dict()

    def newton_step(self, mats, t, dp, chi, dT0=None, dpress=None, eta_dt=None, dd_prev=None, dd=None,
                    mat_id=None, raise_on_notconv=True, stream=None, **opts):
        """One implicit step of the mechanical problem (hm_newton_step).

        mats: [n_mat, 9] host material table; t, dp, chi: CUDA float64 [N, 3]
        start-of-step interface state; dT0, eta_dt, dd_prev [N, 3], dpress [N]
        optional CUDA float64; dd: initial guess (zero if None).  opts: fields
        of hm_newton_opts (max_newton, rtol, atol) and of its linear-solve
        options prefixed lin_ (lin_precond, lin_rtol, ...).  Returns
        (dd, t_new, dp_new, chi_new, report dict)."""
        import torch

        o = NewtonOpts()
        lib().hm_newton_opts_default(ctypes.byref(o))
        for k, v in opts.items():
            if k == "lin":
                raise HMError(HM_EINVAL, "pass linear-solve options as lin_<name>")
            if k.startswith("lin_"):
                _set_fields(o.lin, {k[4:]: v}, "Newton linear-solve")
            else:
                _set_fields(o, {k: v}, "Newton")
        mats = np.ascontiguousarray(np.atleast_2d(mats), dtype=np.float64)
        arr = (InterfaceMaterial * mats.shape[0])()
        for i in range(mats.shape[0]):
            for j, (name, _) in enumerate(InterfaceMaterial._fields_):
                setattr(arr[i], name, float(mats[i, j]))
        f64 = torch.float64
        N = self.ne
        for name, x in (("t", t), ("dp", dp), ("chi", chi), ("dT0", dT0), ("eta_dt", eta_dt),
                        ("dd_prev", dd_prev), ("dd", dd)):
            if x is not None:
                _shape(x, (N, 3), name)
        for name, x in (("dpress", dpress), ("mat_id", mat_id)):
            if x is not None:
                _shape(x, (N,), name)
        dd = torch.zeros(N, 3, dtype=f64, device=t.device) if dd is None else dd.clone()
        outs = [torch.empty(N, 3, dtype=f64, device=t.device) for _ in range(3)]
        # contiguous copies stay referenced here until the call returns, so
        # torch's allocator cannot hand their memory to the next copy
        keep = [x.contiguous() if x is not None else None
                for x in (mat_id, t, dp, chi, dT0, dpress, eta_dt, dd_prev)]
        ptrs = [_dev_ptr(x, torch.int32 if i == 0 else f64) if x is not None else None
                for i, x in enumerate(keep)]
        rep = NewtonReport()
        st = lib().hm_newton_step(self._h, mats.shape[0], ctypes.cast(arr, ctypes.c_void_p), *ptrs,
                                  _dev_ptr(dd, f64), *[_dev_ptr(x, f64) for x in outs],
                                  ctypes.byref(o), ctypes.byref(rep), _stream(stream))
        del keep
        if st != HM_ENOTCONV or raise_on_notconv:
            _check(st)
        return dd, outs[0], outs[1], outs[2], rep.as_dict()

    def precond_apply(self, R, precond=HM_PC_BLOCK3, stream=None):
        """Z = M^-1 R (R: CUDA float64 [nrhs, 3N]) with the solve's preconditioner."""
        import torch

        _vecs(R, self.ndof, "R")
        Z = torch.empty_like(R)
        _check(lib().hm_precond_apply(self._h, precond, R.shape[0], _dev_ptr(R, torch.float64), _ld(R),
                                      _dev_ptr(Z, torch.float64), _ld(Z), _stream(stream)))
        return Z

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_op_destroy(self._h)
            self._h = None


class Batch:
    """Owner of an hm_batch: many operators applied by merged launches
    (captured as one HIP graph; both product phases are queue-driven
    launches over the merged task list).  Keeps its operators alive; the
    batch and its operators are not to be applied concurrently."""

    def __init__(self, ops, use_graph=True, autotune=True, stream=None):
        self.ops = list(ops)
        o = BatchOpts()
        lib().hm_batch_opts_default(ctypes.byref(o))
        o.use_graph = 1 if use_graph else 0
        o.autotune = 1 if autotune else 0
        arr = (ctypes.c_void_p * len(self.ops))(*[op._h for op in self.ops])
        h = ctypes.c_void_p()
        _check(lib().hm_batch_create(len(self.ops), arr, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self._h = h

    def apply(self, Xs, Ys, stream=None):
        """Ys[i] = E_i Xs[i]; each a CUDA float64 tensor [nrhs, 3 N_i] (same nrhs)."""
        import torch

        n = len(self.ops)
        if len(Xs) != n or len(Ys) != n:
            raise HMError(HM_EINVAL, f"expected {n} input and output blocks")
        nrhs = Xs[0].shape[0]
        for k, (op, x, y) in enumerate(zip(self.ops, Xs, Ys)):
            _vecs(x, op.ndof, f"Xs[{k}]", nrhs)
            _vecs(y, op.ndof, f"Ys[{k}]", nrhs)
        xp = (ctypes.c_void_p * n)(*[_dev_ptr(x, torch.float64).value for x in Xs])
        yp = (ctypes.c_void_p * n)(*[_dev_ptr(y, torch.float64).value for y in Ys])
        ldx = (ctypes.c_int64 * n)(*[_ld(x) for x in Xs])
        ldy = (ctypes.c_int64 * n)(*[_ld(y) for y in Ys])
        for x in Xs:
            if x.shape[0] != nrhs:
                raise HMError(HM_EINVAL, "all operators take the same number of columns")
        _check(lib().hm_batch_apply(self._h, nrhs, xp, ldx, yp, ldy, _stream(stream)))
        return Ys

    def info(self) -> dict:
        i = BatchInfo()
        _check(lib().hm_batch_get_info(self._h, ctypes.byref(i)))
        return {"n_ops": i.n_ops, "total_elements": i.total_elements, "use_graph": i.use_graph,
                "leaves_per_task_a": i.leaves_per_task_a, "tune_candidates": list(i.tune_candidates),
                "tune_ms": list(i.tune_ms), "bytes_operators": i.bytes_operators,
                "phase_b_window": i.phase_b_window, "tune_b_candidates": list(i.tune_b_candidates),
                "tune_b_ms": list(i.tune_b_ms)}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_batch_destroy(self._h)
            self._h = None


class Learned:
    """Owner of an hm_learned handle: the MLP correction of the block
    preconditioner (hm_learned_* in the C ABI)."""

    def __init__(self, hidden=64, neighbors=8, seed=0):
        h = ctypes.c_void_p()
        _check(lib().hm_learned_create(hidden, neighbors, seed, ctypes.byref(h)))
        self._h = h
        self.hidden = hidden
        self.neighbors = neighbors
        self.base = HM_PC_BLOCK3

    def set_base(self, base):
        """Base preconditioner of the correction: HM_PC_BLOCK3 (default) or HM_PC_LEAF."""
        _check(lib().hm_learned_set_base(self._h, base))
        self.base = base

    def num_params(self) -> int:
        n = ctypes.c_int64()
        _check(lib().hm_learned_num_params(self._h, ctypes.byref(n)))
        return n.value

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params(), np.float32)
        _check(lib().hm_learned_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p), out.size))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        _check(lib().hm_learned_set_params(self._h, theta.ctypes.data_as(ctypes.c_void_p), theta.size))

    def loss_grad(self, op: Operator, B, X, stream=None):
        """(loss, dL/dtheta) at the current parameters; B, X CUDA float64 [ns, 3N]."""
        import torch

        _vecs(B, op.ndof, "B")
        _vecs(X, op.ndof, "X", B.shape[0])
        g = np.empty(self.num_params(), np.float32)
        loss = ctypes.c_double()
        _check(lib().hm_learned_loss_grad(self._h, op._h, B.shape[0], _dev_ptr(B, torch.float64), _ld(B),
                                          _dev_ptr(X, torch.float64), _ld(X), ctypes.byref(loss),
                                          g.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return loss.value, g

    def train(self, op: Operator, B, X, steps, batch=16, lr=1e-3, stream=None) -> np.ndarray:
        """Adam steps on the samples (B, X) of op's current tangent; returns the loss history."""
        import torch

        _vecs(B, op.ndof, "B")
        _vecs(X, op.ndof, "X", B.shape[0])
        hist = np.zeros(steps)
        _check(lib().hm_learned_train(self._h, op._h, B.shape[0], _dev_ptr(B, torch.float64), _ld(B),
                                      _dev_ptr(X, torch.float64), _ld(X), steps, batch, lr,
                                      hist.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return hist

    def attach(self, op: Operator, stream=None):
        """Predict the correction for op's current tangent and attach it (HM_PC_LEARNED)."""
        _check(lib().hm_learned_attach(op._h, self._h, _stream(stream)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_learned_destroy(self._h)
            self._h = None


def learned_detach(op: Operator):
    lib().hm_learned_detach(op._h)


def learned_features(op: Operator, neighbors: int, stream=None):
    """Pairs and features of op's current tangent: (pe, pf, feat [P, 32], scale)."""
    n = ctypes.c_int64()
    _check(lib().hm_learned_features(op._h, neighbors, 0, ctypes.byref(n), None, None, None, None,
                                     _stream(stream)))
    P = n.value
    pe = np.empty(P, np.int32)
    pf = np.empty(P, np.int32)
    feat = np.empty((P, 32), np.float32)
    scale = np.empty(P, np.float64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().hm_learned_features(op._h, neighbors, P, ctypes.byref(n), ptr(pe), ptr(pf), ptr(feat), ptr(scale),
                                     _stream(stream)))
    return pe, pf, feat, scale


# ---------------------------------------------------------------- flow and the coupled step
def _materials(mats):
    mats = np.ascontiguousarray(np.atleast_2d(mats), dtype=np.float64)
    arr = (InterfaceMaterial * max(mats.shape[0], 1))()
    for i in range(mats.shape[0]):
        for j, (name, _) in enumerate(InterfaceMaterial._fields_):
            setattr(arr[i], name, float(mats[i, j]))
    return mats.shape[0], arr


class Flow:
    """Owner of an hm_flow handle: P1 flow on the triangles of a mesh."""

    def __init__(self, mesh: Mesh, M, mu, perm_law=HM_PERM_CUBIC, k0=0.0, stream=None):
        p = FlowParams(float(M), float(mu), int(perm_law), float(k0))
        h = ctypes.c_void_p()
        _check(lib().hm_flow_create(mesh._h, ctypes.byref(p), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.mesh = mesh
        self.nn = lib().hm_flow_num_nodes(h)
        self.nnz = lib().hm_flow_nnz(h)

    def matrices(self, w, stream=None):
        """(rowptr, col, S, L) host CSR at the hydraulic widths w (CUDA float64 [N])."""
        import torch

        wc = w.contiguous()
        _shape(wc, (self.mesh.ne,), "w")
        rowptr = np.empty(self.nn + 1, np.int64)
        col = np.empty(self.nnz, np.int32)
        S = np.empty(self.nnz)
        L = np.empty(self.nnz)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().hm_flow_matrices(self._h, _dev_ptr(wc, torch.float64), ptr(rowptr), ptr(col), ptr(S), ptr(L),
                                      _stream(stream)))
        return rowptr, col, S, L

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hm_flow_destroy(self._h)
            self._h = None


def coupled_opts(**kw) -> CoupledOpts:
    o = CoupledOpts()
    lib().hm_coupled_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k.startswith("inner_"):
            _set_fields(o.inner, {k[6:]: v}, "inner solve")
        elif k == "scales":
            for i, x in enumerate(v):
                o.scales[i] = float(x)
        else:
            _set_fields(o, {k: v}, "coupled")
    return o


def coupled_step(op: Operator, flow: Flow, mats, t, dp, chi, p_n, w0, dt, dT0=None, eta_dt=None, dd_prev=None,
                 p_o=None, source=None, dn_start=None, dd=None, dpn=None, mat_id=None, raise_on_notconv=True,
                 stream=None, **opts):
    """One coupled implicit step (hm_coupled_step).  Element arrays CUDA
    float64 [N, 3] (t, dp, chi, dT0, eta_dt, dd_prev, dd) or [N] (w0,
    dn_start); nodal arrays [n] (p_n, p_o, source, dpn).  opts: fields of
    hm_coupled_opts (scales as a 4-sequence, inner solve fields as inner_*).
    Returns (dd, dpn, t_new, dp_new, chi_new, report dict)."""
    import torch

    f64 = torch.float64
    N, n = op.ne, flow.nn
    for name, x in (("t", t), ("dp", dp), ("chi", chi), ("dT0", dT0), ("eta_dt", eta_dt), ("dd_prev", dd_prev),
                    ("dd", dd)):
        if x is not None:
            _shape(x, (N, 3), name)
    for name, x in (("w0", w0), ("dn_start", dn_start), ("mat_id", mat_id)):
        if x is not None:
            _shape(x, (N,), name)
    for name, x in (("p_n", p_n), ("p_o", p_o), ("source", source), ("dpn", dpn)):
        if x is not None:
            _shape(x, (n,), name)
    o = coupled_opts(**opts)
    n_mat, arr = _materials(mats)
    dev = t.device
    dd = torch.zeros(N, 3, dtype=f64, device=dev) if dd is None else dd.clone()
    dpn = torch.zeros(n, dtype=f64, device=dev) if dpn is None else dpn.clone()
    outs = [torch.empty(N, 3, dtype=f64, device=dev) for _ in range(3)]
    keep = [x.contiguous() if x is not None else None
            for x in (mat_id, t, dp, chi, dT0, eta_dt, dd_prev, p_n, p_o, source, w0, dn_start)]
    ptrs = [_dev_ptr(x, torch.int32 if i == 0 else f64) if x is not None else None for i, x in enumerate(keep)]
    rep = CoupledReport()
    st = lib().hm_coupled_step(op._h, flow._h, n_mat, ctypes.cast(arr, ctypes.c_void_p), *ptrs, float(dt),
                               _dev_ptr(dd, f64), _dev_ptr(dpn, f64), *[_dev_ptr(x, f64) for x in outs],
                               ctypes.byref(o), ctypes.byref(rep), _stream(stream))
    del keep
    if st != HM_ENOTCONV or raise_on_notconv:
        _check(st)
    return dd, dpn, outs[0], outs[1], outs[2], rep.as_dict()


def scale_update(L_old, L_new, alpha=0.62, rho_min=0.84, rho_max=1.16):
    """The smoothed and clipped scale of Sec. 3.3.2 (hm_scale_update)."""
    out = ctypes.c_double()
    _check(lib().hm_scale_update(float(L_old), float(L_new), float(alpha), float(rho_min), float(rho_max),
                                 ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------- interface law
def interface_update(mats, dd, t, dp, chi, mat_id=None, eta_dt=None, want_D=False, out=None, stream=None):
    """One step of the interface elasto-plastic law (hm_interface_update).

    mats: [n_mat, 9] host array (fields of hm_interface_material in order);
    dd, t, dp, chi: CUDA float64 [N, 3]; mat_id: CUDA int32 [N] or None;
    eta_dt: CUDA float64 [N, 3] or None.  Returns a dict of CUDA tensors
    t, dp, chi [N, 3], cep [N, 3, 3], mode [N] (int32) and, with want_D,
    D = cep + diag(eta_dt).  `out` may supply the output tensors (for
    in-place updates pass the inputs themselves)."""
    import torch

    mats = np.ascontiguousarray(np.atleast_2d(mats), dtype=np.float64)
    n_mat = mats.shape[0]
    arr = (InterfaceMaterial * max(n_mat, 1))()
    for i in range(n_mat):
        for j, (name, _) in enumerate(InterfaceMaterial._fields_):
            setattr(arr[i], name, float(mats[i, j]))
    N = dd.shape[0]
    dev = dd.device
    o = dict(out or {})
    for k in ("t", "dp", "chi"):
        o.setdefault(k, torch.empty(N, 3, dtype=torch.float64, device=dev))
    o.setdefault("cep", torch.empty(N, 3, 3, dtype=torch.float64, device=dev))
    o.setdefault("mode", torch.empty(N, dtype=torch.int32, device=dev))
    if want_D:
        o.setdefault("D", torch.empty(N, 3, 3, dtype=torch.float64, device=dev))
    f64 = torch.float64
    for name, x in (("dd", dd), ("t", t), ("dp", dp), ("chi", chi), ("eta_dt", eta_dt), ("out t", o["t"]),
                    ("out dp", o["dp"]), ("out chi", o["chi"])):
        if x is not None:
            _shape(x, (N, 3), name)
    for name, x in (("mat_id", mat_id), ("out mode", o["mode"])):
        if x is not None:
            _shape(x, (N,), name)
    _shape(o["cep"], (N, 3, 3), "out cep")
    if want_D:
        _shape(o["D"], (N, 3, 3), "out D")
    arrays = [dd, t, dp, chi, mat_id, eta_dt, o["t"], o["dp"], o["chi"], o["cep"], o["mode"]]
    if any(x is not None and not x.is_contiguous() for x in arrays + [o.get("D")]):
        raise HMError(HM_EINVAL, "interface arrays must be contiguous")
    pin = [_dev_ptr(x, f64) for x in (dd, t, dp, chi)]
    mid = _dev_ptr(mat_id, torch.int32) if mat_id is not None else None
    eta = _dev_ptr(eta_dt, f64) if eta_dt is not None else None
    Dp = _dev_ptr(o["D"], f64) if want_D else None
    _check(lib().hm_interface_update(n_mat, ctypes.cast(arr, ctypes.c_void_p), N, mid, *pin,
                                     _dev_ptr(o["t"], f64), _dev_ptr(o["dp"], f64), _dev_ptr(o["chi"], f64),
                                     _dev_ptr(o["cep"], f64), _dev_ptr(o["mode"], torch.int32), eta, Dp,
                                     _stream(stream)))
    return o


# ---------------------------------------------------------------- adaptive time stepping
def timestep_next(dt_n, dt_prev, e_next, e_n, n_its, **opts):
    """Next step size from the paper's controller (hm_timestep_next); opts:
    eps_tol, n_target, growth_max, dt_min, dt_max."""
    o = TimestepOpts()
    lib().hm_timestep_opts_default(ctypes.byref(o))
    _set_fields(o, opts, "time-step")
    out = ctypes.c_double()
    _check(lib().hm_timestep_next(ctypes.byref(o), float(dt_n), float(dt_prev), float(e_next), float(e_n),
                                  int(n_its), ctypes.byref(out)))
    return out.value


def lte_estimate(dd, dt, dd_prev, dt_prev, total, stream=None):
    """Relative truncation-error estimate of a step (hm_lte_estimate); CUDA
    float64 vectors of one length (dd_prev may be None)."""
    import torch

    f64 = torch.float64
    for name, x in (("dd_prev", dd_prev), ("total", total)):
        if x is not None and x.numel() != dd.numel():
            raise HMError(HM_EINVAL, f"{name}: expected {dd.numel()} entries, got {x.numel()}")
    # the contiguous copies are bound to names that live until the call returns
    ddc = dd.contiguous()
    prevc = dd_prev.contiguous() if dd_prev is not None else None
    totc = total.contiguous()
    e = ctypes.c_double()
    _check(lib().hm_lte_estimate(ddc.numel(), _dev_ptr(ddc, f64), float(dt),
                                 _dev_ptr(prevc, f64) if prevc is not None else None,
                                 float(dt_prev), _dev_ptr(totc, f64), ctypes.byref(e), _stream(stream)))
    del ddc, prevc, totc
    return e.value
