"""CPU FP64 oracle for the DD collocation operator, its products and solves.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the GPU path.

What it computes (paper Sec. 3.1, "Solid mechanics" and "Final system"):
  * the exact collocation matrix E of piecewise-constant DD elements, one
    3x3 block per (receiver, source) pair in local frames, element-major
    [s1, s2, n] ordering of DOFs in each element's local frame;
  * Y = E X by direct summation;
  * solutions of the tangent system A11 x = b with A11 = E - eta/dt - C^ep
    (Sec. 3.1.1, mechanical Jacobian) by dense LU, with inactive elements
    carried as identity rows and columns;
  * the closed-form penny-shaped crack opening under uniform pressure and
    uniform shear slip used to pin the oracle itself.

Submodules: `learned` (the learned correction of the block preconditioner,
its loss and gradient), `interface` (the interface elasto-plastic law and
its consistent tangent, Sec. 2.2), `newton` (one implicit step of the
mechanical problem, Sec. 3.1.1) and `timestep` (the truncation-error
estimate and step-size controller, Sec. 3.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C kernel with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        lib.orc_frames.argtypes = [i32, i64, P, P, P, P, P]
        lib.orc_frames.restype = i32
        lib.orc_coplanar_rect_block.argtypes = [d, d, d, d, d, d, P]
        lib.orc_coplanar_rect_block.restype = None
        lib.orc_pk_block.argtypes = [d, d, P, P, i32, P, P, d, P]
        lib.orc_pk_block.restype = None
        lib.orc_assemble.argtypes = [i32, i64, P, i64, P, d, d, i64, P, i64, P, i32, d, P]
        lib.orc_assemble.restype = i32
        lib.orc_rows_matvec.argtypes = [i32, i64, P, i64, P, d, d, i64, P, i32, P, P, i32, d]
        lib.orc_rows_matvec.restype = i32
        lib.orc_grid_table.argtypes = [d, d, i32, i32, d, d, P]
        lib.orc_grid_table.restype = None
        lib.orc_grid_matvec.argtypes = [i32, i32, P, i32, P, P]
        lib.orc_grid_matvec.restype = i32
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


PK_TOL = 1e-13


def frames(mesh):
    """Centroid (vertex mean), frame rows (s1, s2, n) and area per element."""
    lib = _load()
    xyz, conn = _f64(mesh.xyz), _i64(mesh.conn)
    ne = conn.shape[0]
    cent = np.empty((ne, 3))
    fr = np.empty((ne, 3, 3))
    area = np.empty(ne)
    st = lib.orc_frames(conn.shape[1], ne, _p(xyz), _p(conn), _p(cent), _p(fr), _p(area))
    if st != 0:
        raise ValueError("degenerate element")
    return cent, fr, area


def coplanar_rect_block(young, nu, xi1, xi2, ze1, ze2) -> np.ndarray:
    """Closed-form 3x3 block for an axis-aligned source rectangle
    [xi1, xi2] x [ze1, ze2] (offsets from the receiver point in its frame)."""
    out = np.empty(9)
    _load().orc_coplanar_rect_block(young, nu, xi1, xi2, ze1, ze2, _p(out))
    return out.reshape(3, 3)


def pk_block(young, nu, x_recv, frame_recv, verts_src, frame_src, rtol=PK_TOL) -> np.ndarray:
    """3x3 traction block by the Peach-Koehler loop integral (quadrature)."""
    out = np.empty(9)
    x = _f64(x_recv)
    fr = _f64(frame_recv)
    v = _f64(verts_src)
    fs = _f64(frame_src)
    _load().orc_pk_block(young, nu, _p(x), _p(fr), v.shape[0], _p(v), _p(fs), rtol, _p(out))
    return out.reshape(3, 3)


def blocks(mesh, young, nu, rows, cols, method: int = 0, tol: float = PK_TOL) -> np.ndarray:
    """Exact coefficient blocks out[r, c, a, b] = E_{rows[r], cols[c]}^{ab}.

    method 0: coplanar closed form where it applies, PK quadrature elsewhere;
    method 1: PK quadrature everywhere."""
    lib = _load()
    rows, cols = _i64(rows), _i64(cols)
    xyz, conn = _f64(mesh.xyz), _i64(mesh.conn)
    out = np.empty((rows.size, cols.size, 3, 3))
    st = lib.orc_assemble(conn.shape[1], xyz.shape[0], _p(xyz), conn.shape[0], _p(conn), young, nu,
                          rows.size, _p(rows), cols.size, _p(cols), method, tol, _p(out))
    if st != 0:
        raise ValueError(f"oracle assembly failed ({st})")
    return out


def dense(mesh, young, nu, method: int = 0) -> np.ndarray:
    """Dense E as a [3N, 3N] matrix in element-major [s1, s2, n] order."""
    n = mesh.conn.shape[0]
    idx = np.arange(n)
    b = blocks(mesh, young, nu, idx, idx, method)
    return b.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def rows_matvec(mesh, young, nu, rows, X, method: int = 0, tol: float = PK_TOL) -> np.ndarray:
    """Exact rows of E X for selected elements; X is [nrhs, 3N].

    Returns [nrhs, 3 * len(rows)] (DOFs of the selected elements)."""
    lib = _load()
    rows = _i64(rows)
    X = _f64(np.atleast_2d(X))
    xyz, conn = _f64(mesh.xyz), _i64(mesh.conn)
    Y = np.empty((X.shape[0], 3 * rows.size))
    st = lib.orc_rows_matvec(conn.shape[1], xyz.shape[0], _p(xyz), conn.shape[0], _p(conn), young, nu,
                             rows.size, _p(rows), X.shape[0], _p(X), _p(Y), method, tol)
    if st != 0:
        raise ValueError(f"oracle rows failed ({st})")
    return Y


def grid_table(young, nu, nx, ny, h=1.0, hy=None) -> np.ndarray:
    """Coefficient table of a uniform grid of nx x ny rectangles (h x hy)
    sharing one plane and frame, element e = i + nx j: out[dj + ny - 1,
    di + nx - 1] = E between a receiver and the source offset by (di, dj)
    cells (coplanar closed form), shape [2 ny - 1, 2 nx - 1, 3, 3]."""
    hy = h if hy is None else hy
    out = np.empty((2 * ny - 1, 2 * nx - 1, 3, 3))
    _load().orc_grid_table(young, nu, nx, ny, h, hy, _p(out))
    return out


def grid_matvec(table, nx, ny, X) -> np.ndarray:
    """Exact Y = E X on a uniform grid by direct summation over every pair of
    the offset table (OpenMP over receivers); X is [nrhs, 3 nx ny]."""
    X = _f64(np.atleast_2d(X))
    T = _f64(table)
    if T.shape != (2 * ny - 1, 2 * nx - 1, 3, 3) or X.shape[1] != 3 * nx * ny:
        raise ValueError("grid_matvec: shapes do not match the grid")
    Y = np.empty_like(X)
    st = _load().orc_grid_matvec(nx, ny, _p(T), X.shape[0], _p(X), _p(Y))
    if st != 0:
        raise MemoryError("grid_matvec: allocation failed")
    return Y


def grid_matvec_fft(table, nx, ny, X) -> np.ndarray:
    """The same product by circulant embedding: the offset table is laid on a
    (2 ny) x (2 nx) periodic grid (offset d at index -d mod size), so the
    Toeplitz sum is a circular convolution, taken with 2-D FFTs (numpy).  An
    independent route to grid_matvec."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    nrhs = X.shape[0]
    py, px = 2 * ny, 2 * nx
    dj = np.arange(-(ny - 1), ny)
    di = np.arange(-(nx - 1), nx)
    K = np.zeros((3, 3, py, px))
    K[:, :, (-dj[:, None]) % py, (-di[None, :]) % px] = np.asarray(table).transpose(2, 3, 0, 1)
    Kf = np.fft.rfft2(K)
    Xg = np.zeros((nrhs, 3, py, px))
    Xg[:, :, :ny, :nx] = X.reshape(nrhs, ny, nx, 3).transpose(0, 3, 1, 2)
    Xf = np.fft.rfft2(Xg)
    Yf = np.einsum("abyx,cbyx->cayx", Kf, Xf)
    Yg = np.fft.irfft2(Yf, s=(py, px))[:, :, :ny, :nx]
    return Yg.transpose(0, 2, 3, 1).reshape(nrhs, 3 * nx * ny)


def matvec(E: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Direct dense product Y = E X for X [nrhs, 3N] (columns as rows)."""
    return (E @ np.atleast_2d(X).T).T


def tangent_dense(E: np.ndarray, D: np.ndarray | None, active: np.ndarray | None) -> np.ndarray:
    """A11 = E - D on active elements, identity rows/columns on inactive ones.

    D is [N, 3, 3] (eta/dt + C^ep per element, local frame), block diagonal
    (Sec. 3.1.1 mechanical Jacobian)."""
    n = E.shape[0] // 3
    A = E.copy()
    if D is not None:
        for i in range(n):
            A[3 * i:3 * i + 3, 3 * i:3 * i + 3] -= D[i]
    if active is not None:
        act = np.repeat(np.asarray(active, bool), 3)
        A[~act, :] = 0.0
        A[:, ~act] = 0.0
        A[~act, ~act] = 1.0
    return A


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Dense LU solve (LAPACK through numpy)."""
    return np.linalg.solve(A, np.atleast_2d(b).T).T


def penny_opening(r, a, p, young, nu):
    """Sneddon's opening of a penny crack of radius a under uniform pressure p:
    w(r) = 8 (1 - nu^2) p / (pi E) sqrt(a^2 - r^2)."""
    r = np.asarray(r, dtype=np.float64)
    return 8.0 * (1.0 - nu * nu) * p / (np.pi * young) * np.sqrt(np.maximum(a * a - r * r, 0.0))


def penny_slip(r, a, tau, young, nu):
    """Uniform-shear penny crack: slip parallel to the shear stress with
    amplitude 8 (1 - nu) tau sqrt(a^2 - r^2) / (pi (2 - nu) G)."""
    G = young / (2.0 * (1.0 + nu))
    r = np.asarray(r, dtype=np.float64)
    return 8.0 * (1.0 - nu) * tau / (np.pi * (2.0 - nu) * G) * np.sqrt(np.maximum(a * a - r * r, 0.0))
