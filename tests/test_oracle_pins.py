"""Pins of the CPU oracle against what the mathematics fixes.

Each test targets a mistake the oracle could plausibly contain (a dropped
term, a wrong sign, a transposed index, a wrong loop orientation):
  * closed-form self coefficients of a square, evaluated by hand;
  * the coplanar corner formulas against direct high-precision quadrature;
  * the Peach-Koehler loop quadrature against the coplanar closed form
    (two independent derivations of the same coefficient);
  * a closed polyhedral surface under a uniform DD (rigid translation of the
    enclosed body) carries no traction: pins non-coplanar pairs and signs;
  * Sneddon's penny crack under pressure and the uniform-shear penny crack
    (paper Sec. 3.1: piecewise-constant DD with centroid collocation, which
    converges sub-linearly, Sec. 4);
  * symmetry, definiteness, decoupling, nu = 0 identities, invariances,
    additivity and far-field reciprocity.
"""
import mpmath
import numpy as np
import pytest

import oracle
from workloads import Mesh, penny_active_mask, rect_grid, square_fault

YOUNG, NU = 30e9, 0.25
G = YOUNG / (2 * (1 + NU))
EP = YOUNG / (1 - NU * NU)


def test_square_self_coefficients_closed_form(oracle_lib):
    # corner sums at the centre of a square of side h reduce to
    # I0 = -8 sqrt(2) / h and Ixx = Izz = -(4/3)(2 sqrt(2) + 1/sqrt(2)) / h
    for h in (1.0, 0.37, 12.0):
        blk = oracle.coplanar_rect_block(YOUNG, NU, -h / 2, h / 2, -h / 2, h / 2)
        enn = -np.sqrt(2.0) * EP / (np.pi * h)
        ess = -np.sqrt(2.0) * G * (2 - NU) / (np.pi * (1 - NU) * h)
        assert blk[2, 2] == pytest.approx(enn, rel=1e-14)
        assert blk[0, 0] == pytest.approx(ess, rel=1e-14)
        assert blk[1, 1] == pytest.approx(ess, rel=1e-14)
        assert blk[0, 1] == 0.0 and blk[1, 0] == 0.0
        assert np.all(blk[:2, 2] == 0) and np.all(blk[2, :2] == 0)


def test_rectangle_self_coefficients_closed_form(oracle_lib):
    # 2a x 2b rectangle, rho = sqrt(a^2 + b^2):
    # I0 = -4 rho/(ab), Ixx = -(4/3)(rho/(ab) + b/(a rho)), Izz = -(4/3)(rho/(ab) + a/(b rho))
    a, b = 1.0, 0.5
    rho = np.hypot(a, b)
    c0 = G / (4 * np.pi * (1 - NU))
    I0 = -4 * rho / (a * b)
    Ixx = -(4 / 3) * (rho / (a * b) + b / (a * rho))
    Izz = -(4 / 3) * (rho / (a * b) + a / (b * rho))
    blk = oracle.coplanar_rect_block(YOUNG, NU, -a, a, -b, b)
    assert blk[2, 2] == pytest.approx(c0 * I0, rel=1e-14)
    assert blk[0, 0] == pytest.approx(c0 * ((1 - 2 * NU) * I0 + 3 * NU * Ixx), rel=1e-14)
    assert blk[1, 1] == pytest.approx(c0 * ((1 - 2 * NU) * I0 + 3 * NU * Izz), rel=1e-14)


@pytest.mark.parametrize("off", [(2.0, 1.0), (1.5, -3.0), (10.0, 3.0)])
def test_coplanar_corner_formula_vs_quadrature(oracle_lib, off):
    # away from the receiver the integrands are smooth: integrate directly
    mpmath.mp.dps = 20
    x1, x2 = off[0] - 0.5, off[0] + 0.5
    z1, z2 = off[1] - 0.5, off[1] + 0.5
    I0 = mpmath.quad(lambda x, z: (x * x + z * z) ** -1.5, [x1, x2], [z1, z2])
    Ixx = mpmath.quad(lambda x, z: x * x * (x * x + z * z) ** -2.5, [x1, x2], [z1, z2])
    Izz = mpmath.quad(lambda x, z: z * z * (x * x + z * z) ** -2.5, [x1, x2], [z1, z2])
    Ixz = mpmath.quad(lambda x, z: x * z * (x * x + z * z) ** -2.5, [x1, x2], [z1, z2])
    c0 = G / (4 * np.pi * (1 - NU))
    blk = oracle.coplanar_rect_block(YOUNG, NU, x1, x2, z1, z2)
    assert blk[2, 2] == pytest.approx(c0 * float(I0), rel=1e-12)
    assert blk[0, 0] == pytest.approx(c0 * ((1 - 2 * NU) * float(I0) + 3 * NU * float(Ixx)), rel=1e-12)
    assert blk[1, 1] == pytest.approx(c0 * ((1 - 2 * NU) * float(I0) + 3 * NU * float(Izz)), rel=1e-12)
    assert blk[0, 1] == pytest.approx(3 * NU * c0 * float(Ixz), rel=1e-11)


def _unit_square(off=(0.0, 0.0), a=0.5, b=0.5):
    ox, oz = off
    return np.array([[ox - a, oz - b, 0], [ox + a, oz - b, 0], [ox + a, oz + b, 0], [ox - a, oz + b, 0]], float)


def test_pk_matches_coplanar_closed_form(oracle_lib):
    rng = np.random.default_rng(7)
    fr = np.eye(3)
    worst = 0.0
    for _ in range(40):
        a, b = rng.uniform(0.2, 2.0, size=2)
        off = rng.uniform(-6, 6, size=2) if rng.random() < 0.8 else np.zeros(2)
        v = _unit_square(off, a, b)
        if np.all(off == 0) or not (abs(off[0]) < a and abs(off[1]) < b):
            pass
        cf = oracle.coplanar_rect_block(YOUNG, NU, off[0] - a, off[0] + a, off[1] - b, off[1] + b)
        pk = oracle.pk_block(YOUNG, NU, [0, 0, 0], fr, v, fr)
        worst = max(worst, np.abs(cf - pk).max() / np.abs(cf).max())
    assert worst < 1e-10


def _cube(nsub):
    defs = [((0, 0, 0), (0, 1, 0), (1, 0, 0)), ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
            ((0, 0, 0), (1, 0, 0), (0, 0, 1)), ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
            ((0, 0, 0), (0, 0, 1), (0, 1, 0)), ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
    xyz, conn = [], []
    h = 1.0 / nsub
    for o, u, v in defs:
        o, u, v = map(np.array, (o, u, v))
        for j in range(nsub):
            for i in range(nsub):
                p0 = o + u * i * h + v * j * h
                base = len(xyz)
                xyz += [p0, p0 + u * h, p0 + u * h + v * h, p0 + v * h]
                conn.append([base, base + 1, base + 2, base + 3])
    return Mesh(np.array(xyz, float), np.array(conn, np.int64), "cube")


def _icosphere(level):
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, float) / np.linalg.norm(p) for p in v]
    for _ in range(level):
        cache, nf = {}, []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return Mesh(np.array(verts), np.array(f, np.int64), "icosphere")


@pytest.mark.parametrize("mesh_fn", [lambda: _cube(2), lambda: _icosphere(1)], ids=["cube_rect", "icosphere_tri"])
def test_closed_surface_rigid_translation_is_traction_free(oracle_lib, mesh_fn):
    m = mesh_fn()
    cent, fr, _ = oracle.frames(m)
    assert np.all(np.einsum("ij,ij->i", fr[:, 2], cent - cent.mean(0)) > 0)  # outward normals
    E = oracle.dense(m, YOUNG, NU, method=1)
    bvec = np.array([0.3, -0.7, 0.5])
    delta = np.einsum("iab,b->ia", fr, bvec).ravel()
    T = E @ delta
    scale = np.abs(E).max() * np.abs(delta).max()
    assert np.abs(T).max() < 1e-11 * scale
    # one face alone is far from traction-free: the sum is a real cancellation
    assert np.abs(E[:, :3] @ delta[:3]).max() > 1e-3 * scale


def test_penny_crack_pressure_vs_sneddon_and_refinement(oracle_lib):
    p = 1e6
    errs = []
    for n in (16, 32):
        m = square_fault(n)
        act = penny_active_mask(m).astype(bool)
        A = oracle.tangent_dense(oracle.dense(m, YOUNG, NU), None, act)
        b = np.zeros((m.ne, 3))
        b[act, 2] = -p  # t = -p n on the crack faces
        x = oracle.solve_dense(A, b.ravel())[0].reshape(-1, 3)
        cent, _, _ = oracle.frames(m)
        r = np.hypot(cent[:, 0] - n / 2, cent[:, 1] - n / 2)
        w = oracle.penny_opening(r, 0.45 * n, p, YOUNG, NU)
        assert np.all(x[act, 2] > 0)                 # pressure opens the crack
        assert np.all(x[~act] == 0)                  # identity rows, zero load
        assert np.abs(x[:, :2]).max() == 0.0         # exact normal/shear decoupling
        centre_err = abs(x[act, 2].max() / w.max() - 1)
        l2 = np.linalg.norm(x[act, 2] - w[act]) / np.linalg.norm(w[act])
        errs.append((centre_err, l2))
    # 32 x 32: within 2 % at the centre and 6 % in L2; errors shrink with refinement
    assert errs[1][0] < 0.02 and errs[1][1] < 0.06
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1]


def test_penny_crack_pressure_finer_grid_nn_block(oracle_lib):
    # coplanar decoupling (pinned elsewhere) lets the normal block be solved alone
    n, p = 64, 1e6
    m = square_fault(n)
    act = np.nonzero(penny_active_mask(m))[0]
    B = oracle.blocks(m, YOUNG, NU, act, act)[:, :, 2, 2]
    x = np.linalg.solve(B, -p * np.ones(act.size))
    cent, _, _ = oracle.frames(m)
    r = np.hypot(cent[act, 0] - n / 2, cent[act, 1] - n / 2)
    w = oracle.penny_opening(r, 0.45 * n, p, YOUNG, NU)
    l2 = np.linalg.norm(x - w) / np.linalg.norm(w)
    assert abs(x.max() / w.max() - 1) < 0.01 and l2 < 0.035


def test_penny_crack_uniform_shear(oracle_lib):
    n, tau = 32, 1e6
    m = square_fault(n)
    act = penny_active_mask(m).astype(bool)
    A = oracle.tangent_dense(oracle.dense(m, YOUNG, NU), None, act)
    b = np.zeros((m.ne, 3))
    b[act, 0] = -tau
    x = oracle.solve_dense(A, b.ravel())[0].reshape(-1, 3)
    cent, _, _ = oracle.frames(m)
    r = np.hypot(cent[:, 0] - n / 2, cent[:, 1] - n / 2)
    s = oracle.penny_slip(r, 0.45 * n, tau, YOUNG, NU)
    assert abs(x[act, 0].max() / s.max() - 1) < 0.02
    assert np.abs(x[act, 1]).max() < 0.03 * x[act, 0].max()   # small cross slip


def test_uniform_grid_symmetry_definiteness_decoupling(oracle_lib):
    m = square_fault(12)
    E = oracle.dense(m, YOUNG, NU)
    assert np.abs(E - E.T).max() <= 1e-15 * np.abs(E).max()
    np.linalg.cholesky(-E)                                     # -E is SPD
    blk = E.reshape(m.ne, 3, m.ne, 3)
    assert np.all(blk[:, :2, :, 2] == 0) and np.all(blk[:, 2, :, :2] == 0)
    E0 = oracle.dense(m, YOUNG, 0.0).reshape(m.ne, 3, m.ne, 3)
    assert np.allclose(E0[:, 0, :, 0], E0[:, 2, :, 2], rtol=1e-13, atol=0)
    assert np.allclose(E0[:, 1, :, 1], E0[:, 2, :, 2], rtol=1e-13, atol=0)
    assert np.abs(E0[:, 0, :, 1]).max() == 0.0


def test_invariances_translation_rotation_scale_modulus(oracle_lib):
    base = rect_grid(5, 4, 1.0)
    E = oracle.dense(base, YOUNG, NU, method=1)
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    moved = Mesh(base.xyz @ q.T + np.array([12.0, -5.0, 3.0]), base.conn)
    Em = oracle.dense(moved, YOUNG, NU, method=1)
    assert np.abs(Em - E).max() <= 1e-10 * np.abs(E).max()
    lam = 3.5
    Es = oracle.dense(Mesh(base.xyz * lam, base.conn), YOUNG, NU, method=1)
    assert np.abs(Es * lam - E).max() <= 1e-10 * np.abs(E).max()
    E2 = oracle.dense(base, 2 * YOUNG, NU, method=1)
    assert np.abs(E2 - 2 * E).max() <= 1e-12 * np.abs(E).max()


def test_rectangle_equals_two_triangles_off_diagonal(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(6):
        # receiver: a tilted triangle somewhere; source: rectangle vs its halves
        rect = np.array([[0, 0, 0], [2.0, 0, 0], [2.0, 1.0, 0], [0, 1.0, 0]])
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        rect = rect @ q.T
        fs = np.stack([q[:, 0], q[:, 1], q[:, 2]])
        if np.linalg.det(q) < 0:
            fs[2] = -fs[2]
            rect = rect[[0, 3, 2, 1]]
            fs[0] = (rect[1] - rect[0]) / np.linalg.norm(rect[1] - rect[0])
            fs[1] = np.cross(fs[2], fs[0])
        x = rng.uniform(-3, 5, size=3)
        fr, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        fr = fr.T
        fr[2] = np.cross(fr[0], fr[1])
        full = oracle.pk_block(YOUNG, NU, x, fr, rect, fs)
        t1 = oracle.pk_block(YOUNG, NU, x, fr, rect[[0, 1, 2]], fs)
        t2 = oracle.pk_block(YOUNG, NU, x, fr, rect[[0, 2, 3]], fs)
        assert np.abs(full - (t1 + t2)).max() <= 1e-10 * np.abs(full).max()


def test_far_field_reciprocity(oracle_lib):
    # area-weighted reciprocity A_i E_ij^{ab} -> A_j E_ji^{ba}, error O((h/d)^2)
    rng = np.random.default_rng(5)
    tri_i = np.array([[0, 0, 0], [1.0, 0.2, 0], [0.3, 0.9, 0.1]])
    tri_j0 = np.array([[0, 0, 0], [0.7, 0.1, 0.3], [0.1, 0.8, -0.2]])
    _, fri, ai = _tri_frame(tri_i)
    errs = []
    for d in (8.0, 32.0):
        dirv = np.array([0.6, 0.5, 0.62])
        tri_j = tri_j0 + d * dirv / np.linalg.norm(dirv)
        _, frj, aj = _tri_frame(tri_j)
        ci, cj = tri_i.mean(0), tri_j.mean(0)
        Eij = oracle.pk_block(YOUNG, NU, ci, fri, tri_j, frj)
        Eji = oracle.pk_block(YOUNG, NU, cj, frj, tri_i, fri)
        errs.append(np.abs(ai * Eij - aj * Eji.T).max() / np.abs(ai * Eij).max())
    _ = rng
    assert errs[1] < errs[0] / 8.0 and errs[1] < 5e-3


def _tri_frame(t):
    e1, e2 = t[1] - t[0], t[2] - t[0]
    n = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(n)
    s1 = e1 / np.linalg.norm(e1)
    n = n / np.linalg.norm(n)
    return t.mean(0), np.stack([s1, np.cross(n, s1), n]), area


def test_rows_matvec_equals_dense_rows(oracle_lib):
    m = square_fault(10)
    E = oracle.dense(m, YOUNG, NU)
    X = np.random.default_rng(1).standard_normal((3, m.ndof))
    rows = np.array([0, 17, 55, 99])
    Y = oracle.rows_matvec(m, YOUNG, NU, rows, X)
    dof = (3 * rows[:, None] + np.arange(3)).ravel()
    assert np.allclose(Y, (E @ X.T).T[:, dof], rtol=1e-13, atol=1e-13 * np.abs(Y).max())


def test_frames_follow_stated_convention(oracle_lib):
    m = square_fault(2)
    cent, fr, area = oracle.frames(m)
    assert np.allclose(fr[0], np.eye(3))
    assert np.allclose(area, 1.0) and np.allclose(cent[0], [0.5, 0.5, 0.0])


def test_grid_toeplitz_product_equals_dense(oracle_lib):
    # The uniform-grid product (offset table + direct summation) against the
    # dense oracle: square grid, and a ragged grid of non-square rectangles
    # (nx != ny, h != hy), which catches a swapped (di, dj) or a transposed
    # offset sign; and against the PK quadrature alone (method 1), an
    # independent derivation of every table entry.
    from workloads import rhs_columns

    for nx, ny, h, hy in ((32, 32, 1.0, 1.0), (13, 7, 0.5, 1.3)):
        m = rect_grid(nx, ny, h, hy)
        X = rhs_columns(m.ndof, 3, 11)
        ref = oracle.matvec(oracle.dense(m, YOUNG, NU), X)
        T = oracle.grid_table(YOUNG, NU, nx, ny, h, hy)
        Y = oracle.grid_matvec(T, nx, ny, X)
        assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    m = rect_grid(8, 6, 1.0, 0.6)
    X = rhs_columns(m.ndof, 2, 12)
    ref = oracle.matvec(oracle.dense(m, YOUNG, NU, method=1), X)
    Y = oracle.grid_matvec(oracle.grid_table(YOUNG, NU, 8, 6, 1.0, 0.6), 8, 6, X)
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_grid_fft_product_equals_direct_sum(oracle_lib):
    # circulant embedding + FFT against the direct Toeplitz sum, ragged sizes
    from workloads import rhs_columns

    for nx, ny, hy in ((40, 23, 1.0), (5, 17, 2.0), (1, 9, 1.0)):
        T = oracle.grid_table(YOUNG, NU, nx, ny, 1.0, hy)
        X = rhs_columns(3 * nx * ny, 3, 13)
        Yd = oracle.grid_matvec(T, nx, ny, X)
        Yf = oracle.grid_matvec_fft(T, nx, ny, X)
        assert np.abs(Yf - Yd).max() <= 1e-12 * np.abs(Yd).max()


def test_grid_product_symmetric_and_planted_mistakes_fail(oracle_lib):
    # x.(E y) = y.(E x) on a grid of identical elements (E symmetric), and a
    # table with a mirrored offset axis (flips the odd s1-s2 coupling) or
    # with the two shear components swapped (h != hy) is caught by the dense
    # comparison above on the ragged grid
    from workloads import rhs_columns

    nx, ny = 11, 6
    T = oracle.grid_table(YOUNG, NU, nx, ny, 1.0, 0.7)
    x, y = rhs_columns(3 * nx * ny, 2, 14)
    Ex = oracle.grid_matvec(T, nx, ny, x)[0]
    Ey = oracle.grid_matvec(T, nx, ny, y)[0]
    assert abs(x @ Ey - y @ Ex) <= 1e-13 * abs(x @ Ey)
    m = rect_grid(nx, ny, 1.0, 0.7)
    ref = oracle.matvec(oracle.dense(m, YOUNG, NU), x)
    swapped = T.copy()
    swapped[..., 0, 0], swapped[..., 1, 1] = T[..., 1, 1], T[..., 0, 0]
    for bad in (T[:, ::-1].copy(), swapped):
        Yb = oracle.grid_matvec(bad, nx, ny, x)
        assert np.abs(Yb - ref).max() > 1e-6 * np.abs(ref).max()
