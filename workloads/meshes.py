"""Seeded mesh and right-hand-side generators for the fault/fracture workloads.

Only layout and seeded draws live here (see the package docstring).  The
shapes follow the paper's workloads: planar faults meshed by uniform
rectangles, disk-shaped fractures meshed by triangles (three intersecting
fractures, Sec. 5), and a height-confined hydraulic fracture crossing a
vertical strike-slip fault (Sec. 5).  Element sizes are chosen to give the
element counts of the benchmark configurations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    xyz: np.ndarray          # float64 [nv, 3]
    conn: np.ndarray         # int64 [ne, 3 or 4]
    name: str = "mesh"
    meta: dict = field(default_factory=dict)

    @property
    def nvpe(self) -> int:
        return int(self.conn.shape[1])

    @property
    def ne(self) -> int:
        return int(self.conn.shape[0])

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def ndof(self) -> int:
        return 3 * self.ne

    def vertex_means(self) -> np.ndarray:
        """Mean of each element's vertices (layout helper for seeding loads)."""
        return self.xyz[self.conn].mean(axis=1)


def _orthonormal_axes(axes) -> np.ndarray:
    a = np.asarray(axes, dtype=np.float64).reshape(3, 3)
    q, _ = np.linalg.qr(a.T)
    q = q.T
    # keep the orientation of the given first two axes
    for k in range(2):
        if np.dot(q[k], a[k]) < 0:
            q[k] = -q[k]
    q[2] = np.cross(q[0], q[1])
    return q


def rect_grid(nx: int, ny: int, h: float = 1.0, hy: float | None = None,
              origin=(0.0, 0.0, 0.0), axes=None, name="rect_grid") -> Mesh:
    """Uniform grid of nx*ny planar rectangles.

    Element e = i + nx*j covers [i h, (i+1) h] x [j hy, (j+1) hy] in the
    plane spanned by ``axes[0]`` (first in-plane axis) and ``axes[1]``;
    vertices are listed counter-clockwise about ``axes[2]``.
    """
    hy = h if hy is None else hy
    ax = np.eye(3) if axes is None else _orthonormal_axes(axes)
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    u = (ii.ravel() * h)[:, None]
    v = (jj.ravel() * hy)[:, None]
    xyz = np.asarray(origin, dtype=np.float64)[None, :] + u * ax[0][None, :] + v * ax[1][None, :]
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    vid = lambda a, b: a + (nx + 1) * b  # noqa: E731
    conn = np.stack([vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)], axis=1)
    return Mesh(xyz.astype(np.float64), conn.astype(np.int64), name,
                {"nx": nx, "ny": ny, "h": h, "hy": hy, "axes": ax,
                 "origin": np.asarray(origin, dtype=np.float64)})


def square_fault(n: int, h: float = 1.0) -> Mesh:
    """Planar square fault in z = 0 made of n x n squares of side h.

    n = 32 is the small configuration (1,024 elements, 3,072 DOF); n = 256
    is the primary throughput configuration (65,536 elements, 196,608 DOF).
    """
    return rect_grid(n, n, h, name=f"square_fault_{n}x{n}")


def penny_active_mask(mesh: Mesh, radius_fraction: float = 0.45) -> np.ndarray:
    """Elements of a square grid whose centre lies within a centred disk.

    The disk radius is ``radius_fraction`` times the fault side.  Returns a
    uint8 mask [ne] (1 = element on the crack).
    """
    nx, ny, h, hy = (mesh.meta[k] for k in ("nx", "ny", "h", "hy"))
    side = nx * h
    a = radius_fraction * side
    i = np.arange(mesh.ne) % nx
    j = np.arange(mesh.ne) // nx
    cx = (i + 0.5) * h - 0.5 * nx * h
    cy = (j + 0.5) * hy - 0.5 * ny * hy
    return (np.hypot(cx, cy) <= a + 1e-12).astype(np.uint8)


def disk_mesh(radius: float, rings: int, center=(0.0, 0.0, 0.0), axes=None,
              spin: float = 0.0, name="disk") -> Mesh:
    """Concentric-ring triangulation of a disk: 6 k points on ring k.

    Gives 6 * rings**2 triangles, counter-clockwise about ``axes[2]``.
    ``spin`` rotates the in-plane pattern (used to move centroids off
    foreign edges at fracture intersections).
    """
    ax = np.eye(3) if axes is None else _orthonormal_axes(axes)
    pts = [(0.0, 0.0)]
    ring_start = [0]
    for k in range(1, rings + 1):
        ring_start.append(len(pts))
        r = radius * k / rings
        th = spin + 2.0 * np.pi * np.arange(6 * k) / (6 * k)
        pts.extend(zip(r * np.cos(th), r * np.sin(th)))
    pts = np.asarray(pts)
    tris = []
    for k in range(1, rings + 1):
        for s in range(6):
            # inner ring k-1 has k-1 segments per sector, outer ring k has k
            def outer(q):
                return ring_start[k] + (s * k + q) % (6 * k)

            def inner(q):
                if k == 1:
                    return 0
                return ring_start[k - 1] + (s * (k - 1) + q) % (6 * (k - 1))

            for q in range(k):
                tris.append((outer(q), outer(q + 1), inner(q)))
            for q in range(k - 1):
                tris.append((inner(q), outer(q + 1), inner(q + 1)))
    tris = np.asarray(tris, dtype=np.int64)
    xyz = (np.asarray(center, dtype=np.float64)[None, :]
           + pts[:, :1] * ax[0][None, :] + pts[:, 1:2] * ax[1][None, :])
    return Mesh(xyz, tris, name, {"radius": radius, "rings": rings, "axes": ax,
                                  "center": np.asarray(center, dtype=np.float64)})


def rect_tri_mesh(lx: float, ly: float, nx: int, ny: int, center=(0.0, 0.0, 0.0),
                  axes=None, name="rect_tri") -> Mesh:
    """Rectangle lx x ly split into nx*ny cells, each cut into two right triangles."""
    ax = np.eye(3) if axes is None else _orthonormal_axes(axes)
    hx, hy = lx / nx, ly / ny
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    u = ii.ravel() * hx - 0.5 * lx
    v = jj.ravel() * hy - 0.5 * ly
    xyz = (np.asarray(center, dtype=np.float64)[None, :]
           + u[:, None] * ax[0][None, :] + v[:, None] * ax[1][None, :])
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    vid = lambda a, b: a + (nx + 1) * b  # noqa: E731
    t1 = np.stack([vid(i, j), vid(i + 1, j), vid(i + 1, j + 1)], axis=1)
    t2 = np.stack([vid(i, j), vid(i + 1, j + 1), vid(i, j + 1)], axis=1)
    conn = np.empty((2 * nx * ny, 3), dtype=np.int64)
    conn[0::2] = t1
    conn[1::2] = t2
    return Mesh(xyz, conn, name, {"lx": lx, "ly": ly, "nx": nx, "ny": ny, "axes": ax,
                                  "center": np.asarray(center, dtype=np.float64)})


def _merge(meshes, name) -> Mesh:
    xyz, conn, off = [], [], 0
    parts = []
    for m in meshes:
        xyz.append(m.xyz)
        conn.append(m.conn + off)
        parts.append((sum(c.shape[0] for c in conn[:-1]), m.ne))
        off += m.nv
    return Mesh(np.concatenate(xyz), np.concatenate(conn), name,
                {"parts": parts, "submeshes": meshes})


def _point_segment_dist(p, a, b):
    ab = b - a
    t = np.clip(np.einsum("ij,ij->i", p - a, ab) / np.einsum("ij,ij->i", ab, ab), 0.0, 1.0)
    q = a + t[:, None] * ab
    return np.linalg.norm(p - q, axis=1)


def _min_foreign_edge_distance(m_recv: Mesh, m_src: Mesh, band: float) -> float:
    """Smallest distance from receiver vertex-means to source-mesh edges.

    Only receiver points within ``band`` of the source plane are examined
    (others cannot be close to its edges).
    """
    c = m_recv.vertex_means()
    n = m_src.meta["axes"][2]
    o = m_src.xyz[0]
    near = np.abs((c - o) @ n) < band
    if not np.any(near):
        return np.inf
    c = c[near]
    k = m_src.nvpe
    e0 = m_src.xyz[m_src.conn].reshape(-1, 3)
    e1 = m_src.xyz[np.roll(m_src.conn, -1, axis=1)].reshape(-1, 3)
    from scipy.spatial import cKDTree

    mid = 0.5 * (e0 + e1)
    half = 0.5 * np.max(np.linalg.norm(e1 - e0, axis=1))
    tree = cKDTree(mid)
    best = np.inf
    for idx, cand in enumerate(tree.query_ball_point(c, r=band + half)):
        if cand:
            cand = np.asarray(cand)
            d = _point_segment_dist(np.repeat(c[idx:idx + 1], len(cand), 0), e0[cand], e1[cand])
            best = min(best, float(d.min()))
    _ = k
    return best


def three_disks(radius: float = 40.0, rings: int = 76, seed: int = 3001,
                min_edge_frac: float = 0.005) -> Mesh:
    """Three mutually intersecting disk fractures meshed independently.

    Disk A dips 65 degrees; B and C take seeded orientations and centres so
    that every pair of planes intersects inside both disks.  Triangles of a
    later disk that cut through an earlier one are removed (a slit one
    element wide along each intersection), so no element crosses another
    fracture.  Triangulations
    are spun and nudged along their normal (seeded) until every element's
    vertex mean is at least ``min_edge_frac`` times the mesh size away from
    the other disks' edges.
    The default gives about 103,400 triangles (3 x 34,656 minus the slits).
    """
    rng = np.random.default_rng(seed)
    dip = np.deg2rad(65.0)
    nA = np.array([np.sin(dip), 0.0, np.cos(dip)])
    axesA = np.stack([np.array([0.0, 1.0, 0.0]), np.cross(nA, [0.0, 1.0, 0.0]), nA])
    frames = [(np.zeros(3), axesA)]
    while len(frames) < 3:
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        cen = rng.uniform(-8.0, 8.0, size=3)
        ok = True
        for c0, a0 in frames:
            n0 = a0[2]
            s = np.linalg.norm(np.cross(n0, nrm))
            if s < np.sin(np.deg2rad(35.0)):
                ok = False
                break
            # intersection line of the two planes; distance from each centre
            d = np.cross(n0, nrm)
            d /= np.linalg.norm(d)
            A = np.stack([n0, nrm, d])
            p = np.linalg.solve(A, np.array([n0 @ c0, nrm @ cen, 0.0]))
            for cc in (c0, cen):
                v = cc - p
                if np.linalg.norm(v - (v @ d) * d) > 0.6 * radius:
                    ok = False
        if not ok:
            continue
        t = np.cross(nrm, [0.0, 0.0, 1.0] if abs(nrm[2]) < 0.9 else [1.0, 0.0, 0.0])
        t /= np.linalg.norm(t)
        frames.append((cen, np.stack([t, np.cross(nrm, t), nrm])))
    h = radius / rings
    disks = []
    for k, (c, a) in enumerate(frames):
        spin, shift = 0.0, 0.0
        for _ in range(256):
            dk = _drop_crossing(disk_mesh(radius, rings, c + shift * a[2], a, spin=spin, name=f"disk{k}"),
                                disks, radius)
            good = all(
                _min_foreign_edge_distance(dk, o, 2.0 * h) >= min_edge_frac * h
                and _min_foreign_edge_distance(o, dk, 2.0 * h) >= min_edge_frac * h
                for o in disks)
            if good:
                break
            spin = float(rng.uniform(0.0, 2.0 * np.pi))
            shift = float(rng.uniform(-0.5, 0.5)) * h
        else:
            raise RuntimeError("could not place disk away from foreign edges")
        disks.append(dk)
    return _merge(disks, "three_disks")


def _inside(o: Mesh, p: np.ndarray) -> np.ndarray:
    """Points (already projected on o's plane) inside o's footprint."""
    ax, c0 = o.meta["axes"], o.meta["center"]
    d = p - c0
    if "radius" in o.meta:
        return np.linalg.norm(d, axis=-1) <= o.meta["radius"]
    u, v = d @ ax[0], d @ ax[1]
    return (np.abs(u) <= 0.5 * o.meta["lx"]) & (np.abs(v) <= 0.5 * o.meta["ly"])


def _drop_crossing(m: Mesh, others, radius: float = 0.0) -> Mesh:
    """Remove triangles of ``m`` that cut through an earlier fracture
    (vertices on both sides of its plane, inside its footprint): fractures
    meet along a slit one element wide instead of interpenetrating."""
    keep = np.ones(m.ne, dtype=bool)
    for o in others:
        n, c0 = o.meta["axes"][2], o.meta["center"]
        v = m.xyz[m.conn]                        # [ne, 3, 3]
        sd = (v - c0) @ n                        # signed distances of the vertices
        crosses = (sd.min(axis=1) < 0) & (sd.max(axis=1) > 0)
        inplane = v - sd[..., None] * n          # projections on the other plane
        near = _inside(o, inplane).any(axis=1)
        keep &= ~(crosses & near)
    used = np.unique(m.conn[keep])
    remap = -np.ones(m.nv, dtype=np.int64)
    remap[used] = np.arange(used.size)
    meta = dict(m.meta)
    meta["dropped"] = int((~keep).sum())
    return Mesh(m.xyz[used], remap[m.conn[keep]], m.name, meta)


def hf_fault_mesh(h: float = 0.46, seed: int = 5001, min_edge_frac: float = 0.05) -> Mesh:
    """Height-confined hydraulic fracture crossing a vertical strike-slip fault.

    Fracture: 60 m (x) by 20 m (z) in the plane y = 0, centred at the
    origin.  Fault: vertical, 200 m along strike by 100 m high, strike at 30
    degrees to x, centred at (20, 0, 0).  Both are meshed by right
    triangles of leg about ``h``; the fault is shifted along strike by a
    seeded fraction of a cell until vertex means stay ``min_edge_frac * h``
    away from the other mesh's edges.
    """
    rng = np.random.default_rng(seed)
    hf_axes = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, -1.0, 0.0]])
    nx, ny = int(round(60.0 / h)), int(round(20.0 / h))
    hf = rect_tri_mesh(60.0, 20.0, nx, ny, (0.0, 0.0, 0.0), hf_axes, "hf")
    st = np.deg2rad(30.0)
    s1 = np.array([np.cos(st), np.sin(st), 0.0])
    f_axes = np.stack([s1, np.array([0.0, 0.0, 1.0]), np.cross(s1, [0.0, 0.0, 1.0])])
    fx, fy = int(round(200.0 / h)), int(round(100.0 / h))
    shift = 0.0
    for _ in range(64):
        center = np.array([20.0, 0.0, 0.0]) + shift * h * s1
        fault = _drop_crossing(rect_tri_mesh(200.0, 100.0, fx, fy, center, f_axes, "fault"), [hf])
        if (_min_foreign_edge_distance(hf, fault, 2.0 * h) >= min_edge_frac * h
                and _min_foreign_edge_distance(fault, hf, 2.0 * h) >= min_edge_frac * h):
            break
        shift = float(rng.uniform(0.0, 1.0))
    else:
        raise RuntimeError("could not place fault away from fracture edges")
    return _merge([hf, fault], "hf_x_fault")


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def batched_faults(n_meshes: int = 64, seed: int = 4001, nmin: int = 2000,
                   nmax: int = 40000) -> list[Mesh]:
    """Independent planar faults: seeded element counts, aspect ratios 1-4
    and random orientations; square elements of side 1 m."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n_meshes):
        n = int(rng.integers(nmin, nmax + 1))
        a = float(rng.uniform(1.0, 4.0))
        nx = max(1, int(round(np.sqrt(n * a))))
        ny = max(1, int(round(n / nx)))
        R = _random_rotation(rng)
        origin = rng.uniform(-100.0, 100.0, size=3)
        out.append(rect_grid(nx, ny, 1.0, origin=origin, axes=R.T, name=f"fault{m}"))
    return out


def rhs_columns(n: int, ncols: int, seed0: int) -> np.ndarray:
    """ncols seeded N(0,1) vectors of length n; column c uses seed seed0 + c.

    Returned as float64 [ncols, n] (each column contiguous)."""
    return np.stack([np.random.default_rng(seed0 + c).standard_normal(n)
                     for c in range(ncols)]).astype(np.float64)


def gaussian_pressure_traction(mesh: Mesh, peak: float = 5e6, sigma: float = 8.0,
                               seed: int = 3002) -> np.ndarray:
    """Traction load t = (0, 0, -p(x)) per element for a Gaussian pressure
    bump p = peak * exp(-|x - x0|^2 / (2 sigma^2)); x0 is the first
    submesh's centre plus a seeded in-plane offset of at most 5 m."""
    rng = np.random.default_rng(seed)
    sub = mesh.meta.get("submeshes", [mesh])[0]
    ax = sub.meta["axes"]
    c0 = sub.meta.get("center", sub.xyz.mean(axis=0))
    r = rng.uniform(0.0, 5.0)
    th = rng.uniform(0.0, 2.0 * np.pi)
    x0 = c0 + r * (np.cos(th) * ax[0] + np.sin(th) * ax[1])
    x = mesh.vertex_means()
    p = peak * np.exp(-np.sum((x - x0) ** 2, axis=1) / (2.0 * sigma * sigma))
    t = np.zeros((mesh.ne, 3))
    t[:, 2] = -p
    return t.reshape(-1)


def tangent_state(mesh: Mesh, k: int, n_states: int = 20, young: float = 30e9, nu: float = 0.25,
                  rho: float = 2700.0, friction: float = 0.6, dilatancy: float = 0.0,
                  injection=(20.0, 0.0, 0.0), rmax: float = 60.0, seed: int = 5001) -> np.ndarray:
    """Synthetic tangent state k of an injection sequence on a multi-part mesh.

    Returns D [ne, 3, 3] = eta/dt + C^ep in each element's local frame
    (s1, s2, n), the block-diagonal part of the mechanical Jacobian
    A11 = E - eta/dt - C^ep (paper Sec. 3.1.1).  Inside a front of radius
    rmax * sqrt((k + 1) / n_states) around the injection point, elements of
    the first part (the hydraulic fracture) are open (C^ep = 0) and elements
    of the other parts (the fault) have yielded in Coulomb friction along
    s1: C^ep = C - (C N)(gradF^T C) / (gradF^T C N) with gradF = s1 + f n,
    N = s1 + psi n (paper Sec. 2.2).  Elsewhere elements are intact,
    C = diag(Ks, Ks, Kn) with Ks = Kn = E' / h.  The quasi-dynamic term is
    eta = (1/2) diag(G/cs, G/cs, G/cp) (paper Sec. 3.1) over a seeded time
    step 10^U(-1, 2) s.
    """
    rng = np.random.default_rng(seed + k)
    G = young / (2.0 * (1.0 + nu))
    K = young / (3.0 * (1.0 - 2.0 * nu))
    Ep = young / (1.0 - nu * nu)
    cs, cp = np.sqrt(G / rho), np.sqrt((K + 4.0 * G / 3.0) / rho)
    dt = 10.0 ** rng.uniform(-1.0, 2.0)
    eta = 0.5 * np.array([G / cs, G / cs, G / cp])
    x = mesh.vertex_means()
    v = mesh.xyz[mesh.conn]
    if mesh.nvpe == 3:
        area = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    else:
        area = np.linalg.norm(v[:, 1] - v[:, 0], axis=1) * np.linalg.norm(v[:, 3] - v[:, 0], axis=1)
    h = np.sqrt(area)
    kstiff = Ep / h
    radius = rmax * np.sqrt((k + 1.0) / n_states)
    inside = np.linalg.norm(x - np.asarray(injection), axis=1) <= radius
    parts = mesh.meta.get("parts", [(0, mesh.ne)])
    first = np.zeros(mesh.ne, dtype=bool)
    first[parts[0][0]:parts[0][0] + parts[0][1]] = True
    D = np.zeros((mesh.ne, 3, 3))
    D[:, [0, 1, 2], [0, 1, 2]] = kstiff[:, None]                 # intact
    D[inside & first] = 0.0                                      # open
    yielded = inside & ~first
    # with C = K I: C^ep = K (I - N gradF^T / (gradF . N)), N = (1, 0, psi), gradF = (1, 0, f)
    Nv = np.array([1.0, 0.0, dilatancy])
    gF = np.array([1.0, 0.0, friction])
    Cy = np.eye(3) - np.outer(Nv, gF) / (gF @ Nv)
    D[yielded] = kstiff[yielded, None, None] * Cy[None]
    D[:, [0, 1, 2], [0, 1, 2]] += eta[None, :] / dt
    return D


def tangent_rhs(mesh: Mesh, nrhs: int, seed: int, scale: float = 1e6) -> np.ndarray:
    """Right-hand sides for tangent solves: even columns seeded N(0, 1)
    tractions, odd columns normal pressure increments (Gaussian bumps of
    seeded centre and width on the normal component only).  [nrhs, 3 ne]."""
    rng = np.random.default_rng(seed)
    x = mesh.vertex_means()
    out = np.zeros((nrhs, mesh.ne, 3))
    for c in range(nrhs):
        if c % 2 == 0:
            out[c] = rng.standard_normal((mesh.ne, 3))
        else:
            x0 = x[rng.integers(mesh.ne)]
            w = rng.uniform(3.0, 15.0)
            out[c, :, 2] = -np.exp(-np.sum((x - x0) ** 2, axis=1) / (2.0 * w * w))
    return scale * out.reshape(nrhs, -1)
