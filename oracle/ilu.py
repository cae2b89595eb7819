"""CPU FP64 oracle of the paper's sparse approximation of A11 and of its
incomplete LU factorisation (Sec. 3.3.1, solution of the Jacobian system,
second choice of the approximate A11).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the library.
It shares no code with the GPU path: its own cluster and block trees, its
own dense collocation matrix (oracle.dense), its own selection, colouring
and factorisation.

What is computed, in the paper's order:
  1. the near field: the entries of E in the full-rank (inadmissible) leaf
     blocks of the hierarchical partition (cluster tree by median bisection
     of the collocation points along the longest box axis, ties by element
     id; a pair of clusters is admissible when min(diam) <= eta dist with
     vertex bounding boxes, box diagonal and box-to-box distance, dist > 0);
  2. the fraction p of those entries with the largest absolute value: the
     count is k = ceil(p x (number of near-field entries, 9 m n per block))
     and an entry is kept when its magnitude key is at least the k-th
     largest key, the key of a value being the bit pattern of |a| without
     its last 15 bits (a 48-bit integer: exponent and 37 mantissa bits);
  3. A~11 = (kept entries of E) - D on active elements, D = eta/dt + C^ep
     (block diagonal 3x3), every 3x3 diagonal block present in the pattern;
     an inactive element has an identity row and column and no coupling;
  4. an ordering of the unknowns: the elements coloured greedily in
     increasing id (each takes the smallest colour no lower-id neighbour
     holds; neighbours = elements coupled by a pattern entry in either
     direction), then ordered by (colour, id), the three DOFs of an element
     in order s1, s2, n;
  5. ILU(0) of A~11 in that ordering: Gaussian elimination that keeps only
     the positions of the pattern (row by row, eliminating with the earlier
     rows in order), so that (L U)_ij = A~_ij on the pattern;
  6. z = U^-1 L^-1 r.
"""
from __future__ import annotations

import math

import numpy as np

KEY_SHIFT = 15


# ------------------------------------------------------------------ partition
def near_field_blocks(mesh, leaf: int, eta: float):
    """Inadmissible leaf pairs of the hierarchical partition, as a list of
    (target element ids, source element ids)."""
    cent = mesh.xyz[mesh.conn].mean(axis=1)
    v = mesh.xyz[mesh.conn]
    vmin, vmax = v.min(axis=1), v.max(axis=1)
    nodes = []   # (ids, (box min, box max), children or None)

    def build(ids):
        nid = len(nodes)
        nodes.append(None)
        box = (vmin[ids].min(0), vmax[ids].max(0))
        if len(ids) > leaf:
            ext = cent[ids].max(0) - cent[ids].min(0)
            ax = int(np.argmax(ext))
            ids = ids[np.lexsort((ids, cent[ids, ax]))]
            h = len(ids) // 2
            kids = (build(ids[:h]), build(ids[h:]))
            nodes[nid] = (ids, box, kids)
        else:
            nodes[nid] = (ids, box, None)
        return nid

    build(np.arange(mesh.conn.shape[0]))

    def diam(b):
        return float(np.linalg.norm(b[1] - b[0]))

    def dist(a, b):
        return float(np.linalg.norm(np.maximum(0.0, np.maximum(a[0] - b[1], b[0] - a[1]))))

    out = []

    def blocks(t, s):
        bt, bs = nodes[t][1], nodes[s][1]
        d = dist(bt, bs)
        if d > 0.0 and min(diam(bt), diam(bs)) <= eta * d:
            return
        ct, cs = nodes[t][2], nodes[s][2]
        if ct is None and cs is None:
            out.append((nodes[t][0], nodes[s][0]))
        elif ct is None:
            for j in cs:
                blocks(t, j)
        elif cs is None:
            for i in ct:
                blocks(i, s)
        else:
            for i in ct:
                for j in cs:
                    blocks(i, j)

    blocks(0, 0)
    return out


def near_field_mask(n_elem: int, blocks) -> np.ndarray:
    """Boolean [3N, 3N]: the DOF pairs of the near field."""
    M = np.zeros((n_elem, n_elem), dtype=bool)
    for t, s in blocks:
        M[np.ix_(t, s)] = True
    return np.kron(M, np.ones((3, 3), dtype=bool))


# ------------------------------------------------------------------ selection
def magnitude_key(a) -> np.ndarray:
    """48-bit integer key of |a|: the IEEE bit pattern without its last 15 bits
    (non-negative doubles order like their bit patterns)."""
    return np.abs(np.asarray(a, dtype=np.float64)).view(np.uint64) >> np.uint64(KEY_SHIFT)


def select_near_field(E: np.ndarray, near: np.ndarray, p: float):
    """Kept near-field positions (boolean [3N, 3N]) and the threshold key:
    k = ceil(p x #near entries); keep key >= the k-th largest key."""
    keys = magnitude_key(E[near])
    k = max(1, int(math.ceil(p * keys.size)))
    kth = np.sort(keys)[keys.size - k]
    keep = np.zeros_like(near)
    keep[near] = keys >= kth
    return keep, int(kth), k


def tilde_a11(E: np.ndarray, keep: np.ndarray, D: np.ndarray | None, active: np.ndarray | None):
    """Dense storage of A~11 and its pattern (boolean), see the module docstring."""
    n = E.shape[0] // 3
    A = np.where(keep, E, 0.0)
    pat = keep.copy()
    for e in range(n):
        sl = slice(3 * e, 3 * e + 3)
        if D is not None:
            A[sl, sl] -= D[e]
        pat[sl, sl] = True
    if active is not None:
        act = np.repeat(np.asarray(active, bool), 3)
        A[~act, :] = 0.0
        A[:, ~act] = 0.0
        pat[~act, :] = False
        pat[:, ~act] = False
        idx = np.flatnonzero(~act)
        A[idx, idx] = 1.0
        pat[idx, idx] = True
    return A, pat


# ------------------------------------------------------------------ ordering
def greedy_colouring(pat: np.ndarray) -> np.ndarray:
    """Colour of each element: in increasing id, the smallest colour not held
    by a lower-id element coupled to it (either direction)."""
    n = pat.shape[0] // 3
    G = pat.reshape(n, 3, n, 3).any(axis=(1, 3))
    G = G | G.T
    colour = np.full(n, -1, dtype=np.int64)
    for e in range(n):
        used = set(colour[f] for f in np.flatnonzero(G[e, :e]))
        c = 0
        while c in used:
            c += 1
        colour[e] = c
    return colour


def dof_order(colour: np.ndarray) -> np.ndarray:
    """DOFs in elimination order: elements by (colour, id), then s1, s2, n."""
    elems = np.lexsort((np.arange(colour.size), colour))
    return (3 * elems[:, None] + np.arange(3)).ravel()


# ------------------------------------------------------------------ ILU(0)
def ilu0(A: np.ndarray, pat: np.ndarray, order: np.ndarray) -> np.ndarray:
    """ILU(0) of A in the given DOF order: returns the factors packed in one
    array F (in that order): unit lower L below the diagonal, U on and above,
    zero outside the pattern."""
    P = A[np.ix_(order, order)].copy()
    S = pat[np.ix_(order, order)]
    n = P.shape[0]
    for i in range(n):
        for k in np.flatnonzero(S[i, :i]):
            P[i, k] /= P[k, k]
            upd = S[i, k + 1:] & S[k, k + 1:]
            P[i, k + 1:][upd] -= P[i, k] * P[k, k + 1:][upd]
        if P[i, i] == 0.0:
            raise ZeroDivisionError(f"zero pivot at position {i}")
    return np.where(S, P, 0.0)


def ilu0_apply(F: np.ndarray, order: np.ndarray, R: np.ndarray) -> np.ndarray:
    """z = U^-1 L^-1 r for each row of R [nrhs, 3N] (original DOF order)."""
    import scipy.linalg as sl

    R = np.atleast_2d(R)
    L = np.tril(F, -1) + np.eye(F.shape[0])
    U = np.triu(F)
    Z = np.empty_like(R)
    for c in range(R.shape[0]):
        y = sl.solve_triangular(L, R[c, order], lower=True, unit_diagonal=True)
        z = sl.solve_triangular(U, y, lower=False)
        Z[c, order] = z
    return Z
