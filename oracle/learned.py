"""CPU FP64 oracle of the learned correction of the block preconditioner.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the library.  It shares no code with the GPU
path: plain numpy loops and dense algebra, in FP64.

The paper (Sec. 3.3.1) preconditions the inner A11 = E - eta/dt - C^ep
solves with a cheap approximation of A11 (point Jacobi) and has no learned
part; the learned form defined here corrects the 3x3 block-Jacobi inverse
B_e = (A11)_ee^-1 by a linear map over each element's K nearest elements:

    (M^-1 r)_e = B_e r_e + sum_{f in N(e)} W_ef r_f,
    W_ef = (h_e / E') * net(phi_ef)  (zero if e or f is inactive),

net(x) = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3, with output 3a + b
the (a, b) entry of W_ef, h_e = sqrt(area_e), E' = E / (1 - nu^2).  The
training loss over samples (b_s, x_s) with A11 x_s = b_s is

    L = (1/ns) sum_s ||M^-1 b_s - x_s||^2 / ||x_s||^2.

The base may also be any fixed matrix M_base in place of the 3x3 blocks
(the leaf block-Jacobi inverse is one): (M^-1 r) = M_base r + sum over pairs
W_ef r_f.  Wherever a function below takes Bb, a [N, 3, 3] array means the
per-element blocks B_e and a [3N, 3N] array means a dense M_base.

Every function here follows those definitions literally: K-nearest search
by brute force, features from their definitions, the dense preconditioner
matrix built block by block, the gradient by the chain rule written out
layer by layer (pinned against central finite differences in the tests).
"""
from __future__ import annotations

import numpy as np

N_FEAT = 32
N_USED = 20


def unpack(theta, H):
    """Split the flat parameter vector: W1 [32,H], b1 [H], W2 [H,H], b2 [H], W3 [H,9], b3 [9]."""
    t = np.asarray(theta, np.float64)
    sizes = [(N_FEAT, H), (H,), (H, H), (H,), (H, 9), (9,)]
    out, o = [], 0
    for sz in sizes:
        n = int(np.prod(sz))
        out.append(t[o:o + n].reshape(sz))
        o += n
    if o != t.size:
        raise ValueError("parameter count does not match the hidden width")
    return out


def n_params(H):
    return N_FEAT * H + H + H * H + H + H * 9 + 9


def knn_bruteforce(cent, K):
    """For every element e: the min(K, N) elements f with the smallest
    (|c_f - c_e|^2, f), in that order.  Returns pair arrays (pe, pf)."""
    cent = np.asarray(cent, np.float64)
    ne = len(cent)
    k = min(K, ne)
    pe, pf = [], []
    for e in range(ne):
        d2 = [(float(np.sum((cent[f] - cent[e]) ** 2)), f) for f in range(ne)]
        d2.sort()
        for _, f in d2[:k]:
            pe.append(e)
            pf.append(f)
    return np.array(pe, np.int64), np.array(pf, np.int64)


def features(cent, frame, area, D, active, patches, pe, pf, young, nu):
    """Pair features (float64 [P, 32]) and scales h_e / E' (0 if e or f is
    inactive).  frame[e] rows are (s1, s2, n); D [N, 3, 3] or None; active
    [N] bool or None; patches: list of element-index arrays (the groups
    over which the patch means 18-19 are taken)."""
    cent = np.asarray(cent, np.float64)
    frame = np.asarray(frame, np.float64)
    ne = len(cent)
    h = np.sqrt(np.asarray(area, np.float64))
    Ep = young / (1.0 - nu * nu)
    act = np.ones(ne, bool) if active is None else np.asarray(active, bool)
    patch = np.zeros((ne, 2))
    if D is not None:
        for grp in patches:
            members = [int(e) for e in grp]
            actm = [e for e in members if act[e]]
            if not actm:
                continue
            mn = np.mean([D[e][2, 2] * h[e] / Ep for e in actm])
            ms = np.mean([0.5 * (D[e][0, 0] + D[e][1, 1]) * h[e] / Ep for e in actm])
            for e in members:
                patch[e] = (mn, ms)
    P = len(pe)
    F = np.zeros((P, N_FEAT))
    scale = np.zeros(P)
    for p in range(P):
        e, f = int(pe[p]), int(pf[p])
        d = cent[f] - cent[e]
        for a in range(3):
            F[p, a] = frame[e][a] @ d / h[e]
        F[p, 3] = np.sqrt(d @ d) / h[e]
        F[p, 4] = frame[e][2] @ frame[f][2]
        F[p, 5] = frame[e][0] @ frame[f][0]
        F[p, 6] = frame[e][1] @ frame[f][1]
        if D is not None:
            se, sf = h[e] / Ep, h[f] / Ep
            for a in range(3):
                F[p, 7 + a] = D[e][a, a] * se
                F[p, 10 + a] = D[f][a, a] * sf
            F[p, 13] = D[e][0, 2] * se
            F[p, 14] = D[f][0, 2] * sf
            F[p, 15] = D[e][2, 0] * se
        F[p, 16] = h[f] / h[e]
        F[p, 17] = 1.0 if e == f else 0.0
        F[p, 18:20] = patch[e]
        scale[p] = h[e] / Ep if (act[e] and act[f]) else 0.0
    return F, scale


def block_jacobi(A, ne):
    """B_e = inverse of the 3x3 diagonal block (A11)_ee, [N, 3, 3]."""
    return np.array([np.linalg.inv(A[3 * e:3 * e + 3, 3 * e:3 * e + 3]) for e in range(ne)])


def forward(theta, H, F):
    """Network outputs [P, 9] and the activations (z1, a1, z2, a2)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, H)
    z1 = F @ W1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0.0)
    out = a2 @ W3 + b3
    return out, (z1, a1, z2, a2)


def blocks(theta, H, F, scale):
    """W_ef for every pair, [P, 3, 3]."""
    out, _ = forward(theta, H, F)
    return (scale[:, None] * out).reshape(-1, 3, 3)


def dense_preconditioner(Bb, pe, pf, Wb, ne):
    """M^-1 as a dense [3N, 3N] matrix, block by block."""
    if np.ndim(Bb) == 2:
        M = np.array(Bb, dtype=np.float64, copy=True)
    else:
        M = np.zeros((3 * ne, 3 * ne))
        for e in range(ne):
            M[3 * e:3 * e + 3, 3 * e:3 * e + 3] += Bb[e]
    for p in range(len(pe)):
        e, f = int(pe[p]), int(pf[p])
        M[3 * e:3 * e + 3, 3 * f:3 * f + 3] += Wb[p]
    return M


def apply(Bb, pe, pf, Wb, R):
    """Z = M^-1 R for R [ns, 3N], by the sum over pairs."""
    R = np.atleast_2d(np.asarray(R, np.float64))
    dense_base = np.ndim(Bb) == 2
    ne = R.shape[1] // 3 if dense_base else len(Bb)
    Z = np.zeros_like(R)
    for s in range(R.shape[0]):
        r = R[s].reshape(ne, 3)
        z = (Bb @ R[s]).reshape(ne, 3) if dense_base else np.einsum("eab,eb->ea", Bb, r)
        for p in range(len(pe)):
            z[pe[p]] += Wb[p] @ r[pf[p]]
        Z[s] = z.ravel()
    return Z


def loss(theta, H, F, scale, pe, pf, Bb, Bs, Xs):
    Wb = blocks(theta, H, F, scale)
    rho = apply(Bb, pe, pf, Wb, Bs) - Xs
    return float(np.mean(np.sum(rho ** 2, axis=1) / np.sum(Xs ** 2, axis=1)))


def loss_grad(theta, H, F, scale, pe, pf, Bb, Bs, Xs):
    """(L, dL/dtheta) by the chain rule:
    dL/dW_ef = sum_s 2 rho_{s,e} b_{s,f}^T / (ns ||x_s||^2);
    dL/dout_p = scale_p dL/dW_p (flattened row-major); then back through the
    three affine layers and the two ReLUs."""
    Bs = np.atleast_2d(Bs)
    Xs = np.atleast_2d(Xs)
    ns = Bs.shape[0]
    ne = Bs.shape[1] // 3
    W1, b1, W2, b2, W3, b3 = unpack(theta, H)
    out, (z1, a1, z2, a2) = forward(theta, H, F)
    Wb = (scale[:, None] * out).reshape(-1, 3, 3)
    rho = apply(Bb, pe, pf, Wb, Bs) - Xs
    xn = np.sum(Xs ** 2, axis=1)
    L = float(np.mean(np.sum(rho ** 2, axis=1) / xn))
    dW = np.zeros((len(pe), 3, 3))
    for s in range(ns):
        r3 = rho[s].reshape(ne, 3)
        b3v = Bs[s].reshape(ne, 3)
        w = 2.0 / (ns * xn[s])
        for p in range(len(pe)):
            dW[p] += w * np.outer(r3[pe[p]], b3v[pf[p]])
    dout = scale[:, None] * dW.reshape(-1, 9)
    gW3 = a2.T @ dout
    gb3 = dout.sum(0)
    da2 = dout @ W3.T
    dz2 = da2 * (z2 > 0)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(0)
    da1 = dz2 @ W2.T
    dz1 = da1 * (z1 > 0)
    gW1 = F.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g
