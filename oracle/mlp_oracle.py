"""Learned warm start for the CCD iteration: FP64 CPU reference of the
per-amplitude network, its features, targets, loss, gradients and the Adam
update (test infrastructure only: the test-suite, smoke() and the CPU-baseline
leg of bench.py may import it; nothing here is shared with the GPU path).

What is learned.  The iteration of eq. ccd3 is started from the MBPT2
amplitudes t0 = <ab||ij> / eps_ij^ab (eq. ccdGuess).  At the fixed point,
t eps_ij^ab = <ab||ij> + (ladder, ring, one-body and quadratic terms), so the
network predicts the part beyond MBPT2:

    t_ij^ab = (v + y / s) / D,   D = eps_i + eps_j - eps_a - eps_b,
    v = <ab||ij>,  s = L^3 / (1000 MeV fm^3),

and y = 0 gives back the MBPT2 start.  Amplitudes of S_z = +-1 blocks have
v = 0 but are not zero at convergence (the ring term feeds them); the
encoding leaves y free there.

Features of one amplitude (sec. "Two-body interaction" for the relative
momentum transfer q = (k_a - k_b - k_i + k_j) / 2 of <ab|v|ij>, k = 2 pi n / L):
    rho / 0.16,  |q|,  |q'|,  eps_i / 100,  eps_j / 100,  eps_a / 100,  eps_b / 100,  v s
with q' = (k_b - k_a - k_i + k_j) / 2 the transfer of the exchanged element,
energies in MeV and momenta in fm^-1.

Network g: three linear layers, 7 -> 128 -> 128 -> 1, ReLU after the first
two (relu(z) = max(z, 0); its derivative is taken as 0 at z = 0).  The
prediction is antisymmetrised over a <-> b and i <-> j, which swaps the
corresponding energies, maps q to q'
(either single swap) or to -q (both) and flips the sign of v:
    y = ( g(x) - g(x_ab) - g(x_ij) + g(x_abij) ) / 4,
so y (and t) change sign under either swap, as t_ij^ab must.

Loss over M amplitudes: L = (1/M) sum_e (y_e - y*_e)^2 / 2, with the target
y* = (t D - v) s from converged amplitudes.  Adam as in Kingma and Ba (2015),
Algorithm 1.
"""
from __future__ import annotations

import numpy as np

WIDTH = 128
N_IN = 7
RHO0, E0, VSCALE = 0.16, 100.0, 1000.0

# ---------------------------------------------------------------------------
# features and targets
# ---------------------------------------------------------------------------


def features(pnm, ijab):
    """Packed features [M, 8] of the amplitudes t_ij^ab listed as rows (i, j,
    a, b) of ijab, for an oracle.PNM model space."""
    st = pnm.states()
    eps = pnm.fock()
    L = pnm.L
    ku = 2.0 * np.pi / L
    s = L ** 3 / VSCALE
    out = np.zeros((len(ijab), 8))
    for r, (i, j, a, b) in enumerate(ijab):
        ni, nj, na, nb = (st[x, :3].astype(np.float64) for x in (i, j, a, b))
        q = 0.5 * ku * (na - nb - ni + nj)
        qx = 0.5 * ku * (nb - na - ni + nj)
        out[r] = (pnm.rho / RHO0, np.sqrt(q @ q), np.sqrt(qx @ qx),
                  eps[i] / E0, eps[j] / E0, eps[a] / E0, eps[b] / E0, pnm.v(a, b, i, j) * s)
    return out


def denominators(pnm, ijab):
    eps = pnm.fock()
    return np.array([eps[i] + eps[j] - eps[a] - eps[b] for i, j, a, b in ijab])


def targets(pnm, ijab, t):
    """y* = (t D - v) s for amplitudes t of the rows of ijab."""
    s = pnm.L ** 3 / VSCALE
    D = denominators(pnm, ijab)
    v = np.array([pnm.v(a, b, i, j) for i, j, a, b in ijab])
    return (np.asarray(t) * D - v) * s


def amplitudes(pnm, ijab, y):
    """t = (v + y / s) / D (the warm start from predictions y)."""
    s = pnm.L ** 3 / VSCALE
    D = denominators(pnm, ijab)
    v = np.array([pnm.v(a, b, i, j) for i, j, a, b in ijab])
    return (v + np.asarray(y) / s) / D


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

SIGNS = np.array([1.0, -1.0, -1.0, 1.0])


def variants(F):
    """[M, 8] packed features -> [4M, 7] inputs, element-major (row 4e + k):
    identity, a <-> b, i <-> j, both."""
    F = np.asarray(F, dtype=np.float64)
    rho, q, qx, ei, ej, ea, eb, v = (F[:, k] for k in range(8))
    X = np.stack([
        np.stack([rho, q, ei, ej, ea, eb, v], 1),
        np.stack([rho, qx, ei, ej, eb, ea, -v], 1),
        np.stack([rho, qx, ej, ei, ea, eb, -v], 1),
        np.stack([rho, q, ej, ei, eb, ea, v], 1),
    ], 1)
    return X.reshape(-1, N_IN)


def relu(z):
    return np.maximum(z, 0.0)


def drelu(z):
    return (z > 0.0).astype(np.float64)


def g_forward(P, X):
    """Raw network output per input row, with the intermediates."""
    z1 = X @ P["W1"].T + P["b1"]
    h1 = relu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = relu(z2)
    g = h2 @ P["W3"] + P["b3"]
    return g, (X, z1, h1, z2, h2)


def predict(P, F):
    g, _ = g_forward(P, variants(F))
    return (g.reshape(-1, 4) @ SIGNS) / 4.0


def loss_and_grad(P, F, Y):
    """L = (1/M) sum (y - y*)^2 / 2 and dL/dP by backpropagation."""
    M = len(F)
    g, (X, z1, h1, z2, h2) = g_forward(P, variants(F))
    y = (g.reshape(-1, 4) @ SIGNS) / 4.0
    res = y - np.asarray(Y, dtype=np.float64)
    L = 0.5 * np.mean(res ** 2)
    dg = (res[:, None] * SIGNS[None, :] / (4.0 * M)).reshape(-1)
    G = {"W3": h2.T @ dg, "b3": np.sum(dg)}
    dz2 = np.outer(dg, P["W3"]) * drelu(z2)
    G["W2"] = dz2.T @ h1
    G["b2"] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"]) * drelu(z1)
    G["W1"] = dz1.T @ X
    G["b1"] = dz1.sum(0)
    return L, G


def adam(P, G, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1) at step number t >= 1;
    returns new (P, m, v)."""
    Pn, mn, vn = {}, {}, {}
    for k in P:
        mn[k] = beta1 * m[k] + (1.0 - beta1) * G[k]
        vn[k] = beta2 * v[k] + (1.0 - beta2) * G[k] ** 2
        mh = mn[k] / (1.0 - beta1 ** t)
        vh = vn[k] / (1.0 - beta2 ** t)
        Pn[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return Pn, mn, vn


def zeros_like(P):
    return {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in P.items()}
