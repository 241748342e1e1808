"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle
checks.  Nothing here computes any part of the method: it only draws the
workload parameters (cutoffs, densities) and the initial network weights from
numpy's PCG64 generator with recorded seeds, and names the flat layout of the
network parameters that the C ABI uses (include/ccd_mlp.h).
"""
from __future__ import annotations

import numpy as np

C4_SEED = 20161121
C5_SEED = 1611067
MLP_SEED = 65

DENSITIES_10 = [round(0.02 * (k + 1), 2) for k in range(10)]

# flat float32 parameter vector of the warm-start network
WIDTH, N_IN, N_PACK = 128, 7, 8
OFF_W1 = 0                          # [128][8], column 7 unused (zero)
OFF_B1 = OFF_W1 + WIDTH * N_PACK    # [128]
OFF_W2 = OFF_B1 + WIDTH             # [128][128], row = output unit
OFF_B2 = OFF_W2 + WIDTH * WIDTH     # [128]
OFF_W3 = OFF_B2 + WIDTH             # [128]
OFF_B3 = OFF_W3 + WIDTH             # [1]
N_PARAM = 17800                     # OFF_B3 + 1, padded to a multiple of 8


def c4_cutoffs(seed: int = C4_SEED):
    """n^2 cutoffs of the 40 batched solves, order (N, rho) = (14, 0.02) ...
    (66, 0.20), N in {14, 38, 54, 66}."""
    return [int(x) for x in np.random.default_rng(seed).integers(12, 37, size=40)]


def c4_specs(seed: int = C4_SEED):
    cut = c4_cutoffs(seed)
    return [(n, cut[10 * a + b], r) for a, n in enumerate([14, 38, 54, 66])
            for b, r in enumerate(DENSITIES_10)]


def c5_densities(seed: int = C5_SEED):
    """24 training and 16 held-out densities drawn from U[0.02, 0.20] fm^-3."""
    d = np.random.default_rng(seed).uniform(0.02, 0.20, size=40)
    return [float(x) for x in d[:24]], [float(x) for x in d[24:]]


def mlp_init(seed: int = MLP_SEED):
    """Initial parameters, flat float32: weights and biases of each layer
    uniform in +-1/sqrt(fan_in), last bias zero."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAM, dtype=np.float32)
    b1, b2 = 1.0 / np.sqrt(N_IN), 1.0 / np.sqrt(WIDTH)
    w1 = np.zeros((WIDTH, N_PACK), dtype=np.float32)
    w1[:, :N_IN] = rng.uniform(-b1, b1, size=(WIDTH, N_IN))
    p[OFF_W1:OFF_B1] = w1.reshape(-1)
    p[OFF_B1:OFF_W2] = rng.uniform(-b1, b1, size=WIDTH)
    p[OFF_W2:OFF_B2] = rng.uniform(-b2, b2, size=WIDTH * WIDTH)
    p[OFF_B2:OFF_W3] = rng.uniform(-b2, b2, size=WIDTH)
    p[OFF_W3:OFF_B3] = rng.uniform(-b2, b2, size=WIDTH)
    return p


def mlp_unflatten(flat):
    """Flat parameter vector -> dict of float64 arrays W1 [128][7], b1, W2,
    b2, W3, b3 (the structured form the CPU reference takes)."""
    f = np.asarray(flat, dtype=np.float64)
    return {"W1": f[OFF_W1:OFF_B1].reshape(WIDTH, N_PACK)[:, :N_IN].copy(),
            "b1": f[OFF_B1:OFF_W2].copy(),
            "W2": f[OFF_W2:OFF_B2].reshape(WIDTH, WIDTH).copy(),
            "b2": f[OFF_B2:OFF_W3].copy(),
            "W3": f[OFF_W3:OFF_B3].copy(),
            "b3": float(f[OFF_B3])}


def mlp_flatten(P):
    """Inverse of mlp_unflatten (float32)."""
    p = np.zeros(N_PARAM, dtype=np.float32)
    w1 = np.zeros((WIDTH, N_PACK))
    w1[:, :N_IN] = P["W1"]
    p[OFF_W1:OFF_B1] = w1.reshape(-1)
    p[OFF_B1:OFF_W2] = P["b1"]
    p[OFF_W2:OFF_B2] = np.asarray(P["W2"]).reshape(-1)
    p[OFF_B2:OFF_W3] = P["b2"]
    p[OFF_W3:OFF_B3] = P["W3"]
    p[OFF_B3] = P["b3"]
    return p


def pairing_hamiltonian(g, delta=1.0, n_levels=4):
    """The pairing model of eqs. sppairing / intpairing as dense arrays:
    h[s] = delta (p - 1) for state s = 2 (p - 1) + (0 for spin up, 1 for
    spin down), and the antisymmetrised elements <ab||cd> = <ab|V|cd> -
    <ab|V|dc> of V = -g/2 sum_pq a+_{p+} a+_{p-} a_{q-} a_{q+}, whose direct
    elements <p+ p-|V|q+ q-> = <p- p+|V|q- q+> = -g/2 are the only nonzero
    ones (the operator moves a pair of opposite spins from level q to p)."""
    n = 2 * n_levels
    h = np.array([delta * (s // 2) for s in range(n)], dtype=np.float64)

    def direct(a, b, c, d):
        # <ab|V|cd>: a, b one pair of level p (a spin up, b spin down or the
        # reverse), c, d one pair of level q in the same spin order
        if a // 2 != b // 2 or c // 2 != d // 2 or a == b or c == d:
            return 0.0
        if a % 2 != c % 2:
            return 0.0
        return -0.5 * g

    v = np.zeros((n, n, n, n))
    for a in range(n):
        for b in range(n):
            for c in range(n):
                for d in range(n):
                    v[a, b, c, d] = direct(a, b, c, d) - direct(a, b, d, c)
    return h, v

