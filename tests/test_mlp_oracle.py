"""Pins of the warm-start network's CPU reference (oracle/mlp_oracle.py).

The backward pass is checked against torch autograd in float64 and against
central finite differences; the Adam step against torch.optim.Adam; the
antisymmetrised prediction against the swaps it must respect; the features
against a hand-worked momentum transfer and the interaction of the C oracle;
the target encoding against the MBPT2 amplitudes of the C oracle (they map to
y = 0 exactly).
"""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from oracle import oracle
from paper_1611_06765_amd import inputs


def _params(seed=3, scale=1.0):
    P = inputs.mlp_unflatten(inputs.mlp_init(seed))
    P["b3"] = 0.37
    return {k: (np.asarray(v) * scale if k != "b3" else v) for k, v in P.items()}


def _feats(m=23, seed=5):
    r = np.random.default_rng(seed)
    F = np.column_stack([r.uniform(0.1, 1.3, m), r.uniform(0, 3, m), r.uniform(0, 3, m),
                         r.uniform(-0.6, 0.2, m), r.uniform(-0.6, 0.2, m), r.uniform(0, 4, m),
                         r.uniform(0, 4, m), r.normal(0, 0.7, m)])
    return F, r.normal(0, 0.3, m)


def _torch_loss(P, F, Y):
    T = {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=True) for k, v in P.items()}
    X = torch.tensor(M.variants(F))
    h1 = torch.relu(X @ T["W1"].T + T["b1"])
    h2 = torch.relu(h1 @ T["W2"].T + T["b2"])
    g = h2 @ T["W3"] + T["b3"]
    y = (g.reshape(-1, 4) * torch.tensor([1.0, -1.0, -1.0, 1.0])).sum(1) / 4
    L = 0.5 * ((y - torch.tensor(Y)) ** 2).mean()
    L.backward()
    return float(L.detach()), {k: T[k].grad.numpy() for k in T}


def test_gradients_match_torch_autograd():
    P = _params()
    F, Y = _feats()
    L, G = M.loss_and_grad(P, F, Y)
    Lt, Gt = _torch_loss(P, F, Y)
    assert abs(L - Lt) <= 1e-13 * abs(Lt)
    for k in P:
        np.testing.assert_allclose(G[k], Gt[k], rtol=1e-10, atol=1e-15, err_msg=k)


def test_gradients_match_finite_differences():
    P = _params(seed=4)
    F, Y = _feats(m=9, seed=6)
    _, G = M.loss_and_grad(P, F, Y)
    r = np.random.default_rng(0)
    h = 1e-6
    picks = [("W1", (5, 2)), ("W1", (77, 6)), ("b1", (3,)), ("W2", (0, 0)), ("W2", (127, 64)),
             ("b2", (99,)), ("W3", (12,))]
    picks += [("W2", tuple(r.integers(0, 128, 2))) for _ in range(4)]
    for name, idx in picks:
        Pp = {k: np.array(v, copy=True) for k, v in P.items()}
        Pm = {k: np.array(v, copy=True) for k, v in P.items()}
        Pp[name][idx] += h
        Pm[name][idx] -= h
        fd = (M.loss_and_grad(Pp, F, Y)[0] - M.loss_and_grad(Pm, F, Y)[0]) / (2 * h)
        assert abs(fd - G[name][idx]) <= 1e-6 * max(abs(fd), 1e-9), (name, idx, fd, G[name][idx])
    # b3 cancels in the antisymmetrised output
    assert G["b3"] == pytest.approx(0.0, abs=1e-15)


def test_adam_matches_torch():
    P = _params(seed=8)
    F, Y = _feats(m=11, seed=9)
    T = {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=True) for k, v in P.items()}
    opt = torch.optim.Adam(list(T.values()), lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m, v = M.zeros_like(P), M.zeros_like(P)
    Q = {k: np.array(x, dtype=np.float64, copy=True) for k, x in P.items()}
    for step in range(1, 4):
        _, G = M.loss_and_grad(Q, F, Y)
        Q, m, v = M.adam(Q, G, m, v, step, 3e-3)
        opt.zero_grad()
        for k in T:
            T[k].grad = torch.tensor(np.asarray(M.loss_and_grad({kk: T[kk].detach().numpy() for kk in T}, F, Y)[1][k],
                                                dtype=np.float64))
        opt.step()
        for k in T:
            np.testing.assert_allclose(Q[k], T[k].detach().numpy(), rtol=1e-12, atol=1e-15, err_msg=k)


def test_prediction_is_antisymmetric():
    P = _params(seed=11, scale=1.5)
    F, _ = _feats(m=17, seed=12)
    rho, q, qx, ei, ej, ea, eb, v = F.T
    Fab = np.column_stack([rho, qx, q, ei, ej, eb, ea, -v])
    Fij = np.column_stack([rho, qx, q, ej, ei, ea, eb, -v])
    Fboth = np.column_stack([rho, q, qx, ej, ei, eb, ea, v])
    y = M.predict(P, F)
    assert np.max(np.abs(y)) > 1e-3
    np.testing.assert_allclose(M.predict(P, Fab), -y, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(M.predict(P, Fij), -y, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(M.predict(P, Fboth), y, rtol=1e-12, atol=1e-15)
    # a constant network predicts zero
    Z = dict(P)
    Z["W3"] = np.zeros(128)
    assert np.all(M.predict(Z, F) == 0.0)


def _pnm_elements(pnm):
    """All (i, j, a, b) with i<j holes, a<b particles and conserved momentum and spin."""
    st = pnm.states()
    out = []
    for i in range(pnm.N):
        for j in range(i + 1, pnm.N):
            for a in range(pnm.N, pnm.ns):
                for b in range(a + 1, pnm.ns):
                    if np.array_equal(st[a, :3] + st[b, :3], st[i, :3] + st[j, :3]) and \
                            st[a, 3] + st[b, 3] == st[i, 3] + st[j, 3]:
                        out.append((i, j, a, b))
    return np.array(out)


def test_features_hand_example_and_interaction():
    pnm = oracle.PNM(14, 4, 0.08)
    st = pnm.states()
    idx = {tuple(s): k for k, s in enumerate(st)}
    i, j = idx[(0, 0, 0, -1)], idx[(0, 0, 0, 1)]
    a, b = idx[(1, 1, 0, -1)], idx[(-1, -1, 0, 1)]
    F = M.features(pnm, [(i, j, a, b)])[0]
    ku = 2 * np.pi / pnm.L
    # q = (k_a - k_b - k_i + k_j)/2 = ku (1, 1, 0); q' = -q
    assert F[1] == pytest.approx(ku * np.sqrt(2.0), rel=1e-15)
    assert F[2] == pytest.approx(ku * np.sqrt(2.0), rel=1e-15)
    assert F[0] == pytest.approx(0.08 / 0.16, rel=1e-15)
    assert F[7] == pytest.approx(pnm.v(a, b, i, j) * pnm.L ** 3 / 1000.0, rel=1e-14)
    eps = pnm.fock()
    assert F[3:7] == pytest.approx(eps[[i, j, a, b]] / 100.0, rel=1e-15)


def test_mbpt2_amplitudes_encode_to_zero():
    """t0 = v / D (the C oracle's start) gives y* = 0, and y = 0 decodes to t0."""
    pnm = oracle.PNM(14, 4, 0.08)
    o3 = oracle.O3(pnm)
    E = _pnm_elements(pnm)
    t0 = np.array([o3.t(a, b, i, j) for i, j, a, b in E])
    assert np.all(M.denominators(pnm, E) < 0)
    y = M.targets(pnm, E, t0)
    assert np.max(np.abs(y)) <= 1e-12 * np.max(np.abs(t0)) * pnm.L ** 3
    np.testing.assert_allclose(M.amplitudes(pnm, E, np.zeros(len(E))), t0, rtol=1e-13, atol=1e-17)
    # converged amplitudes have nonzero targets, also where v = 0 (S_z = +-1)
    o3.solve(1.0, 1e-10)
    tc = np.array([o3.t(a, b, i, j) for i, j, a, b in E])
    yc = M.targets(pnm, E, tc)
    st = pnm.states()
    same_spin = np.array([st[a, 3] == st[b, 3] for i, j, a, b in E])
    assert np.max(np.abs(yc[same_spin])) > 1e-3
    np.testing.assert_allclose(M.amplitudes(pnm, E, yc), tc, rtol=1e-12, atol=1e-16)
