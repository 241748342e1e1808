"""Learned warm start on the GPU against the CPU reference (oracle/mlp_oracle.py).

Features are computed in FP64 and stored as FP32: they must equal the
reference's to FP32 rounding.  The network's forward and backward run in FP32
on MFMA (sums of 128 products): outputs and gradients must match the FP64
reference to 1e-4 of their scale; the BF16 forward (8-bit mantissa) to 3e-2.
Training must be deterministic and lower the loss, and a network trained on
converged N = 66, n^2 <= 20 amplitudes must shorten held-out n^2 <= 36 solves.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _ctx(specs):
    torch = _torch()
    return ccd.Context([ccd.problem(*s) for s in specs], stream=torch.cuda.current_stream().cuda_stream).bind()


def _params(seed=7, scale=1.0):
    from paper_1611_06765_amd import inputs
    return inputs.mlp_init(seed) * np.float32(scale)


def _dev(a):
    torch = _torch()
    return torch.tensor(np.asarray(a), device="cuda")


def _rand_feats(n, seed=3):
    r = np.random.default_rng(seed)
    return np.column_stack([r.uniform(0.1, 1.3, n), r.uniform(0, 3, n), r.uniform(0, 3, n),
                            r.uniform(-0.6, 0.2, n), r.uniform(-0.6, 0.2, n), r.uniform(0, 4, n),
                            r.uniform(0, 4, n), r.normal(0, 0.7, n)]).astype(np.float32)


@pytest.mark.parametrize("spec", [(14, 4, 0.08), (38, 12, 0.11)])
def test_features_match_oracle(spec):
    from oracle import mlp_oracle as M
    from oracle import oracle
    ctx = _ctx([spec])
    feat = ctx.mlp_features(0).cpu().numpy()
    ijab = ccd.canonical_index(ctx)
    want = M.features(oracle.PNM(*spec), ijab)
    np.testing.assert_allclose(feat, want.astype(np.float32), rtol=2e-7, atol=1e-7)


def test_targets_match_oracle():
    """Targets from amplitudes after three sweeps, against the oracle's amplitudes."""
    from oracle import mlp_oracle as M
    from oracle import oracle
    spec = (14, 4, 0.08)
    ctx = _ctx([spec])
    ctx.iterate(mixing=1.0, tol=0.0, max_iter=3)
    _, tgt = ctx.mlp_features(0, targets=True)
    pnm = oracle.PNM(*spec)
    o3 = oracle.O3(pnm)
    for _ in range(3):
        o3.sweep(1.0)
    ijab = ccd.canonical_index(ctx)
    t = np.array([o3.t(a, b, i, j) for i, j, a, b in ijab])
    want = M.targets(pnm, ijab, t)
    got = tgt.cpu().numpy()
    assert np.max(np.abs(want)) > 1e-3
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6 * np.max(np.abs(want)))


@pytest.mark.parametrize("prec,tol", [(ccd.CCD_PREC_FP32, 1e-4), (ccd.CCD_PREC_BF16, 3e-2)])
def test_forward_matches_oracle(prec, tol):
    from oracle import mlp_oracle as M
    from paper_1611_06765_amd import inputs
    p = _params(scale=2.0)
    F = _rand_feats(1003)
    y = ccd.mlp_forward(_dev(p), _dev(F), prec).cpu().numpy()
    want = M.predict(inputs.mlp_unflatten(p), F.astype(np.float64))
    scale = np.max(np.abs(want))
    assert scale > 1e-2
    assert np.max(np.abs(y - want)) <= tol * scale, np.max(np.abs(y - want)) / scale


def test_loss_and_gradient_match_oracle():
    from oracle import mlp_oracle as M
    from paper_1611_06765_amd import inputs
    p = _params(seed=9, scale=1.5)
    F = _rand_feats(1003, seed=4)
    Y = np.random.default_rng(5).normal(0, 0.2, 1003).astype(np.float32)
    loss, g = ccd.mlp_loss_grad(_dev(p), _dev(F), _dev(Y))
    L, G = M.loss_and_grad(inputs.mlp_unflatten(p), F.astype(np.float64), Y.astype(np.float64))
    assert loss == pytest.approx(L, rel=1e-5)
    gw = inputs.mlp_flatten({k: np.asarray(v) for k, v in G.items()})
    gw[inputs.OFF_B3] = 0.0
    g = g.cpu().numpy()
    scale = np.max(np.abs(gw))
    assert np.max(np.abs(g - gw)) <= 1e-4 * scale
    for lo, hi in [(inputs.OFF_W1, inputs.OFF_B1), (inputs.OFF_W2, inputs.OFF_B2), (inputs.OFF_W3, inputs.OFF_B3)]:
        assert np.linalg.norm(g[lo:hi] - gw[lo:hi]) <= 1e-4 * np.linalg.norm(gw[lo:hi])


def test_adam_steps_match_oracle():
    """Three full-batch Adam steps against the reference update."""
    torch = _torch()
    from oracle import mlp_oracle as M
    from paper_1611_06765_amd import inputs
    p0 = _params(seed=10)
    n = 520
    F = _rand_feats(n, seed=6)
    Y = np.random.default_rng(7).normal(0, 0.2, n).astype(np.float32)
    P = _dev(p0.copy())
    st = ccd.AdamState(P)
    order = torch.arange(3 * n, dtype=torch.int32, device="cuda") % n
    lr = 1e-3
    ccd.mlp_train(P, st, _dev(F), _dev(Y), order, n, lr)
    assert st.step.value == 3
    Q = inputs.mlp_unflatten(p0)
    m, v = M.zeros_like(Q), M.zeros_like(Q)
    for t in range(1, 4):
        _, G = M.loss_and_grad(Q, F.astype(np.float64), Y.astype(np.float64))
        G["b3"] = 0.0
        Q, m, v = M.adam(Q, G, m, v, t, lr)
    got = inputs.mlp_unflatten(P.cpu().numpy())
    _, G0 = M.loss_and_grad(inputs.mlp_unflatten(p0), F.astype(np.float64), Y.astype(np.float64))
    for k in ("W1", "b1", "W2", "b2", "W3"):
        sig = np.abs(np.asarray(G0[k])) > 1e-3 * np.max(np.abs(G0[k]))   # gradient well above FP32 noise
        d = np.abs(np.asarray(got[k]) - np.asarray(Q[k]))[sig]
        assert np.max(d) <= 2e-2 * lr, (k, np.max(d))


def test_training_is_deterministic_and_learns():
    torch = _torch()
    from paper_1611_06765_amd import warmstart
    n = 6000
    F = _dev(_rand_feats(n, seed=8))
    x = F.double()
    # a target with the symmetry of the prediction: odd under a <-> b and under
    # i <-> j (each flips v and exchanges |q| and |q'|)
    Y = (0.3 * x[:, 7] * torch.exp(-0.5 * (x[:, 1] + x[:, 2]))
         / (1.0 + x[:, 5] + x[:, 6] - x[:, 3] - x[:, 4])).float()
    p1, l1 = warmstart.train(F, Y, epochs=12, batch=256, lr=3e-3, seed=1)
    p2, l2 = warmstart.train(F, Y, epochs=12, batch=256, lr=3e-3, seed=1)
    assert torch.equal(p1, p2) and l1 == l2
    assert l1[-1] < 0.2 * l1[0], l1


def test_warm_start_matches_oracle_and_falls_back():
    from oracle import mlp_oracle as M
    from oracle import oracle
    from paper_1611_06765_amd import inputs
    spec = (14, 4, 0.08)
    ctx = _ctx([spec])
    p = _params(seed=12, scale=0.05)
    used = ctx.warm_start(_dev(p), ccd.CCD_PREC_FP32)
    t = ctx.get_amplitudes()
    pnm = oracle.PNM(*spec)
    ijab = ccd.canonical_index(ctx)
    F = M.features(pnm, ijab)
    want = M.amplitudes(pnm, ijab, M.predict(inputs.mlp_unflatten(p), F))
    assert used[0]
    assert np.max(np.abs(t - want)) <= 1e-4 * np.max(np.abs(want))
    assert np.isfinite(ctx.energy()[2])
    # a wild network is rejected: the MBPT2 amplitudes come back bit for bit
    ref = _ctx([spec])
    mb = ref.get_amplitudes()
    used = ctx.warm_start(_dev(_params(seed=12, scale=400.0)), ccd.CCD_PREC_BF16)
    assert not used[0]
    assert np.array_equal(ctx.get_amplitudes(), mb)
    assert ctx.energy()[2] == ref.energy()[2]
    used = ctx.warm_start(None)
    assert not used[0] and np.array_equal(ctx.get_amplitudes(), mb)


def test_learned_start_shortens_heldout_solves():
    """Train on converged N=66, n^2<=20 amplitudes at 8 of the seeded training
    densities; at 4 held-out densities with n^2<=36 the warm start converges
    in fewer sweeps than the MBPT2 start, to the same energy."""
    torch = _torch()
    from paper_1611_06765_amd import inputs, warmstart
    train_d, held = inputs.c5_densities()
    s = torch.cuda.current_stream().cuda_stream
    ctx, r = warmstart.converged_context([(66, 20, d) for d in train_d[:8]], s)
    assert r["status"] == ccd.CCD_OK
    F, Y = warmstart.training_set(ctx)
    params, losses = warmstart.train(F, Y, epochs=10, batch=4096)
    assert losses[-1] < 0.5 * losses[0]
    specs = [(66, 36, d) for d in held[:4]]
    base = _ctx(specs)
    rb = base.iterate(mixing=0.5, tol=1e-6, max_iter=600)
    warm = _ctx(specs)
    used = warm.warm_start(params, ccd.CCD_PREC_BF16)
    assert used.all()
    rw = warm.iterate(mixing=0.5, tol=1e-6, max_iter=600)
    assert rb["status"] == rw["status"] == ccd.CCD_OK
    for p in range(len(specs)):
        e0, e1 = base.energy(p)[2], warm.energy(p)[2]
        assert abs(e0 - e1) <= 1e-6 * abs(e0)
    assert rw["sweeps"].sum() < rb["sweeps"].sum(), (rw["sweeps"], rb["sweeps"])


def test_training_rejects_out_of_range_indices():
    """An order entry outside [0, n_rows) is skipped on the device and the
    call reports CCD_EINVAL; the other amplitudes of the step still train."""
    torch = _torch()
    n = 256
    F = _dev(_rand_feats(n, seed=21))
    Y = _dev(np.random.default_rng(22).normal(0, 0.1, n).astype(np.float32))
    P = _dev(_params(seed=23))
    p0 = P.clone()
    st = ccd.AdamState(P)
    order = torch.arange(n, dtype=torch.int32, device="cuda")
    order[17] = n + 5
    order[40] = -3
    with pytest.raises(ccd.CCDError) as e:
        ccd.mlp_train(P, st, F, Y, order, n, 1e-3)
    assert e.value.status == ccd.CCD_EINVAL and "outside" in str(e.value)
    assert st.step.value == 1 and not torch.equal(P, p0)
