"""Learned warm start of the CCD iteration (include/ccd_mlp.h).

Training data are the method's own converged amplitudes: a batch of solves is
iterated to convergence on the GPU, the library writes the packed features
and the targets y* = (t D - v) s of every canonical amplitude, and the
network is trained with the library's forward / backward / Adam kernels over
seeded permutations of the data.  A warm start then writes
t = (v + y / s) / D for every problem of a context, falling back to the MBPT2
start where the network's energy is implausible.  This module only orders
those calls; every numeric step runs in libccd.so.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ccd, inputs


def converged_context(specs, stream, mixing=0.5, tol=1e-9, max_iter=3000):
    """Context of problems (N, nmax2, rho) iterated in FP64 until |dE| < tol."""
    ctx = ccd.Context([ccd.problem(*s) for s in specs], stream=stream).bind()
    r = ctx.iterate(mixing=mixing, tol=tol, max_iter=max_iter, check_every=16)
    return ctx, r


def training_set(ctx):
    """Packed features and targets of all amplitudes of all problems of ctx."""
    feats, tgts = [], []
    for p in range(ctx.n):
        f, t = ctx.mlp_features(p, targets=True)
        feats.append(f)
        tgts.append(t)
    return torch.cat(feats), torch.cat(tgts)


def train(feat, target, epochs, batch=4096, lr=2e-3, seed=inputs.MLP_SEED, params=None):
    """Adam over `epochs` seeded permutations of the rows, learning rate on a
    half-cosine from lr to lr / 20; returns (params, mean loss per epoch)."""
    dev = feat.device
    if params is None:
        params = torch.tensor(inputs.mlp_init(seed), device=dev)
    state = ccd.AdamState(params)
    rng = np.random.default_rng(seed)
    work = ccd.mlp_work_buffer(batch, dev)
    n = feat.shape[0]
    losses = []
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(dev)
        lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * ep / max(1, epochs))))
        losses.append(ccd.mlp_train(params, state, feat, target, order, batch, lr_ep, work=work))
    return params, losses
