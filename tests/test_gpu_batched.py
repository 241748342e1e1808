"""Batched form: many independent solves in one context, graph replay of
chunks of sweeps, persistent launch shapes and the autotuner.

Launch shapes and graph replay only change how the same kernels are issued:
every variant must give bit-identical amplitudes and energies.  The 40-solve
batch (N in {14, 38, 54, 66} x 10 densities, cutoffs drawn from a seeded
generator) must reproduce each solve run alone in its own context, and its
smallest members the oracle.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")

DENS = [round(0.02 * (k + 1), 2) for k in range(10)]
C4_SEED = 20161121


def c4_cutoffs(seed=C4_SEED):
    """Cutoff n^2 <= nmax2 of each of the 40 solves, in the order
    (N, density) = (14, 0.02), (14, 0.04), ..., (66, 0.20)."""
    return np.random.default_rng(seed).integers(12, 37, size=40)


def c4_problems(seed=C4_SEED):
    cut = c4_cutoffs(seed)
    out = []
    for a, n in enumerate([14, 38, 54, 66]):
        for b, r in enumerate(DENS):
            out.append(ccd.problem(n, int(cut[10 * a + b]), r))
    return out


def _ctx(probs):
    import torch
    assert torch.cuda.is_available()
    return ccd.Context(probs, stream=torch.cuda.current_stream().cuda_stream).bind()


def _all_t(ctx):
    return [ctx.get_amplitudes(p) for p in range(ctx.n)]


MIXED_SET = [(38, 12, 0.06), (66, 20, 0.16), (14, 20, 0.10), (66, 36, 0.16)]


def test_graph_replay_bit_identical_to_eager():
    probs = [ccd.problem(*x) for x in MIXED_SET[:3]]
    a = _ctx(probs)
    ra = a.iterate(mixing=0.6, tol=0.0, max_iter=7, history=True)
    b = _ctx(probs)
    rb = b.iterate(mixing=0.6, tol=0.0, max_iter=7, history=True, check_every=3, graph=True)
    assert np.array_equal(ra["history"], rb["history"])
    for x, y in zip(_all_t(a), _all_t(b)):
        assert np.array_equal(x, y)
    # replaying the cached graphs again continues the same iteration
    ra = a.iterate(mixing=0.6, tol=0.0, max_iter=7, history=True)
    rb = b.iterate(mixing=0.6, tol=0.0, max_iter=7, history=True, check_every=3, graph=True)
    assert np.array_equal(ra["history"], rb["history"])


def test_check_every_does_not_change_convergence():
    probs = [ccd.problem(*x) for x in MIXED_SET[:3]]
    a = _ctx(probs)
    ra = a.iterate(mixing=0.5, tol=1e-8, max_iter=300, history=True)
    b = _ctx(probs)
    rb = b.iterate(mixing=0.5, tol=1e-8, max_iter=300, history=True, check_every=16, graph=True)
    assert ra["status"] == rb["status"] == ccd.CCD_OK
    assert np.array_equal(ra["sweeps"], rb["sweeps"])
    assert np.array_equal(ra["history"], rb["history"], equal_nan=True)
    for p in range(len(probs)):
        assert a.energy(p) == b.energy(p)


@pytest.mark.parametrize("precision,mixed_tol,rule", [(0, 0.0, 0), (0, 0.0, 1), (2, 1e-2, 1)])
def test_chunk_lengths_do_not_change_the_solve(precision, mixed_tol, rule):
    """The host shortens a chunk of sweeps to the sweeps it predicts the
    slowest live problem still needs (no graph replay); the device alone
    decides when each problem stops, so reading its flags after every sweep,
    every 8 sweeps with that prediction, or once per 64 gives the same sweep
    counts, energy histories and energies, in FP64 and in a BF16 phase with
    FP64 refinement (two phases, each with its own prediction)."""
    probs = [ccd.problem(*x) for x in MIXED_SET[:3]]
    out = []
    for every in (1, 8, 64):
        c = _ctx(probs)
        r = c.iterate(mixing=0.5, tol=0.0, tol_rel=1e-9, stop_rule=rule, max_iter=300, history=True,
                      check_every=every, precision=precision, mixed_tol=mixed_tol, refine_sweeps=2)
        assert r["status"] == ccd.CCD_OK
        out.append((r, [c.energy(p) for p in range(len(probs))]))
    for r, e in out[1:]:
        assert np.array_equal(out[0][0]["sweeps"], r["sweeps"])
        assert np.array_equal(out[0][0]["history"], r["history"], equal_nan=True)
        assert out[0][1] == e


TABLES = [
    [1, 1, 1, 1, 1, 1, 0, 0, 0, 0],
    [2, 2, 2, 2, 2, 2, 1, 1, 1, 1],
    [4, 4, 4, 4, 4, 4, 1, 0, 1, 0],
    [0, 0, 0, 0, 0, 0, 1, 1, 1, 1],
]


@pytest.mark.parametrize("prec", [ccd.CCD_PREC_FP64, ccd.CCD_PREC_BF16])
def test_launch_shapes_bit_identical(prec):
    """Persistent grids and the alternative ring tile shapes, all four ring
    size buckets populated (the n^2 <= 36 member has pair blocks of order > 64)."""
    probs = [ccd.problem(*x) for x in MIXED_SET]
    ref = _ctx(probs)
    info = ref.info(3)
    assert info["max_ph"] > 64
    ref.iterate(mixing=0.7, tol=0.0, max_iter=3, precision=prec)
    want = _all_t(ref)
    for tab in TABLES:
        c = _ctx(probs)
        c.set_tuning(tab)
        assert np.array_equal(c.get_tuning(), tab)
        c.iterate(mixing=0.7, tol=0.0, max_iter=3, precision=prec)
        for x, y in zip(want, _all_t(c)):
            assert np.array_equal(x, y), tab


def test_problems_stopping_at_different_sweeps_under_every_launch_shape():
    """Inside a run the energy step of a sweep (which clears the flag of a
    problem that has converged) runs as extra blocks of the next sweep's
    chi_klij launch, beside that launch's own items and the rings.  With
    problems stopping at different sweeps, persistent grids (workgroups that
    take several items) and flags read every sweep or every 8 sweeps, every
    sweep count, energy history and energy equals that of the default shapes
    with the flags read after every sweep."""
    probs = [ccd.problem(n, n2, rho) for n, n2 in ((14, 8), (38, 12), (54, 16), (66, 20))
             for rho in (0.05, 0.1, 0.2)]

    def solve(tab, every, graph=False):
        c = _ctx(probs)
        c.set_tuning(tab)
        r = c.iterate(mixing=0.5, tol=0.0, tol_rel=1e-9, stop_rule=1, max_iter=300, history=True,
                      check_every=every, graph=graph)
        assert r["status"] == ccd.CCD_OK
        return r, [c.energy(p) for p in range(len(probs))]

    ref, e_ref = solve([0] * ccd.CCD_TUNE_LEN, 1)
    assert len(set(ref["sweeps"].tolist())) > 3  # the problems stop at different sweeps
    for tab in [[0] * ccd.CCD_TUNE_LEN] + TABLES:
        for every, graph in ((1, False), (8, False), (8, True)):
            r, e = solve(tab, every, graph)
            assert np.array_equal(ref["sweeps"], r["sweeps"]), (tab, every, graph)
            assert np.array_equal(ref["history"], r["history"], equal_nan=True), (tab, every, graph)
            assert e_ref == e, (tab, every, graph)


def test_autotune_keeps_the_iteration():
    probs = [ccd.problem(*x) for x in MIXED_SET]
    ref = _ctx(probs)
    ref.iterate(mixing=0.5, tol=0.0, max_iter=4)
    c = _ctx(probs)
    c.iterate(mixing=0.5, tol=0.0, max_iter=2)
    tab, best = c.autotune(ccd.CCD_PREC_FP64, reps=3)
    assert np.all(best >= 0.0) and best[ccd.CCD_TUNE_LADDER] > 0.0
    for k, v in enumerate(tab):
        assert v in ((0, 1, 2, 4) if k < ccd.CCD_TUNE_RING_NW32 else (0, 1))
    c.iterate(mixing=0.5, tol=0.0, max_iter=2, graph=True, check_every=2)
    for x, y in zip(_all_t(ref), _all_t(c)):
        assert np.array_equal(x, y)
    with pytest.raises(ccd.CCDError):
        c.set_tuning([3] + [0] * 9)


def test_c4_batch_matches_separate_solves_and_oracle():
    """The 40-solve batch, FP64, two sweeps: each member equals the same solve
    in its own context bit for bit; the N = 14 members match the oracle."""
    from oracle import oracle
    probs = c4_problems()
    big = _ctx(probs)
    h = big.iterate(mixing=0.5, tol=0.0, max_iter=2, history=True, check_every=2, graph=True)["history"]
    for p, pr in enumerate(probs):
        one = _ctx([pr])
        h1 = one.iterate(mixing=0.5, tol=0.0, max_iter=2, history=True)["history"]
        assert np.array_equal(h[p], h1[0]), p
    cut = c4_cutoffs()
    for b in (0, 4, 9):
        o3 = oracle.O3(oracle.PNM(14, int(cut[b]), DENS[b]))
        for s in range(2):
            e = o3.sweep(0.5)
            assert abs(h[b, s] - e) <= 1e-10 * abs(e), (b, s, h[b, s], e)


def test_c4_mixed_batched_converges_to_fp64():
    """The 40 solves batched, BF16 contractions then FP64 refinement, graph
    replay and tuned shapes: every energy within 1e-6 of the FP64 solve."""
    probs = c4_problems()
    ref = _ctx(probs)
    r = ref.iterate(mixing=0.5, tol=1e-9, max_iter=600, check_every=8, graph=True)
    assert r["status"] == ccd.CCD_OK
    mix = _ctx(probs)
    mix.autotune(ccd.CCD_PREC_BF16, reps=2)
    m = mix.iterate(mixing=0.5, tol=1e-9, max_iter=600, precision=ccd.CCD_PREC_BF16, mixed_tol=1e-3,
                    refine_sweeps=3, check_every=8, graph=True)
    assert m["status"] == ccd.CCD_OK
    for p in range(len(probs)):
        e64, em = ref.energy(p)[2], mix.energy(p)[2]
        assert abs(em - e64) <= 1e-6 * abs(e64), (p, em, e64)


def test_extrapolated_stop_rule_bounds_the_error():
    """stop_rule 1: from the MBPT2 start and from a perturbed start (which
    excites every mode), stopping at tol_rel = 1e-7 leaves each energy within
    1e-6 of the converged one; the plain |dE| test is never stricter."""
    probs = [ccd.problem(66, 20, 0.16), ccd.problem(38, 12, 0.06)]
    ref = _ctx(probs)
    ref.iterate(mixing=0.5, tol=1e-11, max_iter=2000, check_every=16)
    e_ref = [ref.energy(p)[2] for p in range(2)]
    for scale in (1.0, 1.6):
        a = _ctx(probs)
        b = _ctx(probs)
        for c in (a, b):
            if scale != 1.0:
                for p in range(2):
                    c.set_amplitudes(c.get_amplitudes(p) * scale, p)
        ra = a.iterate(mixing=0.5, tol=0.0, tol_rel=1e-7, stop_rule=1, max_iter=2000)
        rb = b.iterate(mixing=0.5, tol=0.0, tol_rel=1e-7, stop_rule=0, max_iter=2000)
        assert ra["status"] == rb["status"] == ccd.CCD_OK
        assert np.all(ra["sweeps"] >= rb["sweeps"])
        for p in range(2):
            assert abs(a.energy(p)[2] - e_ref[p]) <= 1e-6 * abs(e_ref[p]), (scale, p)
