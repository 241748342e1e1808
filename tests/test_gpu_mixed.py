"""Mixed-precision contractions (FP32 / BF16 MFMA, FP32 accumulation) with FP64
denominators, update, mixing and energy, then FP64 refinement.

Per term, one sweep in a mixed mode must reproduce the FP64 contribution of
that term to the precision of its operands: FP32 (24-bit mantissa) to 1e-5 of
the term, BF16 (8-bit mantissa, products summed in FP32) to 2e-2 of the term.
A wrong operand or output layout would give O(1) errors.  After refinement the
converged energy must match the FP64 one to 1e-6 relative.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")


def _ctx(probs):
    import torch
    assert torch.cuda.is_available()
    return ccd.Context(probs, stream=torch.cuda.current_stream().cuda_stream).bind()


TERMS = [1, 2, 4, 8, 16, 32, 64]


@pytest.mark.parametrize("prec,rtol", [(ccd.CCD_PREC_FP32, 1e-5), (ccd.CCD_PREC_BF16, 2e-2)])
@pytest.mark.parametrize("mask", TERMS)
def test_term_contribution_matches_fp64(prec, rtol, mask):
    prob = [ccd.problem(38, 12, 0.12)]
    ref = _ctx(prob)
    e0 = ref.energy()[1]
    r64 = ref.iterate(mixing=1.0, tol=0.0, max_iter=1, terms=mask, history=True)["history"][0, 0] - e0
    mix = _ctx(prob)
    rm = mix.iterate(mixing=1.0, tol=0.0, max_iter=1, terms=mask, precision=prec,
                     history=True)["history"][0, 0] - e0
    assert abs(r64) > 1e-6
    assert abs(rm - r64) <= rtol * abs(r64), (mask, rm, r64)


@pytest.mark.parametrize("prec", [ccd.CCD_PREC_FP32, ccd.CCD_PREC_BF16])
def test_refined_energy_matches_fp64(prec):
    """N=66, n^2<=20 at two densities: mixed sweeps to convergence, then FP64
    refinement; the final energy agrees with the converged FP64 energy to 1e-6."""
    probs = [ccd.problem(66, 20, 0.08), ccd.problem(66, 20, 0.16)]
    ref = _ctx(probs)
    r = ref.iterate(mixing=0.5, tol=1e-9, max_iter=400)
    assert r["status"] == ccd.CCD_OK
    mix = _ctx(probs)
    mtol = 1e-3 if prec == ccd.CCD_PREC_BF16 else 1e-6
    m = mix.iterate(mixing=0.5, tol=1e-9, max_iter=400, precision=prec, refine_sweeps=3, mixed_tol=mtol)
    assert m["status"] == ccd.CCD_OK
    for p in range(2):
        e64 = ref.energy(p)[2]
        em = mix.energy(p)[2]
        assert abs(em - e64) <= 1e-6 * abs(e64), (p, em, e64)


def test_mixed_phase_error_is_bounded_before_refinement():
    """The mixed fixed point itself sits close to the FP64 one (FP32 to 1e-5,
    BF16 to 1e-2 relative), so refinement starts near the answer."""
    prob = [ccd.problem(66, 20, 0.12)]
    ref = _ctx(prob)
    ref.iterate(mixing=0.5, tol=1e-9, max_iter=400)
    e64 = ref.energy()[2]
    for prec, rtol in [(ccd.CCD_PREC_FP32, 1e-5), (ccd.CCD_PREC_BF16, 1e-2)]:
        mix = _ctx(prob)
        # refine budget exhausted by the mixed phase: max_iter sweeps, all mixed
        mix.iterate(mixing=0.5, tol=0.0, max_iter=60, precision=prec)
        em = mix.energy()[2]
        assert abs(em - e64) <= rtol * abs(e64), (prec, em, e64)
