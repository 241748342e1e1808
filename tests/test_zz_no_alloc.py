"""ccd_dense_solve_static (the dense CCD on the library's static work area, no
device allocation) against ccd_dense_solve (caller-provided work buffer):
two calls in a row on one GPU, the second on a smaller model space, must give
the same results as the buffered entry point, and a model space beyond the
static area is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")
from paper_1611_06765_amd import inputs  # noqa: E402


def _same(a, b):
    assert a["status"] == b["status"]
    assert a["sweeps"] == b["sweeps"]
    for k in ("e_ref", "e_mbpt2", "e_ccd"):
        assert a[k] == b[k], (k, a[k], b[k])
    assert np.array_equal(a["history"], b["history"])


def test_static_matches_buffered_twice_second_smaller():
    import torch
    assert torch.cuda.is_available()
    stream = torch.cuda.current_stream().cuda_stream
    # pairing model with 8 levels (16 states, 4 particles), then 4 levels (8 states)
    for n_levels, g in ((8, 0.5), (4, -0.5)):
        h, v = inputs.pairing_hamiltonian(g, n_levels=n_levels)
        print(f"static dense solve: {2 * n_levels} states, g = {g}", flush=True)
        a = ccd.dense_solve_static(h, v, 4, mixing=0.7, tol=1e-11, max_iter=300, stream=stream)
        b = ccd.dense_solve(h, v, 4, mixing=0.7, tol=1e-11, max_iter=300, stream=stream)
        assert a["status"] == ccd.CCD_OK
        _same(a, b)
        assert a["e_ccd"] < 0.0


def test_static_refuses_model_space_beyond_its_area():
    h, v = np.zeros(40), np.zeros(40 ** 4)
    with pytest.raises(ccd.CCDError):
        ccd.dense_solve_static(h, v, 4, max_iter=1)
