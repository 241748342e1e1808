"""The committed oracle energies under tests/golden/ (written by
make_oracle_goldens.py from oracle/ alone): well formed, converged by the
stated test, consistent with the oracle as it builds here, and read back by
bench.py's reader."""
import os

import pytest

from conftest import golden

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    if not os.path.exists(os.path.join(GOLDEN, name)):
        pytest.skip(f"{name} not generated")
    return golden(name)


@pytest.mark.parametrize("name,tol", [("oracle_c2_history.txt", 1e-8), ("oracle_c3_history.txt", 1e-10)])
def test_histories_stop_at_the_first_sweep_below_tol(name, tol):
    for r in _rows(name):
        n = int(r[3])
        h = [float(x) for x in r[5:]]
        assert len(h) == n + 1
        d = [abs(h[k + 1] - h[k]) for k in range(n)]
        assert d[-1] < tol and all(x >= tol for x in d[:-1]), r[:3]
        assert all(x < 0.0 for x in h)


@pytest.mark.parametrize("name", ["oracle_c4_converged.txt", "oracle_c5_converged.txt"])
def test_converged_files(name):
    for r in _rows(name):
        assert float(r[7]) < 1e-9
        assert float(r[5]) < 0.0 and float(r[6]) < 0.0


def test_c2_low_density_start_matches_the_oracle_here(orc):
    """E_ref and E_MBPT2 of N = 66, n^2 <= 20, rho = 0.02 as the oracle builds
    them on this machine equal the committed ones."""
    rows = [r for r in _rows("oracle_c2_history.txt") if float(r[2]) == 0.02]
    assert rows
    o3 = orc.O3(orc.PNM(66, 20, 0.02))
    assert o3.eref == pytest.approx(float(rows[0][4]), rel=1e-13)
    assert o3.emp2 == pytest.approx(float(rows[0][5]), rel=1e-13)
    assert o3.sweep(0.5) == pytest.approx(float(rows[0][6]), rel=1e-12)


def test_bench_reader():
    bench = pytest.importorskip("bench")
    rows = _rows("oracle_c3_history.txt")
    e = bench.oracle_energies("oracle_c3_history.txt")
    assert e[(66, 36, 0.16)] == float(rows[0][-1])
    assert bench.oracle_energies("no_such_file.txt") == {}
