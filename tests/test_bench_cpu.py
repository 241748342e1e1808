"""bench.py's roofline bookkeeping on the CPU: the ring's flops split over its
size buckets add up to the library's count, each bucket holds the pairs of its
padded order, and the kernel symbols follow the tuning table."""
import numpy as np
import pytest

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")
bench = pytest.importorskip("bench")


@pytest.mark.parametrize("N,n2", [(66, 20), (66, 36), (38, 12)])
def test_ring_bucket_flops_add_up(N, n2):
    c = ccd.Context([ccd.problem(N, n2, 0.16)])
    f = bench.ring_class_flops(ccd, c)
    assert sum(f.values()) == pytest.approx(c.info()["flops_ring"], rel=1e-15)
    ph = c.export_map(ccd.CCD_MAP_PH_CHANNELS).reshape(-1, 6)
    orders = [max(ph[x, 4], ph[ph[x, 5], 4]) for x in range(len(ph)) if ph[x, 5] >= x]
    for k in f:
        lo, hi = (0, 16) if k == "ring_small" else (int(k[4:]) - 15, int(k[4:]))
        assert any(lo <= o <= hi for o in orders), k
    assert max(orders) <= 80


def test_kernel_symbols():
    t = [0] * 10
    assert bench.kernel_symbol("ladder", t) == "k_ladder64"
    assert bench.kernel_symbol("direct", t) == "void k_direct<0>"
    assert bench.kernel_symbol("ring64", t) == "void k_ringp<0, 64, 16>"
    t[8] = 1
    assert bench.kernel_symbol("ring64", t) == "void k_ringp<0, 64, 8>"
    t[7] = 1
    assert bench.kernel_symbol("ring48", t) == "void k_ringp<0, 48, 3>"


def test_traffic_records_match_the_current_source():
    """The committed counter records are keyed by workload and kernel family
    and hold for the current kernel source (else bench.py reports null)."""
    t = bench.measured_traffic("ring64", bench.TRAFFIC_C2)
    assert t is not None and 50e6 < t < 500e6
    assert bench.measured_traffic("ladder", bench.TRAFFIC_C3) is not None
    assert bench.measured_traffic("ring64", "no such workload") is None
