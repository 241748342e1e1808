"""Twisted boundary conditions in the library's host plan (no GPU): the state
order and hole set against the oracle bit for bit, the channel structure
against brute force, the rectangular cross-channel pairs, the twist mesh
against numpy's Gauss-Legendre rule, and the argument rules."""
import math

import numpy as np
import pytest

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")

PI = math.pi
TWISTS = [(2.5, 0.4, 1.3), (0.7, 1.9, 2.6), (PI, PI, PI), (0.725, 0.725, 0.725), (PI / 2, 0.0, 0.0),
          (5.9, -1.2, 0.3)]


def _ctx(N, nmax2, rho, twist):
    return ccd.Context([ccd.problem(N, nmax2, rho, twist=twist)])


@pytest.mark.parametrize("twist", TWISTS)
@pytest.mark.parametrize("N,nmax2", [(14, 4), (38, 12), (66, 20)])
def test_twisted_basis_and_energies_vs_oracle(orc, N, nmax2, twist):
    c = _ctx(N, nmax2, 0.12, twist)
    p = orc.PNM(N, nmax2, 0.12, twist=twist)
    st = c.export_map(ccd.CCD_MAP_STATES).reshape(-1, 4)
    assert np.array_equal(st, p.states())
    tk, eps, _ = c.export_tables()
    assert np.allclose(tk, p.kinetic(), rtol=1e-14, atol=0)
    assert np.allclose(eps, p.fock(), rtol=1e-12, atol=1e-12)
    assert c.eref() == pytest.approx(p.eref(), rel=1e-13)
    T, V = c.reference_parts()
    assert T == pytest.approx(p.kinetic()[:N].sum(), rel=1e-14)
    assert T + V == pytest.approx(c.eref(), rel=1e-15)


def _brute_ph(st, N):
    groups = {}
    for p in range(N, len(st)):
        for h in range(N):
            key = (int(st[p, 3] - st[h, 3]),) + tuple(int(x) for x in st[p, :3] - st[h, :3])
            groups.setdefault(key, []).append((p, h))
    return groups


@pytest.mark.parametrize("twist", TWISTS[:4])
def test_twisted_cross_channels_bit_exact(orc, twist):
    """Cross channels (Q, sigma) against brute force over the twisted hole set:
    channels whose partner (-Q, -sigma) is empty are left out (no ring term
    lands in them), the rest keep key order, members and partner index."""
    N, nmax2 = 14, 6
    st = orc.PNM(N, nmax2, 0.1, twist=twist).states()
    groups = _brute_ph(st, N)
    keys = sorted(k for k in groups if (-k[0], -k[1], -k[2], -k[3]) in groups)
    c = _ctx(N, nmax2, 0.1, twist)
    ph = c.export_map(ccd.CCD_MAP_PH_CHANNELS).reshape(-1, 6)
    assert len(ph) == len(keys)
    index = {k: x for x, k in enumerate(keys)}
    for x, k in enumerate(keys):
        partner = index[(-k[0], -k[1], -k[2], -k[3])]
        assert list(ph[x]) == [k[1], k[2], k[3], k[0], len(groups[k]), partner]
    mem = np.array([v for k in keys for pr in groups[k] for v in pr], dtype=np.int32)
    assert np.array_equal(c.export_map(ccd.CCD_MAP_PH), mem)


def test_twist_makes_pair_blocks_rectangular():
    """With the hole set off centre, some pairs {Q, -Q} differ in size; the
    ring operation count is 4 n_Q n_-Q^2 per cross channel."""
    c = _ctx(66, 20, 0.16, (0.7, 1.9, 2.6))
    ph = c.export_map(ccd.CCD_MAP_PH_CHANNELS).reshape(-1, 6)
    n, m = ph[:, 4].astype(float), ph[ph[:, 5], 4].astype(float)
    assert np.any(n != m)
    assert c.info()["flops_ring"] == pytest.approx(np.sum(4.0 * n * m * m))
    assert c.info()["max_ph"] <= 80
    periodic = _ctx(66, 20, 0.16, (0.0, 0.0, 0.0)).export_map(ccd.CCD_MAP_PH_CHANNELS).reshape(-1, 6)
    assert np.array_equal(periodic[:, 4], periodic[periodic[:, 5], 4])


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 20])
def test_twist_mesh_matches_numpy(orc, n):
    th, w = ccd.twist_mesh(n)
    th2, w2 = orc.twist_grid(n)
    assert np.allclose(th, th2, rtol=0, atol=1e-14)
    assert np.allclose(w, w2, rtol=1e-13, atol=1e-17)
    assert w.sum() == pytest.approx(1.0, rel=1e-14)


def test_twist_rules():
    # a twisted box takes any even N; odd N and non-finite angles are refused
    _ctx(20, 8, 0.1, (0.3, 0.2, 0.1))
    with pytest.raises(ccd.CCDError) as e:
        _ctx(15, 8, 0.1, (0.3, 0.2, 0.1))
    assert e.value.status == ccd.CCD_ENOTMAGIC
    with pytest.raises(ccd.CCDError) as e:
        _ctx(14, 8, 0.1, (math.nan, 0.0, 0.0))
    assert e.value.status == ccd.CCD_EINVAL
    # the periodic box still needs a closed shell; -0.0 is no twist
    with pytest.raises(ccd.CCDError) as e:
        _ctx(20, 8, 0.1, (-0.0, 0.0, 0.0))
    assert e.value.status == ccd.CCD_ENOTMAGIC
    with pytest.raises(ccd.CCDError):
        ccd.twist_mesh(0)


def test_twisted_problems_share_structure_only_with_equal_twists(orc):
    """A batch of twists keeps each problem's own plan."""
    th, _ = ccd.twist_mesh(2)
    probs = [ccd.problem(14, 6, r, twist=t) for t in th[:3] for r in (0.08, 0.16)]
    c = ccd.Context(probs)
    for k, t in enumerate(th[:3]):
        for j, r in enumerate((0.08, 0.16)):
            st = c.export_map(ccd.CCD_MAP_STATES, 2 * k + j).reshape(-1, 4)
            assert np.array_equal(st, orc.PNM(14, 6, r, twist=t).states())
