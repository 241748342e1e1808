"""C ABI and host plan, without a GPU.

The library must load and export every function include/ccd.h declares; its
host plan (basis, channels, tables) must match what the oracle and brute-force
counting give, bit for bit for integer maps.
"""
import math
import os
import re

import numpy as np
import pytest

from conftest import ROOT

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")


def header_functions():
    names = set()
    for h in ("ccd.h", "ccd_mlp.h", "ccd_nm.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(ccd_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    import ctypes
    lib = ctypes.CDLL(ccd.LIB_PATH)
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ccd.EXPORTED)


def test_library_is_built_for_gfx950():
    data = open(ccd.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _ctx(N, nmax2, rho):
    return ccd.Context([ccd.problem(N, nmax2, rho)])


@pytest.mark.parametrize("N,nmax2,rho", [(14, 4, 0.08), (66, 20, 0.02), (38, 12, 0.11)])
def test_basis_bit_exact_vs_oracle(orc, N, nmax2, rho):
    c = _ctx(N, nmax2, rho)
    got = c.export_map(ccd.CCD_MAP_STATES).reshape(-1, 4)
    want = orc.PNM(N, nmax2, rho).states()
    assert got.dtype == np.int32
    assert np.array_equal(got, want.astype(np.int32))


@pytest.mark.parametrize("N,nmax2,rho", [(14, 4, 0.08), (66, 20, 0.16), (54, 14, 0.1)])
def test_tables_vs_oracle(orc, N, nmax2, rho):
    c = _ctx(N, nmax2, rho)
    p = orc.PNM(N, nmax2, rho)
    tk, eps, w = c.export_tables()
    assert np.allclose(tk, p.kinetic(), rtol=1e-14, atol=0)
    assert np.allclose(eps, p.fock(), rtol=1e-12, atol=1e-12)
    eref = c.eref()
    assert eref == pytest.approx(p.eref(), rel=1e-12)
    L = p.L
    assert c.info()["box_L"] == pytest.approx(L, rel=1e-15)
    # W(m) against the Gaussian transform written out
    for m in range(0, len(w), 7):
        want = sum(V / L ** 3 * (math.pi / k) ** 1.5 * math.exp(-(2 * math.pi / L) ** 2 * m / (4 * k))
                   for V, k in ((200.0, 1.487), (-91.85, 0.465)))
        assert w[m] == pytest.approx(want, rel=1e-14)
    assert len(w) == 4 * nmax2 + 1


def _brute_channels(st, N):
    """Direct channels by brute-force grouping of pairs, ordered by (2S_z, K)."""
    n = len(st)
    hh, pp = {}, {}
    for i in range(N):
        for j in range(i + 1, N):
            key = (int(st[i, 3] + st[j, 3]),) + tuple(int(x) for x in st[i, :3] + st[j, :3])
            hh.setdefault(key, []).append((i, j))
    for a in range(N, n):
        for b in range(a + 1, n):
            key = (int(st[a, 3] + st[b, 3]),) + tuple(int(x) for x in st[a, :3] + st[b, :3])
            if key in hh:
                pp.setdefault(key, []).append((a, b))
    keys = sorted(k for k in hh if k in pp)
    return keys, hh, pp


@pytest.mark.parametrize("N,nmax2", [(14, 4), (14, 6), (38, 8)])
def test_direct_channels_bit_exact(orc, N, nmax2):
    st = orc.PNM(N, nmax2, 0.1).states()
    keys, hh, pp = _brute_channels(st, N)
    c = _ctx(N, nmax2, 0.1)
    ch = c.export_map(ccd.CCD_MAP_CHANNELS).reshape(-1, 6)
    assert len(ch) == len(keys)
    want_ch = np.array([[k[1], k[2], k[3], k[0], len(hh[k]), len(pp[k])] for k in keys], dtype=np.int32)
    assert np.array_equal(ch, want_ch)
    want_hh = np.array([x for k in keys for pr in hh[k] for x in pr], dtype=np.int32)
    want_pp = np.array([x for k in keys for pr in pp[k] for x in pr], dtype=np.int32)
    assert np.array_equal(c.export_map(ccd.CCD_MAP_HH), want_hh)
    assert np.array_equal(c.export_map(ccd.CCD_MAP_PP), want_pp)
    assert c.info()["n_amplitudes"] == sum(len(hh[k]) * len(pp[k]) for k in keys)


def test_amplitude_count_matches_oracle_conservation(orc):
    """Ordered (i, j, a) with a valid b counted by the oracle = 4 x canonical."""
    p = orc.PNM(66, 20, 0.1)
    o3 = orc.O3(p)
    c = _ctx(66, 20, 0.1)
    assert orc.lib().orc_o3_count(o3.o) == 4 * c.info()["n_amplitudes"]


@pytest.mark.parametrize("N,nmax2", [(14, 4), (38, 8)])
def test_ph_channels_bit_exact(orc, N, nmax2):
    st = orc.PNM(N, nmax2, 0.1).states()
    n = len(st)
    groups = {}
    for p in range(N, n):
        for h in range(N):
            key = (int(st[p, 3] - st[h, 3]),) + tuple(int(x) for x in st[p, :3] - st[h, :3])
            groups.setdefault(key, []).append((p, h))
    keys = sorted(groups)
    c = _ctx(N, nmax2, 0.1)
    ph = c.export_map(ccd.CCD_MAP_PH_CHANNELS).reshape(-1, 6)
    assert len(ph) == len(keys)
    index = {k: x for x, k in enumerate(keys)}
    for x, k in enumerate(keys):
        partner = index[(-k[0], -k[1], -k[2], -k[3])]
        assert list(ph[x]) == [k[1], k[2], k[3], k[0], len(groups[k]), partner]
    mem = np.array([v for k in keys for pr in groups[k] for v in pr], dtype=np.int32)
    assert np.array_equal(c.export_map(ccd.CCD_MAP_PH), mem)


def test_operation_counts_match_definition():
    c = _ctx(66, 36, 0.16)
    i = c.info()
    assert i["n_states"] == 1850
    ch = c.export_map(ccd.CCD_MAP_CHANNELS).reshape(-1, 6)
    sz0 = ch[ch[:, 3] == 0]
    M, Nn = sz0[:, 5].astype(float), sz0[:, 4].astype(float)
    # the FP64 pp product runs over the momentum pairs {n_a, n_b} of each block:
    # the distinct momenta of the rows' first states
    st = c.export_map(ccd.CCD_MAP_STATES).reshape(-1, 4)
    pp = c.export_map(ccd.CCD_MAP_PP).reshape(-1, 2)
    off = np.concatenate([[0], np.cumsum(ch[:, 5])])
    Mr = np.array([len({tuple(st[a, :3]) for a in pp[off[k]:off[k + 1], 0]})
                   for k in range(len(ch)) if ch[k, 3] == 0], dtype=float)
    assert np.all((Mr >= M / 2) & (Mr <= (M + 1) / 2))
    assert i["flops_pp"] == pytest.approx(np.sum(2 * Mr * Mr * Nn))
    ph = c.export_map(ccd.CCD_MAP_PH_CHANNELS).reshape(-1, 6)
    assert i["flops_ring"] == pytest.approx(np.sum(4.0 * ph[:, 4].astype(float) ** 3))
    # ordered-pair form of the paper: pp + hh + chi_klij at ordered pairs + ring
    ordered = np.sum(2 * (2 * M) ** 2 * (2 * Nn) + 4 * (2 * M) * (2 * Nn) ** 2) + i["flops_ring"]
    assert i["flops_ordered"] == pytest.approx(ordered)
    assert round(i["flops_ordered"] / 1e9, 2) == 8.33


@pytest.mark.parametrize("N", [3, 10, 15, 67])
def test_not_closed_shell_is_rejected(N):
    with pytest.raises(ccd.CCDError) as e:
        _ctx(N, 8, 0.1)
    assert e.value.status == ccd.CCD_ENOTMAGIC


def test_invalid_arguments():
    with pytest.raises(ccd.CCDError) as e:
        _ctx(14, 4, -0.1)
    assert e.value.status == ccd.CCD_EINVAL
    with pytest.raises(ccd.CCDError) as e:
        _ctx(14, 0, 0.1)
    assert e.value.status == ccd.CCD_EINVAL
    with pytest.raises(ccd.CCDError) as e:
        _ctx(66, 4, 0.1)  # no particle states
    assert e.value.status == ccd.CCD_ENOTMAGIC


def test_device_calls_before_binding_fail_cleanly():
    c = _ctx(14, 4, 0.08)
    with pytest.raises(ccd.CCDError) as e:
        c.iterate(1.0, 1e-10, 5)
    assert e.value.status == ccd.CCD_ESTATE
    with pytest.raises(ccd.CCDError) as e:
        c.get_amplitudes()
    assert e.value.status == ccd.CCD_ESTATE


def test_batched_plan_keeps_problems_separate(orc):
    probs = [ccd.problem(14, 4, 0.08), ccd.problem(38, 12, 0.05), ccd.problem(66, 20, 0.2)]
    c = ccd.Context(probs)
    for p, (N, n2, rho) in enumerate([(14, 4, 0.08), (38, 12, 0.05), (66, 20, 0.2)]):
        got = c.export_map(ccd.CCD_MAP_STATES, p).reshape(-1, 4)
        assert np.array_equal(got, orc.PNM(N, n2, rho).states().astype(np.int32))
        single = ccd.Context([probs[p]])
        assert c.info(p) == single.info(0)
    assert c.workspace_size() > 0


def test_build_step_does_not_need_the_library():
    """The build module imports without loading libccd.so (fresh checkouts)."""
    import subprocess
    import sys
    code = ("import sys, paper_1611_06765_amd.build_lib as b; "
            "assert 'paper_1611_06765_amd.ccd' not in sys.modules; print(b.LIB)")
    subprocess.check_call([sys.executable, "-c", code], cwd=ROOT)


def test_size_limits():
    """The largest cutoff the W table supports (n^2 <= 64) plans; N = 114 has
    particle-hole blocks beyond the ring kernels' 80 and is refused with a
    reason; a cutoff beyond 64 is refused."""
    c = _ctx(66, 64, 0.16)
    i = c.info()
    assert i["n_states"] == 4218 and i["lut_size"] == 257 and i["max_ph"] <= 80
    with pytest.raises(ccd.CCDError) as e:
        _ctx(114, 20, 0.16)
    assert e.value.status == ccd.CCD_EINVAL and "particle-hole" in str(e.value)
    with pytest.raises(ccd.CCDError) as e:
        _ctx(66, 65, 0.16)
    assert e.value.status == ccd.CCD_EINVAL


def test_measure_ceilings_checks_its_arguments():
    import numpy as np
    out = np.zeros(5)
    st = ccd._lib.ccd_measure_ceilings(None, 1 << 30, None, out.ctypes.data_as(ccd._dp))
    assert st == ccd.CCD_EINVAL
    st = ccd._lib.ccd_measure_ceilings(ccd._vp(4096 + 8), 1 << 30, None, out.ctypes.data_as(ccd._dp))
    assert st == ccd.CCD_EINVAL  # misaligned


@pytest.mark.parametrize("n,nh", [(1, 1), (49, 4), (8, 0), (8, 8)])
def test_dense_solver_limits(n, nh):
    import ctypes
    b = ctypes.c_size_t()
    assert ccd._lib.ccd_dense_workspace_size(n, nh, ctypes.byref(b)) == ccd.CCD_EINVAL


def test_pairing_hamiltonian_two_constructions_agree(orc):
    """The input module's pairing elements (direct, then antisymmetrised) equal
    the oracle's (signed pair factors), and the model's E_ref = 2 delta - g."""
    import numpy as np
    from paper_1611_06765_amd import inputs
    for g in (-1.0, -0.3, 0.7):
        h1, v1 = inputs.pairing_hamiltonian(g)
        h2, v2 = orc.pairing_model(g)
        assert np.array_equal(h1, h2) and np.array_equal(v1, v2)
        eref = h1[:4].sum() + 0.5 * sum(v1[i, j, i, j] for i in range(4) for j in range(4))
        assert eref == pytest.approx(2.0 - g, abs=1e-14)


def test_kernel_family_names():
    """The timing families in the order the header documents them."""
    names = [ccd._lib.ccd_kernel_name(i).decode() for i in range(ccd._lib.ccd_kernel_families())]
    assert names == ["init", "direct", "dsum", "dchi", "ring_small", "ring32", "ring48", "ring64", "ring80",
                     "ladder", "update", "energy"]
    assert ccd._lib.ccd_kernel_name(-1) == b"" and ccd._lib.ccd_kernel_name(len(names)) == b""
