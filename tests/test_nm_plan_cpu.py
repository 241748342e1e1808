"""The nuclear-matter plan of the C ABI (include/ccd_nm.h) against the oracle,
on the CPU: states bit for bit, the element the kernels use, Fock and
reference energies, and the set of canonical amplitudes.  No GPU work."""
import numpy as np
import pytest

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")


def _pair(orc, A, n2, rho, species=2):
    m = orc.NM(A, n2, rho, species=species)
    c = ccd.NMContext(ccd.nm_problem(A, n2, rho, species=species))
    return m, c


@pytest.mark.parametrize("A,n2,species", [(4, 1, 2), (28, 4, 2), (76, 9, 2), (14, 4, 1), (66, 20, 1)])
def test_states_bit_exact(orc, A, n2, species):
    m, c = _pair(orc, A, n2, 0.16, species)
    st = c.export_map(ccd.CCD_NM_MAP_STATES).reshape(-1, 5)
    assert np.array_equal(st[:, :4], m.states())
    assert np.array_equal(st[:, 4], m.isospins())
    assert c.info()["n_holes"] == A


@pytest.mark.parametrize("A,n2,species", [(28, 4, 2), (76, 9, 2), (14, 4, 1)])
def test_fock_and_reference_energies(orc, A, n2, species):
    m, c = _pair(orc, A, n2, 0.12, species)
    tk, eps, eref = c.export_tables()
    assert np.allclose(tk, m.kinetic(), rtol=1e-13, atol=0)
    assert np.allclose(eps, m.fock(), rtol=1e-12, atol=1e-12)
    assert eref == pytest.approx(m.eref(), rel=1e-12)


def test_element_against_oracle_every_spin_isospin_kind(orc):
    m, c = _pair(orc, 28, 4, 0.16)
    st, tz = m.states(), m.isospins()
    rng = np.random.default_rng(23)
    kinds = set()
    n = m.ns
    checked = 0
    while checked < 3000:
        a, b, r = (int(x) for x in rng.integers(0, n, 3))
        tgt = st[a, :3] + st[b, :3] - st[r, :3]
        cand = np.nonzero(np.all(st[:, :3] == tgt, axis=1))[0]
        if len(cand) == 0:
            continue
        s = int(rng.choice(cand))
        want = m.v(a, b, r, s)
        got = c.element(a, b, r, s)
        assert got == pytest.approx(want, rel=1e-12, abs=1e-15), (a, b, r, s)
        if want != 0.0:
            kinds.add((int(tz[a] + tz[b]), int(st[a, 3] + st[b, 3])))
        checked += 1
    assert kinds == {(t, s) for t in (-2, 0, 2) for s in (-2, 0, 2)} - {(-2, -2), (-2, 2), (2, -2), (2, 2)}


@pytest.mark.parametrize("A,n2", [(4, 1), (28, 4)])
def test_canonical_amplitudes_are_the_oracle_set(orc, A, n2):
    m, c = _pair(orc, A, n2, 0.1)
    idx = c.canonical_index()
    assert len(idx) == c.info()["n_amplitudes"]
    assert np.all(idx[:, 0] < idx[:, 1]) and np.all(idx[:, 2] < idx[:, 3])
    o3 = orc.O3(m)
    ijab, _ = o3.export()
    sel = (ijab[:, 0] < ijab[:, 1]) & (ijab[:, 2] < ijab[:, 3])
    want = {tuple(x) for x in ijab[sel]}
    assert {tuple(x) for x in idx} == want


def test_not_closed_shell_refused():
    for A in (2, 8, 30):
        with pytest.raises(ccd.CCDError):
            ccd.NMContext(ccd.nm_problem(A, 4, 0.16))


def test_kernel_families():
    """The timing families in the order the header documents them."""
    lib = ccd._lib
    names = [lib.ccd_nm_kernel_name(f).decode() for f in range(8)]
    assert names == ["gather", "rowcol", "dchi", "gemm_chi", "gemm_ladder_ring", "update", "energy", "ladder_pp"]
    assert lib.ccd_nm_kernel_name(8) == b"" and lib.ccd_nm_kernel_name(-1) == b""


@pytest.mark.parametrize("n2,rho", [(4, 0.16), (20, 0.16), (36, 0.08)])
def test_neutron_ladder_over_momentum_pairs_matches_the_neutron_path(n2, rho):
    """With neutrons only the isospin path's pp ladder over momentum pairs
    (its grouping of each block's rows by the first state's momentum, the
    pairing of its label pairs and the classes the plan derives) must come to
    exactly the momentum-pair products of the neutron path: the same pair
    counts in every block give the same flops, counted independently."""
    c = ccd.NMContext(ccd.nm_problem(66 if n2 >= 20 else 14, n2, rho, species=1))
    flops = {k: v[2] for k, v in c.kernel_times().items()}
    p = ccd.Context([ccd.problem(66 if n2 >= 20 else 14, n2, rho)])
    assert flops["ladder_pp"] == p.info(0)["flops_pp"]
    assert flops["ladder_pp"] > 0


@pytest.mark.parametrize("A,n2", [(28, 4), (76, 9), (108, 20)])
def test_every_isospin_block_takes_the_momentum_pair_form(A, n2):
    """Symmetric matter: every block's pp ladder goes over its momentum pairs,
    counted here from the exported pair lists: the distinct momenta of the
    pairs' first states, times the products the block's kind needs (one
    difference and one element class for S_z = 0 pairs of like particles and
    |S_z| = 1 pairs of unlike ones, two of each for S_z = T_z = 0, none for
    |S_z| = |T_z| = 1, where the element vanishes).  A block left to the product
    over label pairs would be missing from the sum."""
    c = ccd.NMContext(ccd.nm_problem(A, n2, 0.16))
    info = c.info()
    kt = c.kernel_times()
    blocks = c.export_map(ccd.CCD_NM_MAP_CHANNELS).reshape(info["n_channels"], 7)
    pp = c.export_map(ccd.CCD_NM_MAP_PP).reshape(-1, 2)
    st = c.export_map(ccd.CCD_NM_MAP_STATES).reshape(-1, 5)
    want, row = 0.0, 0
    for kx, ky, kz, sz2, tz2, nhh, npp in blocks:
        firsts = {tuple(st[a, :3]) for a in pp[row:row + npp, 0]}
        row += npp
        prods = 4 if (sz2, tz2) == (0, 0) else (1 if (sz2 == 0) != (tz2 == 0) else 0)
        want += 2.0 * prods * len(firsts) ** 2 * nhh
    assert row == len(pp)
    assert kt["ladder_pp"][2] == pytest.approx(want, rel=1e-15) and want > 0
    assert info["flops_per_sweep"] == pytest.approx(kt["gemm_chi"][2] + kt["gemm_ladder_ring"][2] +
                                                    kt["ladder_pp"][2], rel=1e-15)
