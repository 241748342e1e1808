"""Pins of the oracle's symmetric nuclear matter (protons and neutrons, the
isospin loop of the model-space passage and the full Minnesota operator with
its V_T channel) against what the paper and the mathematics fix: Table 1's
magic numbers doubled, an independent construction of the spin-isospin
element from Pauli matrices, exact diagonalisation of two nucleons, the
MBPT2 and third-order identities, the dense form O1 against the
intermediates form O3, isospin symmetry, and the pure-neutron limit."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

from conftest import golden

MIN = dict(VR=200.0, kR=1.487, VT=-178.0, kT=0.639, VS=-91.85, kS=0.465)


def test_snm_magic_numbers_table1_doubled(orc):
    """Closed shells of symmetric nuclear matter are Table 1's fillings
    doubled (4, 28, 76, 108, 132, 228); other nucleon numbers are refused."""
    magic = [int(r[0]) for r in golden("snm_magic.txt")]
    for A in magic:
        m = orc.NM(A, 9, 0.16)
        st, tz = m.states(), m.isospins()
        holes = st[:A]
        assert np.sum(tz[:A] < 0) == A // 2 and np.sum(tz[:A] > 0) == A // 2
        # the holes are whole momenta with all four spin-isospin states
        mom = {tuple(x) for x in holes[:, :3]}
        assert len(mom) * 4 == A
    for A in range(2, 232, 2):
        if A in magic:
            continue
        with pytest.raises(ValueError):
            orc.NM(A, 9, 0.16)


def test_snm_basis_is_pnm_basis_times_isospin(orc):
    for n2 in (1, 4, 9, 20):
        s = orc.NM(4, n2, 0.1)
        p = orc.PNM(2, n2, 0.1)
        assert s.ns == 2 * p.ns
        st, tz = s.states(), s.isospins()
        # loop order: momentum, then spin, then isospin innermost
        assert np.array_equal(st[0::2], p.states()) and np.array_equal(st[1::2], p.states())
        assert np.all(tz[0::2] == -1) and np.all(tz[1::2] == 1)


def _pauli_spin_isospin_operators():
    """The three channel operators on |s1 t1, s2 t2> (kron order spin1,
    iso1, spin2, iso2) from P_s = (1 + s1.s2)/2 and P_t = (1 + t1.t2)/2."""
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.array([[1, 0], [0, -1]], dtype=complex)
    e = np.eye(2)

    def on(a, b, c, d):
        return np.kron(np.kron(np.kron(a, b), c), d)

    Ps = 0.5 * (np.eye(16) + sum(on(s, e, s, e) for s in (sx, sy, sz)))
    Pt = 0.5 * (np.eye(16) + sum(on(e, s, e, s) for s in (sx, sy, sz)))
    one = np.eye(16)
    ex = one - Ps @ Pt
    ops = {"R": 0.5 * ex, "T": 0.25 * (one + Ps) @ ex, "S": 0.25 * (one - Ps) @ ex}
    assert all(np.max(np.abs(o.imag)) < 1e-15 for o in ops.values())
    return {k: o.real for k, o in ops.items()}


def _ft_numeric(V, kappa, q):
    if q == 0.0:
        f = lambda r: 4 * math.pi * r * r * V * math.exp(-kappa * r * r)
    else:
        f = lambda r: 4 * math.pi * r * r * V * math.exp(-kappa * r * r) * math.sin(q * r) / (q * r)
    val, _ = integrate.quad(f, 0.0, 40.0, limit=400, epsabs=1e-13, epsrel=1e-13)
    return val


def test_snm_element_independent_construction(orc):
    """<pq||rs> of the full Minnesota operator between nucleons of any spin
    and isospin: spatial part a numerical Fourier integral, spin-isospin part
    from Pauli matrices (index 0 = spin up / isospin up = neutron)."""
    m = orc.NM(28, 4, 0.16)
    st, tz = m.states(), m.isospins()
    L = m.L
    ops = _pauli_spin_isospin_operators()
    pars = {"R": (MIN["VR"], MIN["kR"]), "T": (MIN["VT"], MIN["kT"]), "S": (MIN["VS"], MIN["kS"])}
    one = lambda x: 2 * (st[x, 3] < 0) + (tz[x] < 0)
    idx = lambda a, b: 4 * one(a) + one(b)

    def vdir(a, b, c, d):
        na, nb, nc, nd = (st[x, :3] for x in (a, b, c, d))
        if np.any(na + nb != nc + nd):
            return 0.0
        q = 0.5 * (2 * math.pi / L) * (na - nb - nc + nd)
        qn = float(np.sqrt(q @ q))
        tot = 0.0
        for ch, (V, k) in pars.items():
            si = ops[ch][idx(a, b), idx(c, d)]
            if si != 0.0:
                tot += _ft_numeric(V, k, qn) / L ** 3 * si
        return tot

    rng = np.random.default_rng(17)
    n = m.ns
    kinds = set()
    checked = 0
    while checked < 80:
        a, b, c = (int(x) for x in rng.integers(0, n, 3))
        if checked % 2 == 0:
            # every other sample: a proton and a neutron of equal spin (the
            # triplet channels only V_T and V_R reach)
            b = int(rng.choice([x for x in range(n) if tz[x] != tz[a] and st[x, 3] == st[a, 3]]))
        target = st[a, :3] + st[b, :3] - st[c, :3]
        cands = [d for d in range(n) if np.all(st[d, :3] == target)]
        if not cands:
            continue
        d = cands[rng.integers(len(cands))]
        want = vdir(a, b, c, d) - vdir(a, b, d, c)
        got = m.v(a, b, c, d)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-12), (a, b, c, d)
        if want != 0.0:
            kinds.add((tz[a] + tz[b], st[a, 3] + st[b, 3]))
        checked += 1
    # pn pairs in spin triplets (the V_T channel) were among the nonzero ones
    assert (0, 2) in kinds or (0, -2) in kinds


def test_snm_conservation_and_symmetries(orc):
    m = orc.NM(28, 4, 0.12)
    st, tz = m.states(), m.isospins()
    n = m.ns
    rng = np.random.default_rng(5)
    for _ in range(600):
        a, b, c, d = (int(x) for x in rng.integers(0, n, 4))
        v = m.v(a, b, c, d)
        assert v == pytest.approx(-m.v(b, a, c, d), abs=1e-14)
        assert v == pytest.approx(-m.v(a, b, d, c), abs=1e-14)
        assert v == pytest.approx(m.v(c, d, a, b), abs=1e-14)
        if v != 0.0:
            assert np.all(st[a, :3] + st[b, :3] == st[c, :3] + st[d, :3])
            assert st[a, 3] + st[b, 3] == st[c, 3] + st[d, 3]
            assert tz[a] + tz[b] == tz[c] + tz[d]


def test_like_nucleons_feel_the_neutron_matter_force(orc):
    """Between two neutrons (or two protons) the element equals the pure
    neutron matter element of the same momenta and spins at the same box side
    (the V_T channel vanishes between like nucleons)."""
    m = orc.NM(28, 4, 0.16)
    p = orc.PNM(14, 4, 0.08)  # L = (14 / 0.08)^(1/3) = (28 / 0.16)^(1/3)
    assert m.L == pytest.approx(p.L, rel=1e-15)
    st, tz = m.states(), m.isospins()
    pst = p.states()
    key = {tuple(x): k for k, x in enumerate(pst)}
    rng = np.random.default_rng(9)
    checked = 0
    while checked < 200:
        a, b, c, d = (int(x) for x in rng.integers(0, m.ns, 4))
        if not (tz[a] == tz[b] == tz[c] == tz[d]):
            continue
        pa, pb, pc, pd = (key[tuple(st[x])] for x in (a, b, c, d))
        assert m.v(a, b, c, d) == pytest.approx(p.v(pa, pb, pc, pd), rel=1e-13, abs=1e-15)
        checked += 1


def test_neutron_only_species_is_pnm(orc):
    a = orc.NM(14, 4, 0.08, species=1)
    b = orc.PNM(14, 4, 0.08)
    assert np.array_equal(a.states(), b.states())
    assert np.array_equal(a.fock(), b.fock())
    oa, ob = orc.O3(a), orc.O3(b)
    assert oa.emp2 == ob.emp2
    assert oa.sweep(0.7) == ob.sweep(0.7)


@pytest.mark.parametrize("nmax2,rho", [(1, 0.05), (2, 0.08)])
def test_proton_neutron_pair_ccd_is_exact(orc, nmax2, rho):
    """A proton and a neutron (the first two states: zero momentum, both spin
    down, so S_z = -1, T_z = 0): T1 vanishes by momentum conservation and T2^2
    annihilates two-nucleon states, so converged CCD equals the lowest
    eigenvalue of H in the K = 0, S_z = -1, T_z = 0 two-body sector, which the
    triplet channel V_T binds."""
    m = orc.NM(2, nmax2, rho, open_ok=True)
    st, tz = m.states(), m.isospins()
    assert (st[0, 3], st[1, 3], tz[0], tz[1]) == (-1, -1, -1, 1)
    tk = m.kinetic()
    pairs = [(a, b) for a in range(m.ns) for b in range(a + 1, m.ns)
             if np.all(st[a, :3] + st[b, :3] == 0) and st[a, 3] + st[b, 3] == -2 and tz[a] + tz[b] == 0]
    H = np.array([[m.v(a, b, c, d) + (tk[a] + tk[b] if x == y else 0.0)
                   for y, (c, d) in enumerate(pairs)] for x, (a, b) in enumerate(pairs)])
    exact = np.linalg.eigvalsh(H)[0] - m.eref()
    assert exact < -0.1
    o3 = orc.O3(m)
    hist = o3.solve(0.5, 1e-12, 4000)
    assert abs(hist[-1] - hist[-2]) < 1e-12
    assert hist[-1] == pytest.approx(exact, rel=1e-9)
    if m.ns <= 60:
        o1 = orc.O1(tk, m.dense_v(), 2)
        e = o1.ecorr
        for _ in range(4000):
            en = o1.sweep(0.5)
            if abs(en - e) < 1e-12:
                break
            e = en
        assert en == pytest.approx(exact, rel=1e-9)


def test_snm_first_iteration_energy_is_mbpt2(orc):
    m = orc.NM(4, 2, 0.1)
    v, eps = m.dense_v(), m.fock()
    A, n = 4, m.ns
    h, pp = slice(0, A), slice(A, n)
    D = eps[h, None, None, None] + eps[None, h, None, None] - eps[None, None, pp, None] - eps[None, None, None, pp]
    vv = v[h, h, pp, pp]
    e2 = 0.25 * np.sum(vv * vv / D)
    assert orc.O3(m).emp2 == pytest.approx(e2, rel=1e-12)


def _third_order(m, v, eps, A):
    n = m.ns
    H, P = range(A), range(A, n)
    D2 = lambda i, j, a, b: eps[i] + eps[j] - eps[a] - eps[b]
    d4 = d5 = d3 = 0.0
    for i, j in itertools.product(H, H):
        for a, b in itertools.product(P, P):
            x = v[i, j, a, b]
            if x == 0.0:
                continue
            dij = D2(i, j, a, b)
            for c, d in itertools.product(P, P):
                y = v[c, d, a, b]
                if y != 0.0:
                    d4 += v[i, j, c, d] * y * x / (D2(i, j, c, d) * dij)
            for k, l in itertools.product(H, H):
                y = v[k, l, i, j]
                if y != 0.0:
                    d5 += v[a, b, k, l] * y * x / (dij * D2(k, l, a, b))
            for k in H:
                for c in P:
                    y = v[b, k, j, c]
                    if y != 0.0:
                        d3 += x * y * v[a, c, i, k] / (dij * D2(i, k, a, c))
    return d4 / 8.0, d5 / 8.0, d3


def test_snm_linear_terms_reproduce_third_order_diagrams(orc):
    """One linear sweep from t^(0) adds diagrams (4), (5) and (3) of eqs.
    diag3-diag5 (diagram (3) read with <bk|v|jc>), by brute force, A = 4,
    n^2 <= 1 (28 states)."""
    m = orc.NM(4, 1, 0.12)
    v, eps = m.dense_v(), m.fock()
    d4, d5, d3 = _third_order(m, v, eps, 4)
    for mask, want in ((orc.T_PP, d4), (orc.T_HH, d5), (orc.T_RING, d3), (orc.T_LINEAR, d3 + d4 + d5)):
        assert abs(want) > 1e-6
        o3 = orc.O3(m)
        assert o3.sweep(1.0, mask) - o3.emp2 == pytest.approx(want, rel=1e-10)
        o1 = orc.O1(m.kinetic(), v, 4)
        assert o1.sweep(1.0, mask) - o1.emp2 == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("mask", [1, 2, 4, 8, 16, 32, 64, 127])
def test_snm_o1_and_o3_agree_per_term(orc, mask):
    m = orc.NM(4, 1, 0.1)
    o1 = orc.O1(m.kinetic(), m.dense_v(), 4)
    o3 = orc.O3(m)
    assert o1.emp2 == pytest.approx(o3.emp2, rel=1e-13)
    for _ in range(3):
        assert o1.sweep(0.8, mask) == pytest.approx(o3.sweep(0.8, mask), rel=1e-12)
    ijab, tv = o3.export()
    for (i, j, a, b), t in zip(ijab[::5], tv[::5]):
        assert o1.t(a, b, i, j) == pytest.approx(t, rel=1e-10, abs=1e-15)


def test_snm_isospin_mirror_symmetry(orc):
    """Without Coulomb the Minnesota force is isospin symmetric, so swapping
    protons and neutrons maps every amplitude onto an equal one after any
    number of sweeps (A = 28, n^2 <= 4)."""
    m = orc.NM(28, 4, 0.16)
    st, tz = m.states(), m.isospins()
    key = {(tuple(st[x]), int(tz[x])): x for x in range(m.ns)}
    mirror = np.array([key[(tuple(st[x]), -int(tz[x]))] for x in range(m.ns)])
    o3 = orc.O3(m)
    o3.sweep(0.7)
    o3.sweep(0.7)
    ijab, tv = o3.export()
    sel = np.random.default_rng(2).choice(len(tv), 400, replace=False)
    for k in sel:
        i, j, a, b = (mirror[x] for x in ijab[k])
        assert o3.t(a, b, i, j) == pytest.approx(tv[k], rel=1e-12, abs=1e-16)
