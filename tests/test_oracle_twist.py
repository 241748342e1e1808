"""Pins of the oracle's twisted boundary conditions (the twist-averaging passage
and its algorithm in sec. "Developing a CCD code for infinite matter"):
momenta k = (2 pi n + theta) / L, the holes filled by energy for each twist,
and the Gauss-Legendre twist average.

Each pin is something other than the oracle itself: an integral done by hand,
a closed-form Fermi sea, an invariance that follows from momentum conservation,
exact diagonalisation, the dense form of the iteration, or the infinite-matter
kinetic energy.
"""
import itertools
import math

import numpy as np
import pytest

from test_oracle_pins import _W

HB2M = 41.47
PI = math.pi


def test_twist_grid_integrates_even_powers(orc):
    """Weights w_x w_y w_z / pi^3 sum to 1; an n-point rule on [0, pi] is exact
    for theta^2 and theta^4 once n >= 3: <theta^2> = pi^2/3, <theta^4> = pi^4/5."""
    for n in (3, 4, 5):
        th, w = orc.twist_grid(n)
        assert th.shape == (n ** 3, 3) and np.all((th > 0) & (th < PI))
        assert w.sum() == pytest.approx(1.0, rel=1e-14)
        assert (w * th[:, 0] ** 2).sum() == pytest.approx(PI ** 2 / 3, rel=1e-13)
        assert (w * th[:, 2] ** 4).sum() == pytest.approx(PI ** 4 / 5, rel=1e-13)


@pytest.mark.parametrize("rho", [0.08, 0.16])
def test_two_neutrons_twist_averaged_kinetic_energy(orc, rho):
    """N = 2: for theta in [0, pi)^3 both neutrons sit at n = 0, so
    T(theta) = 2 (hbar^2/2m) |theta|^2 / L^2, and its average over the twists is
    (hbar^2/m) pi^2 / L^2."""
    th, w = orc.twist_grid(3)
    T = 0.0
    for t, wi in zip(th, w):
        p = orc.PNM(2, 4, rho, twist=t)
        assert np.all(p.states()[:2, :3] == 0)
        T += wi * p.kinetic()[:2].sum()
    L = (2.0 / rho) ** (1.0 / 3.0)
    assert T == pytest.approx(HB2M * PI ** 2 / L ** 2, rel=1e-12)


def test_antiperiodic_sixteen_neutrons_closed_form(orc):
    """theta = (pi, pi, pi): k = 2 pi (n + 1/2) / L.  The eight corners
    n in {0, -1}^3 have |n + 1/2|^2 = 3/4 and close a shell of 16, so
    T = 16 (hbar^2/2m) 3 pi^2 / L^2.  Their pairwise |dn|^2 are 0 (8 ordered
    pairs), 1 (24), 2 (24), 3 (8), so with only singlets interacting
    E_ref = T + 36 W(0) + 12 W(1) + 12 W(2) + 4 W(3)."""
    p = orc.PNM(16, 4, 0.1, twist=(PI, PI, PI))
    st = p.states()
    fs = sorted(map(tuple, np.unique(st[:16, :3], axis=0)))
    assert fs == sorted(itertools.product((-1, 0), repeat=3))
    assert tuple(st[16, :3]) not in fs
    L = p.L
    T = 16 * 0.5 * HB2M * 3 * (PI / L) ** 2
    assert p.kinetic()[:16].sum() == pytest.approx(T, rel=1e-13)
    eref = T + 36 * _W(0, L) + 12 * _W(1, L) + 12 * _W(2, L) + 4 * _W(3, L)
    assert p.eref() == pytest.approx(eref, rel=1e-12)


def test_small_twist_keeps_the_correlation_energy(orc):
    """A twist that keeps the hole set cancels in every denominator
    (eps_i + eps_j - eps_a - eps_b loses 4 pi theta.(n_i + n_j - n_a - n_b) = 0
    by momentum conservation) and in every matrix element, so each CCD iterate
    has the periodic energy; E_ref moves by N (hbar^2/2m) |theta|^2 / L^2 since
    the periodic Fermi sea has sum n = 0."""
    th = np.array([0.02, 0.03, 0.05])
    p0 = orc.PNM(14, 4, 0.08)
    p1 = orc.PNM(14, 4, 0.08, twist=th)
    assert set(map(tuple, p0.states()[:14])) == set(map(tuple, p1.states()[:14]))
    assert [tuple(x) for x in p0.states()[:14]] != [tuple(x) for x in p1.states()[:14]]
    shift = 14 * 0.5 * HB2M * float(th @ th) / p0.L ** 2
    assert p1.eref() - p0.eref() == pytest.approx(shift, abs=1e-10)
    o0, o1 = orc.O3(p0), orc.O3(p1)
    assert o1.emp2 == pytest.approx(o0.emp2, rel=1e-12)
    for _ in range(4):
        assert o1.sweep(0.8) == pytest.approx(o0.sweep(0.8), rel=1e-12)


@pytest.mark.parametrize("twist", [(0.7, 1.9, 2.6), (3.0, 0.2, 1.4)])
def test_twisted_two_neutrons_ccd_is_exact(orc, twist):
    """Two neutrons with a twist: CCD is still exact (T2^2 |Phi> = 0), so the
    converged E_ref + Delta E is the lowest eigenvalue of the two-body
    Hamiltonian with twisted kinetic energies in the sector of the hole pair."""
    p = orc.PNM(2, 4, 0.08, twist=twist)
    st = p.states()
    tk = p.kinetic()
    K = st[0, :3] + st[1, :3]
    pairs = [(a, b) for a in range(p.ns) for b in range(a + 1, p.ns)
             if np.all(st[a, :3] + st[b, :3] == K) and st[a, 3] + st[b, 3] == 0]
    H = np.zeros((len(pairs), len(pairs)))
    for x, (a, b) in enumerate(pairs):
        for y, (c, d) in enumerate(pairs):
            H[x, y] = p.v(a, b, c, d) + (tk[a] + tk[b] if x == y else 0.0)
    exact = np.linalg.eigvalsh(H)[0] - p.eref()
    hist = orc.O3(p).solve(0.7, 1e-13, 3000)
    assert hist[-1] == pytest.approx(exact, rel=1e-9)


def test_twisted_holes_are_the_lowest_states(orc):
    """For any twist the states are the periodic basis reordered, every hole
    lies at or below every particle in kinetic energy, and the two spins of a
    momentum stay adjacent (down first)."""
    base = orc.PNM(38, 12, 0.1)
    ref = sorted(map(tuple, base.states()))
    rng = np.random.default_rng(7)
    for _ in range(8):
        th = rng.uniform(0.0, 2 * PI, 3)
        p = orc.PNM(38, 12, 0.1, twist=th)
        st = p.states()
        assert sorted(map(tuple, st)) == ref
        tk = p.kinetic()
        assert tk[:38].max() <= tk[38:].min() * (1 + 1e-12)
        assert np.all(st[0::2, :3] == st[1::2, :3])
        assert np.all(st[0::2, 3] == -1) and np.all(st[1::2, 3] == 1)


def test_twisted_element_equals_its_integer_form(orc):
    """<pq||rs> from the twisted momenta (q = (k_p - k_q - k_r + k_s) / 2, as
    the element is defined) equals its form in integer momentum differences,
    because the twists cancel."""
    p = orc.PNM(14, 4, 0.08, twist=(2.5, 0.4, 1.3))
    st = p.states()
    rng = np.random.default_rng(3)
    done = 0
    while done < 200:
        a, b, c = rng.integers(0, p.ns, 3)
        want = st[a, :3] + st[b, :3] - st[c, :3]
        d = [x for x in range(p.ns) if np.all(st[x, :3] == want)]
        if not d:
            continue
        d = d[rng.integers(0, len(d))]
        assert p.v(a, b, c, d) == pytest.approx(p.v_fast(a, b, c, d), rel=1e-12, abs=1e-15)
        done += 1


@pytest.mark.parametrize("mask", [4, 16, 127])
def test_twisted_o1_and_o3_agree(orc, mask):
    """A twist that moves holes (the hole set is no longer inversion symmetric,
    so cross channels Q and -Q differ in size): dense eq. ccd3 and the
    intermediates form still agree sweep by sweep."""
    th = (2.5, 0.4, 1.3)
    p = orc.PNM(14, 2, 0.1, twist=th)
    p0 = orc.PNM(14, 2, 0.1)
    assert set(map(tuple, p.states()[:14])) != set(map(tuple, p0.states()[:14]))
    o1 = orc.O1(p.kinetic(), p.dense_v(), 14)
    o3 = orc.O3(p)
    assert o1.emp2 == pytest.approx(o3.emp2, rel=1e-13)
    for _ in range(3):
        assert o1.sweep(0.8, mask) == pytest.approx(o3.sweep(0.8, mask), rel=1e-12)


@pytest.mark.parametrize("N", [38, 114])
def test_twist_average_brings_kinetic_energy_to_infinite_matter(orc, N):
    """The finite-size error of T/N against 3 hbar^2 k_F^2 / 10m
    (k_F^3 = 3 pi^2 rho) shrinks at least five-fold from periodic to
    twist-averaged (5 points per direction) boundary conditions."""
    rho = 0.16
    kf = (3 * PI ** 2 * rho) ** (1.0 / 3.0)
    t_inf = 3 * HB2M * kf ** 2 / 10
    t_pbc = orc.PNM(N, 20, rho).kinetic()[:N].sum() / N
    th, w = orc.twist_grid(5)
    t_tabc = sum(wi * orc.PNM(N, 20, rho, twist=t).kinetic()[:N].sum() / N for t, wi in zip(th, w))
    assert abs(t_tabc - t_inf) < 0.2 * abs(t_pbc - t_inf)
