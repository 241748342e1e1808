"""The identity behind the ladder over momentum pairs, checked on the oracle's
own interaction (no GPU): in an S_z = 0 block (the only blocks with a nonzero
pp ladder) the rows come in momentum pairs {p, K - p} whose two spin rows
(p up, q down) and (p down, q up) have opposite elements <ab||cd> with every
column, and the two spin columns of a pair are opposite with every row.  So
the product over spin pairs equals the product over momentum pairs on
t(up, down) - t(down, up).  The library's pair count per block is checked
against the blocks it exports."""
import numpy as np
import pytest

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")


def _blocks(c):
    ch = c.export_map(ccd.CCD_MAP_CHANNELS).reshape(-1, 6)
    pp = c.export_map(ccd.CCD_MAP_PP).reshape(-1, 2)
    off = np.concatenate([[0], np.cumsum(ch[:, 5])])
    return [(ch[k], pp[off[k]:off[k + 1]]) for k in range(len(ch)) if ch[k, 3] == 0]


def _pairs(st, rows):
    """momentum pair -> {spin of a: row}, keyed by the momentum of a"""
    out = {}
    for r, (a, b) in enumerate(rows):
        slot = out.setdefault(tuple(st[a, :3]), {})
        assert st[a, 3] not in slot, "two rows of one block share a and its spin"
        slot[int(st[a, 3])] = r
    return out


@pytest.mark.parametrize("case", [(14, 4, 0.08, None), (38, 8, 0.12, None), (14, 6, 0.1, (2.5, 0.4, 1.3))])
def test_spin_rows_of_a_momentum_pair_are_opposite(orc, case):
    N, n2, rho, tw = case
    kw = {} if tw is None else {"twist": tw}
    p = orc.PNM(N, n2, rho, **kw)
    c = ccd.Context([ccd.problem(N, n2, rho, **kw)])
    st = p.states()
    assert np.array_equal(c.export_map(ccd.CCD_MAP_STATES).reshape(-1, 4), st)
    rng = np.random.default_rng(11)
    checked = 0
    for ch, rows in _blocks(c):
        pairs = _pairs(st, rows)
        # the two rows of a pair have the same momenta (a, b) with spins swapped
        for slot in pairs.values():
            if len(slot) == 2:
                (a1, b1), (a2, b2) = rows[slot[1]], rows[slot[-1]]
                assert np.array_equal(st[a1, :3], st[a2, :3]) and np.array_equal(st[b1, :3], st[b2, :3])
        for slot in list(pairs.values())[:6]:
            if len(slot) < 2:
                continue
            up, dn = rows[slot[1]], rows[slot[-1]]
            for j in rng.choice(len(rows), size=min(len(rows), 6), replace=False):
                cc, dd = rows[j]
                v_up = p.v(up[0], up[1], cc, dd)
                v_dn = p.v(dn[0], dn[1], cc, dd)
                assert v_dn == pytest.approx(-v_up, rel=1e-12, abs=1e-15)
                # and the columns: <ab||c d> of the two spin columns of a pair
                v_c1 = p.v(cc, dd, up[0], up[1])
                v_c2 = p.v(cc, dd, dn[0], dn[1])
                assert v_c2 == pytest.approx(-v_c1, rel=1e-12, abs=1e-15)
                checked += 1
    assert checked > 20


@pytest.mark.parametrize("N,n2", [(14, 4), (66, 20), (66, 36)])
def test_pair_count_is_half_the_rows(N, n2):
    """Every pair of a periodic closed shell has two spin rows: a pair {p, p}
    would need K = 2p with p a particle, but |K| <= 2 k_F."""
    c = ccd.Context([ccd.problem(N, n2, 0.16)])
    st = c.export_map(ccd.CCD_MAP_STATES).reshape(-1, 4)
    total_rows = total_pairs = 0
    flops = 0.0
    for ch, rows in _blocks(c):
        pairs = _pairs(st, rows)
        assert all(len(s) == 2 for s in pairs.values())
        total_rows += len(rows)
        total_pairs += len(pairs)
        flops += 2.0 * len(pairs) ** 2 * ch[4]
    assert total_rows == 2 * total_pairs
    assert c.info()["flops_pp"] == pytest.approx(flops)
