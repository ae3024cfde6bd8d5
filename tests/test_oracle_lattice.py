"""Pins of the oracle's velocity sets against the vectors printed in the paper
(Eq. 23, 31, 36; weights Eq. 24) and against exact isotropy identities."""
import itertools
import os
from fractions import Fraction

import pytest

from oracle import lattice as L

G = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    with open(os.path.join(G, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(tuple(int(x) for x in line.split()))
    return rows


def test_d3q19_matches_eq23_order():
    assert L.D3Q19.c_list == _read("velocities_eq23_d3q19.txt")


def test_d3q6_matches_eq31_order():
    assert L.D3Q6.c_list == _read("velocities_eq31_d3q6.txt")
    assert L.D3Q7.c_list[1:] == L.D3Q6.c_list and L.D3Q7.c_list[0] == (0, 0, 0)


def test_d3q27_covers_eq36_and_fills_the_missing_corner():
    printed = _read("velocities_eq36_d3q27_printed.txt")
    assert len(printed) == 26 and len(set(printed)) == 26
    ours = set(L.D3Q27.c_list)
    assert ours == set(itertools.product((-1, 0, 1), repeat=3))
    assert ours - set(printed) == {(1, -1, 1)}
    # the first 19 follow Eq. 23 / the printed order
    assert L.D3Q27.c_list[:19] == printed[:19]


def test_d3q19_weights_eq24():
    table = {r[0]: Fraction(r[1], r[2]) for r in _read("weights_eq24_d3q19.txt")}
    for c, w in zip(L.D3Q19.c_list, L.D3Q19.w_frac):
        assert w == table[sum(x * x for x in c)]


def _moment(lat, idx):
    s = Fraction(0)
    for c, w in zip(lat.c_list, lat.w_frac):
        p = Fraction(1)
        for a in idx:
            p *= c[a]
        s += w * p
    return s


@pytest.mark.parametrize("lat", [L.D3Q19, L.D3Q27], ids=lambda l: l.name)
def test_flow_lattice_isotropy_to_fourth_order(lat):
    cs2 = Fraction(1, 3)
    assert lat.cs2_frac == cs2
    d = lambda a, b: 1 if a == b else 0
    assert _moment(lat, ()) == 1
    for a in range(3):
        assert _moment(lat, (a,)) == 0
        for b in range(3):
            assert _moment(lat, (a, b)) == cs2 * d(a, b)
            for c in range(3):
                assert _moment(lat, (a, b, c)) == 0
                for e in range(3):
                    want = cs2 ** 2 * (d(a, b) * d(c, e) + d(a, c) * d(b, e) + d(a, e) * d(b, c))
                    assert _moment(lat, (a, b, c, e)) == want


def test_d3q27_weights_are_tensor_product():
    assert sorted(set(L.D3Q27.w_frac)) == [Fraction(1, 216), Fraction(1, 54), Fraction(2, 27), Fraction(8, 27)]


@pytest.mark.parametrize("lat,cs2", [(L.D3Q6, Fraction(1, 3)), (L.D3Q7, Fraction(1, 4))], ids=["Q6", "Q7"])
def test_scalar_lattices(lat, cs2):
    assert sum(lat.w_frac) == 1
    assert lat.cs2_frac == cs2
    for a in range(3):
        assert _moment(lat, (a,)) == 0
        for b in range(3):
            assert _moment(lat, (a, b)) == (cs2 if a == b else 0)


@pytest.mark.parametrize("lat", [L.D3Q19, L.D3Q27, L.D3Q6, L.D3Q7], ids=lambda l: l.name)
def test_opposites_are_pairs(lat):
    for q, c in enumerate(lat.c_list):
        o = int(lat.opp[q])
        assert lat.c_list[o] == tuple(-x for x in c)
        assert lat.w_frac[o] == lat.w_frac[q]
