"""Velocity sets and weights (oracle; test infrastructure only).

D3Q19: velocities in the order printed in Eq. 23, weights Eq. 24.
D3Q27: {-1,0,1}^3 (Eq. 36). The printed Eq. 36 lists only seven of the eight
       corner vectors; (1,-1,1) is missing. All eight are used. Order: the
       D3Q19 list, then the corners as +/- pairs. The weights are not printed in
       the paper; they are the tensor product of the one-dimensional weights
       (1/6, 2/3, 1/6), i.e. 8/27, 2/27, 1/54, 1/216.
D3Q6:  Eq. 31, weight 1/6.
D3Q7:  D3Q6 plus a rest velocity (not in the paper): w0 = 1/4, w = 1/8, so the
       lattice sound speed squared of the scalar lattice is 1/4.

In every set, index 0 is the rest velocity when present and the moving
velocities come in opposite pairs, so opp(i) = i+1 for i odd (counting the rest
velocity as index 0) -- this is checked, not assumed, by ``opposite``.
"""
from fractions import Fraction

import torch

_Q19 = [
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
]
_CORNERS = [
    (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
    (1, -1, 1), (-1, 1, -1), (1, -1, -1), (-1, 1, 1),
]
_Q6 = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def _w19(c):
    n2 = sum(x * x for x in c)
    return {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}[n2]


def _w27(c):
    one_d = {0: Fraction(2, 3), 1: Fraction(1, 6), -1: Fraction(1, 6)}
    return one_d[c[0]] * one_d[c[1]] * one_d[c[2]]


class Lattice:
    """A discrete velocity set: integer velocities c (Q,3), weights w (Q,),
    opposite index opp (Q,), sound speed squared cs2 (exact rational)."""

    def __init__(self, name, vel, weights):
        self.name = name
        self.c_list = list(vel)
        self.w_frac = list(weights)
        self.Q = len(vel)
        self.c = torch.tensor(vel, dtype=torch.float64)
        self.ci = torch.tensor(vel, dtype=torch.int64)
        self.w = torch.tensor([float(x) for x in weights], dtype=torch.float64)
        self.opp = torch.tensor([self.c_list.index(tuple(-x for x in v)) for v in vel])
        cs2 = sum(wq * v[0] * v[0] for wq, v in zip(weights, vel))
        self.cs2_frac = Fraction(cs2)
        self.cs2 = float(cs2)


D3Q19 = Lattice("D3Q19", _Q19, [_w19(c) for c in _Q19])
D3Q27 = Lattice("D3Q27", _Q19 + _CORNERS, [_w27(c) for c in _Q19 + _CORNERS])
D3Q6 = Lattice("D3Q6", _Q6, [Fraction(1, 6)] * 6)
D3Q7 = Lattice("D3Q7", [(0, 0, 0)] + _Q6, [Fraction(1, 4)] + [Fraction(1, 8)] * 6)
