"""Cumulants of a D3Q27 distribution via the truncated moment generating
function (oracle; test infrastructure only).

Eq. 54 defines the cumulants as derivatives at zero of the logarithm of the
(two-sided Laplace transform) moment generating function. On D3Q27 only the
moments with every exponent <= 2 are independent, so the generating function is
taken in the ring of polynomials in (X, Y, Z) truncated at degree 2 in each
variable. An element is stored as its 27 coefficients a[i, j, k] of
X^i Y^j Z^k, shape (3, 3, 3, n) for n nodes.

Moments -> generating function: coefficient = m_ijk / (i! j! k!).
Cumulants: C_ijk = i! j! k! [X^i Y^j Z^k] ln(M).  ln(1 + G) is the power
series sum_{k=1..6} (-1)^(k+1) G^k / k, exact here because G has no constant
term and every product raises the total degree by at least one, so G^7 = 0 in
the truncated ring (the maximum degree is 6). exp is the series
sum_{k=0..6} L^k / k!, exact for the same reason.
"""
import math

import torch

_FACT = torch.tensor([1.0, 1.0, 2.0], dtype=torch.float64)
# (3,3,3) table of i! j! k!
FACT3 = (_FACT[:, None, None] * _FACT[None, :, None] * _FACT[None, None, :])


def _mul_table():
    """Index triples (c, a, b) over flattened (i,j,k) -> 9 i + 3 j + k such that
    X^a X^b = X^c with every exponent <= 2 (216 of the 27 x 27 pairs)."""
    ia, ib, ic = [], [], []
    for i1 in range(3):
        for j1 in range(3):
            for k1 in range(3):
                for i2 in range(3 - i1):
                    for j2 in range(3 - j1):
                        for k2 in range(3 - k1):
                            ia.append((i1 * 3 + j1) * 3 + k1)
                            ib.append((i2 * 3 + j2) * 3 + k2)
                            ic.append(((i1 + i2) * 3 + (j1 + j2)) * 3 + (k1 + k2))
    return torch.tensor(ia), torch.tensor(ib), torch.tensor(ic)


_IA, _IB, _IC = _mul_table()


def mul(a, b):
    """Product in the truncated ring; a, b: (3,3,3,n) -> (3,3,3,n)."""
    n = a.shape[-1]
    prod = a.reshape(27, n)[_IA] * b.reshape(27, n)[_IB]
    out = torch.zeros(27, n, dtype=prod.dtype)
    out = out.index_add(0, _IC, prod)
    return out.reshape(3, 3, 3, n)


def log1p(g):
    """ln(1 + g) for g with zero constant term."""
    acc = torch.zeros_like(g)
    p = g
    for k in range(1, 7):
        acc = acc + ((-1.0) ** (k + 1) / k) * p
        if not bool(p.any()):      # every higher power is exactly zero as well
            break
        p = mul(p, g)
    return acc


def exp(l):
    """exp(l) for l with zero constant term."""
    acc = torch.zeros_like(l)
    acc[0, 0, 0] = 1.0
    p = l
    for k in range(1, 7):
        acc = acc + p / math.factorial(k)
        if not bool(p.any()):
            break
        p = mul(p, l)
    return acc


def cumulants_from_moments(m):
    """m: normalised moments m_ijk (3,3,3,n) with m_000 = 1 -> cumulants
    C_ijk (3,3,3,n), C_000 = 0 (ln 1)."""
    g = m / FACT3[..., None]
    g = g.clone()
    g[0, 0, 0] = 0.0
    return log1p(g) * FACT3[..., None]


def moments_from_cumulants(c):
    """Inverse of cumulants_from_moments: C (with C_000 ignored) -> m, m_000 = 1."""
    l = (c / FACT3[..., None]).clone()
    l[0, 0, 0] = 0.0
    return exp(l) * FACT3[..., None]
