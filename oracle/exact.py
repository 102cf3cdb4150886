"""Exact rational moments and cumulants for tiny integer data (TEST
INFRASTRUCTURE ONLY: only tests may import this module).

Two routes that share nothing but the data, so that agreement between them
pins both:

* ``cumulant_recursive`` -- the centred recursion of Section 3.2 (eq. cum_r):
  c_2 = m_2, c_3 = m_3 and, for d >= 4, the central moment minus the sum over
  partitions into >= 2 parts of size >= 2 of products of lower cumulants;
* ``cumulant_moebius`` -- the classical formula quoted in Section 5.3
  (eq. cumfmom) on RAW (non-centred) moments: the sum over all set partitions,
  singletons included, weighted by (|zeta|-1)! (-1)^(|zeta|-1).

Plain Python loops over ``fractions.Fraction``: for n <= 4, t <= 64, d <= 6.

``cumulant_moebius_int`` is route (b) again for integer data at orders up to
10 (B(10) = 115975 partitions): the moment sums of every subset of positions
are formed once, as Python integers, and the weighted sum is carried as the
integer t^d * cumulant, so no fraction is reduced inside the loop.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial


def set_partitions(items):
    """All set partitions of the list ``items`` (each part keeps the items'
    order).  Element k goes into one of the parts opened so far or a new one."""
    items = list(items)
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for sub in set_partitions(rest):
        # first element in a new part of its own, or prepended to an existing part
        yield [[first]] + sub
        for r in range(len(sub)):
            yield sub[:r] + [[first] + sub[r]] + sub[r + 1:]


def to_fractions(X):
    return [[Fraction(int(v)) if float(v).is_integer() else Fraction(v) for v in row] for row in X]


def mean(X):
    t = len(X)
    n = len(X[0])
    return [sum(X[l][i] for l in range(t)) / t for i in range(n)]


def centre(X):
    mu = mean(X)
    return [[x - m for x, m in zip(row, mu)] for row in X]


def moment(X, idx):
    """(1/t) sum_l prod_k x_{l, idx_k}  (Def. of the d-th moment)."""
    t = len(X)
    s = Fraction(0)
    for row in X:
        p = Fraction(1)
        for i in idx:
            p *= row[i]
        s += p
    return s / t


def cumulant_recursive(Xc, idx, _memo=None):
    """Cumulant at multi-index idx of CENTRED data by eq. cum_r."""
    idx = tuple(idx)
    d = len(idx)
    if _memo is None:
        _memo = {}
    key = tuple(sorted(idx))
    if key in _memo:
        return _memo[key]
    m = moment(Xc, idx)
    if d < 4:
        _memo[key] = m
        return m
    total = Fraction(0)
    for part in set_partitions(range(d)):
        if len(part) < 2 or any(len(p) < 2 for p in part):
            continue
        prod = Fraction(1)
        for p in part:
            prod *= cumulant_recursive(Xc, [idx[a] for a in p], _memo)
        total += prod
    val = m - total
    _memo[key] = val
    return val


def cumulant_moebius(X, idx):
    """Cumulant at multi-index idx of RAW data by eq. cumfmom (Section 5.3)."""
    idx = tuple(idx)
    total = Fraction(0)
    for part in set_partitions(range(len(idx))):
        z = len(part)
        w = factorial(z - 1) * (-1) ** (z - 1)
        prod = Fraction(1)
        for p in part:
            prod *= moment(X, [idx[a] for a in p])
        total += w * prod
    return total


def partition_masks(d):
    """Every set partition of d positions as a tuple of part bit masks.
    Position k joins one of the parts opened so far or opens a new one."""
    out = []

    def grow(k, parts):
        if k == d:
            out.append(tuple(parts))
            return
        bit = 1 << k
        for r in range(len(parts)):
            parts[r] |= bit
            grow(k + 1, parts)
            parts[r] ^= bit
        parts.append(bit)
        grow(k + 1, parts)
        parts.pop()

    grow(0, [])
    return out


def cumulant_moebius_int(X, idx, parts=None):
    """Cumulant at multi-index idx of RAW integer data by eq. cumfmom (Section
    5.3), exactly, as a Fraction.  S(B) = sum_l prod_{k in B} x_{l, idx_k}
    is an integer for every position set B, and a partition into z parts
    contributes (z-1)! (-1)^(z-1) prod_B S(B) / t^z, so t^d times the
    cumulant is the integer sum of (z-1)! (-1)^(z-1) t^(d-z) prod_B S(B).
    ``parts`` may pass partition_masks(len(idx)) in, to share it between
    calls."""
    idx = tuple(idx)
    d = len(idx)
    t = len(X)
    rows = [[int(v) for v in row] for row in X]
    if any(float(a) != b for row, r in zip(X, rows) for a, b in zip(row, r)):
        raise ValueError("integer data only")
    sums = [0] * (1 << d)
    for row in rows:
        vals = [row[i] for i in idx]
        prod = [1] * (1 << d)
        for mask in range(1, 1 << d):
            low = mask & -mask
            prod[mask] = prod[mask ^ low] * vals[low.bit_length() - 1]
            sums[mask] += prod[mask]
    if parts is None:
        parts = partition_masks(d)
    tpow = [t ** e for e in range(d + 1)]
    total = 0
    for zeta in parts:
        z = len(zeta)
        term = factorial(z - 1) * tpow[d - z]
        if z % 2 == 0:
            term = -term
        for mask in zeta:
            term *= sums[mask]
        total += term
    return Fraction(total, t ** d)
