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
