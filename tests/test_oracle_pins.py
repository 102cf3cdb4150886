"""Pins for the CPU oracle: every check here compares the oracle with
something other than itself -- numbers the paper prints, textbook closed
forms, a second exact formula on raw moments, library routines, and
invariants the mathematics fixes.  No GPU."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parts_by_sigma(orc, d, min_part):
    P = orc.partitions(d, min_part=min_part, min_parts=1)
    out = {}
    for lab in P:
        s = int(lab.max()) + 1
        out[s] = out.get(s, 0) + 1
    return P, out


# ---------------------------------------------------------------- combinatorics
def test_partition_counts_printed(orc):
    g = json.load(open(os.path.join(GOLDEN, "partition_counts.json")))
    for key, val in g["S_prime"].items():
        d, s = map(int, key.split(","))
        _, by = _parts_by_sigma(orc, d, 2)
        assert by.get(s, 0) == val, (d, s)
    for key, val in g["N"].items():
        d = int(key)
        _, by = _parts_by_sigma(orc, d, 2)
        assert sum((s - 1) * c for s, c in by.items() if s >= 2) == val
    _, by4 = _parts_by_sigma(orc, 4, 1)
    assert by4[2] == g["S_4_2_all_parts"]


@pytest.mark.parametrize("d", range(1, 9))
def test_partitions_match_stirling_and_bell(orc, d):
    P, by = _parts_by_sigma(orc, d, 1)
    # Stirling numbers of the second kind by the explicit formula (eq. n1)
    for s in range(1, d + 1):
        S = sum((-1) ** (s - j) * math.comb(s, j) * j ** d for j in range(s + 1)) // math.factorial(s)
        assert by.get(s, 0) == S
    # each label vector is a valid restricted-growth string, all distinct
    seen = set()
    for lab in P:
        mx = -1
        for a in lab:
            assert a <= mx + 1
            mx = max(mx, a)
        seen.add(tuple(lab))
    assert len(seen) == len(P)


def test_F_recurrence_and_sigma_max(orc):
    # F(d) = number of partitions with no singleton; F(d+1) = B(d) - F(d) (eq. req)
    def F(d):
        return len(orc.partitions(d, min_part=2, min_parts=1)) if d >= 2 else 0

    def B(d):
        return len(orc.partitions(d, min_part=1, min_parts=1))

    assert [F(d) for d in range(2, 7)] == [1, 1, 4, 11, 41]
    for d in range(1, 10):
        assert F(d + 1) == B(d) - F(d)
    for d in range(2, 9):
        P = orc.partitions(d, 2, 2)
        smax = max((int(l.max()) + 1 for l in P), default=1)
        assert smax == max(1, d // 2) or (d < 4 and len(P) == 0)


def test_recursion_partitions_brute_force(orc):
    # parts >= 2, at least 2 parts: compare with a brute-force labelling of d positions
    for d in range(2, 8):
        got = {tuple(l) for l in orc.partitions(d, 2, 2)}
        want = set()
        for lab in itertools.product(range(d), repeat=d):
            # canonical (first-appearance) labels only
            ren, nxt, can = {}, 0, []
            for a in lab:
                if a not in ren:
                    ren[a] = nxt
                    nxt += 1
                can.append(ren[a])
            if tuple(can) != lab:
                continue
            sizes = [lab.count(r) for r in range(nxt)]
            if nxt >= 2 and min(sizes) >= 2:
                want.add(lab)
        assert got == want


# ---------------------------------------------------------------- exact routes
def test_exact_routes_agree():
    """Centred recursion (eq. cum_r) == Moebius sum over raw moments (eq. cumfmom)."""
    X = workloads.dyadic_integers(t=16, n=3, seed=5)
    X = X + np.array([1.0, -2.0, 3.0])  # non-zero means: the Moebius route sees raw data
    Xf = exact.to_fractions(X)
    Xc = exact.centre(Xf)
    for d in range(2, 6):
        for idx in itertools.combinations_with_replacement(range(3), d):
            assert exact.cumulant_recursive(Xc, idx) == exact.cumulant_moebius(Xf, idx), idx
    for idx in [(0, 0, 0, 0, 0, 0), (0, 1, 2, 0, 1, 2), (2, 2, 1, 1, 0, 0), (0, 0, 1, 1, 1, 2)]:
        assert exact.cumulant_recursive(Xc, idx) == exact.cumulant_moebius(Xf, idx), idx


def test_oracle_equals_exact_on_dyadic_data(orc):
    """On zero-mean small-integer data with t a power of two every FP64 step is
    exact, so the oracle must equal the rational value exactly."""
    X = workloads.dyadic_integers(t=32, n=3, seed=11)
    _, K = orc.cumulants_dense(X, 6)
    Xf = exact.to_fractions(X)
    Xc = exact.centre(Xf)
    memo = {}
    for d in range(2, 7):
        for idx in itertools.product(range(3), repeat=d):
            want = exact.cumulant_recursive(Xc, idx, memo)
            assert Fraction(float(want)) == want  # representable
            assert K[d][idx] == float(want), (d, idx)
    # and against the independent raw-moment route with a shifted copy
    Xs = X + 7.0
    _, Ks = orc.cumulants_dense(Xs, 6)
    Xsf = exact.to_fractions(Xs)
    for idx in [(0, 1, 2, 2), (1, 1, 1, 1, 1), (0, 0, 1, 1, 2, 2), (2, 0, 1, 0, 2, 1)]:
        assert Ks[len(idx)][idx] == float(exact.cumulant_moebius(Xsf, idx)), idx


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("k", [1, 5, 16, 31])
def test_bernoulli_closed_forms(orc, k):
    t = 64
    x = workloads.bernoulli_column(t, k, seed=k)
    _, K = orc.cumulants_dense(x, 6)
    p = Fraction(k, t)
    q = 1 - p
    want = {
        2: p * q,
        3: p * q * (1 - 2 * p),
        4: p * q * (1 - 6 * p * q),
        5: p * q * (1 - 2 * p) * (1 - 12 * p * q),
        6: p * q * (1 - 30 * p * q + 120 * p * p * q * q),
    }
    for d in range(2, 7):
        got = K[d].reshape(-1)[0]
        assert abs(got - float(want[d])) <= 1e-15 * max(1.0, abs(float(want[d]))), (d, got, float(want[d]))


def test_univariate_textbook(orc):
    x = workloads.laplace_mix(t=4000, n=1, seed=3)
    _, K = orc.cumulants_dense(x, 6)
    xc = x[:, 0] - x[:, 0].mean()
    m = {r: np.mean(xc ** r) for r in range(2, 7)}
    want = {
        2: m[2],
        3: m[3],
        4: m[4] - 3 * m[2] ** 2,
        5: m[5] - 10 * m[3] * m[2],
        6: m[6] - 15 * m[4] * m[2] - 10 * m[3] ** 2 + 30 * m[2] ** 3,
    }
    for d in range(2, 7):
        got = K[d].reshape(-1)[0]
        assert abs(got - want[d]) <= 1e-10 * abs(m[d] if d > 2 else m[2]) + 1e-13, d


def test_covariance_and_printed_fourth_cumulant(orc):
    X = workloads.t_wishart(t=3000, n=5, seed=2)
    mean, K = orc.cumulants_dense(X, 4)
    np.testing.assert_allclose(mean, X.mean(axis=0), rtol=1e-13, atol=1e-13)
    C = np.cov(X, rowvar=False, bias=True)
    np.testing.assert_allclose(K[2], C, rtol=1e-12, atol=1e-12 * np.abs(C).max())
    Xc = X - X.mean(axis=0)
    M3 = np.einsum("li,lj,lk->ijk", Xc, Xc, Xc) / len(X)
    np.testing.assert_allclose(K[3], M3, rtol=0, atol=1e-11 * np.abs(M3).max())
    # eq. c4: c_ijkl = m_ijkl - c_ij c_kl - c_ik c_jl - c_il c_jk
    M4 = np.einsum("li,lj,lk,lm->ijkm", Xc, Xc, Xc, Xc) / len(X)
    K4 = M4 - (np.einsum("ij,km->ijkm", C, C) + np.einsum("ik,jm->ijkm", C, C) + np.einsum("im,jk->ijkm", C, C))
    np.testing.assert_allclose(K[4], K4, rtol=0, atol=1e-10 * np.abs(M4).max())


# ---------------------------------------------------------------- structure
def test_identical_columns_and_rank_one(orc):
    x = workloads.t_gamma_mix(t=2000, n=2, seed=8)[:, :1]
    _, K1 = orc.cumulants_dense(x, 6)
    _, Kn = orc.cumulants_dense(np.repeat(x, 3, axis=1), 6)
    a = np.array([0.5, -2.0, 1.5])
    _, Kr = orc.cumulants_dense(x * a[None, :], 6)
    for d in range(2, 7):
        u = K1[d].reshape(-1)[0]
        assert np.all(np.abs(Kn[d] - u) <= 1e-12 * abs(u) + 1e-14)
        outer = a
        for _ in range(d - 1):
            outer = np.multiply.outer(outer, a)
        np.testing.assert_allclose(Kr[d], u * outer, rtol=1e-10, atol=1e-12 * abs(u) * 3 ** d)


def test_gaussian_higher_cumulants_vanish(orc):
    rng = np.random.default_rng(4)
    t = 200_000
    X = rng.standard_normal((t, 2)) @ np.array([[1.0, 0.0], [0.5, 1.0]]).T
    _, K = orc.cumulants_dense(X, 6)
    for d in range(3, 7):
        # App. A: std of a d-th moment estimate < sqrt(M_2d / t); M_2d of a unit-ish
        # Gaussian is (2d-1)!!; allow 6 standard errors
        m2d = math.prod(range(2 * d - 1, 0, -2)) * 1.25 ** d
        assert np.abs(K[d]).max() < 6 * math.sqrt(m2d / t) * 4, d


def test_laplace_even_cumulants(orc):
    rng = np.random.default_rng(9)
    X = rng.laplace(0.0, 1.0, size=(400_000, 2))
    _, K = orc.cumulants_dense(X, 6)
    # Laplace(0,1): kappa_2k = 2 (2k-1)!  -> 2, 12, 240
    assert abs(K[2][0, 0] - 2) < 0.05 and abs(K[4][0, 0, 0, 0] - 12) < 1.5
    assert abs(K[6][(0,) * 6] - 240) < 80
    assert abs(K[4][0, 0, 1, 1]) < 0.3


# ---------------------------------------------------------------- invariants
def _perm_apply(T, perm):
    return np.transpose(T, perm)


def test_full_permutation_symmetry(orc):
    X = workloads.dyadic_integers(t=64, n=3, seed=1)
    _, K = orc.cumulants_dense(X, 6)
    for d in range(2, 7):
        for perm in itertools.permutations(range(d)):
            assert np.array_equal(K[d], _perm_apply(K[d], perm)), (d, perm)
    Xf = workloads.t_wishart(t=500, n=3, seed=6)
    _, Kf = orc.cumulants_dense(Xf, 5)
    for d in range(2, 6):
        scale = np.abs(Kf[d]).max()
        for perm in itertools.permutations(range(d)):
            assert np.abs(Kf[d] - _perm_apply(Kf[d], perm)).max() <= 1e-13 * scale


def test_shift_scale_and_row_permutation(orc):
    X = workloads.dyadic_integers(t=64, n=3, seed=2)
    _, K = orc.cumulants_dense(X, 6)
    _, Ks = orc.cumulants_dense(X + np.array([3.0, -5.0, 11.0]), 6)
    _, K2 = orc.cumulants_dense(2.0 * X, 6)
    rng = np.random.default_rng(0)
    _, Kp = orc.cumulants_dense(X[rng.permutation(len(X))], 6)
    for d in range(2, 7):
        assert np.array_equal(K[d], Ks[d]), d
        assert np.array_equal(K2[d], (2.0 ** d) * K[d]), d
        assert np.array_equal(Kp[d], K[d]), d


def test_column_permutation_and_multilinearity(orc):
    X = workloads.laplace_mix(t=3000, n=4, seed=12)
    _, K = orc.cumulants_dense(X, 5)
    perm = np.array([2, 0, 3, 1])
    _, Kp = orc.cumulants_dense(X[:, perm], 5)
    A = np.random.default_rng(1).standard_normal((3, 4))
    _, KA = orc.cumulants_dense(X @ A.T, 5)
    for d in range(2, 6):
        assert np.array_equal(Kp[d], K[d][np.ix_(*([perm] * d))]), d
        T = K[d]
        for _ in range(d):  # contract every mode with A (the last mode each time)
            T = np.tensordot(T, A, axes=([d - 1], [1]))
            T = np.moveaxis(T, -1, 0)
        np.testing.assert_allclose(KA[d], T, rtol=0, atol=1e-9 * np.abs(T).max())


# ---------------------------------------------------------------- modes and storage
def test_sampled_mode_equals_dense(orc):
    X = workloads.t_gamma_mix(t=700, n=4, seed=4)
    mean, K = orc.cumulants_dense(X, 6)
    _, Xc = orc.center(X)
    rng = np.random.default_rng(2)
    for d in range(2, 7):
        idx = rng.integers(0, 4, size=(40, d))
        got = orc.cumulant_at(Xc, idx)
        want = np.array([K[d][tuple(i)] for i in idx])
        assert np.array_equal(got, want), d


def test_block_counts_and_fold(orc):
    for n, b, d in [(6, 2, 2), (5, 2, 3), (7, 3, 4), (16, 2, 4), (48, 4, 4), (24, 3, 6), (64, 4, 5)]:
        nbar = -(-n // b)
        # C(nbar+d-1, d) blocks (the printed binomial C(nbar+d-1, nbar) is a misprint)
        assert orc.block_elems(n, d, b) == b ** d * math.comb(nbar + d - 1, d)
    assert orc.block_elems(6, 2, 2) == 6 * 4
    n, b, d = 5, 2, 3
    rng = np.random.default_rng(0)
    dense = rng.standard_normal((n,) * d)
    blocks = orc.fold(dense, b)
    offs = np.arange(blocks.size)
    idx = orc.block_indices(n, d, b, offs)
    for o, ix in zip(offs, idx):
        if ix[0] < 0:
            assert blocks[o] == 0.0
        else:
            assert blocks[o] == dense[tuple(ix)]
            j = ix // b
            assert np.all(np.diff(j) >= 0)
    # every sorted multi-index appears at least once (redundant copies in diagonal blocks)
    have = {tuple(sorted(ix)) for ix in idx if ix[0] >= 0}
    assert have == set(itertools.combinations_with_replacement(range(n), d))


def test_high_orders_against_raw_moment_route(orc):
    """Orders 7 and 8 (the paper's method reaches order 10): the FP64 oracle
    on shifted small-integer data against the Moebius route on raw moments."""
    X = workloads.dyadic_integers(t=16, n=2, seed=4, lo=-1, hi=1) + np.array([2.0, -1.0])
    _, K = orc.cumulants_dense(X, 8)
    Xf = exact.to_fractions(X)
    for idx in [(0,) * 7, (0, 1, 0, 1, 1, 0, 1), (1,) * 8, (0, 0, 0, 1, 1, 1, 0, 1)]:
        want = exact.cumulant_moebius(Xf, idx)
        assert Fraction(float(want)) == want
        assert K[len(idx)][idx] == float(want), idx


@pytest.mark.parametrize("n,dmax,seed", [(3, 9, 5), (2, 10, 6)])
def test_orders_9_and_10_against_raw_moment_route(orc, n, dmax, seed):
    """Orders 8 to 10, the top of the range the paper claims (Section 1.1):
    the FP64 oracle (centred recursion, eq. cum_r) on shifted small-integer
    data equals eq. cumfmom of Section 5.3 on the raw moments, evaluated
    exactly with integers, at every sorted multi-index and at permutations
    of some.  Every value here is a short dyadic fraction, so equality is
    bit for bit."""
    X = workloads.dyadic_integers(t=16, n=n, seed=seed, lo=-2, hi=3) + np.array([2.0, -1.0, 3.0][:n])
    _, K = orc.cumulants_dense(X, dmax)
    rng = np.random.default_rng(seed)
    nonzero = 0
    for d in range(dmax - 2, dmax + 1):
        parts = exact.partition_masks(d)
        idxs = list(itertools.combinations_with_replacement(range(n), d))
        idxs += [tuple(rng.permutation(idxs[k])) for k in rng.choice(len(idxs), size=4, replace=False)]
        for idx in idxs:
            want = exact.cumulant_moebius_int(X, idx, parts)
            assert Fraction(float(want)) == want, idx
            assert K[d][idx] == float(want), (idx, K[d][idx], float(want))
            nonzero += want != 0
    assert nonzero > 20


@pytest.mark.parametrize("d", [7, 8, 9, 10])
def test_sampled_mode_equals_dense_high_orders(orc, d):
    """The per-entry route (the recursion evaluated at chosen multi-indices)
    gives the dense routine's bits at orders 7 to 10 too, on float data."""
    n = 3 if d <= 9 else 2
    X = workloads.laplace_mix(t=400, n=n, seed=40 + d)
    _, K = orc.cumulants_dense(X, d)
    _, Xc = orc.center(X)
    rng = np.random.default_rng(d)
    idx = np.concatenate([rng.integers(0, n, size=(40, d)), np.repeat(np.arange(n)[:, None], d, axis=1)])
    got = orc.cumulant_at(Xc, idx)
    want = np.array([K[d][tuple(i)] for i in idx])
    assert np.array_equal(got, want)
