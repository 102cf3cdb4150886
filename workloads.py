"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws data: it holds none of the moment or cumulant
arithmetic.  Every generator is deterministic in its seed (numpy PCG64) and
returns FP64 arrays of shape (t, n), rows = samples, columns = variables (the
data matrix of Section 1.3).

The paper times its method on unnamed "illustrative data" with n = 60,
t = 2e5 and orders 4 and 5 and says t ~ 1e5 is typical for d = 4; the five
workloads below stand in for that data with heavy-tailed, skewed, correlated
and volatility-clustered columns of the stated shapes.
"""
from __future__ import annotations

import math

import numpy as np

# (name, n, b, d_max, t, device precision)
WORKLOADS = {
    "t-wishart-n16-t5000": dict(n=16, b=2, d_max=4, t=5_000, prec="f64", seed=1701001),
    "t-gamma-mix-n48-t100000": dict(n=48, b=4, d_max=4, t=100_000, prec="f32", seed=1701002),
    "laplace-mix-n24-t200000": dict(n=24, b=3, d_max=6, t=200_000, prec="bf16x2", seed=1701003),
    "batch512-t-corr-n32": dict(n=32, b=4, d_max=4, t=None, prec="f32", seed=1701004, n_sets=512),
    "ar1-garch-n64-t50000": dict(n=64, b=4, d_max=5, t=50_000, prec="f32", seed=1701005),
}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _wishart_chol(rng, n, dof):
    G = rng.standard_normal((n, dof))
    return np.linalg.cholesky(G @ G.T)


def t_wishart(t=5_000, n=16, nu=6.0, seed=1701001):
    """Student-t(nu) latent times the Cholesky factor of a Wishart(I, n+4) draw."""
    rng = _rng(seed)
    L = _wishart_chol(rng, n, n + 4)
    Z = rng.standard_t(nu, size=(t, n))
    return Z @ L.T


def t_gamma_mix(t=100_000, n=48, seed=1701002):
    """Half the columns Student-t(5), half Gamma(2,1)-2 (skewed, zero mean),
    mixed by a Haar-random orthogonal matrix."""
    rng = _rng(seed)
    h = n // 2
    S = np.empty((t, n))
    S[:, :h] = rng.standard_t(5.0, size=(t, h))
    S[:, h:] = rng.gamma(2.0, 1.0, size=(t, n - h)) - 2.0
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    return S @ Q.T


def laplace_mix(t=200_000, n=24, seed=1701003):
    """i.i.d. Laplace(0,1) latent times a dense N(0, 1/n) mixing matrix."""
    rng = _rng(seed)
    A = rng.normal(0.0, 1.0 / math.sqrt(n), size=(n, n))
    Z = rng.laplace(0.0, 1.0, size=(t, n))
    return Z @ A.T


def batch_t_corr(n_sets=512, n=32, t_lo=500, t_hi=20_000, seed=1701004):
    """n_sets datasets: t_i log-uniform in [t_lo, t_hi], Student-t(nu_i) latent
    with nu_i in {4, 6, 10}, correlated by a random correlation matrix (a
    Wishart(I, n+4) draw scaled to unit diagonal)."""
    rng = _rng(seed)
    out = []
    for _ in range(n_sets):
        ti = int(round(math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))))
        nu = float(rng.choice([4.0, 6.0, 10.0]))
        G = rng.standard_normal((n, n + 4))
        W = G @ G.T
        dinv = 1.0 / np.sqrt(np.diag(W))
        R = W * dinv[:, None] * dinv[None, :]
        L = np.linalg.cholesky(R)
        Z = rng.standard_t(nu, size=(ti, n))
        out.append(Z @ L.T)
    return out


def ar1_garch(t=50_000, n=64, rho=0.6, omega=0.05, alpha=0.1, beta=0.85, burn=1_000, seed=1701005):
    """Gaussian innovations with AR(1) correlation across variables
    (Sigma_ij = rho^|i-j|) and per-column GARCH(1,1) volatility along samples."""
    rng = _rng(seed)
    idx = np.arange(n)
    Sigma = rho ** np.abs(idx[:, None] - idx[None, :])
    L = np.linalg.cholesky(Sigma)
    E = rng.standard_normal((t + burn, n)) @ L.T
    X = np.empty((t + burn, n))
    h = np.ones(n)
    xprev = np.zeros(n)
    for l in range(t + burn):
        h = omega + alpha * xprev * xprev + beta * h
        xprev = np.sqrt(h) * E[l]
        X[l] = xprev
    return X[burn:]


def generate(name, t=None):
    """The named workload (a list of arrays for the batched one).  ``t``
    overrides the sample count for a smaller draw of the same recipe."""
    w = WORKLOADS[name]
    if name.startswith("t-wishart"):
        return t_wishart(t=t or w["t"], n=w["n"], seed=w["seed"])
    if name.startswith("t-gamma"):
        return t_gamma_mix(t=t or w["t"], n=w["n"], seed=w["seed"])
    if name.startswith("laplace"):
        return laplace_mix(t=t or w["t"], n=w["n"], seed=w["seed"])
    if name.startswith("batch"):
        return batch_t_corr(n_sets=w["n_sets"], n=w["n"], seed=w["seed"])
    if name.startswith("ar1"):
        return ar1_garch(t=t or w["t"], n=w["n"], seed=w["seed"])
    raise KeyError(name)


def dyadic_integers(t=64, n=4, lo=-3, hi=3, seed=0, skew=True):
    """Small integer data whose columns sum to exactly zero (so the mean is 0
    and every product and sum is exact in FP64, FP32 and the BF16 splits).
    With ``skew`` the entries lean positive before balancing, so odd-order
    cumulants are non-zero."""
    rng = _rng(seed)
    if skew:
        vals = np.arange(lo, hi + 1)
        w = np.exp(0.35 * vals)
        X = rng.choice(vals, size=(t, n), p=w / w.sum()).astype(np.int64)
    else:
        X = rng.integers(lo, hi + 1, size=(t, n))
    for i in range(n):
        s = int(X[:, i].sum())
        while s != 0:
            r = int(rng.integers(t))
            step = -1 if s > 0 else 1
            if lo <= X[r, i] + step <= hi:
                X[r, i] += step
                s += step
    return X.astype(np.float64)


def bernoulli_column(t, k, seed=0):
    """A 0/1 column with exactly k ones among t samples, in random order."""
    rng = _rng(seed)
    x = np.zeros(t)
    x[:k] = 1.0
    rng.shuffle(x)
    return x[:, None]
