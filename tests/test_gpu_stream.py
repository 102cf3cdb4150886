"""Streaming windows against the CPU oracle on the window's samples: batches
added (and removed) one by one must give the cumulants of their
concatenation (the moment sums are additive over disjoint sample ranges,
eq. mapred; the re-centring to the window's mean is exact algebra)."""
import sys

import numpy as np
import pytest

import workloads
from errmeasure import e_d

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-6, "bf16x2": 5e-5, "bf16x3": 1e-6, "f16x2": 1e-6}


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_05420_amd as pc

    return torch, pc


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(got, want):
    den = np.abs(want).max()
    return np.abs(got - want).max() / (den if den > 0 else 1.0)


def check_window(orc, st, Xw, dmax, b, tol, exact=False):
    mean, K = st.cumulants()
    import torch

    torch.cuda.synchronize()
    om, OK = orc.cumulants_dense(Xw, dmax)
    assert np.abs(mean.cpu().numpy() - om).max() <= 1e-13 * max(1.0, np.abs(Xw).max())
    for d in range(2, dmax + 1):
        want = orc.fold(OK[d], b)
        got = K[d].cpu().numpy()
        if exact:
            assert np.array_equal(got, want), (d, np.abs(got - want).max())
        else:
            e = rel(got, want)
            say(f"  e_{d} = {e:.3e}")
            assert e <= tol, (d, e)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2", "bf16x3", "f16x2"])
def test_stream_equals_concatenation(dev, orc, prec):
    torch, pc = dev
    n, b, dmax = 13, 4, 5
    ts = [700, 1500, 333, 2048, 1]
    Xs = [workloads.t_gamma_mix(t=t, n=n, seed=500 + i) + 2.0 for i, t in enumerate(ts)]
    st = pc.Stream(n, dmax, b, prec)
    for X in Xs:
        st.add(torch.from_numpy(X).cuda())
    assert st.count() == sum(ts)
    say(f"stream prec={prec} t={sum(ts)}")
    check_window(orc, st, np.concatenate(Xs), dmax, b, TOL[prec])
    st.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16x2"])
def test_stream_rolling_window(dev, orc, prec):
    """Add five batches, remove the first two: the cumulants of the last three."""
    torch, pc = dev
    n, b, dmax = 9, 3, 6
    ts = [1200, 800, 2500, 640, 1717]
    Xs = [workloads.laplace_mix(t=t, n=n, seed=600 + i) for i, t in enumerate(ts)]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    st = pc.Stream(n, dmax, b, prec)
    for X in Xd:
        st.add(X)
    st.remove(Xd[0])
    st.remove(Xd[1])
    assert st.count() == sum(ts[2:])
    say(f"rolling window prec={prec}")
    check_window(orc, st, np.concatenate(Xs[2:]), dmax, b, TOL[prec])
    # slide once more: add a new batch, drop the oldest
    Xn = workloads.laplace_mix(t=999, n=n, seed=700)
    st.add(torch.from_numpy(Xn).cuda())
    st.remove(Xd[2])
    check_window(orc, st, np.concatenate(Xs[3:] + [Xn]), dmax, b, TOL[prec])
    st.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2", "bf16x3", "f16x2"])
def test_stream_integer_exact(dev, orc, prec):
    """Zero-sum small-integer batches with shift 0: the window's mean is 0 and
    every sum is exact, so the cumulants are bit-exact."""
    torch, pc = dev
    n, b, dmax = 6, 4, 6
    Xs = [workloads.dyadic_integers(t=t, n=n, seed=t, lo=-2, hi=2) for t in (128, 256, 64)]
    st = pc.Stream(n, dmax, b, prec, shift=np.zeros(n))
    for X in Xs:
        st.add(torch.from_numpy(X).cuda())
    check_window(orc, st, np.concatenate(Xs), dmax, b, 0.0, exact=True)
    st.remove(torch.from_numpy(Xs[1]).cuda())
    check_window(orc, st, np.concatenate([Xs[0], Xs[2]]), dmax, b, 0.0, exact=True)
    st.close()


def test_stream_far_shift_ragged(dev, orc):
    """A shift three standard deviations away from the mean, ragged blocks."""
    torch, pc = dev
    n, b, dmax = 11, 4, 5
    X = workloads.ar1_garch(t=4000, n=n, seed=8)
    shift = X.mean(axis=0) + 3.0 * X.std(axis=0)
    st = pc.Stream(n, dmax, b, "f64", shift=shift)
    st.add(torch.from_numpy(X[:1500]).cuda())
    st.add(torch.from_numpy(X[1500:]).cuda())
    check_window(orc, st, X, dmax, b, 1e-10)
    st.close()


def test_stream_errors(dev):
    torch, pc = dev
    st = pc.Stream(5, 4, 2, "f64")
    with pytest.raises(pc.CumulantError):
        st.cumulants()  # empty window
    X = torch.from_numpy(workloads.t_wishart(t=100, n=5, seed=1)).cuda()
    with pytest.raises(pc.CumulantError):
        st.remove(X)  # nothing added
    st.add(X)
    with pytest.raises(pc.CumulantError):
        st.remove(torch.from_numpy(workloads.t_wishart(t=101, n=5, seed=2)).cuda())  # more than present
    st.reset()
    assert st.count() == 0
    with pytest.raises(pc.CumulantError):
        st.cumulants()
    st.close()


def check_moebius(orc, st, Xw, dmax, b, tol, exact=False):
    import torch

    mean, K = st.cumulants(method="moebius")
    torch.cuda.synchronize()
    om, OK = orc.cumulants_dense(Xw, dmax)
    assert np.abs(mean.cpu().numpy() - om).max() <= 1e-13 * max(1.0, np.abs(Xw).max())
    for d in range(2, dmax + 1):
        want = orc.fold(OK[d], b)
        got = K[d].cpu().numpy()
        if exact:
            assert np.array_equal(got, want), (d, np.abs(got - want).max())
        else:
            e = rel(got, want)
            say(f"  general formula e_{d} = {e:.3e}")
            assert e <= tol, (d, e)


@pytest.mark.parametrize("n,b,dmax", [(9, 3, 6), (5, 2, 8)])
def test_moebius_on_raw_moments(dev, orc, n, b, dmax):
    """The general formula (eq. cumfmom) on raw moments (shift 0) of data whose
    mean is small against its spread, against the oracle's recursion on
    centred data."""
    torch, pc = dev
    Xs = [workloads.t_gamma_mix(t=t, n=n, seed=800 + t) + 0.25 for t in (1500, 2200)]
    st = pc.Stream(n, dmax, b, "f64", shift=np.zeros(n))
    for X in Xs:
        st.add(torch.from_numpy(X).cuda())
    say(f"general formula n={n} b={b} dmax={dmax}")
    check_moebius(orc, st, np.concatenate(Xs), dmax, b, 1e-10)
    st.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2", "bf16x3", "f16x2"])
def test_moebius_integer_exact(dev, orc, prec):
    """Zero-mean small-integer data, t = 512, shift 0: every moment and every
    product of the formula is a short dyadic number, so the general formula
    and the recursion agree bit for bit."""
    torch, pc = dev
    n, b, dmax = 6, 4, 6
    Xs = [workloads.dyadic_integers(t=t, n=n, seed=900 + t, lo=-2, hi=2) for t in (256, 128, 128)]
    st = pc.Stream(n, dmax, b, prec, shift=np.zeros(n))
    for X in Xs:
        st.add(torch.from_numpy(X).cuda())
    check_moebius(orc, st, np.concatenate(Xs), dmax, b, 0.0, exact=True)
    st.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stream_high_order_window(dev, orc, prec):
    """d_max = 8: the window's cumulants of orders 7 and 8 come from the
    first-position formula over the kept central moments; against the
    oracle's dense recursion on the window's samples."""
    torch, pc = dev
    n, b, dmax = 4, 3, 8
    Xs = [workloads.laplace_mix(t=t, n=n, seed=950 + t) + 0.5 for t in (900, 700, 1100)]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    st = pc.Stream(n, dmax, b, prec)
    for X in Xd:
        st.add(X)
    st.remove(Xd[0])
    say(f"high-order window prec={prec}")
    Xw = np.concatenate(Xs[1:])
    mean, K = st.cumulants()
    torch.cuda.synchronize()
    om, OK = orc.cumulants_dense(Xw, dmax)
    assert np.abs(mean.cpu().numpy() - om).max() <= 1e-13 * max(1.0, np.abs(Xw).max())
    tol = 1e-10 if prec == "f64" else 1e-6
    for d in range(2, dmax + 1):
        want = orc.fold(OK[d], b)
        e = e_d(K[d].cpu().numpy(), want, d, Xw - om)
        say(f"  e_{d} = {e:.3e}")
        assert e <= tol, (d, e)
    st.close()
