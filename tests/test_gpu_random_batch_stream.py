"""Seeded random configurations of the batch and streaming paths against the
dense CPU oracle: variables, block size, order, precision, dataset count and
sizes (t_i = 1 included), and random add / remove sequences over a window.
Each case prints its configuration before it runs.

Errors are e_d, relative to the largest oracle entry of each order (with two
samples the odd cumulants vanish in exact arithmetic and are scaled by the
moments instead), held to the path's target; the FP32-staged paths are held to
the target times the cancellation max|M_d| / max|kappa_d|
(tests/errmeasure.py)."""
import sys

import numpy as np
import pytest

import workloads
from errmeasure import bound, e_d

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-6, "bf16x2": 5e-5, "bf16x3": 1e-6, "f16x2": 1e-6}
PRECS = ["f64", "f32", "bf16x2", "bf16x3"]


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_05420_amd as pc

    return torch, pc


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check(orc, X, mean, K, d_max, b, tol, prec, shift=None):
    """Parity of one window (a stream sums about `shift`, which these tests
    keep near the data's mean)."""
    om, OK = orc.cumulants_dense(X, d_max)
    assert np.abs(mean - om).max() <= 1e-13 * max(1.0, np.abs(X).max())
    for d in range(2, d_max + 1):
        want = orc.fold(OK[d], b)
        got = K[d]
        if len(X) == 1 and shift is None:
            assert not np.any(got), d
            continue
        e = e_d(got, want, d, X - om)
        tl = bound(tol, prec, len(X), orc, X - om, OK[d], d)
        say(f"  e_{d} = {e:.3e} (tolerance {tl:.3e})")
        assert e <= tl, (d, e, tl)


def batch_cases(count=10, seed=17010, precs=None):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.integers(1, 17))
        d_max = int(rng.integers(2, 7))
        if n ** d_max > 200_000:
            continue
        b = int(rng.integers(1, n + 1))
        sets = int(rng.integers(1, 13))
        ts = [int(x) for x in rng.choice([1, 2, 3, 63, 64, 65, 300, 1000, 2500], size=sets)]
        prec = PRECS[int(rng.integers(0, 4))] if precs is None else precs[int(rng.integers(0, len(precs)))]
        out.append((n, b, d_max, prec, ts, int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("n,b,d_max,prec,ts,seed", batch_cases() + batch_cases(count=5, seed=17016, precs=["f16x2"]))
def test_random_batch(dev, orc, n, b, d_max, prec, ts, seed):
    torch, pc = dev
    say(f"batch n={n} b={b} d_max={d_max} prec={prec} t={ts}")
    Xs = [workloads.t_gamma_mix(t=t, n=n, seed=seed + i) + 1.0 for i, t in enumerate(ts)]
    batch = pc.Batch(ts, n, d_max, b, prec)
    try:
        means, K = batch.run([torch.from_numpy(X).cuda() for X in Xs])
        torch.cuda.synchronize()
        for s, X in enumerate(Xs):
            check(orc, X, means[s].cpu().numpy(), {d: K[s][d].cpu().numpy() for d in K[s]}, d_max, b, TOL[prec], prec)
    finally:
        batch.close()


def stream_cases(count=10, seed=17011, precs=None):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.integers(1, 13))
        d_max = int(rng.integers(2, 7))
        if n ** d_max > 200_000:
            continue
        b = int(rng.integers(1, n + 1))
        method = ["recursion", "moebius"][int(rng.integers(0, 2))]
        # the general formula subtracts products of raw moments: FP64 only here
        if method == "moebius":
            prec = "f64"
        else:
            prec = PRECS[int(rng.integers(0, 4))] if precs is None else precs[int(rng.integers(0, len(precs)))]
        out.append((n, b, d_max, prec, method, int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("n,b,d_max,prec,method,seed", stream_cases() + stream_cases(count=5, seed=17017, precs=["f16x2"]))
def test_random_stream_sequence(dev, orc, n, b, d_max, prec, method, seed):
    """Twelve random adds and removes about a fixed shift near the data's
    mean; the window is checked after the sixth and the last operation."""
    torch, pc = dev
    say(f"stream n={n} b={b} d_max={d_max} prec={prec} method={method} seed={seed}")
    rng = np.random.default_rng(seed)
    shift = np.full(n, 0.5)
    st = pc.Stream(n, d_max, b, prec, shift=shift)
    window = []
    try:
        for op in range(12):
            if len(window) >= 2 and rng.random() < 0.4:
                k = int(rng.integers(0, len(window)))
                st.remove(window.pop(k)[1])
            else:
                t = int(rng.choice([1, 2, 17, 64, 500, 1500]))
                X = workloads.laplace_mix(t=t, n=n, seed=seed + op) + 0.5
                Xd = torch.from_numpy(X).cuda()
                st.add(Xd)
                window.append((X, Xd))
            if op in (5, 11):
                Xw = np.concatenate([x for x, _ in window])
                assert st.count() == len(Xw)
                mean, K = st.cumulants(method=method)
                torch.cuda.synchronize()
                check(orc, Xw, mean.cpu().numpy(), {d: K[d].cpu().numpy() for d in K}, d_max, b, TOL[prec], prec, shift)
    finally:
        st.close()
