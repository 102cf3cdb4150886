"""Orders 7..10 (the paper states its method is practical up to the tenth
order): exact on small-integer data for every path, and FP64 against the
dense oracle on floating-point data."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_05420_amd as pc

    return torch, pc


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2", "bf16x3"])
@pytest.mark.parametrize("n,b,dmax", [(3, 2, 10), (3, 1, 9), (4, 3, 8)])
def test_high_order_integer_exact(dev, orc, prec, n, b, dmax):
    torch, pc = dev
    say(f"high-order integer prec={prec} n={n} b={b} d_max={dmax}")
    X = workloads.dyadic_integers(t=64, n=n, seed=dmax + n, lo=-1, hi=1)
    _, OK = orc.cumulants_dense(X, dmax)
    _, K = pc.cumulants(torch.from_numpy(X).cuda(), dmax, b, prec)
    torch.cuda.synchronize()
    for d in range(2, dmax + 1):
        want = orc.fold(OK[d], b)
        got = K[d].cpu().numpy()
        assert np.array_equal(got, want), (d, np.abs(got - want).max())


def test_high_order_float_fp64(dev, orc):
    torch, pc = dev
    n, b, dmax, t = 4, 3, 8, 1500
    X = workloads.laplace_mix(t=t, n=n, seed=8)
    _, OK = orc.cumulants_dense(X, dmax)
    _, K = pc.cumulants(torch.from_numpy(X).cuda(), dmax, b, "f64")
    for d in range(2, dmax + 1):
        want = orc.fold(OK[d], b)
        e = np.abs(K[d].cpu().numpy() - want).max() / np.abs(want).max()
        say(f"  e_{d} = {e:.3e}")
        assert e <= 1e-10, (d, e)
