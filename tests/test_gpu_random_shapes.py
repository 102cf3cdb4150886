"""Seeded random configurations against the dense CPU oracle: variables,
block size (ragged or not), order, sample count, precision and every tuned
knob (inner block size, task shape, work-item target).  Each case prints its
configuration before it runs.

The error of order d is e_d, relative to the largest oracle entry of that
order (with t = 2 the odd cumulants vanish in exact arithmetic and are
scaled by the moments instead), held to the path's target; the FP32-staged
paths are held to the target times the cancellation max|M_d| / max|kappa_d|
(tests/errmeasure.py)."""
import sys

import numpy as np
import pytest

import workloads
from errmeasure import bound, e_d

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-6, "bf16x2": 5e-5, "bf16x3": 1e-6, "f16x2": 1e-6}
PRECS = ["f64", "f32", "bf16x2", "bf16x3"]


def cases(count=30, seed=1701, precs=None):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.integers(1, 21))
        d_max = int(rng.integers(2, 7))
        if n ** d_max > 400_000:
            continue
        b = int(rng.integers(1, n + 1))
        t = int(rng.choice([1, 2, 3, 63, 64, 65, 500, 1777, 3000]))
        prec = PRECS[int(rng.integers(0, 4))] if precs is None else precs[int(rng.integers(0, len(precs)))]
        inner = int(rng.integers(1, b + 1))
        shape = ["32x32", "32x64"][int(rng.integers(0, 2))]
        target = int(rng.choice([64, 1024, 16384]))
        out.append((n, b, d_max, t, prec, inner, shape, target, int(rng.integers(1 << 30))))
    return out


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_05420_amd as pc

    return torch, pc


@pytest.mark.parametrize("n,b,d_max,t,prec,inner,shape,target,seed",
                         cases() + cases(count=12, seed=1716, precs=["f16x2"]))
def test_random_configuration(dev, orc, n, b, d_max, t, prec, inner, shape, target, seed):
    torch, pc = dev
    print(f"case n={n} b={b} d_max={d_max} t={t} prec={prec} inner_b={inner} {shape} {target}",
          file=sys.stderr, flush=True)
    X = workloads.t_gamma_mix(t=t, n=n, seed=seed) + 1.5
    pc.set_tuning(t, n, d_max, b, prec, shape, target, inner_b=inner)
    try:
        mean, K = pc.cumulants(torch.from_numpy(X).cuda(), d_max, b, prec)
        torch.cuda.synchronize()
    finally:
        pc.set_tuning(t, n, d_max, b, prec, None)
    om, OK = orc.cumulants_dense(X, d_max)
    assert np.abs(mean.cpu().numpy() - om).max() <= 1e-14 * np.abs(X).max()
    for d in range(2, d_max + 1):
        want = orc.fold(OK[d], b)
        got = K[d].cpu().numpy()
        if t == 1:
            assert not np.any(got), d
            continue
        e = e_d(got, want, d, X - om)
        tol = bound(TOL[prec], prec, t, orc, X - om, OK[d], d)
        print(f"  e_{d} = {e:.3e} (tolerance {tol:.3e})", file=sys.stderr, flush=True)
        assert e <= tol, (d, e, tol)
