"""The allocation-free entry point, cum_cumulants_noalloc, against
cum_cumulants through the C ABI: the same configuration gives bitwise the
same mean and cumulants, on two calls in a row, the second with fewer
samples (so the fixed scratch still holds the first call's contents)."""
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


@pytest.mark.parametrize("n,b,dmax,prec,sizes", [
    (16, 2, 5, "f32", (30_000, 9_000)),
    (13, 3, 4, "bf16x3", (20_000, 777)),
    (11, 4, 6, "f16x2", (25_000, 4_000)),
    (8, 2, 8, "f32", (12_000, 3_001)),   # d_max >= 7: staged in FP64, lower central moments in the scratch
])
def test_noalloc_matches_cumulants(dev, n, b, dmax, prec, sizes):
    torch, pc = dev
    print(f"noalloc n={n} b={b} d_max={dmax} prec={prec} t={sizes}", file=sys.stderr, flush=True)
    data = {t: torch.from_numpy(workloads.laplace_mix(t=t, n=n, seed=5000 + t)).cuda() for t in sizes}
    # the existing entry point first: its results, and the device tables of both sizes
    ref = {t: pc.cumulants(data[t], dmax, b, prec) for t in sizes}
    torch.cuda.synchronize()
    for t in sizes:
        mean = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        out = {d: torch.full((pc.layout(n, d, b)["elems"],), float("nan"), dtype=torch.float64, device="cuda")
               for d in range(2, dmax + 1)}
        pc.cumulants_noalloc(data[t], dmax, b, prec, mean, out)
        torch.cuda.synchronize()
        rmean, rK = ref[t]
        assert torch.equal(mean, rmean), t
        for d in range(2, dmax + 1):
            assert torch.equal(out[d], rK[d]), (t, d)
