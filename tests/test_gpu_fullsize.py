"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (autotuned), on sampled stored entries: random positions plus
every pure-diagonal entry, each computed by the oracle's per-index routine.
Also the largest supported n."""
import sys

import numpy as np
import pytest

import workloads

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


def diagonal_block_offsets(pc, n, d, b, count, rng):
    """Stored offsets in blocks with repeated block indices, where the
    redundant copies live (random positions, the canonical copy or not)."""
    L = pc.layout(n, d, b)
    be, nbar = L["block_elems"], L["nbar"]
    out = []
    while len(out) < count:
        j = np.sort(rng.integers(0, nbar, size=d))
        k = rng.integers(1, d)
        j[k] = j[k - 1]  # a repeated block index (j stays sorted)
        i = j * b + rng.integers(0, b, size=d)
        if i.max() >= n:
            continue
        i = rng.permutation(i)  # any copy: the in-block digits need not be sorted
        base = pc.stored_offset(n, d, b, sorted(i.tolist())) // be * be
        dig = [x - (x // b) * b for x in i]
        # position of this (permuted) copy inside the block of the sorted block tuple
        order = np.argsort([x // b for x in i], kind="stable")
        inb = 0
        for k in order:
            inb = inb * b + dig[k]
        out.append(base + inb)
    return np.array(out, dtype=np.int64)


def sampled_check(pc, orc, Xc, K, n, dmax, b, precs, count, seed):
    rng = np.random.default_rng(seed)
    for d in range(2, dmax + 1):
        elems = pc.layout(n, d, b)["elems"]
        offs = rng.choice(elems, size=min(count, elems), replace=False)
        diag = [pc.stored_offset(n, d, b, [i] * d) for i in range(n)]
        offs = np.unique(np.concatenate([offs, diag, diagonal_block_offsets(pc, n, d, b, count // 2, rng)]))
        idx = orc.block_indices(n, d, b, offs)
        keep = idx[:, 0] >= 0
        offs, idx = offs[keep], idx[keep]
        want = orc.cumulant_at(Xc, idx)
        den = np.abs(want).max()
        for p in precs:
            e = np.abs(K[p][d][offs] - want).max() / den
            say(f"  d={d} {p}: e = {e:.3e} over {len(offs)} entries")
            assert e <= TOL[p], (d, p, e)


@pytest.mark.parametrize("name,precs", [
    ("t-gamma-mix-n48-t100000", ["f64", "f32", "bf16x3", "bf16x2", "f16x2"]),
    ("laplace-mix-n24-t200000", ["f64", "bf16x2", "bf16x3", "f32", "f16x2"]),
    ("ar1-garch-n64-t50000", ["f64", "f32", "bf16x3", "f16x2"]),
])
def test_workload_full_size(dev, orc, name, precs):
    torch, pc = dev
    w = workloads.WORKLOADS[name]
    n, b, dmax = w["n"], w["b"], w["d_max"]
    say(f"{name}: n={n} b={b} d_max={dmax} t={w['t']}")
    X = workloads.generate(name)
    Xd = torch.from_numpy(X).cuda()
    K = {}
    for p in precs:
        tuned = pc.autotune(Xd, dmax, b, p)
        say(f"  {p}: tuned {tuned}")
        _, k1 = pc.cumulants(Xd, dmax, b, p)
        _, k2 = pc.cumulants(Xd, dmax, b, p)
        torch.cuda.synchronize()
        K[p] = {d: k1[d].cpu().numpy() for d in k1}
        for d in k1:  # deterministic at the tuned configuration
            assert torch.equal(k1[d], k2[d]), (p, d)
    _, Xc = orc.center(X)
    sampled_check(pc, orc, Xc, K, n, dmax, b, precs, count=250 if dmax >= 6 else 400, seed=17)
    for p in precs:
        pc.set_tuning(len(X), n, dmax, b, p, None)


def test_largest_n(dev, orc):
    """n = 112 variables (the largest the staged layout holds), ragged b."""
    torch, pc = dev
    n, b, dmax, t = 112, 9, 4, 3000
    X = workloads.t_gamma_mix(t=t, n=n, seed=21)
    Xd = torch.from_numpy(X).cuda()
    K = {}
    for p in ["f64", "f32", "bf16x3", "f16x2"]:
        _, k = pc.cumulants(Xd, dmax, b, p)
        K[p] = {d: k[d].cpu().numpy() for d in k}
    _, Xc = orc.center(X)
    sampled_check(pc, orc, Xc, K, n, dmax, b, ["f64", "f32", "bf16x3", "f16x2"], count=400, seed=3)
    with pytest.raises(pc.CumulantError):
        pc.cumulants(torch.zeros((10, 113), dtype=torch.float64, device="cuda"), 4, 4, "f32")
