"""Batched cumulants (many datasets, uneven sample counts, one graph) against
the CPU oracle, graph-replay determinism and the per-dataset timestamps."""
import sys

import numpy as np
import pytest

import workloads
from errmeasure import bound, e_d

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


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2", "bf16x3", "f16x2"])
def test_batch_matches_oracle_and_replays(dev, orc, prec):
    torch, pc = dev
    n, b, dmax = 13, 4, 5
    rng = np.random.default_rng(3)
    ts = [int(x) for x in rng.integers(1, 3000, size=23)] + [1, 64, 65]
    say(f"batch prec={prec} sets={len(ts)} n={n} b={b}")
    Xs = [workloads.t_gamma_mix(t=t, n=n, seed=100 + i) for i, t in enumerate(ts)]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    batch = pc.Batch(ts, n, dmax, b, prec)
    means, K = batch.run(Xd)
    torch.cuda.synchronize()
    got = [{d: K[s][d].cpu().numpy() for d in K[s]} for s in range(len(ts))]
    for s, X in enumerate(Xs):
        om, OK = orc.cumulants_dense(X, dmax)
        assert np.abs(means[s].cpu().numpy() - om).max() <= 1e-14 * max(1.0, np.abs(X).max())
        for d in range(2, dmax + 1):
            want = orc.fold(OK[d], b)
            if ts[s] == 1:
                assert not np.any(got[s][d])
                continue
            e = rel(got[s][d], want)
            assert e <= TOL[prec], (s, ts[s], d, e)
    # replay with fresh output buffers: same bits
    means2, K2 = batch.run(Xd)
    torch.cuda.synchronize()
    for s in range(len(ts)):
        for d in range(2, dmax + 1):
            assert np.array_equal(K2[s][d].cpu().numpy(), got[s][d]), (s, d)
    start, ticks, hz = batch.timestamps()
    assert hz > 0 and all(tk >= start for tk in ticks)
    batch.close()


def test_batch_integer_exact_and_autotune(dev, orc):
    torch, pc = dev
    n, b, dmax = 6, 4, 6
    ts = [64, 128, 256, 32, 512]
    Xs = [workloads.dyadic_integers(t=t, n=n, seed=t, lo=-2, hi=2) for t in ts]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    for prec in ["f64", "f32", "bf16x2", "bf16x3", "f16x2"]:
        say(f"batch integer prec={prec}")
        batch = pc.Batch(ts, n, dmax, b, prec)
        best = batch.autotune(Xd)
        assert best["ms"] > 0
        _, K = batch.run(Xd)
        torch.cuda.synchronize()
        for s, X in enumerate(Xs):
            _, OK = orc.cumulants_dense(X, dmax)
            for d in range(2, dmax + 1):
                assert np.array_equal(K[s][d].cpu().numpy(), orc.fold(OK[d], b)), (prec, s, d)
        batch.close()


def test_batch_workload_sampled(dev, orc):
    """The 512-dataset workload (n = 32, b = 4, d <= 4, t_i log-uniform in
    [500, 20000]) at its full size, FP32 path, in the autotuned configuration
    the benchmark times; sampled datasets checked."""
    torch, pc = dev
    w = workloads.WORKLOADS["batch512-t-corr-n32"]
    Xs = workloads.generate("batch512-t-corr-n32")
    ts = [len(X) for X in Xs]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    batch = pc.Batch(ts, w["n"], w["d_max"], w["b"], "f32")
    say(f"batch512 autotuned: {batch.autotune(Xd)}")
    _, K = batch.run(Xd)
    torch.cuda.synchronize()
    for s in [0, 7, 100, 255, 511]:
        say(f"batch512 dataset {s} t={ts[s]}")
        _, OK = orc.cumulants_dense(Xs[s], 4) if ts[s] <= 3000 else (None, None)
        if OK is not None:
            for d in range(2, 5):
                assert rel(K[s][d].cpu().numpy(), orc.fold(OK[d], 4)) <= TOL["f32"]
        else:
            _, Xc = orc.center(Xs[s])
            rng = np.random.default_rng(s)
            for d in range(2, 5):
                elems = pc.layout(32, d, 4)["elems"]
                offs = rng.choice(elems, size=150, replace=False)
                diag = [pc.stored_offset(32, d, 4, [i] * d) for i in range(32)]
                offs = np.unique(np.concatenate([offs, diag]))
                idx = orc.block_indices(32, d, 4, offs)
                want = orc.cumulant_at(Xc, idx)
                assert rel(K[s][d].cpu().numpy()[offs], want) <= TOL["f32"]
    batch.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_high_order_integer_exact(dev, orc, prec):
    """Orders to 9 in a batch (orders 7 and above by the first-position
    formula over each dataset's lower central moments), bit-exact on
    small-integer data."""
    torch, pc = dev
    n, b, dmax = 3, 2, 9
    ts = [64, 32, 128, 16]
    say(f"batch high-order integer prec={prec} n={n} b={b} d_max={dmax}")
    Xs = [workloads.dyadic_integers(t=t, n=n, seed=40 + t, lo=-1, hi=1) for t in ts]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    batch = pc.Batch(ts, n, dmax, b, prec)
    _, K = batch.run(Xd)
    torch.cuda.synchronize()
    for s, X in enumerate(Xs):
        _, OK = orc.cumulants_dense(X, dmax)
        for d in range(2, dmax + 1):
            got = K[s][d].cpu().numpy()
            want = orc.fold(OK[d], b)
            assert np.array_equal(got, want), (s, d, np.abs(got - want).max())
    batch.close()


def test_batch_high_order_float(dev, orc):
    """Orders to 8 over ragged blocks (b = 3 does not divide n = 4) on
    floating-point data, FP64 path."""
    torch, pc = dev
    n, b, dmax = 4, 3, 8
    ts = [700, 1500, 65, 2000]
    say(f"batch high-order float n={n} b={b} d_max={dmax}")
    Xs = [workloads.t_gamma_mix(t=t, n=n, seed=300 + i) for i, t in enumerate(ts)]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    batch = pc.Batch(ts, n, dmax, b, "f64")
    _, K = batch.run(Xd)
    torch.cuda.synchronize()
    for s, X in enumerate(Xs):
        _, OK = orc.cumulants_dense(X, dmax)
        for d in range(2, dmax + 1):
            e = rel(K[s][d].cpu().numpy(), orc.fold(OK[d], b))
            assert e <= 1e-10, (s, d, e)
    batch.close()


@pytest.mark.parametrize("groups", [3, 8])
def test_batch_groups_bitwise_and_oracle(dev, orc, groups, monkeypatch):
    """Datasets finalised in groups (each group's chunk sum and finalisation
    on a side stream beside the next group's contraction) give bitwise the
    results of one group, which match the oracle; replays keep the bits and
    every dataset gets its finalisation stamp."""
    torch, pc = dev
    n, b, dmax = 7, 3, 5
    rng = np.random.default_rng(groups)
    ts = [int(x) for x in rng.integers(1, 2500, size=19)] + [1, 64]
    say(f"batch groups={groups} sets={len(ts)} n={n} b={b} d_max={dmax}")
    Xs = [workloads.t_gamma_mix(t=t, n=n, seed=700 + i) for i, t in enumerate(ts)]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    monkeypatch.setenv("CUM_BATCH_GROUPS", "1")
    one = pc.Batch(ts, n, dmax, b, "f32")
    _, K1 = one.run(Xd)
    monkeypatch.setenv("CUM_BATCH_GROUPS", str(groups))
    grp = pc.Batch(ts, n, dmax, b, "f32")
    for rep in range(2):
        _, K = grp.run(Xd)
        torch.cuda.synchronize()
        for s in range(len(ts)):
            for d in range(2, dmax + 1):
                assert torch.equal(K[s][d], K1[s][d]), (rep, s, d)
    start, ticks, hz = grp.timestamps()
    assert hz > 0 and all(tk > start for tk in ticks)
    for s, X in enumerate(Xs):
        if ts[s] < 2:
            continue
        om, OK = orc.cumulants_dense(X, dmax)
        for d in range(2, dmax + 1):
            e = e_d(K[s][d].cpu().numpy(), orc.fold(OK[d], b), d, X - om)
            assert e <= bound(1e-6, "f32", ts[s], orc, X - om, OK[d], d), (s, ts[s], d, e)
    one.close()
    grp.close()
