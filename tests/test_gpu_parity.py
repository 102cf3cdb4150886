"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (normwise, e_d = max|gpu - oracle| / max|oracle| over the compared
entries of order d):
  * FP64 path: 1e-10, and bit-exact on small-integer data whose sums are exact;
  * FP32 and BF16x3 paths: 1e-6, and bit-exact on small-integer data (every
    product and partial sum is exactly representable there);
  * BF16x2 path: 5e-5 (each Khatri-Rao operand is carried as two BF16 terms,
    16 significant bits: a relative residual of up to 2^-18 per operand, which
    near-cancelling entries such as the third cumulant of nearly symmetric
    data amplify), and bit-exact on small-integer data;
  * FP16x2 path (FP16 hi and 2^11-scaled lo, 22 bits per operand, after a
    per-variable power-of-two scaling): 1e-6, and bit-exact on small-integer
    data.  Orders up to 6 (from order 7 on the calls that centre their own
    data stage in FP64, and moment_blocks refuses it).
"""
import sys

import numpy as np
import pytest

import workloads
from errmeasure import bound

pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "bf16x2", "bf16x3"]
CPRECS = PRECS + ["f16x2"]  # precisions of cum_cumulants
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


def run_gpu(dev, X, d_max, b, prec):
    torch, pc = dev
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    mean, K = pc.cumulants(Xd, d_max, b, prec)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), {d: K[d].cpu().numpy() for d in K}


def stored_sample(orc, n, d, b, count, seed):
    """Random stored offsets plus every pure-diagonal entry, padding dropped."""
    import paper_1701_05420_amd as pc

    elems = pc.layout(n, d, b)["elems"]
    rng = np.random.default_rng(seed)
    offs = rng.choice(elems, size=min(count, elems), replace=False)
    diag = [pc.stored_offset(n, d, b, [i] * d) for i in range(n)]
    offs = np.unique(np.concatenate([offs, diag]))
    idx = orc.block_indices(n, d, b, offs)
    keep = idx[:, 0] >= 0
    return offs[keep], idx[keep]


# ---------------------------------------------------------------- exact data
@pytest.mark.parametrize("prec", CPRECS)
@pytest.mark.parametrize("n,b,shift", [(6, 4, 0.0), (5, 2, 3.0), (9, 3, -2.0)])
def test_integer_data_bit_exact(dev, orc, prec, n, b, shift):
    say(f"integer bit-exact prec={prec} n={n} b={b} shift={shift}")
    X = workloads.dyadic_integers(t=256, n=n, seed=n + b, lo=-2, hi=2) + shift
    mean, K = run_gpu(dev, X, 6, b, prec)
    omean, OK = orc.cumulants_dense(X, 6)
    assert np.array_equal(mean, omean)
    for d in range(2, 7):
        want = orc.fold(OK[d], b)
        assert np.array_equal(K[d], want), (d, np.abs(K[d] - want).max())


@pytest.mark.parametrize("prec", CPRECS)
@pytest.mark.parametrize("n,b,dmax", [(9, 4, 5), (7, 3, 6), (10, 5, 4)])
def test_inner_block_sizes_integer_exact(dev, orc, prec, n, b, dmax):
    """Every inner block size of the contraction gives the exact cumulants."""
    torch, pc = dev
    t = 256
    X = workloads.dyadic_integers(t=t, n=n, seed=n * b, lo=-2, hi=2) + 1.0
    _, OK = orc.cumulants_dense(X, dmax)
    Xd = torch.from_numpy(X).cuda()
    for bi in range(1, b + 1):
        say(f"inner block size prec={prec} n={n} b={b} dmax={dmax} inner_b={bi}")
        pc.set_tuning(t, n, dmax, b, prec, "32x64", 1024, inner_b=bi)
        _, K = pc.cumulants(Xd, dmax, b, prec)
        for d in range(2, dmax + 1):
            want = orc.fold(OK[d], b)
            got = K[d].cpu().numpy()
            assert np.array_equal(got, want), (bi, d, np.abs(got - want).max())
    pc.set_tuning(t, n, dmax, b, prec, None)
    with pytest.raises(pc.CumulantError):
        pc.set_tuning(t, n, dmax, b, prec, "32x64", 1024, inner_b=b + 1)


@pytest.mark.parametrize("prec", CPRECS)
def test_unfold_integer_exact(dev, orc, prec):
    torch, pc = dev
    say(f"unfold prec={prec}")
    X = workloads.dyadic_integers(t=128, n=7, seed=3, lo=-2, hi=2)
    _, OK = orc.cumulants_dense(X, 5)
    Xd = torch.from_numpy(X).cuda()
    _, K = pc.cumulants(Xd, 5, 3, prec)
    for d in range(2, 6):
        dense = pc.unfold(K[d], 7, d, 3).cpu().numpy()
        assert np.array_equal(dense, OK[d]), d


# ---------------------------------------------------------------- small dense
@pytest.mark.parametrize("prec", CPRECS)
def test_t_wishart_n16_dense(dev, orc, prec):
    say(f"t-wishart n16 t5000 dense prec={prec}")
    X = workloads.generate("t-wishart-n16-t5000")
    mean, K = run_gpu(dev, X, 4, 2, prec)
    omean, OK = orc.cumulants_dense(X, 4)
    assert np.abs(mean - omean).max() <= 1e-14 * np.abs(X).max()
    for d in range(2, 5):
        e = rel(K[d], orc.fold(OK[d], 2))
        say(f"  e_{d} = {e:.3e}")
        assert e <= TOL[prec], (d, e)


@pytest.mark.parametrize("prec", CPRECS)
# (9, 8) at d = 6 and (34, 34) at d = 4 hold too many lower-order entries per
# block to stage them in LDS: the recursion reads them from memory
@pytest.mark.parametrize("n,b,t,dmax", [(7, 3, 3000, 6), (11, 4, 2000, 5), (13, 13, 1500, 4), (9, 1, 1000, 4),
                                        (9, 8, 1500, 6), (34, 34, 1000, 4)])
def test_ragged_small_dense(dev, orc, prec, n, b, t, dmax):
    say(f"ragged dense prec={prec} n={n} b={b} t={t} dmax={dmax}")
    X = workloads.t_gamma_mix(t=t, n=n, seed=n * 7 + b)
    mean, K = run_gpu(dev, X, dmax, b, prec)
    _, OK = orc.cumulants_dense(X, dmax)
    for d in range(2, dmax + 1):
        e = rel(K[d], orc.fold(OK[d], b))
        say(f"  e_{d} = {e:.3e}")
        assert e <= TOL[prec], (d, e)


@pytest.mark.parametrize("prec", CPRECS)
def test_moment_blocks_multi_tile_sampled(dev, orc, prec):
    """n = 37, b = 5: several work-group tiles per order and a ragged block."""
    torch, pc = dev
    n, b, t = 37, 5, 4000
    say(f"moment_blocks n={n} b={b} t={t} prec={prec}")
    X = workloads.laplace_mix(t=t, n=n, seed=5)
    _, Xc = orc.center(X)
    Xd = torch.from_numpy(Xc).cuda()
    if prec != "f64":
        Xd = Xd.float()
    for d in range(2, 6):
        M = pc.moment_blocks(Xd, d, b, prec).cpu().numpy()
        offs, idx = stored_sample(orc, n, d, b, 400, seed=d)
        want = np.array([np.mean(np.prod(Xc[:, ix], axis=1)) for ix in idx])
        e = rel(M[offs], want)
        say(f"  moment e_{d} = {e:.3e}")
        assert e <= TOL[prec], (d, e)
        if d == 3:
            # each distinct variable tuple is summed once: every stored copy
            # holds exactly the value of the canonical (sorted) copy
            all_offs = np.arange(M.size)
            idx = orc.block_indices(n, d, b, all_offs)
            real = idx[:, 0] >= 0
            canon = np.array([pc.stored_offset(n, d, b, list(ix)) for ix in idx[real]])
            assert np.array_equal(M[all_offs[real]], M[canon])
            assert not np.any(M[all_offs[~real]])


def test_f16x2_moment_blocks_orders(dev):
    """cum_moment_blocks contracts the data it is given in the precision asked
    for, and the FP16 split holds orders up to 6 only (CUM_EUNSUPPORTED)."""
    torch, pc = dev
    Xd = torch.from_numpy(workloads.t_gamma_mix(t=1000, n=6, seed=2)).cuda().float()
    assert pc.moment_blocks(Xd, 6, 2, "f16x2").shape[0] == pc.layout(6, 6, 2)["elems"]
    with pytest.raises(pc.CumulantError):
        pc.moment_blocks(Xd, 7, 2, "f16x2")


def test_f16x2_scaling_extremes(dev, orc):
    """The FP16 split's per-variable powers of two: columns 2^-40 .. 2^40
    apart, a far outlier, a constant column and data far from zero.  With
    every entry divided by its variables' column scales (exact powers of two),
    e_d stays within the FP32-staged bound; each variable's own cumulants (the
    pure diagonal) are within 1e-6 of the oracle relative to themselves,
    times max(1, |m_d| / |c_d|) for the cancellation in c_d; all finite."""
    torch, pc = dev
    n, b, dmax, t = 7, 3, 6, 3000
    cs = np.ldexp(1.0, np.array([-40, -13, 0, 7, 21, 40, 0]))
    X = workloads.t_gamma_mix(t=t, n=n, seed=77) * cs[None, :]
    X[123, 2] += 200.0 * np.abs(X[:, 2]).max()  # one far outlier
    X[:, 6] = 5.0                                 # a constant column
    X = X + 1e3 * cs[None, :]                     # far from zero
    say("f16x2 scaling extremes")
    _, K = run_gpu(dev, X, dmax, b, "f16x2")
    _, OK = orc.cumulants_dense(X, dmax)
    Xc = X - X.mean(axis=0)
    for d in range(2, dmax + 1):
        got, want = K[d], orc.fold(OK[d], b)
        assert np.all(np.isfinite(got)), d
        idx = orc.block_indices(n, d, b, np.arange(got.size))
        real = idx[:, 0] >= 0
        norm = np.ones(got.size)
        norm[real] = np.prod(cs[idx[real]], axis=1)
        e = rel(got / norm, want / norm)
        tol = bound(TOL["f16x2"], "f16x2", t, orc, Xc / cs[None, :], orc.fold(OK[d], b) / norm, d)
        say(f"  e_{d} (scaled) = {e:.3e} (tolerance {tol:.3e})")
        assert e <= tol, (d, e, tol)
        for i in range(n - 1):
            off = pc.stored_offset(n, d, b, [i] * d)
            m = np.mean(Xc[:, i] ** d)
            w = want[off]
            assert abs(got[off] - w) <= 1e-6 * max(abs(w), abs(m)), (i, d, got[off], w, m)


# ---------------------------------------------------------------- properties
def test_deterministic_and_shift_invariant(dev):
    X = workloads.t_gamma_mix(t=20_000, n=20, seed=1)
    for prec in CPRECS:
        say(f"determinism prec={prec}")
        _, K1 = run_gpu(dev, X, 5, 4, prec)
        _, K2 = run_gpu(dev, X, 5, 4, prec)
        for d in K1:
            assert np.array_equal(K1[d], K2[d]), (prec, d)
    _, Ka = run_gpu(dev, X, 5, 4, "f64")
    _, Kb = run_gpu(dev, X + 1000.0, 5, 4, "f64")
    for d in Ka:
        assert rel(Kb[d], Ka[d]) < 1e-7, d


def test_edge_cases(dev, orc):
    torch, pc = dev
    say("edge cases")
    # t = 1: centred data are all zero
    X = np.array([[1.5, -2.0, 3.25]])
    _, K = run_gpu(dev, X, 4, 2, "f64")
    for d in K:
        assert not np.any(K[d])
    # d_max = 2 is the biased covariance
    X = workloads.t_wishart(t=777, n=5, seed=4)
    _, K = run_gpu(dev, X, 2, 5, "f64")
    C = np.cov(X, rowvar=False, bias=True)
    assert rel(K[2], C.reshape(-1)) < 1e-12
    # one variable, one-element blocks
    x = workloads.laplace_mix(t=5000, n=1, seed=2)
    _, K = run_gpu(dev, x, 6, 1, "f64")
    _, OK = orc.cumulants_dense(x, 6)
    for d in range(2, 7):
        assert abs(K[d][0] - OK[d].reshape(-1)[0]) <= 1e-10 * abs(OK[d].reshape(-1)[0])
    # workspace too small is refused before anything runs
    Xd = torch.from_numpy(X).cuda()
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(pc.CumulantError):
        pc.cumulants(Xd, 4, 2, "f64", ws=ws)


def test_center_entry_point(dev, orc):
    torch, pc = dev
    X = workloads.ar1_garch(t=3000, n=9, seed=3) + 50.0
    for prec in ["f64", "f32"]:
        mean, Xc = pc.center(torch.from_numpy(X).cuda(), prec)
        om, oXc = orc.center(X)
        assert np.abs(mean.cpu().numpy() - om).max() <= 1e-15 * np.abs(om).max()
        got = Xc.cpu().numpy().astype(np.float64)
        want = oXc if prec == "f64" else oXc.astype(np.float32).astype(np.float64)
        tol = 1e-13 if prec == "f64" else 1.2e-7
        assert np.abs(got - want).max() <= tol * np.abs(oXc).max()


def test_autotune_and_tuned_configs(dev, orc):
    """Every tile shape / chunking the autotuner may pick gives the oracle's
    result to the path's tolerance, deterministically."""
    torch, pc = dev
    X = workloads.t_gamma_mix(t=30_000, n=24, seed=9)
    Xd = torch.from_numpy(X).cuda()
    _, Xc = orc.center(X)
    offs_idx = {d: stored_sample(orc, 24, d, 4, 200, seed=d) for d in range(2, 6)}
    want = {d: orc.cumulant_at(Xc, offs_idx[d][1]) for d in offs_idx}
    for prec in CPRECS:
        for bi in [4, 2, 1]:
            for shape in ["32x32", "32x64"]:
                for target in [256, 1024, 4096]:
                    say(f"tuned prec={prec} inner_b={bi} shape={shape} target={target}")
                    pc.set_tuning(30_000, 24, 5, 4, prec, shape, target, inner_b=bi)
                    _, K1 = pc.cumulants(Xd, 5, 4, prec)
                    _, K2 = pc.cumulants(Xd, 5, 4, prec)
                    for d in range(2, 6):
                        g = K1[d].cpu().numpy()
                        assert np.array_equal(g, K2[d].cpu().numpy())
                        e = rel(g[offs_idx[d][0]], want[d])
                        assert e <= TOL[prec], (prec, bi, shape, target, d, e)
        pc.set_tuning(30_000, 24, 5, 4, prec, None)
        best = pc.autotune(Xd, 5, 4, prec)
        say(f"autotune {prec}: {best}")
        assert best["shape"] in (0, 2) and best["ms"] > 0 and 1 <= best["inner_b"] <= 4
        pc.set_tuning(30_000, 24, 5, 4, prec, None)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16x2"])
def test_graph_capture_replays(dev, orc, prec):
    """After one call of a shape, cum_cumulants allocates nothing and issues
    only kernels, so it can be captured in a HIP graph: every replay (with
    eager work and synchronisations between replays) gives the eager bits."""
    torch, pc = dev
    n, b, dmax, t = 16, 2, 4, 5000
    X = workloads.generate("t-wishart-n16-t5000")
    Xd = torch.from_numpy(X).cuda()
    ws = torch.empty(pc.workspace_size(t, n, dmax, b, prec), dtype=torch.uint8, device="cuda")
    out = {d: torch.empty(pc.layout(n, d, b)["elems"], dtype=torch.float64, device="cuda") for d in range(2, dmax + 1)}
    mean = torch.empty(n, dtype=torch.float64, device="cuda")
    pc.cumulants(Xd, dmax, b, prec, ws=ws, out=out)  # tables for the shape exist from here on
    torch.cuda.synchronize()
    ref = {d: out[d].clone() for d in out}
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pc.cumulants(Xd, dmax, b, prec, ws=ws, out=out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        for d in out:
            out[d].fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for d in out:
            assert torch.equal(out[d], ref[d]), (rep, d)
        _, _ = pc.cumulants(Xd[: t // 2], dmax, b, prec)  # eager work in between
        torch.cuda.synchronize()
    _, OK = orc.cumulants_dense(X, dmax)
    for d in out:
        assert rel(out[d].cpu().numpy(), orc.fold(OK[d], b)) <= TOL[prec]


def test_side_stream_without_workspace(dev, orc):
    """Calls on a stream other than the current one, with no workspace or
    outputs passed in: the binding allocates them for that stream, so work
    queued meanwhile on the current stream cannot reuse them while the
    call's kernels run.  Same bits as a call on the current stream."""
    torch, pc = dev
    n, b, dmax, t = 12, 3, 4, 20_000
    X = workloads.t_gamma_mix(t=t, n=n, seed=31)
    Xd = torch.from_numpy(X).cuda()
    _, ref = pc.cumulants(Xd, dmax, b, "f32")
    mref = pc.moment_blocks(pc.center(Xd, "f32")[1], 3, b)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        _, K = pc.cumulants(Xd, dmax, b, "f32", stream=s)
        mean_c, Xc = pc.center(Xd, "f32", stream=s)
        M = pc.moment_blocks(Xc, 3, b, stream=s)
        # traffic on the current stream that would reuse freed blocks at once
        junk = [torch.full((1 << 20,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(8)]
        del junk
        torch.cuda.synchronize()
        for d in ref:
            assert torch.equal(K[d], ref[d]), (rep, d)
        assert torch.equal(M, mref), rep
    _, OK = orc.cumulants_dense(X, dmax)
    for d in ref:
        assert rel(ref[d].cpu().numpy(), orc.fold(OK[d], b)) <= TOL["f32"]
