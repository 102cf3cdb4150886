"""The error measure every parity tolerance is stated in.

e_d = max |gpu - oracle| / max |oracle| over the compared entries of order d
(normwise, infinity norm).  One degenerate case has no such scale: with two
samples the centred data are x and -x, so every odd moment and every odd
cumulant is zero in exact arithmetic and the oracle's entries are rounding
noise.  There, and only there, the scale is s_d = max_i mean_l |x~_li|^d,
which bounds every entry of M_d (Hoelder's inequality).

The tolerance e_d is held to (``bound``) is the path's target (1e-10 FP64,
1e-6 FP32 and the three-term BF16 split, 5e-5 the two-term split), times
max(1, rho_d) for the FP32-staged paths, rho_d = max|M_d| / max|kappa_d|.
Those paths sum each stage of 64 samples in FP32 before carrying the sum into
FP64, so a moment carries FP32 roundings relative to the moment itself; the
cumulant inherits them amplified by the cancellation of its recursion, rho_d.
Measured: e_4 = 1.65e-6 at rho_4 = 2.47 on 63 samples (a CPU emulation of the
same FP32 sums gives 1.3e-6; rounding the data to FP32 alone 1.2e-7), and
e_5 = 1.14e-6 at rho_5 = 2.63 on 1434 samples."""
import numpy as np

def e_d(got, want, d, Xc=None):
    """Relative error of order d.  Xc: the centred samples the cumulants are
    of, needed only to recognise (and scale) the two-sample odd orders."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = float(np.abs(want).max()) if want.size else 0.0
    if Xc is not None and len(Xc) == 2 and d % 2 == 1:
        scale = float((np.abs(Xc) ** d).mean(axis=0).max())
    diff = float(np.abs(got - want).max()) if want.size else 0.0
    if scale == 0.0:
        return diff
    return diff / scale


def rho(orc, Xc, kappa_dense, d):
    """max|M_d| / max|kappa_d| over all entries (the oracle's dense moment)."""
    k = float(np.abs(kappa_dense).max())
    m = float(np.abs(orc.moment_dense(np.ascontiguousarray(Xc), d)).max())
    return m / k if k > 0 else 1.0


def bound(tol, prec, t, orc=None, Xc=None, kappa_dense=None, d=None):
    """The tolerance of e_d for a path of precision prec on t samples (see
    the module text): tol, times max(1, rho_d) for the FP32-staged paths."""
    if prec == "f64" or orc is None or t <= 2:
        # (with two samples the odd orders are scaled by s_d in e_d already)
        return tol
    return tol * max(1.0, rho(orc, Xc, kappa_dense, d))
