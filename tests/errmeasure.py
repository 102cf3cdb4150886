"""The error measure every parity tolerance is stated in.

e_d = max |gpu - oracle| / max |oracle| over the compared entries of order d
(normwise, infinity norm).  One degenerate case has no such scale: with two
samples the centred data are x and -x, so every odd moment and every odd
cumulant is zero in exact arithmetic and the oracle's entries are rounding
noise.  There, and only there, the scale is s_d = max_i mean_l |x~_li|^d,
which bounds every entry of M_d (Hoelder's inequality)."""
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
