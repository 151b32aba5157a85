"""TEST INFRASTRUCTURE ONLY: O(N^2) numpy brute force for tiny inputs.

An implementation of the near-field force written independently of the C
oracle, used to pin it: every ordered pair (i, j) is formed explicitly, the
displacement takes the minimum periodic image, and the pair is kept when the
periodic cell offset of j from i is within R on every axis (Sec. 3.4.1, the
(2R+1)^3 neighbouring cells).  With K >= 2R+3 every near-field separation is
below half the box, so the minimum image is the neighbouring-cell image.

The force law is Eq. 3 with eps_s = 2.16 eps_p (Sec. 3.2), evaluated with
``numpy.polynomial.polynomial.polyval``, or Eq. 2 (Plummer, eps_p as given)
written as the gradient of the potential -(r^2 + eps_p^2)^(-1/2) with
``numpy.power``.  This module pins the oracle's pair
enumeration, image choice and summation; the force law itself is pinned by the
closed-form tests (Newton's law outside eps_s, the C2 matching conditions that
define the spline, and the Plummer small-r limit of Eq. 2).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as npoly


def cells(pos: np.ndarray, box: float, cpd: int) -> np.ndarray:
    """Periodic integer cell coordinates, n x 3, via numpy floor in FP64."""
    t = pos.astype(np.float64) * (float(cpd) / float(box))
    return np.mod(np.floor(t).astype(np.int64), cpd)


def forces(pos: np.ndarray, box: float, cpd: int, radius: int, eps_plummer: float,
           sinks=None, chunk: int = 256, law: str = "spline", absolute: bool = False):
    """FP64 accelerations of ``sinks`` (all if None) and the ordered pair count.

    With ``absolute`` the first result is instead, per sink and component, the
    sum of the absolute summands sum_j |f d_ij,a| (f >= 0 for both laws), and
    the second the per-sink number of near-field sources."""
    x = pos.astype(np.float64)
    n = x.shape[0]
    c = cells(pos, box, cpd)
    eps = 2.16 * eps_plummer
    idx = np.arange(n) if sinks is None else np.asarray(sinks, dtype=np.int64)
    out = np.zeros((idx.size, 3))
    counts = np.zeros(idx.size, np.int64)
    npairs = 0
    for b in range(0, idx.size, chunk):
        ii = idx[b:b + chunk]
        d = x[None, :, :] - x[ii, None, :]
        d -= box * np.rint(d / box)                      # minimum image
        dc = c[None, :, :] - c[ii, None, :]
        dc = np.mod(dc + radius, cpd) - radius           # periodic cell offset
        near = np.all(np.abs(dc) <= radius, axis=2)
        near[np.arange(ii.size), ii] = False             # no self-force
        r = np.sqrt(np.sum(d * d, axis=2))
        u = r / eps
        with np.errstate(divide="ignore", invalid="ignore"):
            newton = 1.0 / r ** 3
        soft = npoly.polyval(u, [10.0, -15.0, 6.0]) / eps ** 3
        if law == "plummer":
            f = np.power(r * r + eps_plummer ** 2, -1.5)
        elif law == "spline":
            f = np.where(u < 1.0, soft, newton)
        else:
            raise ValueError(law)
        f = np.where(near & (r > 0), f, 0.0)
        if absolute:
            out[b:b + ii.size] = np.einsum("ij,ijk->ik", f, np.abs(d))
            counts[b:b + ii.size] = near.sum(axis=1)
        else:
            out[b:b + ii.size] = np.einsum("ij,ijk->ik", f, d)
        npairs += int(near.sum())
    return (out, counts) if absolute else (out, npairs)
