"""Helpers shared by the GPU parity tests (no GPU work at import time)."""
import numpy as np

import oracle

# Accuracy bar of the forward force (fractional error per particle against the
# FP64 oracle): median <= 1e-6 and 99.9th percentile <= 1e-4.
MEDIAN_TOL = 1e-6
P999_TOL = 1e-4
# Adjoint: relative 2-norm error over the compared particles <= 1e-4.
VJP_TOL = 1e-4


def frac_err(acc, ref):
    """Per-particle ||a - a_ref|| / ||a_ref||, particles with a_ref = 0 dropped."""
    acc = np.asarray(acc, np.float64)
    ref = np.asarray(ref, np.float64)
    nrm = np.linalg.norm(ref, axis=1)
    keep = nrm > 0
    return np.linalg.norm(acc[keep] - ref[keep], axis=1) / nrm[keep]


def err_stats(e):
    return {"median": float(np.median(e)), "p99": float(np.percentile(e, 99)),
            "p999": float(np.percentile(e, 99.9)), "max": float(e.max())}


def oracle_bin_boxes(boxes):
    """Oracle binning of a box list, assembled into the concatenated layout."""
    offs, perms, rels = [], [], []
    first = 0
    for b in boxes:
        _, o, p, r = oracle.bin(b.pos, b.box, b.cpd)
        offs.append(o[:-1].astype(np.int64) + first)
        perms.append(p.astype(np.int64) + first)
        rels.append(r)
        first += b.n
    offs.append(np.array([first]))
    return (np.concatenate(offs).astype(np.int32), np.concatenate(perms).astype(np.int32),
            np.concatenate(rels, axis=0))


def pair_count(boxes):
    """Exact number of ordered near-field pairs: sum_c n_c S_c - N (oracle binning)."""
    total = 0
    for b in boxes:
        _, o, _, _ = oracle.bin(b.pos, b.box, b.cpd)
        K, R = b.cpd, b.radius
        n = np.diff(o).astype(np.int64).reshape(K, K, K)
        s = np.zeros_like(n)
        for ox in range(-R, R + 1):
            for oy in range(-R, R + 1):
                for oz in range(-R, R + 1):
                    s += np.roll(n, (ox, oy, oz), axis=(0, 1, 2))
        total += int((n * s).sum()) - b.n
    return total


# Unit roundoff of FP32.
U32 = 2.0 ** -24


def single_sum_bound_violations(single, comp, ref, s_abs, count):
    """Number of (sink, component) entries where the single-accumulator result
    departs from the oracle by more than the compensated result does plus the
    rounding one FP32 running sum allows.

    Both modes add the same computed pair terms t (each an exact product folded
    in by one fused multiply-add), so
      |single - sum t| <= (n - 1) u sum|t|      (one running sum of n terms),
      |comp - sum t|   <= (63 + 5) u sum|t|     (sums of <= 64 terms, folded
                                                 with TwoSum, a few roundings),
    to first order in u = 2^-24, with n = count + 1 (the sink's own zero term).
    sum|t| is taken as twice the oracle's sum of absolute summands ``s_abs``,
    which covers the FP32 terms' own relative error.  Hence
      |single - ref| <= |comp - ref| + 2 (count + 1 + 68) u s_abs."""
    single = np.asarray(single, np.float64)
    comp = np.asarray(comp, np.float64)
    lim = np.abs(comp - ref) + 2.0 * (np.asarray(count)[:, None] + 69) * U32 * s_abs
    return int((np.abs(single - ref) > lim).sum())


def oracle_abs_boxes(boxes):
    """oracle.force_abs of every particle of a box list, concatenated (empty
    boxes contribute nothing), matching oracle_forces_boxes' order."""
    s, c = [], []
    for b in boxes:
        if b.n == 0:
            continue
        sb, cb = oracle.force_abs(b.pos, b.box, b.cpd, b.radius, b.eps_plummer)
        s.append(sb)
        c.append(cb)
    return np.concatenate(s), np.concatenate(c)
