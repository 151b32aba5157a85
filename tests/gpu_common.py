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
