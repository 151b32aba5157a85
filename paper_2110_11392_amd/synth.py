"""Seeded synthetic inputs for the near-field force.

This module draws particle positions, cotangents and sample indices only.  It
holds none of the method's arithmetic (no binning, no forces) and imports
nothing from the HIP path or from the oracle, so both sides can be fed from it.

The paper's own workloads are a z=0 LCDM snapshot (Sec. 3.5.4) and a uniform
random set used for the Ewald test (Sec. 3.5.2); neither is available, so these
generators stand in for them:

* ``uniform``   -- i.i.d. uniform positions in the periodic box (the Ewald-test
  shape: random particles, tens of particles per cell).
* ``clustered`` -- half uniform background, half in isotropic Gaussian blobs of
  widths 0.2 to 2 cell widths with log-uniform weights.  This gives the very
  uneven cell occupancy of a clustered snapshot (dense halo cells next to
  near-empty voids), which is what stresses load balance and FP32 accumulation
  (Sec. 3.5.4, near-field error "islands").

Every array is produced by ``numpy.random.Generator(PCG64(seed))`` in a fixed
draw order, so a (config, seed) pair always yields the same bytes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _wrap_to_f32(x64: np.ndarray, box: float) -> np.ndarray:
    """Wrap FP64 coordinates into [0, box), round to FP32, and fold any value that
    rounded up to exactly ``box`` back to 0 so every coordinate lies in [0, box)."""
    x = np.mod(x64, box).astype(np.float32)
    x[x >= np.float32(box)] = np.float32(0.0)
    return x


def uniform(n: int, seed: int, box: float = 1.0) -> np.ndarray:
    """n x 3 FP32 positions, i.i.d. uniform in [0, box)."""
    rng = _rng(seed)
    u = rng.random((n, 3), dtype=np.float32)
    if box == 1.0:
        return np.ascontiguousarray(u)
    return np.ascontiguousarray(_wrap_to_f32(u.astype(np.float64) * box, box))


def clustered(n: int, n_blobs: int, cpd: int, seed: int, box: float = 1.0) -> np.ndarray:
    """n x 3 FP32 positions: n - n//2 uniform background particles plus n//2
    particles in ``n_blobs`` isotropic Gaussian blobs.

    Blob centres are uniform in the box; blob widths are
    sigma = w * exp(U(ln 0.2, ln 2)) with w = box / cpd the cell width; blob
    weights are exp(U(0, ln 100)) and blob particle counts are multinomial in
    those weights.  The particle order is randomly permuted so that storage order
    carries no spatial information.
    """
    rng = _rng(seed)
    w = box / cpd
    n_blob_part = n // 2
    n_bg = n - n_blob_part
    bg = rng.random((n_bg, 3)) * box
    parts = [bg]
    if n_blobs > 0 and n_blob_part > 0:
        centres = rng.random((n_blobs, 3)) * box
        sigma = w * np.exp(rng.uniform(math.log(0.2), math.log(2.0), size=n_blobs))
        weight = np.exp(rng.uniform(0.0, math.log(100.0), size=n_blobs))
        counts = rng.multinomial(n_blob_part, weight / weight.sum())
        owner = np.repeat(np.arange(n_blobs), counts)
        offs = rng.standard_normal((n_blob_part, 3)) * sigma[owner, None]
        parts.append(centres[owner] + offs)
    else:
        parts.append(rng.random((n_blob_part, 3)) * box)
    x64 = np.concatenate(parts, axis=0)
    perm = rng.permutation(n)
    return np.ascontiguousarray(_wrap_to_f32(x64[perm], box))


def gaussian_weights(n: int, seed: int) -> np.ndarray:
    """n x 3 FP32 cotangent vectors w_i ~ N(0, I)."""
    rng = _rng(seed)
    return np.ascontiguousarray(rng.standard_normal((n, 3)).astype(np.float32))


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct particle indices in [0, n), sorted ascending (int64)."""
    rng = _rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


@dataclasses.dataclass
class Box:
    """One periodic box of the workload (unit masses, G*m = 1)."""
    pos: np.ndarray        # n x 3 FP32 in [0, box)
    box: float             # side length L
    cpd: int               # cells per dimension K
    radius: int            # near-field radius R in cells
    eps_plummer: float     # Plummer-equivalent softening length

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def config(name: str, scale: Optional[int] = None) -> List[Box]:
    """The five synthetic workloads (L = 1, R = 2 everywhere).

    C1  N = 4096 uniform, K = 8.
    C2  N = 128^3 clustered with 2000 blobs, K = 32 (64 per cell on average).
    C3  N = 256^3 clustered with 20000 blobs, K = 64.
    C4  64 independent boxes, N_b log-uniform in [32^3, 128^3],
        K_b = max(7, round((N_b/64)^(1/3))), round(N_b/1024) blobs each.
    C5  N = 64^3 clustered with 256 blobs, K = 16 (the differentiation case).

    ``scale`` (C4 only) keeps the first ``scale`` boxes, for small test runs.
    """
    name = name.upper()
    if name == "C1":
        n = 4096
        return [Box(uniform(n, 1101), 1.0, 8, 2, 1.0 / 640.0)]
    if name == "C2":
        n = 128 ** 3
        return [Box(clustered(n, 2000, 32, 1102), 1.0, 32, 2, 1.0 / 5120.0)]
    if name == "C3":
        n = 256 ** 3
        return [Box(clustered(n, 20000, 64, 1103), 1.0, 64, 2, 1.0 / 10240.0)]
    if name == "C4":
        rng = _rng(1104)
        sizes = np.rint(np.exp(rng.uniform(math.log(32768.0), math.log(2097152.0),
                                           size=64))).astype(np.int64)
        boxes = []
        count = 64 if scale is None else min(scale, 64)
        for b in range(count):
            nb = int(sizes[b])
            kb = max(7, int(round((nb / 64.0) ** (1.0 / 3.0))))
            pos = clustered(nb, int(round(nb / 1024.0)), kb, 1104 * 1000 + b)
            boxes.append(Box(pos, 1.0, kb, 2, 1.0 / (40.0 * nb ** (1.0 / 3.0))))
        return boxes
    if name == "C5":
        n = 64 ** 3
        return [Box(clustered(n, 256, 16, 1105), 1.0, 16, 2, 1.0 / 2560.0)]
    raise ValueError(f"unknown workload {name!r}")


def c5_cotangent() -> np.ndarray:
    """Gaussian FP32 cotangent for C5 (seed 1105 + 1)."""
    return gaussian_weights(64 ** 3, 1106)


def c5_fd_coords(k: int = 256) -> np.ndarray:
    """k (particle, axis) pairs for the C5 finite-difference check (seed 1105 + 2)."""
    rng = _rng(1107)
    idx = rng.choice(64 ** 3, size=k, replace=False).astype(np.int64)
    axis = rng.integers(0, 3, size=k).astype(np.int64)
    return np.stack([idx, axis], axis=1)
