"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the FP64 C oracle.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this module.  It never imports the HIP package.

``build()`` compiles ``abacus_oracle.c`` with ``-O2 -ffp-contract=off`` (one IEEE
rounding per written operation) into ``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abacus_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library; returns its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                        "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    vp = ctypes.c_void_p
    lib.oracle_bin.argtypes = [i64, vp, dbl, i32, vp, vp, vp, vp]
    lib.oracle_forces.argtypes = [i64, vp, dbl, i32, i32, dbl, i32, i64, vp, vp, vp]
    lib.oracle_vjp.argtypes = [i64, vp, vp, dbl, i32, i32, dbl, i32, i64, vp, vp]
    lib.oracle_force_abs.argtypes = [i64, vp, dbl, i32, i32, dbl, i32, i64, vp, vp, vp]
    lib.oracle_fd.argtypes = [i64, vp, vp, dbl, i32, i32, dbl, i32, i64, i32, dbl, vp]
    lib.oracle_density.argtypes = [i64, vp, dbl, i32, i32, dbl, i64, vp, vp]
    lib.oracle_multipoles.argtypes = [i64, vp, dbl, i32, i32, i32, vp]
    lib.oracle_multipole_terms.argtypes = [i32, i32]
    lib.oracle_multipole_terms.restype = i64
    lib.oracle_kick_drift.argtypes = [i64, vp, vp, vp, dbl, i32, dbl, dbl, vp, vp, vp, vp]
    lib.oracle_timestep.argtypes = [vp, dbl, dbl, dbl, dbl]
    lib.oracle_timestep.restype = dbl
    for f in ("oracle_bin", "oracle_forces", "oracle_force_abs", "oracle_vjp", "oracle_fd", "oracle_density",
              "oracle_multipoles", "oracle_kick_drift"):
        getattr(lib, f).restype = ctypes.c_int
    lib.oracle_spline_over_plummer.restype = dbl
    lib.oracle_spline_over_plummer.argtypes = []
    lib.oracle_pair_f.restype = dbl
    lib.oracle_pair_f.argtypes = [dbl, dbl]
    lib.oracle_pair_h.restype = dbl
    lib.oracle_pair_h.argtypes = [dbl, dbl]
    lib.oracle_plummer_f.restype = dbl
    lib.oracle_plummer_f.argtypes = [dbl, dbl]
    lib.oracle_plummer_h.restype = dbl
    lib.oracle_plummer_h.argtypes = [dbl, dbl]
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _pos(pos) -> np.ndarray:
    p = np.ascontiguousarray(pos, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("positions must be n x 3")
    return p


# Force laws: Eq. 3 spline with eps_s = 2.16 eps_p, or Eq. 2 Plummer with eps_p.
LAWS = {"spline": 0, "plummer": 1}


def _law(law: str) -> int:
    if law not in LAWS:
        raise ValueError(f"unknown force law {law!r}")
    return LAWS[law]


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def spline_over_plummer() -> float:
    return _load().oracle_spline_over_plummer()


def pair_f(r: float, eps_s: float) -> float:
    """f(r) of Eq. 3 (F = f(r) d)."""
    return _load().oracle_pair_f(float(r), float(eps_s))


def pair_h(r: float, eps_s: float) -> float:
    """h(r) = f'(r)/r of Eq. 3."""
    return _load().oracle_pair_h(float(r), float(eps_s))


def plummer_f(r: float, eps_p: float) -> float:
    """f(r) of Eq. 2 (F = f(r) d)."""
    return _load().oracle_plummer_f(float(r), float(eps_p))


def plummer_h(r: float, eps_p: float) -> float:
    """h(r) = f'(r)/r of Eq. 2."""
    return _load().oracle_plummer_h(float(r), float(eps_p))


def bin(pos, box: float, cpd: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Returns (cell[n], offsets[K^3+1], perm[n], rel[n,4]) as the oracle defines them."""
    p = _pos(pos)
    n = p.shape[0]
    cell = np.empty(n, np.int32)
    offs = np.empty(cpd ** 3 + 1, np.int32)
    perm = np.empty(n, np.int32)
    rel = np.empty((n, 4), np.float32)
    _check(_load().oracle_bin(n, _ptr(p), float(box), int(cpd), _ptr(cell), _ptr(offs),
                              _ptr(perm), _ptr(rel)), "oracle_bin")
    return cell, offs, perm, rel


def forces(pos, box: float, cpd: int, radius: int, eps_plummer: float,
           sinks: Optional[np.ndarray] = None, law: str = "spline") -> Tuple[np.ndarray, int]:
    """FP64 near-field accelerations (box units) of ``sinks`` (all if None) and the
    number of ordered pairs summed."""
    p = _pos(pos)
    n = p.shape[0]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.shape[0]
    acc = np.zeros((ns, 3), np.float64)
    npairs = ctypes.c_int64(0)
    _check(_load().oracle_forces(n, _ptr(p), float(box), int(cpd), int(radius), float(eps_plummer),
                                 _law(law), ns, _ptr(s), _ptr(acc), ctypes.byref(npairs)),
           "oracle_forces")
    return acc, int(npairs.value)


def force_abs(pos, box: float, cpd: int, radius: int, eps_plummer: float,
              sinks: Optional[np.ndarray] = None,
              law: str = "spline") -> Tuple[np.ndarray, np.ndarray]:
    """Per sink: sum_j |f(r_ij) d_ij,a| per component (box units) and the number
    of near-field sources summed -- the scale that bounds the rounding of any
    summation order of the sink's acceleration."""
    p = _pos(pos)
    n = p.shape[0]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.shape[0]
    out = np.zeros((ns, 3), np.float64)
    cnt = np.zeros(ns, np.int64)
    _check(_load().oracle_force_abs(n, _ptr(p), float(box), int(cpd), int(radius),
                                    float(eps_plummer), _law(law), ns, _ptr(s), _ptr(out),
                                    _ptr(cnt)), "oracle_force_abs")
    return out, cnt


def vjp(pos, w, box: float, cpd: int, radius: int, eps_plummer: float,
        sinks: Optional[np.ndarray] = None, law: str = "spline") -> np.ndarray:
    """FP64 gradient of sum_i w_i . a_i with respect to the positions of ``sinks``."""
    p = _pos(pos)
    wv = np.ascontiguousarray(w, dtype=np.float32)
    n = p.shape[0]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.shape[0]
    g = np.zeros((ns, 3), np.float64)
    _check(_load().oracle_vjp(n, _ptr(p), _ptr(wv), float(box), int(cpd), int(radius),
                              float(eps_plummer), _law(law), ns, _ptr(s), _ptr(g)), "oracle_vjp")
    return g


def fd(pos, w, box: float, cpd: int, radius: int, eps_plummer: float, k: int, axis: int,
       h: float, law: str = "spline") -> float:
    """Central difference D(h) of sum_i w_i . a_i along x_{k,axis}, binning frozen."""
    p = _pos(pos)
    wv = np.ascontiguousarray(w, dtype=np.float32)
    out = ctypes.c_double(0.0)
    _check(_load().oracle_fd(p.shape[0], _ptr(p), _ptr(wv), float(box), int(cpd), int(radius),
                             float(eps_plummer), _law(law), int(k), int(axis), float(h),
                             ctypes.byref(out)),
           "oracle_fd")
    return float(out.value)


def density(pos, box: float, cpd: int, radius: int, b: float,
            sinks: Optional[np.ndarray] = None) -> np.ndarray:
    """Apodized top-hat density sum_{r<b} (1 - r^2/b^2), self included (Sec. 3.4.4)."""
    p = _pos(pos)
    n = p.shape[0]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.shape[0]
    rho = np.zeros(ns, np.float64)
    _check(_load().oracle_density(n, _ptr(p), float(box), int(cpd), int(radius), float(b), ns,
                                  _ptr(s), _ptr(rho)), "oracle_density")
    return rho


def multipole_terms(order: int, reduced: bool = False) -> int:
    return int(_load().oracle_multipole_terms(int(order), 1 if reduced else 0))


def multipoles(pos, box: float, cpd: int, order: int, reduced: bool = False) -> np.ndarray:
    """Cell multipoles of Eq. 4 (K^3 x terms FP64, box units, about cell centres):
    the complete basis of order p, or its (p+1)^2 reduction."""
    p = _pos(pos)
    out = np.zeros((cpd ** 3, multipole_terms(order, reduced)), np.float64)
    _check(_load().oracle_multipoles(p.shape[0], _ptr(p), float(box), int(cpd), int(order),
                                     1 if reduced else 0, _ptr(out)), "oracle_multipoles")
    return out


def kick_drift(pos, vel, acc, box: float, cpd: int, kick: float, drift: float):
    """One kick and drift with the Eq. 1 statistics: returns (pos', vel',
    cell_stats (K^3 x 2: v_rms, a_max), box_stats (min_c v_rms/a_max, v_rms, a_max, N))."""
    p = _pos(pos)
    v = np.ascontiguousarray(vel, dtype=np.float32)
    a = np.ascontiguousarray(acc, dtype=np.float32)
    if v.shape != p.shape or a.shape != p.shape:
        raise ValueError("pos, vel and acc must all be n x 3")
    po = np.empty_like(p)
    vo = np.empty_like(v)
    cs = np.zeros((cpd ** 3, 2), np.float64)
    bs = np.zeros(4, np.float64)
    _check(_load().oracle_kick_drift(p.shape[0], _ptr(p), _ptr(v), _ptr(a), float(box), int(cpd),
                                     float(kick), float(drift), _ptr(po), _ptr(vo), _ptr(cs),
                                     _ptr(bs)), "oracle_kick_drift")
    return po, vo, cs, bs


def timestep(box_stats, a: float, H: float, eta_acc: float, eta_H: float) -> float:
    """Eq. 1 from the statistics of kick_drift."""
    bs = np.ascontiguousarray(box_stats, dtype=np.float64)
    return float(_load().oracle_timestep(_ptr(bs), float(a), float(H), float(eta_acc),
                                         float(eta_H)))


def fd_richardson(pos, w, box, cpd, radius, eps_plummer, k, axis, h, law="spline") -> float:
    """Richardson-extrapolated central difference (4 D(h/2) - D(h)) / 3."""
    d1 = fd(pos, w, box, cpd, radius, eps_plummer, k, axis, h, law)
    d2 = fd(pos, w, box, cpd, radius, eps_plummer, k, axis, h / 2, law)
    return (4.0 * d2 - d1) / 3.0
