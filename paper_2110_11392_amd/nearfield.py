"""PyTorch-facing API of the near-field force.

PyTorch supplies device memory and the stream; every computation is one of the
library's HIP kernels, reached through the C ABI in ``_lib``.

    spec = BoxSpec(n, box=1.0, cpd=32, radius=2, eps_plummer=1/5120)
    nf = NearField([spec])                  # resolves sizes, owns the workspace
    binned = nf.bin(pos)                    # pos: (n, 3) float32 on the GPU
    acc = nf.forces(binned)                 # (n, 3) float32, original order
    grad = nf.forces_vjp(binned, w)         # d/dpos sum(w * acc)

    acc = near_field(pos, 1.0, 32, 2, 1/5120)   # autograd.Function form
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib


@dataclasses.dataclass(frozen=True)
class BoxSpec:
    """One periodic box: n particles, side ``box``, ``cpd`` cells per dimension,
    near-field radius ``radius`` (cells), Plummer-equivalent softening and the
    optional top-hat radius of the density estimate (0: none)."""
    n: int
    box: float
    cpd: int
    radius: int
    eps_plummer: float
    density_radius: float = 0.0

    def astuple(self):
        return (self.n, self.box, self.cpd, self.radius, self.eps_plummer, self.density_radius)


ACCUMULATION = {"compensated": _lib.COMPENSATED, "chunked": _lib.CHUNKED,
                "single": _lib.SINGLE_ACC}
# Force laws: the spline of Eq. 3 (eps_s = 2.16 eps_p) or Plummer's Eq. 2.
LAWS = {"spline": 0, "plummer": _lib.PLUMMER}


@dataclasses.dataclass
class Binned:
    """Device arrays produced by ``NearField.bin`` (see include/abacus_nf.h)."""
    cell_offsets: torch.Tensor   # int32, cells_total + 1
    perm: torch.Tensor           # int32, n_total
    rel: torch.Tensor            # float32, n_total x 4
    status: torch.Tensor         # int32, 1

    def cstruct(self) -> _lib.Binned:
        return _lib.Binned(self.cell_offsets.data_ptr(), self.perm.data_ptr(),
                           self.rel.data_ptr(), self.status.data_ptr())

    def check_status(self) -> None:
        """Raise if the binning flagged bad coordinates, or a cell too full for
        the pair kernels, which then evaluate nothing (synchronises)."""
        st = int(self.status.item())
        if st & _lib.STATUS_BADPOS:
            raise ValueError("non-finite or out-of-range particle coordinate (|x K/L| >= 2^30)")
        if st & _lib.STATUS_CELLFULL:
            raise ValueError("a cell holds more than 2^28 particles: beyond the pair kernels' "
                             "offsets; use more cells per dimension")


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class NearField:
    """Resolved box list plus a reusable device workspace; ``law`` selects the
    force law of every call ("spline", Eq. 3, or "plummer", Eq. 2)."""

    def __init__(self, boxes: Sequence[BoxSpec], device=None, law: str = "spline"):
        if law not in LAWS:
            raise ValueError(f"unknown force law {law!r}")
        self.law = law
        lib = _lib.load()
        self.specs: List[BoxSpec] = list(boxes)
        self._boxes = _lib.box_array([b.astuple() for b in self.specs])
        self.nboxes = len(self.specs)
        n_total, cells_total = ctypes.c_int64(0), ctypes.c_int64(0)
        _lib.check(lib.abacus_nf_layout(self._boxes, self.nboxes, ctypes.byref(n_total),
                                        ctypes.byref(cells_total)), "abacus_nf_layout")
        nbytes = ctypes.c_size_t(0)
        _lib.check(lib.abacus_nf_workspace_bytes(self._boxes, self.nboxes, ctypes.byref(nbytes)),
                   "abacus_nf_workspace_bytes")
        self.n_total = int(n_total.value)
        self.cells_total = int(cells_total.value)
        self.workspace_bytes = int(nbytes.value)
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self._lib = lib

    # -- helpers -----------------------------------------------------------
    def _flags(self, accumulation: str) -> int:
        if accumulation not in ACCUMULATION:
            raise ValueError(f"unknown accumulation {accumulation!r}")
        return ACCUMULATION[accumulation] | LAWS[self.law]

    def _check_pos(self, pos: torch.Tensor):
        if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("positions must be an (n, 3) float32 tensor")
        if pos.shape[0] != self.n_total:
            raise ValueError(f"expected {self.n_total} particles, got {pos.shape[0]}")
        if pos.device != self.device or not pos.is_contiguous():
            raise ValueError("positions must be contiguous on the workspace's device")

    def alloc_binned(self) -> Binned:
        d = self.device
        return Binned(torch.empty(self.cells_total + 1, dtype=torch.int32, device=d),
                      torch.empty(self.n_total, dtype=torch.int32, device=d),
                      torch.empty((self.n_total, 4), dtype=torch.float32, device=d),
                      torch.empty(1, dtype=torch.int32, device=d))

    # -- entry points --------------------------------------------------------
    def bin(self, pos: torch.Tensor, out: Optional[Binned] = None, check: bool = False) -> Binned:
        self._check_pos(pos)
        out = out if out is not None else self.alloc_binned()
        cs = out.cstruct()
        _lib.check(self._lib.abacus_nf_bin(self._boxes, self.nboxes, _ptr(pos), ctypes.byref(cs),
                                           _ptr(self.workspace), self.workspace_bytes, _stream()),
                   "abacus_nf_bin")
        if check:
            out.check_status()
        return out

    def forces(self, binned: Binned, accumulation: str = "compensated",
               out: Optional[torch.Tensor] = None, momentum: bool = False,
               count_pairs: bool = False, momentum_out: Optional[torch.Tensor] = None,
               pairs_out: Optional[torch.Tensor] = None,
               density_out: Optional[torch.Tensor] = None
               ) -> Tuple[torch.Tensor, Optional[torch.Tensor], Optional[torch.Tensor]]:
        """Accelerations (n, 3) in original order; optionally the per-box FP64
        momentum sums (nboxes, 4) and the evaluated pair count (1,) int64.  With
        ``density_out`` (a contiguous (n,) float32 tensor; every box needs a
        density radius) the same pass also writes the top-hat density estimate."""
        if density_out is not None and (density_out.dtype != torch.float32
                                        or tuple(density_out.shape) != (self.n_total,)
                                        or not density_out.is_contiguous()
                                        or density_out.device != self.device):
            raise ValueError("density_out must be a contiguous (n,) float32 tensor")
        flags = self._flags(accumulation) | (_lib.COUNT_PAIRS if count_pairs else 0)
        acc = out if out is not None else torch.empty((self.n_total, 3), dtype=torch.float32,
                                                      device=self.device)
        mom = momentum_out
        if mom is None and momentum:
            mom = torch.empty((self.nboxes, 4), dtype=torch.float64, device=self.device)
        pairs = pairs_out
        if pairs is None and count_pairs:
            pairs = torch.empty(1, dtype=torch.int64, device=self.device)
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_forces(self._boxes, self.nboxes, ctypes.byref(cs), _ptr(acc),
                                              _ptr(density_out), _ptr(mom), _ptr(pairs), flags,
                                              _ptr(self.workspace), self.workspace_bytes,
                                              _stream()),
                   "abacus_nf_forces")
        return acc, mom, pairs

    def forces_f64(self, binned: Binned, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Accelerations (n, 3) in FP64, original order: the FP64 pair kernel."""
        acc = out if out is not None else torch.empty((self.n_total, 3), dtype=torch.float64,
                                                      device=self.device)
        if acc.dtype != torch.float64 or tuple(acc.shape) != (self.n_total, 3) or \
                not acc.is_contiguous():
            raise ValueError("out must be a contiguous (n, 3) float64 tensor")
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_forces_f64(self._boxes, self.nboxes, ctypes.byref(cs),
                                                  _ptr(acc), LAWS[self.law],
                                                  _ptr(self.workspace), self.workspace_bytes,
                                                  _stream()),
                   "abacus_nf_forces_f64")
        return acc

    def forces_vjp_f64(self, binned: Binned, w: torch.Tensor,
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Adjoint of forces_f64 for an FP64 cotangent w (n, 3), original order:
        the FP64 adjoint pair kernel.  Returns (n, 3) FP64."""
        if w.dtype != torch.float64 or tuple(w.shape) != (self.n_total, 3) or \
                not w.is_contiguous() or w.device != self.device:
            raise ValueError("w must be a contiguous (n, 3) float64 tensor on the device")
        grad = out if out is not None else torch.empty((self.n_total, 3), dtype=torch.float64,
                                                       device=self.device)
        if grad.dtype != torch.float64 or tuple(grad.shape) != (self.n_total, 3) or \
                not grad.is_contiguous():
            raise ValueError("out must be a contiguous (n, 3) float64 tensor")
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_forces_vjp_f64(self._boxes, self.nboxes, ctypes.byref(cs),
                                                      _ptr(w), _ptr(grad), LAWS[self.law],
                                                      _ptr(self.workspace), self.workspace_bytes,
                                                      _stream()),
                   "abacus_nf_forces_vjp_f64")
        return grad

    def forces_vjp(self, binned: Binned, w: torch.Tensor, accumulation: str = "compensated",
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if w.dtype != torch.float32 or tuple(w.shape) != (self.n_total, 3) or not w.is_contiguous():
            raise ValueError("cotangent must be a contiguous (n, 3) float32 tensor")
        grad = out if out is not None else torch.empty((self.n_total, 3), dtype=torch.float32,
                                                       device=self.device)
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_forces_vjp(self._boxes, self.nboxes, ctypes.byref(cs),
                                                  _ptr(w), _ptr(grad), self._flags(accumulation),
                                                  _ptr(self.workspace), self.workspace_bytes,
                                                  _stream()),
                   "abacus_nf_forces_vjp")
        return grad

    def _slab_out(self, out: Optional[torch.Tensor]) -> torch.Tensor:
        if out is None:
            return torch.empty((self.n_total, 3), dtype=torch.float32, device=self.device)
        if out.dtype != torch.float32 or tuple(out.shape) != (self.n_total, 3) or \
                not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous (n, 3) float32 tensor on the device")
        return out

    def forces_slab(self, binned: Binned, x_begin: int, x_end: int,
                    accumulation: str = "compensated",
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Accelerations of the sinks in the slabs x in [x_begin, x_end) of every
        box, bit-identical to those rows of ``forces``; other rows of ``out``
        are left as they were (uninitialised when ``out`` is None)."""
        acc = self._slab_out(out)
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_forces_slab(self._boxes, self.nboxes, ctypes.byref(cs),
                                                   int(x_begin), int(x_end), _ptr(acc),
                                                   self._flags(accumulation),
                                                   _ptr(self.workspace), self.workspace_bytes,
                                                   _stream()),
                   "abacus_nf_forces_slab")
        return acc

    def forces_vjp_slab(self, binned: Binned, x_begin: int, x_end: int, w: torch.Tensor,
                        accumulation: str = "compensated",
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """``forces_vjp`` for the particles of the slabs x in [x_begin, x_end)
        of every box; other rows of ``out`` are left as they were."""
        if w.dtype != torch.float32 or tuple(w.shape) != (self.n_total, 3) or not w.is_contiguous():
            raise ValueError("cotangent must be a contiguous (n, 3) float32 tensor")
        grad = self._slab_out(out)
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_forces_vjp_slab(self._boxes, self.nboxes,
                                                       ctypes.byref(cs), int(x_begin), int(x_end),
                                                       _ptr(w), _ptr(grad),
                                                       self._flags(accumulation),
                                                       _ptr(self.workspace),
                                                       self.workspace_bytes, _stream()),
                   "abacus_nf_forces_vjp_slab")
        return grad


    def multipoles(self, binned: Binned, order: int, reduced: bool = False,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Cell multipoles of Eq. 4 about every cell centre, (cells_total, terms)
        FP64 in box units: the complete basis of ``order`` or its (p+1)^2
        reduction (see include/abacus_nf.h)."""
        flags = _lib.REDUCED if reduced else 0
        terms = ctypes.c_int64(0)
        _lib.check(self._lib.abacus_nf_multipole_terms(int(order), flags, ctypes.byref(terms)),
                   "abacus_nf_multipole_terms")
        nbytes = ctypes.c_size_t(0)
        _lib.check(self._lib.abacus_nf_multipoles_workspace_bytes(
            self._boxes, self.nboxes, int(order), flags, ctypes.byref(nbytes)),
            "abacus_nf_multipoles_workspace_bytes")
        if getattr(self, "_mp_ws", None) is None or self._mp_ws.numel() < nbytes.value:
            self._mp_ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8,
                                      device=self.device)
        shape = (self.cells_total, int(terms.value))
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=self.device)
        elif out.dtype != torch.float64 or tuple(out.shape) != shape or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous {shape} float64 tensor")
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_multipoles(self._boxes, self.nboxes, ctypes.byref(cs),
                                                  int(order), flags, _ptr(out), _ptr(self._mp_ws),
                                                  self._mp_ws.numel(), _stream()),
                   "abacus_nf_multipoles")
        return out

    def kick_drift(self, binned: Binned, pos: torch.Tensor, vel: torch.Tensor,
                   acc: torch.Tensor, kick, drift, cell_stats: bool = False,
                   box_stats: bool = True) -> Tuple[Optional[torch.Tensor], Optional[torch.Tensor]]:
        """One leapfrog kick and drift of ``vel`` and ``pos`` in place (``binned``
        must be the binning of ``pos`` before the call); returns the optional
        per-cell (v_rms, a_max) and per-box (min_c v_rms/a_max, v_rms, a_max, N)
        FP64 statistics of Eq. 1.  ``kick`` / ``drift``: one factor for every box
        or a sequence of nboxes factors."""
        self._check_pos(pos)
        for name, t in (("vel", vel), ("acc", acc)):
            if t.dtype != torch.float32 or tuple(t.shape) != (self.n_total, 3) or \
                    not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"{name} must be a contiguous (n, 3) float32 tensor")
        k = [float(kick)] * self.nboxes if not hasattr(kick, "__len__") else [float(x) for x in kick]
        d = [float(drift)] * self.nboxes if not hasattr(drift, "__len__") else [float(x) for x in drift]
        if len(k) != self.nboxes or len(d) != self.nboxes:
            raise ValueError("kick and drift need one factor per box")
        karr = (ctypes.c_double * self.nboxes)(*k)
        darr = (ctypes.c_double * self.nboxes)(*d)
        cs = torch.empty((self.cells_total, 2), dtype=torch.float64, device=self.device) \
            if cell_stats else None
        bs = torch.empty((self.nboxes, 4), dtype=torch.float64, device=self.device) \
            if box_stats else None
        nbytes = ctypes.c_size_t(0)
        _lib.check(self._lib.abacus_nf_kick_drift_workspace_bytes(self._boxes, self.nboxes,
                                                                  ctypes.byref(nbytes)),
                   "abacus_nf_kick_drift_workspace_bytes")
        ws = self.workspace
        if nbytes.value > ws.numel():
            if getattr(self, "_kdk_ws", None) is None or self._kdk_ws.numel() < nbytes.value:
                self._kdk_ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            ws = self._kdk_ws
        b = binned.cstruct()
        _lib.check(self._lib.abacus_nf_kick_drift(self._boxes, self.nboxes, ctypes.byref(b), karr,
                                                  darr, _ptr(pos), _ptr(vel), _ptr(acc), _ptr(cs),
                                                  _ptr(bs), _ptr(ws), ws.numel(), _stream()),
                   "abacus_nf_kick_drift")
        return cs, bs

    # -- tuning ------------------------------------------------------------------
    def autotune(self, binned: Binned, accumulation: str = "compensated") -> dict:
        """Time the candidate launch shapes on this input and keep the fastest
        (synchronises; do not call while capturing a graph)."""
        scratch = torch.empty((max(self.n_total, 1), 3), dtype=torch.float32, device=self.device)
        fwd, adj = _lib.Tuning(), _lib.Tuning()
        cs = binned.cstruct()
        _lib.check(self._lib.abacus_nf_autotune(self._boxes, self.nboxes, ctypes.byref(cs),
                                                _ptr(scratch), self._flags(accumulation),
                                                _ptr(self.workspace), self.workspace_bytes,
                                                _stream(), ctypes.byref(fwd), ctypes.byref(adj)),
                   "abacus_nf_autotune")
        return {"forward": fwd.asdict(), "adjoint": adj.asdict()}

    def get_tuning(self, kernel: int, accumulation: str = "compensated") -> dict:
        t = _lib.Tuning()
        _lib.check(self._lib.abacus_nf_get_tuning(self._boxes, self.nboxes,
                                                  self._flags(accumulation), kernel,
                                                  ctypes.byref(t)), "abacus_nf_get_tuning")
        return t.asdict()

    def set_tuning(self, kernel: int, tuning: Optional[dict],
                   accumulation: str = "compensated") -> None:
        t = None if tuning is None else ctypes.byref(_lib.Tuning(**tuning))
        _lib.check(self._lib.abacus_nf_set_tuning(self._boxes, self.nboxes,
                                                  self._flags(accumulation), kernel, t),
                   "abacus_nf_set_tuning")


class _NearFieldFn(torch.autograd.Function):
    """acc = near-field accelerations of pos; backward is the hand-written adjoint
    kernel on the binning saved by forward (binning is piecewise constant in pos,
    so it contributes no gradient)."""

    @staticmethod
    def forward(ctx, pos, nf: NearField, accumulation: str):
        binned = nf.bin(pos.contiguous())
        acc, _, _ = nf.forces(binned, accumulation)
        ctx.nf = nf
        ctx.binned = binned
        ctx.accumulation = accumulation
        return acc

    @staticmethod
    def backward(ctx, grad_acc):
        g = ctx.nf.forces_vjp(ctx.binned, grad_acc.contiguous().float(), ctx.accumulation)
        return g, None, None


class _NearFieldF64Fn(torch.autograd.Function):
    """The FP64 kernels: acc (FP64) = near-field accelerations of pos; backward
    is the FP64 adjoint kernel on the saved binning, the gradient returned in
    the dtype of pos."""

    @staticmethod
    def forward(ctx, pos, nf: NearField):
        binned = nf.bin(pos.contiguous())
        acc = nf.forces_f64(binned)
        ctx.nf = nf
        ctx.binned = binned
        ctx.pos_dtype = pos.dtype
        return acc

    @staticmethod
    def backward(ctx, grad_acc):
        g = ctx.nf.forces_vjp_f64(ctx.binned, grad_acc.contiguous().double())
        return g.to(ctx.pos_dtype), None


PRECISIONS = ("fp32", "fp64")


def near_field(pos: torch.Tensor, box: float, cpd: int, radius: int, eps_plummer: float,
               accumulation: str = "compensated", nf: Optional[NearField] = None,
               law: str = "spline", precision: str = "fp32") -> torch.Tensor:
    """Near-field accelerations of one periodic box, differentiable in ``pos``
    (FP32 positions; the binning is held fixed under differentiation).

    ``precision`` "fp32" runs the FP32 kernels, and ``accumulation`` is how each
    sink's FP32 sum is formed, in the forward and the adjoint alike: "single"
    (one running FP32 accumulator, as the paper's kernel), "chunked" (FP32
    partials over at most 64 sources added to it) or "compensated" (those
    partials folded into an FP32 sum and error term).  "fp64" runs the FP64
    kernels (plain FP64 sums; ``accumulation`` does not apply) and returns FP64
    accelerations."""
    if precision not in PRECISIONS:
        raise ValueError(f"unknown precision {precision!r}; one of {list(PRECISIONS)}")
    if accumulation not in ACCUMULATION:
        raise ValueError(f"unknown accumulation {accumulation!r}; "
                         f"one of {sorted(ACCUMULATION)}")
    if nf is None:
        nf = NearField([BoxSpec(pos.shape[0], box, cpd, radius, eps_plummer)], device=pos.device,
                       law=law)
    if precision == "fp64":
        return _NearFieldF64Fn.apply(pos, nf)
    return _NearFieldFn.apply(pos, nf, accumulation)


def timestep(box_stats, a: float, H: float, eta_acc: float, eta_H: float) -> float:
    """Eq. 1 for one box from its four kick-drift statistics (host arithmetic)."""
    arr = (ctypes.c_double * 4)(*[float(x) for x in box_stats])
    return float(_lib.load().abacus_nf_timestep(arr, float(a), float(H), float(eta_acc),
                                                float(eta_H)))


def timing_enable(enable: bool = True) -> None:
    _lib.check(_lib.load().abacus_nf_timing_enable(1 if enable else 0), "timing_enable")


def timing_reset() -> None:
    _lib.check(_lib.load().abacus_nf_timing_reset(), "timing_reset")


def timing_read(kernel: int) -> Tuple[float, int]:
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _lib.check(_lib.load().abacus_nf_timing_read(kernel, ctypes.byref(ms), ctypes.byref(n)),
               "timing_read")
    return float(ms.value), int(n.value)
