#!/usr/bin/env python3
"""Throughput of the MI355X near-field force path.

One step = one pass of the whole path over one batch of synthetic input,
already resident in HBM: cell binning, work plan, forward pair kernel with the
FP64 momentum reduction, and the adjoint (VJP) pair kernel with its work plan.

Prints ONE JSON line.  ``value`` is the pair interactions evaluated per second
over the whole step (every ordered near-field pair is evaluated once by the
forward kernel and once by the adjoint kernel), in G/s.  Per-kernel durations
come from HIP events the library records around its kernels on the stream they
run on.

Workloads (``--workload``):
  C4 (default)  64 uneven clustered boxes, N_b log-uniform in [32^3, 128^3]:
                the batched path (one persistent launch per kernel for all
                boxes, autotuned, replayed from a HIP graph; ``value`` is the
                graph replay), measured beside 64 sequential per-box calls with
                the built-in shapes.
  C3            clustered single box N = 256^3, K = 64.
  C2            clustered single box N = 128^3, K = 32.
  C5, C1        the small differentiation / uniform cases.

Beside the headline the line carries the error of the timed outputs against
the FP64 oracle on sampled sinks (the same oracle calls, timed, give
``cpu_baseline``), the single-box configurations C2 and C3 as ``configs``, and
the widened rows (density, Plummer, FP64 kernel, multipoles, kick-drift) on C3.

    python bench.py [--steps K] [--warmup W] [--workload C4|C3|C2|C5|C1]
                    [--accumulation compensated|chunked|single] [--no-cpu-baseline]
                    [--no-configs] [--no-rows]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per ordered pair: 26 FLOP for the forward interaction
# (Sec. 3.4.4 counts about 26 including the reciprocal square root) and 47 FLOP
# for the adjoint interaction (force, f'(r)/r, the (w_j - w_k) projection and
# two three-component updates).
FLOP_FWD = 26.0
FLOP_ADJ = 47.0
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 x 2.4 GHz.
PEAK_FP32_TFLOPS = 157.3

WORKLOADS = {
    "C1": "uniform N=4096 K=8 R=2 eps_p=1/640",
    "C2": "clustered N=2097152 (2000 blobs) K=32 R=2 eps_p=1/5120",
    "C3": "clustered N=16777216 (20000 blobs) K=64 R=2 eps_p=1/10240",
    "C4": "64 clustered boxes, N_b log-uniform in [32^3, 128^3], K_b=(N_b/64)^(1/3), R=2",
    "C5": "clustered N=262144 (256 blobs) K=16 R=2 eps_p=1/2560",
}
# HBM traffic of the dominant kernel from rocprofv3 counter runs, kept beside
# the profiles; used only while the kernel source is unchanged.
TRAFFIC_FILES = {"C4": "profiles/hbm_traffic_c4_batch64.json"}
# VALU instruction counters of the pair kernels, same rule.
VALU_FILES = {"C4": "profiles/valu_counters_c4_batch64.json"}
KERNEL_SOURCES = {"forward": "paper_2110_11392_amd/csrc/pairs.hip",
                  "adjoint": "paper_2110_11392_amd/csrc/vjp.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(kernel):
    with open(os.path.join(ROOT, KERNEL_SOURCES[kernel]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_bytes(workload, kernel):
    """HBM bytes per launch of `kernel`, or None if not measured for this source."""
    path = TRAFFIC_FILES.get(workload)
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    with open(os.path.join(ROOT, path)) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("source_sha256") != source_sha(kernel):
        return None
    kib = k["fetch_kib"] * rec["copy_fetch_factor"] + k["write_kib"] * rec["copy_write_factor"]
    return kib * 1024.0


def algorithmic_bytes(kernel, n, cells):
    """The HBM bytes one launch of the pair kernel cannot avoid: every particle's
    binned offsets (16 B) and permutation entry (4 B) read once, its result
    (12 B) written once, the cotangent (12 B) read once by the adjoint, and one
    4-byte cell offset per cell."""
    per_particle = 16 + 4 + 12 + (12 if kernel == "adjoint" else 0)
    return float(per_particle * n + 4 * cells)


def valu_issue(workload, avg):
    """Counter-derived VALU figures of the pair kernels (rocprofv3 SQ counters
    kept beside the profiles), valid only while the kernel source is unchanged:
    VALU instructions per pair, the useful-lane fraction and the issue rate in
    VALU instructions per SIMD per 4 cycles (a wave64 instruction occupies a
    16-lane SIMD for 4 cycles, so 1.0 is one instruction stream's full rate)."""
    path = VALU_FILES.get(workload)
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    with open(os.path.join(ROOT, path)) as f:
        rec = json.load(f)
    out = {"source": path}
    for kernel in ("forward", "adjoint"):
        k = rec.get("kernels", {}).get(kernel)
        if not k or k.get("source_sha256") != source_sha(kernel):
            continue
        out[kernel] = dict(k["derived"])
    return out if len(out) > 1 else None


def exact_pairs(cell_offsets, boxes):
    """sum_c n_c S_c - N from the cell offsets (S_c = particles in c's stencil)."""
    import numpy as np
    off = cell_offsets.astype(np.int64)
    total = 0
    base = 0
    for b in boxes:
        K, R = b.cpd, b.radius
        n = np.diff(off[base:base + K ** 3 + 1]).reshape(K, K, K)
        s = np.zeros_like(n)
        for ox in range(-R, R + 1):
            for oy in range(-R, R + 1):
                for oz in range(-R, R + 1):
                    s += np.roll(n, (ox, oy, oz), axis=(0, 1, 2))
        total += int((n * s).sum()) - b.n
        base += K ** 3
    return total


def host_cpu():
    """The host CPU model and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return model, nproc


def oracle_sample(boxes, wvec, n_sinks, seed):
    """FP64 oracle forces and adjoint on ~n_sinks sinks drawn in proportion to
    N_b (global indices into the concatenated particles), with the single-thread
    time of those oracle calls: the CPU baseline in the metric's unit."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2110_11392_amd import synth
    n_all = sum(b.n for b in boxes)
    idx, ref_a, ref_g = [], [], []
    pairs, dt = 0, 0.0
    first = 0
    for k, b in enumerate(boxes):
        m = min(b.n, max(1, int(round(n_sinks * b.n / n_all)))) if b.n else 0
        if m:
            s = synth.sample_indices(b.n, m, seed + k)
            t0 = time.perf_counter()
            ra, npairs = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, s)
            rg = oracle.vjp(b.pos, wvec[first:first + b.n], b.box, b.cpd, b.radius,
                            b.eps_plummer, s)
            dt += time.perf_counter() - t0
            pairs += 2 * npairs
            idx.append(first + s)
            ref_a.append(ra)
            ref_g.append(rg)
        first += b.n
    idx = np.concatenate(idx)
    model, nproc = host_cpu()
    baseline = {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
                "sample": f"the accuracy sample: {idx.size} sinks of the same workload drawn in "
                          f"proportion to N_b, FP64 forces + adjoint of those sinks, {pairs} pair "
                          f"evaluations in {dt:.1f} s on one thread (including the oracle's "
                          f"binning of each sampled box)",
                "cpu_model": model, "host_cores_available": nproc}
    return (idx, np.concatenate(ref_a), np.concatenate(ref_g)), baseline


def accuracy(sample, acc, grad, seed):
    """Per-particle fractional force error (median, 99.9th percentile) and the
    adjoint's relative 2-norm error with its per-particle median / 99.9th
    percentile, of outputs `acc`, `grad` (all particles) on the oracle sample."""
    import numpy as np
    idx, ra, rg = sample
    a = acc[idx].astype(np.float64)
    g = grad[idx].astype(np.float64)
    nrm = np.linalg.norm(ra, axis=1)
    keep = nrm > 0
    e = np.linalg.norm(a[keep] - ra[keep], axis=1) / nrm[keep]
    gn = np.linalg.norm(rg, axis=1)
    gkeep = gn > 0
    ge = np.linalg.norm(g[gkeep] - rg[gkeep], axis=1) / gn[gkeep]
    return {
        "sinks": int(idx.size), "sampling": f"in proportion to N_b, seeds {seed}+b",
        "force_frac_err_median": float(np.median(e)),
        "force_frac_err_p999": float(np.percentile(e, 99.9)),
        "adjoint_rel_err": float(np.linalg.norm(g - rg) / np.linalg.norm(rg)),
        "adjoint_frac_err_median": float(np.median(ge)),
        "adjoint_frac_err_p999": float(np.percentile(ge, 99.9)),
        "tolerances": {"force_median": 1e-6, "force_p999": 1e-4, "adjoint_rel": 1e-4},
    }


class Stepper:
    """Preallocated buffers and one step of the path for a list of boxes."""

    def __init__(self, anf, torch, boxes, accumulation, dev, pos=None, wvec=None):
        import numpy as np
        from paper_2110_11392_amd import synth
        self.torch = torch
        self.nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)
                                 for b in boxes], device=dev)
        nf = self.nf
        self.pos = pos if pos is not None else \
            torch.from_numpy(np.concatenate([b.pos for b in boxes])).to(dev)
        self.wvec = wvec if wvec is not None else \
            torch.from_numpy(synth.gaussian_weights(nf.n_total, 4242)).to(dev)
        self.binned = nf.alloc_binned()
        self.acc = torch.empty((nf.n_total, 3), dtype=torch.float32, device=dev)
        self.grad = torch.empty_like(self.acc)
        self.mom = torch.empty((nf.nboxes, 4), dtype=torch.float64, device=dev)
        self.accumulation = accumulation

    def step(self):
        nf = self.nf
        nf.bin(self.pos, out=self.binned)
        nf.forces(self.binned, self.accumulation, out=self.acc, momentum_out=self.mom)
        nf.forces_vjp(self.binned, self.wvec, self.accumulation, out=self.grad)

    def capture(self):
        torch = self.torch
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.step()
        graph.replay()
        torch.cuda.synchronize()
        return graph


def measure_rows(anf, torch, st, boxes, accumulation, reps=5):
    """The widened rows, each timed by the library's own HIP events over `reps`
    launches outside the main step: the density estimate fused into the
    forward kernel, the Plummer law, the FP64 pair kernels, the cell multipoles
    (p = 8, complete and reduced) and the kick-drift step.  Returns per-row
    figures."""
    import numpy as np
    from paper_2110_11392_amd import synth
    nf = st.nf
    dev = st.pos.device
    rows = {}

    def kernel_ms(slot, fn):
        fn()
        torch.cuda.synchronize()
        anf.timing_reset()
        anf.timing_enable(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        anf.timing_enable(False)
        ms, n = anf.timing_read(slot)
        return ms / n if n else float("nan")

    fwd = kernel_ms(0, lambda: nf.forces(st.binned, accumulation, out=st.acc))
    # density: b = 0.4 cell (below half a cell, so cells two apart skip it), every box
    specs = [anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer, 0.4 * b.box / b.cpd)
             for b in boxes]
    nfd = anf.NearField(specs, device=dev)
    nfd.set_tuning(0, nf.get_tuning(0, accumulation), accumulation)
    rho = torch.empty(nf.n_total, dtype=torch.float32, device=dev)
    dens = kernel_ms(0, lambda: nfd.forces(st.binned, accumulation, out=st.acc, density_out=rho))
    rows["density"] = {"forward_ms": fwd, "forward_with_density_ms": dens,
                       "overhead": dens / fwd - 1.0, "radius_cells": 0.4}
    del nfd
    # Plummer law (its own launch shapes: the built-in ones)
    nfp = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)
                         for b in boxes], device=dev, law="plummer")
    plum = kernel_ms(0, lambda: nfp.forces(st.binned, accumulation, out=st.acc))
    rows["plummer"] = {"forward_ms": plum}
    del nfp
    # the FP64 pair kernel (built-in shape, whole work items)
    acc64 = torch.empty((nf.n_total, 3), dtype=torch.float64, device=dev)
    f64 = kernel_ms(0, lambda: nf.forces_f64(st.binned, out=acc64))
    rows["fp64_forward"] = {"forward_ms": f64, "vs_fp32": f64 / fwd}
    # and its adjoint, against the FP32 adjoint of the main step's shapes
    w64 = st.wvec.to(torch.float64)
    adj = kernel_ms(1, lambda: nf.forces_vjp(st.binned, st.wvec, accumulation, out=st.acc))
    a64 = kernel_ms(1, lambda: nf.forces_vjp_f64(st.binned, w64, out=acc64))
    rows["fp64_adjoint"] = {"adjoint_ms": a64, "vs_fp32": a64 / adj}
    del acc64, w64
    # one GPU's share of a box split into slabs along x: 8 shares of K/8 sink
    # slabs, each reading its neighbour slabs, forward and adjoint per share
    if len(boxes) == 1 and boxes[0].cpd % 8 == 0:
        K = boxes[0].cpd
        shares = [(g * K // 8, (g + 1) * K // 8) for g in range(8)]
        f_sh = [kernel_ms(0, lambda x=x: nf.forces_slab(st.binned, x[0], x[1], accumulation,
                                                        out=st.acc)) for x in shares]
        a_sh = [kernel_ms(1, lambda x=x: nf.forces_vjp_slab(st.binned, x[0], x[1], st.wvec,
                                                            accumulation, out=st.acc))
                for x in shares]
        rows["slab_shares"] = {
            "shares": 8, "sink_slabs_per_share": K // 8,
            "forward_ms": f_sh, "adjoint_ms": a_sh,
            "forward_sum_over_whole": sum(f_sh) / fwd, "adjoint_sum_over_whole": sum(a_sh) / adj,
            "forward_max_over_mean": max(f_sh) * 8 / sum(f_sh),
            "adjoint_max_over_mean": max(a_sh) * 8 / sum(a_sh)}
    # multipoles, p = 8
    n, cells = nf.n_total, nf.cells_total
    out_c = torch.empty((cells, 165), dtype=torch.float64, device=dev)
    out_r = torch.empty((cells, 81), dtype=torch.float64, device=dev)
    mp_c = kernel_ms(4, lambda: nf.multipoles(st.binned, 8, out=out_c))
    mp_r = kernel_ms(4, lambda: nf.multipoles(st.binned, 8, reduced=True, out=out_r))
    # algorithmic bytes: 16 B offsets per particle + offsets 4 B per cell read,
    # 165 doubles per cell written (reduced: + complete rows read back, 81 written)
    bytes_c = 16.0 * n + 4.0 * cells + 8.0 * 165 * cells
    bytes_r = bytes_c + 8.0 * 165 * cells + 8.0 * 81 * cells
    rows["multipoles_p8"] = {
        "complete_ms": mp_c, "reduced_ms": mp_r,
        "complete_gbps": bytes_c / (mp_c * 1e-3) / 1e9,
        "reduced_gbps": bytes_r / (mp_r * 1e-3) / 1e9,
        "hbm_peak_gbps": 8000.0,
        "complete_frac_hbm": bytes_c / (mp_c * 1e-3) / 8e12,
        "fp64_tflops_at_384_flop_per_particle": 384.0 * n / (mp_c * 1e-3) / 1e12,
        "fp64_peak_tflops": 78.6}
    del out_c, out_r
    # kick-drift on copies of the state (the main step's inputs stay untouched),
    # first in the workload's original particle order, then with the particles
    # stored in cell order (the layout the paper's slabs keep), where the
    # gathers through the permutation are contiguous.  Each call gets the
    # binning of the positions it moves, as in a time step (the statistics'
    # cells are the cells of that binning); only the kick-drift is timed.
    pos = st.pos.clone()
    vel = torch.from_numpy(synth.gaussian_weights(n, 77) * np.float32(0.05)).to(dev)
    acc = st.acc.clone()
    nf.forces(st.binned, accumulation, out=acc)
    # algorithmic bytes: pos, vel read and written, acc read (12 B each), perm
    # 4 B per particle; offsets 4 B and statistics 16 B per cell
    bytes_kd = (12.0 * 5 + 4.0) * n + 20.0 * cells
    bd_o = nf.alloc_binned()

    def kd_step(bd, p, v, a):
        nf.bin(p, out=bd)
        nf.kick_drift(bd, p, v, a, 1e-9, 1e-9, cell_stats=True)
    kd = kernel_ms(5, lambda: kd_step(bd_o, pos, vel, acc))
    nf.bin(pos, out=bd_o)
    order = bd_o.perm.long()
    pos_c, vel_c, acc_c = pos[order].contiguous(), vel[order].contiguous(), acc[order].contiguous()
    bd_c = nf.alloc_binned()
    kdc = kernel_ms(5, lambda: kd_step(bd_c, pos_c, vel_c, acc_c))
    rows["kick_drift"] = {"original_order_ms": kd, "cell_order_ms": kdc,
                          "original_order_gbps": bytes_kd / (kd * 1e-3) / 1e9,
                          "cell_order_gbps": bytes_kd / (kdc * 1e-3) / 1e9,
                          "cell_order_frac_hbm": bytes_kd / (kdc * 1e-3) / 8e12,
                          "algorithmic_bytes": bytes_kd}
    return rows


def binning_row(ms, n, cells, step_ms):
    """The binning against the HBM line.  Algorithmic bytes: the position read
    twice (cell assignment, then the cell offsets of the sorted slots), the
    cell id written and read back, the 16-byte offsets and 4-byte permutation
    written (52 B per particle), and 4 B of cell offset per cell.  The stable
    LSD radix sort moves 24 B per particle in each of its 8-bit passes."""
    bits = max(1, math.ceil(math.log2(max(cells, 2))))
    b = 52.0 * n + 4.0 * (cells + 1)
    return {"ms": ms, "algorithmic_bytes": b, "gbps": b / (ms * 1e-3) / 1e9,
            "frac_hbm": b / (ms * 1e-3) / 8e12, "radix_passes": (bits + 7) // 8,
            "share_of_step": ms / step_ms}


def timed(torch, fn, steps):
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(steps):
        fn()
        log(f"[bench] step {k + 1}/{steps} enqueued")
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def run_config(anf, torch, name, accumulation, dev, steps, warmup, autotune, keep=False):
    """One single-box configuration: tuned shapes, `steps` eager steps timed."""
    from paper_2110_11392_amd import synth
    log(f"[bench] config {name}: generating")
    boxes = synth.config(name)
    st = Stepper(anf, torch, boxes, accumulation, dev)
    for _ in range(warmup):
        st.step()
    torch.cuda.synchronize()
    st.binned.check_status()
    tuning = None
    if autotune:
        tuning = st.nf.autotune(st.binned, accumulation)
        st.step()
        torch.cuda.synchronize()
    pairs = exact_pairs(st.binned.cell_offsets.cpu().numpy(), boxes)
    anf.timing_reset()
    anf.timing_enable(True)
    ms = timed(torch, st.step, steps)
    anf.timing_enable(False)
    avg = {k: (lambda r: r[0] / r[1] if r[1] else float("nan"))(anf.timing_read(i))
           for k, i in (("forward", 0), ("adjoint", 1), ("bin", 2), ("plan", 3))}
    rec = {"workload": f"{name}: {WORKLOADS[name]}", "n": st.nf.n_total,
           "pairs_per_evaluation": pairs, "steps": steps, "ms_per_step": ms,
           "value": 2.0 * pairs / (ms * 1e-3) / 1e9, "unit": "Gpairs/s", "timed": "eager calls",
           "kernel_ms": avg, "tuning": tuning,
           "forward_gpairs_per_s": pairs / (avg["forward"] * 1e-3) / 1e9,
           "adjoint_gpairs_per_s": pairs / (avg["adjoint"] * 1e-3) / 1e9,
           "forward_frac_fp32": FLOP_FWD * pairs / (avg["forward"] * 1e-3) / 1e12
           / PEAK_FP32_TFLOPS,
           "adjoint_frac_fp32": FLOP_ADJ * pairs / (avg["adjoint"] * 1e-3) / 1e12
           / PEAK_FP32_TFLOPS,
           "adjoint_over_forward": avg["adjoint"] / avg["forward"]}
    return rec, (st, boxes) if keep else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C4", choices=sorted(WORKLOADS))
    ap.add_argument("--accumulation", default="compensated",
                    choices=["compensated", "chunked", "single"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle comparison of the timed outputs (and its timing)")
    ap.add_argument("--accuracy-sinks", type=int, default=10000,
                    help="sinks of the oracle comparison, drawn in proportion to N_b")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of timing candidates")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the measurement of the step replayed from a HIP graph")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-box configurations C2 and C3 beside the headline")
    ap.add_argument("--config-steps", type=int, default=5)
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the density / Plummer / FP64 / multipole / kick-drift figures")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the near-field path here runs on a single MI355X "
              "(--gpus 1). One GPU's share of a box split into x-slabs is timed in "
              "rows.slab_shares; runs over several GPUs are not measured here.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return

    import paper_2110_11392_amd as anf
    from paper_2110_11392_amd import synth

    log(f"[bench] generating {args.workload}")
    boxes = synth.config(args.workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    st = Stepper(anf, torch, boxes, args.accumulation, dev)
    nf = st.nf

    log("[bench] warmup")
    for _ in range(args.warmup):
        st.step()
    torch.cuda.synchronize()
    st.binned.check_status()
    tuning = {"forward": nf.get_tuning(0, args.accumulation),
              "adjoint": nf.get_tuning(1, args.accumulation)}
    if not args.no_autotune:
        log("[bench] autotune")
        tuning = nf.autotune(st.binned, args.accumulation)
        log(f"[bench] tuned {tuning}")
        st.step()
        torch.cuda.synchronize()
    pairs = exact_pairs(st.binned.cell_offsets.cpu().numpy(), boxes)
    log(f"[bench] pairs per evaluation: {pairs}")

    anf.timing_reset()
    anf.timing_enable(True)
    ms_eager = timed(torch, st.step, args.steps)
    anf.timing_enable(False)
    kt = {name: anf.timing_read(k) for name, k in
          (("forward", 0), ("adjoint", 1), ("bin", 2), ("plan", 3))}
    avg = {name: (ms / n if n else float("nan")) for name, (ms, n) in kt.items()}

    graph_ms = None
    if not args.no_graph:
        log("[bench] graph capture")
        graph = st.capture()
        graph_ms = timed(torch, graph.replay, args.steps)
        log(f"[bench] graph replay {graph_ms:.3f} ms/step")
    # the outputs of the last timed step, compared with the oracle below
    acc_out = st.acc.cpu().numpy()
    grad_out = st.grad.cpu().numpy()
    mom_out = st.mom.cpu().numpy()

    sequential_ms = None
    plain = None
    if args.workload == "C4":
        log("[bench] 64 sequential per-box calls, built-in shapes, no graph")
        per_box = []
        first = 0
        for b in boxes:
            per_box.append(Stepper(anf, torch, [b], args.accumulation, dev,
                                   pos=st.pos[first:first + b.n],
                                   wvec=st.wvec[first:first + b.n]))
            first += b.n

        def sequential():
            for s in per_box:
                s.step()
        sequential()
        torch.cuda.synchronize()
        sequential_ms = timed(torch, sequential, args.steps)
        log(f"[bench] sequential {sequential_ms:.3f} ms/step")
        # the plain single-box path: the same calls with one FP32 running sum
        # per sink (the paper kernel's accumulation), built-in shapes
        for s in per_box:
            s.accumulation = "single"
        sequential()
        torch.cuda.synchronize()
        anf.timing_reset()
        anf.timing_enable(True)
        plain_ms = timed(torch, sequential, args.steps)
        anf.timing_enable(False)
        pk = {name: anf.timing_read(k)[0] / args.steps for name, k in
              (("forward", 0), ("adjoint", 1), ("bin", 2), ("plan", 3))}
        plain = {"accumulation": "single", "shapes": "built-in", "calls": "64 per-box calls per step",
                 "ms_per_step": plain_ms, "value": 2.0 * pairs / (plain_ms * 1e-3) / 1e9,
                 "kernel_ms_per_step": pk,
                 "adjoint_frac_fp32": FLOP_ADJ * pairs / (pk["adjoint"] * 1e-3) / 1e12
                 / PEAK_FP32_TFLOPS}
        plain_acc = torch.cat([s.acc for s in per_box]).cpu().numpy()
        plain_grad = torch.cat([s.grad for s in per_box]).cpu().numpy()
        log(f"[bench] plain single-box {plain_ms:.3f} ms/step")
        del per_box

    resid = float((np.abs(mom_out[:, :3]).max(axis=1) / mom_out[:, 3]).max())
    fwd_tflops = FLOP_FWD * pairs / (avg["forward"] * 1e-3) / 1e12
    adj_tflops = FLOP_ADJ * pairs / (avg["adjoint"] * 1e-3) / 1e12
    dominant = "adjoint" if avg["adjoint"] >= avg["forward"] else "forward"
    achieved = adj_tflops if dominant == "adjoint" else fwd_tflops
    tbytes = traffic_bytes(args.workload, dominant)
    ms_value = graph_ms if (args.workload == "C4" and graph_ms is not None) else ms_eager
    out = {
        "metric": "near-field pair interactions/s (G) + particle updates/s; adjoint/forward time",
        "value": 2.0 * pairs / (ms_value * 1e-3) / 1e9,
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_value,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "n": nf.n_total, "boxes": nf.nboxes, "pairs_per_evaluation": pairs,
                   "accumulation": args.accumulation,
                   "step": "bin + forward(+FP64 momentum) + adjoint",
                   "timed": "graph replay" if ms_value == graph_ms else "eager calls",
                   "tuning": tuning},
        "ms_per_step_eager": ms_eager,
        "ms_per_step_graph_replay": graph_ms,
        "forward_gpairs_per_s": pairs / (avg["forward"] * 1e-3) / 1e9,
        "adjoint_gpairs_per_s": pairs / (avg["adjoint"] * 1e-3) / 1e9,
        "particle_updates_per_s": nf.n_total / ((avg["bin"] + avg["plan"] + avg["forward"]) * 1e-3),
        "adjoint_over_forward": avg["adjoint"] / avg["forward"],
        "kernel_ms": avg,
        "binning": binning_row(avg["bin"], nf.n_total, nf.cells_total, ms_value),
        "momentum_residual": resid,
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": tbytes,
                     "algorithmic_flop_per_launch": (FLOP_ADJ if dominant == "adjoint"
                                                     else FLOP_FWD) * pairs,
                     "algorithmic_bytes_per_launch": algorithmic_bytes(dominant, nf.n_total,
                                                                       nf.cells_total),
                     "forward_tflops": fwd_tflops, "adjoint_tflops": adj_tflops,
                     "valu": valu_issue(args.workload, avg)},
    }
    if sequential_ms is not None:
        out["sequential_per_box_ms_per_step"] = sequential_ms
        out["batched_speedup_vs_sequential"] = sequential_ms / ms_value
    if plain is not None:
        out["plain_single_box"] = plain
    if not args.no_cpu_baseline:
        log(f"[bench] oracle comparison of the timed outputs on {args.accuracy_sinks} sinks")
        sample, baseline = oracle_sample(boxes, st.wvec.cpu().numpy(), args.accuracy_sinks, 4250)
        out["accuracy"] = accuracy(sample, acc_out, grad_out, 4250)
        out["cpu_baseline"] = baseline
        if plain is not None:
            plain["accuracy"] = accuracy(sample, plain_acc, plain_grad, 4250)
        log(f"[bench] accuracy {out['accuracy']}")
    rows_src = (st, boxes)
    if not args.no_configs:
        out["configs"] = {}
        for name in ("C2", "C3"):
            if name == args.workload:
                continue
            rec, kept = run_config(anf, torch, name, args.accumulation, dev, args.config_steps,
                                   2, not args.no_autotune, keep=(name == "C3"))
            out["configs"][name] = rec
            log(f"[bench] config {name}: {rec['value']:.1f} Gpairs/s")
            if kept is not None:
                rows_src = kept
    if not args.no_rows:
        rst, rboxes = rows_src
        log(f"[bench] widened rows on {rboxes[0].n if len(rboxes) == 1 else 'the batch'}")
        out["rows"] = measure_rows(anf, torch, rst, rboxes, args.accumulation)
        out["rows"]["workload"] = ("C3: " + WORKLOADS["C3"]) if rst is not st else \
            out["config"]["workload"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
