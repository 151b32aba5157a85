#!/usr/bin/env python3
"""Throughput of the MI355X near-field force path.

One step = one pass of the whole path over one batch of synthetic input,
already resident in HBM: cell binning, work plan, forward pair kernel with the
FP64 momentum reduction, and the adjoint (VJP) pair kernel with its work plan.

Prints ONE JSON line.  ``value`` is the pair interactions evaluated per second
over the whole step (every ordered near-field pair is evaluated once by the
forward kernel and once by the adjoint kernel), in G/s.  Per-kernel durations
come from HIP events the library records around its kernels on the stream they
run on.  The default workload is the clustered single box N = 128^3, K = 32.

    python bench.py [--steps K] [--warmup W] [--workload C2|C3|C5|C1]
                    [--accumulation compensated|chunked|single] [--no-cpu-baseline]
"""
import argparse
import json
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
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed)
# x 2.4 GHz.
PEAK_FP32_TFLOPS = 157.3

WORKLOADS = {
    "C1": "uniform N=4096 K=8 R=2 eps_p=1/640",
    "C2": "clustered N=2097152 (2000 blobs) K=32 R=2 eps_p=1/5120",
    "C3": "clustered N=16777216 (20000 blobs) K=64 R=2 eps_p=1/10240",
    "C5": "clustered N=262144 (256 blobs) K=16 R=2 eps_p=1/2560",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def cpu_baseline(box, budget_s=12.0):
    """The FP64 oracle (single thread) on a bounded sample of sinks of the same
    workload: forward forces plus the adjoint for those sinks."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2110_11392_amd import synth
    w = synth.gaussian_weights(box.n, 4242)
    order = synth.sample_indices(box.n, min(box.n, 200000), 4243)
    rng = np.random.default_rng(4244)
    rng.shuffle(order)
    pairs = 0
    sinks_done = 0
    t0 = time.perf_counter()
    chunk = 500
    while time.perf_counter() - t0 < budget_s and sinks_done < order.size:
        s = np.sort(order[sinks_done:sinks_done + chunk])
        _, npairs = oracle.forces(box.pos, box.box, box.cpd, box.radius, box.eps_plummer, s)
        oracle.vjp(box.pos, w, box.box, box.cpd, box.radius, box.eps_plummer, s)
        pairs += 2 * npairs
        sinks_done += s.size
    dt = time.perf_counter() - t0
    return {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{sinks_done} random sinks of the same workload, FP64 forces + adjoint, "
                      f"{pairs} pair evaluations in {dt:.1f} s (single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--accumulation", default="compensated",
                    choices=["compensated", "chunked", "single"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of timing candidates")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the extra measurement of the step replayed from a HIP graph")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the near-field path here runs on a single MI355X "
              "(--gpus 1); multi-GPU sharding is a design note, not a measured path.",
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
    box = boxes[0]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes],
                       device=dev)
    pos = torch.from_numpy(np.concatenate([b.pos for b in boxes])).to(dev)
    wvec = torch.from_numpy(synth.gaussian_weights(nf.n_total, 4242)).to(dev)
    binned = nf.alloc_binned()
    acc = torch.empty((nf.n_total, 3), dtype=torch.float32, device=dev)
    grad = torch.empty_like(acc)
    mom = torch.empty((nf.nboxes, 4), dtype=torch.float64, device=dev)

    def step():
        nf.bin(pos, out=binned)
        nf.forces(binned, args.accumulation, out=acc, momentum_out=mom)
        nf.forces_vjp(binned, wvec, args.accumulation, out=grad)

    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    binned.check_status()
    tuning = {"forward": nf.get_tuning(0, args.accumulation),
              "adjoint": nf.get_tuning(1, args.accumulation)}
    if not args.no_autotune:
        log("[bench] autotune")
        tuning = nf.autotune(binned, args.accumulation)
        log(f"[bench] tuned {tuning}")
        step()
        torch.cuda.synchronize()
    pairs = exact_pairs(binned.cell_offsets.cpu().numpy(), boxes)
    log(f"[bench] pairs per evaluation: {pairs}")

    anf.timing_reset()
    anf.timing_enable(True)
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(args.steps):
        step()
        log(f"[bench] step {k + 1}/{args.steps} enqueued")
    t1.record(stream)
    torch.cuda.synchronize()
    anf.timing_enable(False)
    ms_total = t0.elapsed_time(t1)
    ms_step = ms_total / args.steps
    kt = {name: anf.timing_read(k) for name, k in
          (("forward", 0), ("adjoint", 1), ("bin", 2), ("plan", 3))}
    avg = {name: (ms / n if n else float("nan")) for name, (ms, n) in kt.items()}
    graph_ms = None
    if not args.no_graph:
        log("[bench] graph capture")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        graph.replay()
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(args.steps):
            graph.replay()
        g1.record(stream)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / args.steps
        log(f"[bench] graph replay {graph_ms:.3f} ms/step")
    m = mom.cpu().numpy()
    resid = float(np.abs(m[:, :3]).max() / m[:, 3].max())

    fwd_tflops = FLOP_FWD * pairs / (avg["forward"] * 1e-3) / 1e12
    adj_tflops = FLOP_ADJ * pairs / (avg["adjoint"] * 1e-3) / 1e12
    dominant = "adjoint" if avg["adjoint"] >= avg["forward"] else "forward"
    achieved = adj_tflops if dominant == "adjoint" else fwd_tflops
    out = {
        "metric": "near-field pair interactions/s (G) + particle updates/s; adjoint/forward time",
        "value": 2.0 * pairs / (ms_step * 1e-3) / 1e9,
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "n": nf.n_total, "pairs_per_evaluation": pairs,
                   "accumulation": args.accumulation,
                   "step": "bin + forward(+FP64 momentum) + adjoint",
                   "tuning": tuning},
        "ms_per_step_graph_replay": graph_ms,
        "forward_gpairs_per_s": pairs / (avg["forward"] * 1e-3) / 1e9,
        "adjoint_gpairs_per_s": pairs / (avg["adjoint"] * 1e-3) / 1e9,
        "particle_updates_per_s": nf.n_total / ((avg["bin"] + avg["plan"] + avg["forward"]) * 1e-3),
        "adjoint_over_forward": avg["adjoint"] / avg["forward"],
        "kernel_ms": avg,
        "momentum_residual": resid,
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "flop_per_pair": FLOP_ADJ if dominant == "adjoint" else FLOP_FWD,
                     "forward_tflops": fwd_tflops, "adjoint_tflops": adj_tflops},
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(box)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
