"""GPU parity at the full benchmark sizes and of the quantities checked only
loosely elsewhere, against the FP64 oracle, through the C ABI:

  * the adjoint on C2 and C3 (the sizes the benchmark times) on 10^4 sampled
    sinks, compensated and chunked: relative 2-norm error <= 1e-4;
  * the whole 64-box batch C4 in the launch configuration the benchmark times
    (autotuned shapes, bin + forces + adjoint replayed from a HIP graph),
    forward and adjoint on 10^4 sinks sampled in proportion to N_b;
  * the per-box FP64 momentum sums against an exact sum of the returned FP32
    accelerations and, for C1, against the oracle's accelerations;
  * the single-accumulator forward mode against the oracle within the bound
    that rounding in one FP32 running sum allows (Higham's recursive-summation
    bound on the sum of absolute summands, from the oracle);
  * the C5 adjoint against central differences on all 256 sampled
    coordinates, plain and Richardson-extrapolated.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from gpu_common import (MEDIAN_TOL, P999_TOL, VJP_TOL, err_stats, frac_err,
                        single_sum_bound_violations)
from paper_2110_11392_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def anf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd
    return paper_2110_11392_amd


def make_nf(anf, boxes):
    return anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)
                          for b in boxes])


def upload(boxes):
    return torch.from_numpy(np.ascontiguousarray(np.concatenate([b.pos for b in boxes]))).cuda()


def sinks_in_proportion(boxes, total, seed):
    """About `total` sinks over the boxes, in proportion to N_b (at least one per
    non-empty box), as local indices per box."""
    n_all = sum(b.n for b in boxes)
    out = []
    for k, b in enumerate(boxes):
        m = min(b.n, max(1, int(round(total * b.n / n_all)))) if b.n else 0
        out.append(synth.sample_indices(b.n, m, seed + k) if m else np.zeros(0, np.int64))
    return out


def vjp_report(g, ref):
    rel = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    return rel, err_stats(frac_err(g, ref))


# ---------------------------------------------------------------------------
# adjoint at the benchmark sizes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["C2", "C3"])
def test_vjp_configs_sampled(anf, name):
    b = synth.config(name)[0]
    sinks = synth.sample_indices(b.n, 10000, 1100 + int(name[1]) + 11)
    w = synth.gaussian_weights(b.n, 1100 + int(name[1]) + 12)
    say(f"[vjp] {name} n={b.n} sampled={sinks.size}")
    nf = make_nf(anf, [b])
    bd = nf.bin(torch.from_numpy(b.pos).cuda())
    wt = torch.from_numpy(w).cuda()
    res = {acc: nf.forces_vjp(bd, wt, acc).cpu().numpy()[sinks]
           for acc in ("compensated", "chunked")}
    ref = oracle.vjp(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, sinks)
    for acc, g in res.items():
        rel, st = vjp_report(g, ref)
        say(f"  {acc}: relative 2-norm error {rel:.3g}; per particle {st}")
        assert rel <= VJP_TOL
        assert st["median"] <= 1e-5


# ---------------------------------------------------------------------------
# the whole batch, in the benchmark's launch configuration
# ---------------------------------------------------------------------------

def test_c4_full_batch_graph_replay(anf):
    boxes = synth.config("C4")
    n_total = sum(b.n for b in boxes)
    say(f"[C4] {len(boxes)} boxes, n={n_total}")
    nf = make_nf(anf, boxes)
    pos = upload(boxes)
    w = synth.gaussian_weights(n_total, 1104 + 12)
    wt = torch.from_numpy(w).cuda()
    binned = nf.alloc_binned()
    acc = torch.empty((n_total, 3), dtype=torch.float32, device="cuda")
    grad = torch.empty_like(acc)
    mom = torch.empty((len(boxes), 4), dtype=torch.float64, device="cuda")

    def step():
        nf.bin(pos, out=binned)
        nf.forces(binned, "compensated", out=acc, momentum_out=mom)
        nf.forces_vjp(binned, wt, "compensated", out=grad)

    step()
    torch.cuda.synchronize()
    binned.check_status()
    tuning = nf.autotune(binned, "compensated")
    say(f"  tuned {tuning}")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    results = []
    for rep in range(2):
        acc.zero_()
        grad.zero_()
        graph.replay()
        torch.cuda.synchronize()
        results.append((acc.cpu().numpy(), grad.cpu().numpy(), mom.cpu().numpy()))
    assert all(np.array_equal(results[0][k].view(np.uint64 if k == 2 else np.uint32),
                              results[1][k].view(np.uint64 if k == 2 else np.uint32))
               for k in range(3))
    a, g, m = results[0]
    sinks = sinks_in_proportion(boxes, 10000, 1104 + 20)
    refs_a, refs_g, got_a, got_g = [], [], [], []
    first = 0
    for k, b in enumerate(boxes):
        s = sinks[k]
        if s.size:
            ra, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, s)
            rg = oracle.vjp(b.pos, w[first:first + b.n], b.box, b.cpd, b.radius, b.eps_plummer,
                            s)
            refs_a.append(ra)
            refs_g.append(rg)
            got_a.append(a[first + s])
            got_g.append(g[first + s])
        # per-box momentum: the FP64 sums of this box's returned accelerations
        ab = a[first:first + b.n].astype(np.float64)
        for c in range(3):
            exact = math.fsum(ab[:, c])
            assert abs(m[k, c] - exact) <= reduction_bound(b.n) * np.abs(ab[:, c]).sum()
        first += b.n
    st = err_stats(frac_err(np.concatenate(got_a), np.concatenate(refs_a)))
    rel, gst = vjp_report(np.concatenate(got_g), np.concatenate(refs_g))
    say(f"  forces ({sum(s.size for s in sinks)} sinks): {st}")
    say(f"  adjoint: relative 2-norm error {rel:.3g}; per particle {gst}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL
    assert rel <= VJP_TOL


# ---------------------------------------------------------------------------
# FP64 momentum sums
# ---------------------------------------------------------------------------

def reduction_bound(n):
    """Relative bound (to the sum of absolute values) of the FP64 reduction:
    every partial passes through at most ceil(n / 2^18) sequential additions per
    thread (1024 chunks of 256 threads per box) and at most 64 more in the
    fixed wave / block / final tree, each adding one FP64 rounding of at most
    2^-53 of the running magnitude (first-order recursive-summation bound)."""
    return (math.ceil(max(n, 1) / 2 ** 18) + 64) * U64


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_momentum_matches_fp64_sums(anf, name):
    boxes = synth.config(name)
    b = boxes[0]
    say(f"[momentum] {name} n={b.n}")
    nf = make_nf(anf, boxes)
    bd = nf.bin(upload(boxes))
    acc, mom, _ = nf.forces(bd, "compensated", momentum=True)
    torch.cuda.synchronize()
    a = acc.cpu().numpy().astype(np.float64)
    m = mom.cpu().numpy()[0]
    lim = reduction_bound(b.n)
    for c in range(3):
        exact = math.fsum(a[:, c])
        scale = np.abs(a[:, c]).sum()
        say(f"  sum a_{'xyz'[c]}: gpu {m[c]:.17g} exact {exact:.17g} "
            f"|diff|/sum|a| {abs(m[c] - exact) / scale:.3g} (bound {lim:.3g})")
        assert abs(m[c] - exact) <= lim * scale
    # each norm: two roundings in the sum of squares (the squares of FP32 values
    # are exact in FP64) and one in the square root
    norms = np.sqrt(a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1] + a[:, 2] * a[:, 2])
    exact_n = math.fsum(norms)
    say(f"  sum |a|: gpu {m[3]:.17g} exact {exact_n:.17g}")
    assert abs(m[3] - exact_n) <= (lim + 4 * U64) * exact_n
    resid = np.abs(m[:3]).max() / m[3]
    say(f"  momentum residual |sum a| / sum |a| = {resid:.3g}")
    if name == "C1":
        # against the oracle: |sum_i a_i - sum_i r_i| <= sum_i |a_i - r_i| per
        # component and |sum |a_i| - sum |r_i|| <= sum |a_i - r_i| (triangle
        # inequality), where the oracle's own sum_i r_i is zero up to FP64
        # rounding (pair antisymmetry, Eq. 3)
        ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer)
        diff = np.abs(a - ref)
        rnorm = np.linalg.norm(ref, axis=1)
        slack = 1e-12 * rnorm.sum()
        for c in range(3):
            assert abs(m[c] - math.fsum(ref[:, c])) <= diff[:, c].sum() + slack
        assert abs(m[3] - math.fsum(rnorm)) <= np.linalg.norm(a - ref, axis=1).sum() + slack
        say(f"  oracle: sum |r| {math.fsum(rnorm):.17g}, |sum r| / sum |r| "
            f"{np.abs(ref.sum(axis=0)).max() / rnorm.sum():.3g}")


# ---------------------------------------------------------------------------
# the single-accumulator forward mode
# ---------------------------------------------------------------------------

def test_single_accumulator_c2_sampled(anf):
    """C2 in the single mode: within the one-running-sum rounding bound of the
    compensated result on every sampled sink, with its measured error beside
    the compensated one's."""
    boxes = synth.config("C2")
    b = boxes[0]
    sinks = synth.sample_indices(b.n, 10000, 1102 + 7)
    nf = make_nf(anf, boxes)
    bd = nf.bin(upload(boxes))
    got = {}
    for accumulation in ("single", "compensated"):
        acc, _, _ = nf.forces(bd, accumulation)
        got[accumulation] = acc.cpu().numpy()[sinks]
    ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, sinks)
    s_abs, cnt = oracle.force_abs(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, sinks)
    for accumulation, a in got.items():
        say(f"[single] C2 {accumulation}: {err_stats(frac_err(a, ref))}")
    bad = single_sum_bound_violations(got["single"], got["compensated"], ref, s_abs, cnt)
    assert bad == 0


# ---------------------------------------------------------------------------
# C5 adjoint against central differences on every sampled coordinate
# ---------------------------------------------------------------------------

def test_vjp_c5_all_fd_coordinates(anf):
    b = synth.config("C5")[0]
    w = synth.c5_cotangent()
    coords = synth.c5_fd_coords(256)
    say(f"[fd] C5: {len(coords)} coordinates, h = 1e-4, plain and Richardson")
    nf = make_nf(anf, [b])
    bd = nf.bin(torch.from_numpy(b.pos).cuda())
    g = nf.forces_vjp(bd, torch.from_numpy(w).cuda()).cpu().numpy().astype(np.float64)
    h = 1e-4
    plain, rich, plain_ok = [], [], []
    for k, ax in coords:
        k, ax = int(k), int(ax)
        d1 = oracle.fd(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, k, ax, h)
        d2 = oracle.fd(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, k, ax, h / 2)
        dr = (4.0 * d2 - d1) / 3.0
        nk = np.linalg.norm(g[k])
        plain.append(abs(g[k, ax] - d1) / nk)
        rich.append(abs(g[k, ax] - dr) / nk)
        # the plain difference errs by its h^2 truncation term, which d1 - dr
        # estimates; beyond that the adjoint may differ by its own tolerance
        plain_ok.append(abs(g[k, ax] - d1) <= abs(d1 - dr) + VJP_TOL * nk)
    plain, rich = np.array(plain), np.array(rich)
    say(f"  plain D(h):  median {np.median(plain):.3g} max {plain.max():.3g}")
    say(f"  Richardson:  median {np.median(rich):.3g} max {rich.max():.3g}")
    assert all(plain_ok)
    assert np.median(rich) < 1e-5 and rich.max() < 1e-3
