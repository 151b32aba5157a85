"""GPU parity of the HIP near-field path against the FP64 oracle.

Every test calls the library through its C ABI (via the ctypes binding) and
compares with ``oracle/`` on the same seeded inputs:
  * binning: bit-exact (cell offsets, permutation, FP32 offsets);
  * forces: fractional error median <= 1e-6 and 99.9th percentile <= 1e-4;
  * adjoint: relative 2-norm error <= 1e-4 against the FP64 gradient;
  * pair coverage: the debug counter equals sum_c n_c S_c - N exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import (MEDIAN_TOL, P999_TOL, VJP_TOL, err_stats, frac_err, oracle_abs_boxes,
                        oracle_bin_boxes, pair_count, single_sum_bound_violations)
from paper_2110_11392_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nfmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd as anf
    return anf


def make_nf(anf, boxes):
    specs = [anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes]
    return anf.NearField(specs)


def upload(boxes):
    pos = np.concatenate([b.pos for b in boxes], axis=0) if boxes else np.zeros((0, 3), np.float32)
    return torch.from_numpy(np.ascontiguousarray(pos)).cuda()


def small_boxes():
    return {
        "C1": synth.config("C1"),
        "uniform_K7": [synth.Box(synth.uniform(3001, 9), 1.0, 7, 2, 1 / 600)],
        "clustered_K9_R1": [synth.Box(synth.clustered(5000, 12, 9, 10), 1.0, 9, 1, 1 / 700)],
        "one_cell_crowd": [synth.Box((np.float32(0.5) + np.float32(0.001) *
                                      synth.uniform(1500, 11)).astype(np.float32),
                                     1.0, 8, 2, 1 / 2000)],
        "box_3p7_K11": [synth.Box(synth.uniform(4000, 12, 3.7), 3.7, 11, 2, 3.7 / 640)],
        # K = 2R + 1: the cell R below an item's lower cell is the cell R above
        # its upper cell, so the paired edge runs of two-cell items coincide
        "clustered_K5_edges": [synth.Box(synth.clustered(3000, 8, 5, 18), 1.0, 5, 2, 1 / 400)],
        "clustered_K6_edges": [synth.Box(synth.clustered(3500, 8, 6, 19), 1.0, 6, 2, 1 / 450)],
        # 3000 particles in cell (4, 4, 1) beside 8 per cell elsewhere: two-cell
        # items of pencil (4, 4) pair a 3000-particle edge run with an 8-particle
        # one (47 chunks, one lane set active after the first)
        "edge_crowd_K8": [synth.Box(np.concatenate([
            synth.uniform(4096, 20),
            (np.array([4.5, 4.5, 1.5], np.float32) / np.float32(8) +
             np.float32(0.08) * (synth.uniform(3000, 21) - np.float32(0.5))).astype(np.float32)]),
            1.0, 8, 2, 1 / 800)],
        # softening just below / above half a cell: the Newton-only path for
        # cells two apart is on / off
        "soft_0p45_cell": [synth.Box(synth.clustered(3000, 10, 8, 16), 1.0, 8, 2,
                                     0.45 / 8 / 2.16)],
        "soft_0p60_cell": [synth.Box(synth.clustered(3000, 10, 8, 17), 1.0, 8, 2,
                                     0.60 / 8 / 2.16)],
        "batch_ragged": [synth.Box(synth.clustered(2500, 6, 8, 13), 1.0, 8, 2, 1 / 500),
                         synth.Box(np.zeros((0, 3), np.float32), 1.0, 5, 2, 1 / 500),
                         synth.Box(synth.uniform(1, 14), 2.0, 5, 2, 1 / 500),
                         synth.Box(synth.clustered(4100, 9, 10, 15), 1.0, 10, 2, 1 / 700)],
    }


# ---------------------------------------------------------------------------
# binning
# ---------------------------------------------------------------------------

def check_bin(anf, boxes, label):
    say(f"[bin] {label}: n={sum(b.n for b in boxes)} boxes={len(boxes)}")
    nf = make_nf(anf, boxes)
    bd = nf.bin(upload(boxes))
    torch.cuda.synchronize()
    o_off, o_perm, o_rel = oracle_bin_boxes(boxes)
    assert int(bd.status.item()) == 0
    assert np.array_equal(bd.cell_offsets.cpu().numpy(), o_off)
    assert np.array_equal(bd.perm.cpu().numpy(), o_perm)
    assert np.array_equal(bd.rel.cpu().numpy().view(np.uint32), o_rel.view(np.uint32))


@pytest.mark.parametrize("name", list(small_boxes().keys()))
def test_bin_bit_exact_small(nfmod, name):
    check_bin(nfmod, small_boxes()[name], name)


@pytest.mark.parametrize("name", ["C5", "C2"])
def test_bin_bit_exact_configs(nfmod, name):
    check_bin(nfmod, synth.config(name), name)


def many_boxes(count):
    rng = np.random.default_rng(31)
    boxes = []
    for k in range(count):
        K = int(rng.integers(1, 7))
        n = int(rng.integers(0, 40))
        L = float(rng.choice([0.5, 1.0, 3.0]))
        boxes.append(synth.Box(synth.uniform(n, 3100 + k, L), L, K, (K - 1) // 2, L / K / 50))
    return boxes


@pytest.mark.parametrize("count", [1000, 1100])
def test_bin_and_forces_of_many_boxes(nfmod, count):
    """Batches of 1000 and 1100 small boxes (0 to 39 particles, K 1..6): the
    binning's box lookup reads the boxes' first particles from LDS up to 1024
    boxes and searches the box table itself beyond; both are bit-exact, and the
    forces of every particle match the oracle."""
    boxes = many_boxes(count)
    check_bin(nfmod, boxes, f"{count} boxes")
    acc, _, pairs = gpu_forces(nfmod, boxes, count_pairs=True)
    assert pairs == pair_count(boxes)
    ref, idx = oracle_forces_boxes(boxes)
    alone = np.linalg.norm(ref, axis=1) == 0
    assert (acc[idx[alone]] == 0).all()
    st = err_stats(frac_err(acc[idx[~alone]], ref[~alone]))
    say(f"  forces {st}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL


@pytest.mark.parametrize("label,boxes", [
    # no particle at all: every offset is 0
    ("all_empty", [synth.Box(np.zeros((0, 3), np.float32), 1.0, 5, 2, 1 / 500),
                   synth.Box(np.zeros((0, 3), np.float32), 2.0, 6, 2, 1 / 500)]),
    # one cell per box (R = 0, K = 1): the sort has no pass at all
    ("single_cell", [synth.Box(synth.uniform(300, 21), 1.0, 1, 0, 1 / 500)]),
    # empty cells before the first and after the last occupied cell
    ("sparse_corner", [synth.Box((np.float32(0.95) + np.float32(0.04) *
                                  synth.uniform(200, 22)).astype(np.float32), 1.0, 9, 2, 1 / 900)]),
])
def test_bin_offsets_edge_cases(nfmod, label, boxes):
    check_bin(nfmod, boxes, label)


def test_bin_adversarial_faces_and_wrap(nfmod):
    K = 8
    rng = np.random.default_rng(3)
    faces = (rng.integers(-2 * K, 3 * K, size=(3000, 3)) / K).astype(np.float32)
    tiny = (rng.integers(-3, 4, size=(500, 3)) * np.float32(1e-30)).astype(np.float32)
    near_one = np.nextafter(np.float32(1.0), np.float32(0.0)) * np.ones((10, 3), np.float32)
    pos = np.concatenate([faces, tiny, near_one, np.ones((3, 3), np.float32)])
    check_bin(nfmod, [synth.Box(pos, 1.0, K, 2, 1 / 640)], "faces/wrap")


def test_bin_flags_bad_positions(nfmod):
    pos = synth.uniform(1000, 21)
    pos[17, 2] = np.nan
    pos[400, 0] = np.inf
    nf = make_nf(nfmod, [synth.Box(pos, 1.0, 8, 2, 1 / 640)])
    bd = nf.bin(upload([synth.Box(pos, 1.0, 8, 2, 1 / 640)]))
    with pytest.raises(ValueError):
        bd.check_status()
    good = synth.uniform(1000, 22)
    bd = nf.bin(torch.from_numpy(good).cuda())
    bd.check_status()


# ---------------------------------------------------------------------------
# forward forces
# ---------------------------------------------------------------------------

def gpu_forces(anf, boxes, accumulation="compensated", momentum=False, count_pairs=False):
    nf = make_nf(anf, boxes)
    bd = nf.bin(upload(boxes))
    acc, mom, pairs = nf.forces(bd, accumulation, momentum=momentum, count_pairs=count_pairs)
    torch.cuda.synchronize()
    return (acc.cpu().numpy(), None if mom is None else mom.cpu().numpy(),
            None if pairs is None else int(pairs.item()))


def oracle_forces_boxes(boxes, sinks_per_box=None):
    """Oracle accelerations; sinks_per_box[b] = local indices or None (all)."""
    refs, idx = [], []
    first = 0
    for k, b in enumerate(boxes):
        s = None if sinks_per_box is None else sinks_per_box[k]
        if b.n == 0:
            continue
        a, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, s)
        refs.append(a)
        idx.append(first + (np.arange(b.n) if s is None else np.asarray(s)))
        first += b.n
    return np.concatenate(refs), np.concatenate(idx)


@pytest.mark.parametrize("name", list(small_boxes().keys()))
@pytest.mark.parametrize("accumulation", ["compensated", "chunked", "single"])
def test_forces_small_full(nfmod, name, accumulation):
    anf = nfmod
    boxes = small_boxes()[name]
    say(f"[forces] {name} {accumulation}")
    acc, _, pairs = gpu_forces(anf, boxes, accumulation, count_pairs=True)
    assert pairs == pair_count(boxes)
    ref, idx = oracle_forces_boxes(boxes)
    e = frac_err(acc[idx], ref)
    st = err_stats(e)
    say(f"  errors {st}")
    assert np.all(np.isfinite(acc))
    if accumulation != "single":
        assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL
    else:
        # one FP32 running sum per sink: within the recursive-summation bound
        # of the compensated result (derivation in gpu_common)
        comp, _, _ = gpu_forces(anf, boxes, "compensated")
        s_abs, cnt = oracle_abs_boxes(boxes)
        assert single_sum_bound_violations(acc[idx], comp[idx], ref, s_abs, cnt) == 0


@pytest.mark.parametrize("name", ["C5", "C2", "C3"])
def test_forces_configs_sampled(nfmod, name):
    boxes = synth.config(name)
    b = boxes[0]
    sinks = synth.sample_indices(b.n, 10000, 1100 + int(name[1]) + 7)
    say(f"[forces] {name} n={b.n} sampled={sinks.size}")
    res = {}
    for accumulation in ("compensated", "chunked"):
        acc, mom, _ = gpu_forces(nfmod, boxes, accumulation, momentum=True)
        res[accumulation] = (acc, mom)
    ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, sinks)
    for accumulation, (acc, mom) in res.items():
        st = err_stats(frac_err(acc[sinks], ref))
        resid = np.abs(mom[0, :3]).max() / mom[0, 3]
        say(f"  {accumulation}: {st} momentum residual {resid:.3g}")
        assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL
        assert resid < 1e-5


def test_pair_count_c2(nfmod):
    boxes = synth.config("C2")
    say("[pairs] C2")
    _, _, pairs = gpu_forces(nfmod, boxes, count_pairs=True)
    assert pairs == pair_count(boxes)


def test_forces_deterministic_and_translation_invariant(nfmod):
    K = 16
    rng = np.random.default_rng(77)
    pos = (rng.integers(0, 2 ** 20, size=(60000, 3)) / 2 ** 20).astype(np.float32)
    # a dense clump, kept on a dyadic grid so that whole-cell shifts stay exact in FP32
    pos[:20000] = (np.float32(0.3125) + (pos[:20000] - np.float32(0.5)) * np.float32(0.0625))
    shift = np.array([5, -3, 7]) / K
    moved = np.mod(pos.astype(np.float64) + shift, 1.0).astype(np.float32)
    assert np.array_equal(np.mod(moved.astype(np.float64) - shift, 1.0).astype(np.float32), pos)
    b0 = [synth.Box(pos, 1.0, K, 2, 1 / 1500)]
    b1 = [synth.Box(moved, 1.0, K, 2, 1 / 1500)]
    say("[determinism/translation] n=60000 K=16")
    a0, _, _ = gpu_forces(nfmod, b0)
    a0b, _, _ = gpu_forces(nfmod, b0)
    a1, _, _ = gpu_forces(nfmod, b1)
    assert np.array_equal(a0.view(np.uint32), a0b.view(np.uint32))
    assert np.array_equal(a0.view(np.uint32), a1.view(np.uint32))


def test_batched_equals_single_boxes(nfmod):
    boxes = synth.config("C4", scale=6)
    say(f"[batch] C4 first 6 boxes n={[b.n for b in boxes]}")
    acc_b, mom_b, _ = gpu_forces(nfmod, boxes, momentum=True)
    first = 0
    for k, b in enumerate(boxes):
        a, m, _ = gpu_forces(nfmod, [b], momentum=True)
        assert np.array_equal(acc_b[first:first + b.n].view(np.uint32), a.view(np.uint32))
        assert np.array_equal(mom_b[k], m[0])
        first += b.n
    sinks = [synth.sample_indices(b.n, 1500, 1104 + 7 + k) for k, b in enumerate(boxes)]
    ref, idx = oracle_forces_boxes(boxes, sinks)
    st = err_stats(frac_err(acc_b[idx], ref))
    say(f"  errors {st}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def test_vjp_c5_against_oracle_and_fd(nfmod):
    b = synth.config("C5")[0]
    w = synth.c5_cotangent()
    coords = synth.c5_fd_coords(256)
    say("[vjp] C5")
    nf = make_nf(nfmod, [b])
    bd = nf.bin(torch.from_numpy(b.pos).cuda())
    g = nf.forces_vjp(bd, torch.from_numpy(w).cuda()).cpu().numpy()
    sinks = synth.sample_indices(b.n, 20000, 1105 + 9)
    ref = oracle.vjp(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, sinks)
    rel = np.linalg.norm(g[sinks] - ref) / np.linalg.norm(ref)
    st = err_stats(frac_err(g[sinks], ref))
    say(f"  relative 2-norm error {rel:.3g}; per particle {st}")
    assert rel <= VJP_TOL
    # central differences in FP64 (h = 1e-4), Richardson-extrapolated
    fd_err = []
    for k, a in coords[:64]:
        d = oracle.fd_richardson(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, int(k),
                                 int(a), 1e-4)
        fd_err.append(abs(g[k, a] - d) / np.linalg.norm(g[k]))
    fd_err = np.array(fd_err)
    say(f"  vs Richardson FD: median {np.median(fd_err):.3g} max {fd_err.max():.3g}")
    assert np.median(fd_err) < 1e-5 and fd_err.max() < 1e-3


def test_vjp_small_all_modes(nfmod):
    boxes = small_boxes()["batch_ragged"]
    say("[vjp] batch_ragged")
    nf = make_nf(nfmod, boxes)
    pos = upload(boxes)
    bd = nf.bin(pos)
    n = pos.shape[0]
    w = synth.gaussian_weights(n, 99)
    refs = []
    first = 0
    for b in boxes:
        if b.n:
            refs.append(oracle.vjp(b.pos, w[first:first + b.n], b.box, b.cpd, b.radius,
                                   b.eps_plummer))
        first += b.n
    ref = np.concatenate(refs)
    for accumulation in ("compensated", "chunked", "single"):
        g = nf.forces_vjp(bd, torch.from_numpy(w).cuda(), accumulation).cpu().numpy()
        rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        say(f"  {accumulation}: relative error {rel:.3g}")
        assert rel <= VJP_TOL


@pytest.mark.parametrize("name", ["edge_crowd_K8", "clustered_K5_edges", "clustered_K6_edges"])
def test_vjp_paired_edge_runs(nfmod, name):
    """Adjoint on boxes whose two-cell items pair edge runs of very different
    lengths (a crowded cell against sparse ones) or where the two edge cells
    are one cell (K = 2R + 1), in every accumulation mode."""
    boxes = small_boxes()[name]
    b = boxes[0]
    say(f"[vjp] {name}")
    nf = make_nf(nfmod, boxes)
    bd = nf.bin(upload(boxes))
    w = synth.gaussian_weights(b.n, 98)
    ref = oracle.vjp(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer)
    for accumulation in ("compensated", "chunked", "single"):
        g = nf.forces_vjp(bd, torch.from_numpy(w).cuda(), accumulation).cpu().numpy()
        rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        st = err_stats(frac_err(g, ref))
        say(f"  {accumulation}: relative error {rel:.3g} per particle {st}")
        assert rel <= VJP_TOL
        if accumulation != "single":
            assert st["median"] <= 1e-5


@pytest.mark.parametrize("name", ["one_cell_crowd", "soft_0p60_cell", "clustered_K9_R1"])
def test_vjp_pairs_inside_softening(nfmod, name):
    """Adjoint where many pairs lie inside eps_s (the crowd has nearly all of
    them there), so the spline branch's F (v + T d) with T = h (d.v) / f is
    exercised, not only the Newton one; per-particle check against the oracle."""
    boxes = small_boxes()[name]
    say(f"[vjp] {name}")
    nf = make_nf(nfmod, boxes)
    bd = nf.bin(upload(boxes))
    b = boxes[0]
    w = synth.gaussian_weights(b.n, 123)
    ref = oracle.vjp(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer)
    g = nf.forces_vjp(bd, torch.from_numpy(w).cuda()).cpu().numpy()
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    per = np.linalg.norm(g - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    say(f"  relative error {rel:.3g}, per-particle median {np.median(per):.3g}, "
        f"99.9% {np.percentile(per, 99.9):.3g}")
    assert rel <= VJP_TOL
    assert np.median(per) <= 1e-5


@pytest.mark.parametrize("accumulation", ["compensated", "chunked", "single"])
def test_autograd_matches_vjp(nfmod, accumulation):
    b = synth.config("C1")[0]
    pos = torch.from_numpy(b.pos).cuda().requires_grad_(True)
    acc = nfmod.near_field(pos, b.box, b.cpd, b.radius, b.eps_plummer, accumulation)
    w = torch.from_numpy(synth.gaussian_weights(b.n, 5)).cuda()
    (acc * w).sum().backward()
    # the autograd form is the library's forward and adjoint in that mode
    nf = make_nf(nfmod, [b])
    bd = nf.bin(torch.from_numpy(b.pos).cuda())
    direct, _, _ = nf.forces(bd, accumulation)
    assert torch.equal(acc.detach(), direct)
    ref = oracle.vjp(b.pos, w.cpu().numpy(), b.box, b.cpd, b.radius, b.eps_plummer)
    g = pos.grad.cpu().numpy()
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= VJP_TOL
    with pytest.raises(ValueError):
        nfmod.near_field(pos, b.box, b.cpd, b.radius, b.eps_plummer, "kahan")
