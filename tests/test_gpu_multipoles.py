"""GPU parity of the cell multipoles (Eq. 4) against the FP64 oracle.

Both sides sum the same FP32 cell-relative offsets (the binning is bit-exact)
in FP64, so the only differences are rounding order: each complete term must
agree within 1e-13 of the sum of the absolute values of its summands, and each
reduced term within 1e-11 of the largest such sum in its cell row (the reduction
combines up to a few dozen terms with integer-ratio coefficients).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2110_11392_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def anf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd as m
    return m


def complete_indices(p):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


def abs_sums(b, p):
    """Per cell and complete term, sum_q |x^a y^b z^c| (box units) from the
    oracle's binning."""
    _, offs, _, rel = oracle.bin(b.pos, b.box, b.cpd)
    w = b.box / b.cpd
    d = np.abs(rel[:, :3].astype(np.float64)) * w
    cell = np.repeat(np.arange(b.cpd ** 3), np.diff(offs))
    out = np.zeros((b.cpd ** 3, len(complete_indices(p))))
    for k, (a, bb, c) in enumerate(complete_indices(p)):
        out[:, k] = np.bincount(cell, weights=d[:, 0] ** a * d[:, 1] ** bb * d[:, 2] ** c,
                                minlength=b.cpd ** 3)
    return out


def run(anf, boxes, p, reduced):
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes])
    pos = torch.from_numpy(np.ascontiguousarray(np.concatenate([b.pos for b in boxes]))).cuda()
    bd = nf.bin(pos)
    return nf, bd, nf.multipoles(bd, p, reduced).cpu().numpy()


def check(boxes, p, reduced, got):
    row = 0
    for b in boxes:
        ncell = b.cpd ** 3
        ref = oracle.multipoles(b.pos, b.box, b.cpd, p, reduced)
        mine = got[row:row + ncell]
        sums = abs_sums(b, p)
        if reduced:
            tol = 1e-11 * sums.max(axis=1, keepdims=True) + 1e-300
        else:
            tol = 1e-13 * sums + 1e-300
        err = np.abs(mine - ref)
        bad = np.argwhere(err > tol)
        assert bad.size == 0, (b.n, p, reduced, bad[:5], mine[tuple(bad[0])], ref[tuple(bad[0])])
        row += ncell
    assert row == got.shape[0]


def crowd():
    # 1500 particles in one cell: the cell takes all 64 lanes of a wave
    return [synth.Box((np.float32(0.5) + np.float32(0.001) * synth.uniform(1500, 11))
                      .astype(np.float32), 1.0, 8, 2, 1 / 2000)]


CASES = {
    "C1": lambda: synth.config("C1"),
    "clustered_K9": lambda: [synth.Box(synth.clustered(5000, 12, 9, 10), 1.0, 9, 1, 1 / 700)],
    "one_cell_crowd": crowd,
    "box_3p7_K11": lambda: [synth.Box(synth.uniform(4000, 12, 3.7), 3.7, 11, 2, 3.7 / 640)],
    "batch_ragged": lambda: [synth.Box(synth.clustered(2500, 6, 8, 13), 1.0, 8, 2, 1 / 500),
                             synth.Box(np.zeros((0, 3), np.float32), 1.0, 5, 2, 1 / 500),
                             synth.Box(synth.uniform(1, 14), 2.0, 5, 2, 1 / 500),
                             synth.Box(synth.clustered(4100, 9, 70, 15), 1.0, 70, 2, 1 / 700)],
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("reduced", [False, True])
def test_multipoles_order8_small(anf, name, reduced):
    boxes = CASES[name]()
    say(f"[multipoles] {name} p=8 reduced={reduced}")
    _, _, got = run(anf, boxes, 8, reduced)
    check(boxes, 8, reduced, got)


@pytest.mark.parametrize("p", range(0, 9))
def test_multipoles_every_order(anf, p):
    boxes = [synth.Box(synth.clustered(3000, 10, 7, 300 + p), 1.0, 7, 2, 1 / 500)]
    say(f"[multipoles] orders p={p}")
    for reduced in (False, True):
        _, _, got = run(anf, boxes, p, reduced)
        check(boxes, p, reduced, got)


def test_multipoles_c2_full_and_deterministic(anf):
    boxes = synth.config("C2")
    say(f"[multipoles] C2 n={boxes[0].n} p=8")
    nf, bd, got = run(anf, boxes, 8, False)
    check(boxes, 8, False, got)
    again = nf.multipoles(bd, 8).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), again.view(np.uint64))
    red = nf.multipoles(bd, 8, reduced=True).cpu().numpy()
    check(boxes, 8, True, red)


def test_multipoles_reject_bad_arguments(anf):
    boxes = synth.config("C1")
    nf, bd, _ = run(anf, boxes, 2, False)
    with pytest.raises(Exception):
        nf.multipoles(bd, 9)
    with pytest.raises(Exception):
        nf.multipoles(bd, -1)


def random_boxes(i):
    """One to three boxes from a seeded generator: K 1..12 (R plays no part in
    the multipoles), sides 0.3, 1 and 2.5, 0 to 3000 particles uniform,
    clustered or piled into a few cells."""
    rng = np.random.default_rng(9600 + i)
    boxes = []
    for k in range(int(rng.integers(1, 4))):
        K = int(rng.integers(1, 13))
        L = float(rng.choice([0.3, 1.0, 2.5]))
        n = int(rng.integers(0, 3001))
        seed = 9700 + 10 * i + k
        kind = int(rng.integers(3))
        if kind == 0:
            pos = synth.uniform(n, seed, L)
        elif kind == 1:
            pos = synth.clustered(n, max(1, n // 250), K, seed, L)
        else:   # a few crowded cells: up to n particles in one cell
            pos = ((np.float32(0.5) + np.float32(0.004) * synth.uniform(n, seed)) *
                   np.float32(L)).astype(np.float32)
        boxes.append(synth.Box(pos, L, K, 0, L / K / 100))
    return boxes


@pytest.mark.parametrize("i", range(8))
def test_multipoles_random(anf, i):
    boxes = random_boxes(i)
    p = int(np.random.default_rng(9800 + i).integers(0, 9))
    say(f"[multipoles] random {i} p={p}: " +
        ", ".join(f"n={b.n} K={b.cpd} L={b.box}" for b in boxes))
    for reduced in (False, True):
        _, _, got = run(anf, boxes, p, reduced)
        check(boxes, p, reduced, got)
