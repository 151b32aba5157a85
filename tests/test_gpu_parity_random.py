"""Seeded random configurations against the FP64 oracle, in full.

Each case is one to three boxes drawn from a seeded generator: near-field
radius R in 0..4 (R = 3 is the largest whose tail items are split into 2R + 1
slices, R = 4 is never split, and a batch of mixed radii is never split),
K from 2R + 1 to 2R + 8, box sides 0.3, 1 and 2.5, 0 to 2500 particles
uniform or clustered, the spline softening from 0.005 to 0.8 cell widths
(above 1/2 cell every cell takes the spline select) and either force law.
Every particle is compared:
  * the debug pair counter equals the exact pair count from the cell counts;
  * forces (compensated): median <= 1e-6 and 99.9th percentile <= 1e-4 over
    particles with a neighbour; exactly 0 for particles without one;
  * adjoint (compensated): relative 2-norm error <= 1e-4.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import MEDIAN_TOL, P999_TOL, VJP_TOL, err_stats, frac_err, pair_count
from paper_2110_11392_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_CASES = 18   # 16 drawn, then two fixed single-box R = 3 cases (7-slice tail splits)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def anf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd as m
    return m


def random_case(i):
    if i == 16:
        return [synth.Box(synth.clustered(3000, 12, 9, 9216), 1.0, 9, 3, 0.02 / 2.16 / 9)], \
            "spline"
    if i == 17:
        return [synth.Box(synth.uniform(2000, 9217, 2.5), 2.5, 8, 3, 0.55 / 2.16 * 2.5 / 8)], \
            "spline"
    rng = np.random.default_rng(9100 + i)
    law = "plummer" if rng.random() < 0.25 else "spline"
    nb = 1 if i % 2 == 0 else int(rng.integers(2, 4))
    boxes = []
    for k in range(nb):
        R = int(rng.integers(0, 5))
        K = int(rng.integers(2 * R + 1, 2 * R + 9))
        L = float(rng.choice([1.0, 2.5, 0.3]))
        n = int(rng.integers(0, 2501)) if rng.random() < 0.9 else 0
        seed = 9200 + 10 * i + k
        if rng.random() < 0.5:
            pos = synth.uniform(n, seed, L)
        else:
            pos = synth.clustered(n, max(1, n // 200), K, seed, L)
        eps_cells = float(np.exp(rng.uniform(np.log(0.005), np.log(0.8))))
        boxes.append(synth.Box(pos, L, K, R, eps_cells / 2.16 * L / K))
    return boxes, law


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_configuration(anf, case):
    boxes, law = random_case(case)
    desc = ", ".join(f"n={b.n} K={b.cpd} R={b.radius} L={b.box}" for b in boxes)
    say(f"[random {case}] {law}: {desc}")
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes],
                       law=law)
    pos = np.ascontiguousarray(np.concatenate([b.pos for b in boxes]))
    bd = nf.bin(torch.from_numpy(pos).cuda())
    bd.check_status()
    w = synth.gaussian_weights(nf.n_total, 9300 + case)
    acc, _, pairs = nf.forces(bd, count_pairs=True)
    grad = nf.forces_vjp(bd, torch.from_numpy(w).cuda())
    acc, grad, pairs = acc.cpu().numpy(), grad.cpu().numpy(), int(pairs.item())
    assert pairs == pair_count(boxes)
    refs, grefs = [], []
    first = 0
    for b in boxes:
        if b.n:
            refs.append(oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, law=law)[0])
            grefs.append(oracle.vjp(b.pos, w[first:first + b.n], b.box, b.cpd, b.radius,
                                    b.eps_plummer, law=law))
        first += b.n
    if not refs:
        return
    ref, gref = np.concatenate(refs), np.concatenate(grefs)
    alone = np.linalg.norm(ref, axis=1) == 0
    assert (acc[alone] == 0).all() and (grad[alone] == 0).all()
    if (~alone).any():
        st = err_stats(frac_err(acc[~alone], ref[~alone]))
        rel_g = np.linalg.norm(grad - gref) / np.linalg.norm(gref)
        say(f"  forces {st}; adjoint relative error {rel_g:.3g}")
        assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL
        assert rel_g <= VJP_TOL


def dyadic(pos):
    q = np.floor(np.asarray(pos, np.float64) * 2.0 ** 20) / 2.0 ** 20
    q[q >= 1.0] = 0.0
    return q.astype(np.float32)


# FP64 kernels at the radii and grids above, on dyadic positions (L = 1, K a
# power of two): the stored FP32 cell offsets are then exact, so the FP64
# kernels must match the oracle to FP64 rounding, forces within 1e-12 at the
# median and 1e-9 at the maximum, the adjoint within 1e-12 in relative 2-norm.
FP64_CASES = {
    "K1_R0": [(2000, 1, 0, 0.02)],
    "K2_R0": [(1500, 2, 0, 0.3)],
    "K8_R3": [(3000, 8, 3, 0.01)],
    "K16_R4": [(3000, 16, 4, 0.04)],
    "mixed_R": [(1200, 4, 1, 0.05), (0, 2, 0, 0.1), (2500, 8, 3, 0.7), (1800, 16, 4, 0.01)],
}


@pytest.mark.parametrize("law", ["spline", "plummer"])
@pytest.mark.parametrize("name", list(FP64_CASES))
def test_fp64_radii_and_grids(anf, name, law):
    specs = FP64_CASES[name]
    boxes = [synth.Box(dyadic(synth.clustered(n, max(1, n // 300), K, 9400 + k)), 1.0, K, R,
                       eps_cells / 2.16 / K)
             for k, (n, K, R, eps_cells) in enumerate(specs)]
    say(f"[random fp64] {name} {law}")
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes],
                       law=law)
    bd = nf.bin(torch.from_numpy(np.ascontiguousarray(np.concatenate([b.pos for b in boxes])))
                .cuda())
    w32 = synth.gaussian_weights(nf.n_total, 9500)
    w = w32.astype(np.float64)   # the same values: the oracle takes them in FP32
    acc = nf.forces_f64(bd).cpu().numpy()
    grad = nf.forces_vjp_f64(bd, torch.from_numpy(w).cuda()).cpu().numpy()
    first = 0
    for b in boxes:
        if b.n:
            sl = slice(first, first + b.n)
            ref, _ = oracle.forces(b.pos, 1.0, b.cpd, b.radius, b.eps_plummer, law=law)
            gref = oracle.vjp(b.pos, w32[sl], 1.0, b.cpd, b.radius, b.eps_plummer, law=law)
            st = err_stats(frac_err(acc[sl], ref))
            rel2 = np.linalg.norm(grad[sl] - gref) / np.linalg.norm(gref)
            say(f"  n={b.n} K={b.cpd} R={b.radius}: forces {st}; adjoint relative 2-norm "
                f"{rel2:.3g}")
            assert st["median"] <= 1e-12 and st["max"] <= 1e-9
            assert rel2 <= 1e-12
        first += b.n
