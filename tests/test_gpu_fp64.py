"""GPU parity of the FP64 pair kernel (``abacus_nf_forces_f64``).

On positions that are multiples of 2^-20 in a unit box with K a power of two,
the cell offsets are exact in FP32, so the kernel and the FP64 oracle sum the
same exact separations and differ only by FP64 rounding: per-particle
fractional error below 1e-12 at the median and 1e-9 at the maximum (sums of up
to a few thousand terms with partial cancellation).  On a clustered workload
with arbitrary FP32 positions the stored offsets carry one FP32 rounding, so
the FP64 kernel must simply be no worse than the FP32 kernel against the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import MEDIAN_TOL, P999_TOL, err_stats, frac_err
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


def dyadic(pos):
    q = np.floor(np.asarray(pos, np.float64) * 2.0 ** 20) / 2.0 ** 20
    q[q >= 1.0] = 0.0
    return q.astype(np.float32)


@pytest.mark.parametrize("law", ["spline", "plummer"])
@pytest.mark.parametrize("case", ["clustered_K8", "uniform_K16_R1", "soft_0p6_cell",
                                  "edge_crowd_K8"])
def test_fp64_matches_oracle_to_fp64_rounding(anf, law, case):
    # edge_crowd_K8: 3000 particles in cell (4, 4, 1) beside 8 per cell, so
    # two-cell items pair a long edge run with a short one
    crowd = np.concatenate([synth.uniform(4096, 504),
                            np.array([4.5, 4.5, 1.5]) / 8 +
                            0.08 * (synth.uniform(3000, 505).astype(np.float64) - 0.5)])
    spec = {"clustered_K8": (synth.clustered(6000, 10, 8, 501), 8, 2, 1 / 700),
            "uniform_K16_R1": (synth.uniform(8000, 502), 16, 1, 1 / 1000),
            "soft_0p6_cell": (synth.clustered(4000, 8, 8, 503), 8, 2, 0.6 / 8 / 2.16),
            "edge_crowd_K8": (crowd, 8, 2, 1 / 800)}[case]
    pos, K, R, eps = spec
    pos = dyadic(pos)
    say(f"[fp64] {case} {law}")
    nf = anf.NearField([anf.BoxSpec(pos.shape[0], 1.0, K, R, eps)], law=law)
    bd = nf.bin(torch.from_numpy(pos).cuda())
    _, _, _, rel = oracle.bin(pos, 1.0, K)
    assert np.all(rel[:, :3].astype(np.float64) * 2.0 ** 24 ==
                  np.round(rel[:, :3].astype(np.float64) * 2.0 ** 24))
    acc = nf.forces_f64(bd).cpu().numpy()
    ref, _ = oracle.forces(pos, 1.0, K, R, eps, law=law)
    st = err_stats(frac_err(acc, ref))
    say(f"  {st}")
    assert st["median"] <= 1e-12 and st["max"] <= 1e-9


@pytest.mark.parametrize("law", ["spline", "plummer"])
def test_fp64_on_c2_no_worse_than_fp32(anf, law):
    b = synth.config("C2")[0]
    say(f"[fp64] C2 {law}")
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)], law=law)
    bd = nf.bin(torch.from_numpy(b.pos).cuda())
    a64 = nf.forces_f64(bd).cpu().numpy()
    a32, _, _ = nf.forces(bd)
    a32 = a32.cpu().numpy()
    sinks = synth.sample_indices(b.n, 3000, 1102 + 7)
    ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, sinks, law=law)
    s64 = err_stats(frac_err(a64[sinks], ref))
    s32 = err_stats(frac_err(a32[sinks], ref))
    say(f"  fp64 {s64}\n  fp32 {s32}")
    assert s64["median"] <= MEDIAN_TOL and s64["p999"] <= P999_TOL
    assert s64["median"] <= s32["median"]


def test_fp64_batch_and_ragged(anf):
    boxes = [synth.Box(dyadic(synth.clustered(2500, 6, 8, 13)), 1.0, 8, 2, 1 / 500),
             synth.Box(np.zeros((0, 3), np.float32), 1.0, 4, 1, 1 / 500),
             synth.Box(dyadic(synth.uniform(1, 14)), 1.0, 5, 2, 1 / 500),
             synth.Box(dyadic(synth.clustered(4100, 9, 16, 15)), 1.0, 16, 2, 1 / 700)]
    say("[fp64] ragged batch")
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes])
    pos = np.ascontiguousarray(np.concatenate([b.pos for b in boxes]))
    acc = nf.forces_f64(nf.bin(torch.from_numpy(pos).cuda())).cpu().numpy()
    first = 0
    for b in boxes:
        if b.n > 1:
            ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer)
            st = err_stats(frac_err(acc[first:first + b.n], ref))
            assert st["median"] <= 1e-12 and st["max"] <= 1e-9, st
        elif b.n == 1:
            assert np.all(acc[first] == 0.0)
        first += b.n
