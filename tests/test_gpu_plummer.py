"""GPU parity of the Plummer force law (Eq. 2, ``ABACUS_NF_PLUMMER``).

With the Plummer flag every pair takes f = (r^2 + eps_p^2)^(-3/2): the same
instruction sequence as the Newton branch of the spline law, with eps_p^2 in
place of the tiny r^2 guard.  Checks against the FP64 oracle with law="plummer":
  * forces: fractional error median <= 1e-6 and 99.9th percentile <= 1e-4;
  * adjoint: relative 2-norm error <= 1e-4, and against finite differences;
  * launch shapes give bit-identical results, as for the spline law;
  * the law flag changes the answer (the spline result differs).
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import MEDIAN_TOL, P999_TOL, VJP_TOL, err_stats, frac_err
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


def bits(t):
    return t.detach().cpu().numpy().view(np.uint32)


def make(anf, boxes, law="plummer"):
    specs = [anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes]
    nf = anf.NearField(specs, law=law)
    pos = torch.from_numpy(np.ascontiguousarray(np.concatenate([b.pos for b in boxes]))).cuda()
    return nf, nf.bin(pos)


CASES = {
    "C1": lambda: synth.config("C1"),
    "clustered_K9_R1": lambda: [synth.Box(synth.clustered(5000, 12, 9, 10), 1.0, 9, 1, 1 / 700)],
    # softening of several cells: the Plummer core spans the whole stencil
    "wide_soft_K8": lambda: [synth.Box(synth.clustered(3000, 10, 8, 16), 1.0, 8, 2, 0.3)],
    "batch_ragged": lambda: [synth.Box(synth.clustered(2500, 6, 8, 13), 1.0, 8, 2, 1 / 500),
                             synth.Box(np.zeros((0, 3), np.float32), 1.0, 5, 2, 1 / 500),
                             synth.Box(synth.uniform(1, 14), 2.0, 5, 2, 1 / 500),
                             synth.Box(synth.clustered(4100, 9, 10, 15), 1.0, 10, 2, 1 / 700)],
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("accumulation", ["compensated", "chunked"])
def test_plummer_forces_small(anf, name, accumulation):
    boxes = CASES[name]()
    say(f"[plummer forces] {name} {accumulation}")
    nf, bd = make(anf, boxes)
    acc, _, _ = nf.forces(bd, accumulation)
    acc = acc.cpu().numpy()
    first = 0
    errs = []
    for b in boxes:
        if b.n:
            ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, law="plummer")
            errs.append(frac_err(acc[first:first + b.n], ref))
        first += b.n
    e = np.concatenate(errs)
    st = err_stats(e)
    say(f"  {st}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL


def test_plummer_differs_from_spline(anf):
    boxes = synth.config("C1")
    nf_p, bd_p = make(anf, boxes)
    nf_s, bd_s = make(anf, boxes, law="spline")
    a_p, _, _ = nf_p.forces(bd_p)
    a_s, _, _ = nf_s.forces(bd_s)
    assert not np.allclose(a_p.cpu().numpy(), a_s.cpu().numpy(), rtol=1e-4)


def test_plummer_c2_sampled(anf):
    boxes = synth.config("C2")
    b = boxes[0]
    say(f"[plummer forces] C2 n={b.n}")
    nf, bd = make(anf, boxes)
    acc, _, _ = nf.forces(bd)
    sinks = synth.sample_indices(b.n, 4000, 1102 + 7)
    ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer, sinks, law="plummer")
    st = err_stats(frac_err(acc.cpu().numpy()[sinks], ref))
    say(f"  {st}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL


def test_plummer_vjp_c5_against_oracle_and_fd(anf):
    boxes = synth.config("C5")
    b = boxes[0]
    w = synth.c5_cotangent()
    say(f"[plummer vjp] C5 n={b.n}")
    nf, bd = make(anf, boxes)
    g = nf.forces_vjp(bd, torch.from_numpy(w).cuda()).cpu().numpy().astype(np.float64)
    sinks = synth.sample_indices(b.n, 3000, 4242)
    ref = oracle.vjp(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, sinks, law="plummer")
    rel = np.linalg.norm(g[sinks] - ref) / np.linalg.norm(ref)
    say(f"  relative 2-norm error {rel:.3e}")
    assert rel <= VJP_TOL
    # central differences in FP64 (h = 1e-4), Richardson-extrapolated
    fd_err = []
    for k, a in synth.c5_fd_coords(64):
        d = oracle.fd_richardson(b.pos, w, b.box, b.cpd, b.radius, b.eps_plummer, int(k),
                                 int(a), 1e-4, law="plummer")
        fd_err.append(abs(g[k, a] - d) / np.linalg.norm(g[k]))
    fd_err = np.array(fd_err)
    say(f"  vs Richardson FD: median {np.median(fd_err):.3g} max {fd_err.max():.3g}")
    assert np.median(fd_err) < 1e-5 and fd_err.max() < 1e-3


def test_plummer_launch_shapes_bit_identical(anf):
    boxes = synth.config("C5")
    nf, bd = make(anf, boxes)
    w = torch.from_numpy(synth.c5_cotangent()).cuda()
    ref_a, _, _ = nf.forces(bd)
    ref_g = nf.forces_vjp(bd, w)
    ref_a, ref_g = bits(ref_a), bits(ref_g)
    try:
        for shape in (dict(unroll=2, pipeline=1, span=1, grid_mult=1, split=1),
                      dict(unroll=8, pipeline=0, span=3, grid_mult=2, split=0)):
            say(f"[plummer shape] {shape}")
            nf.set_tuning(0, shape)
            nf.set_tuning(1, dict(shape, unroll=min(shape["unroll"], 4), grid_mult=1))
            a, _, _ = nf.forces(bd)
            g = nf.forces_vjp(bd, w)
            assert np.array_equal(bits(a), ref_a), shape
            assert np.array_equal(bits(g), ref_g), shape
    finally:
        nf.set_tuning(0, None)
        nf.set_tuning(1, None)


def test_plummer_autograd_matches_oracle(anf):
    b = synth.config("C1")[0]
    pos = torch.from_numpy(b.pos).cuda().requires_grad_(True)
    acc = anf.near_field(pos, b.box, b.cpd, b.radius, b.eps_plummer, law="plummer")
    w = torch.from_numpy(synth.gaussian_weights(b.n, 5)).cuda()
    (acc * w).sum().backward()
    ref = oracle.vjp(b.pos, w.cpu().numpy(), b.box, b.cpd, b.radius, b.eps_plummer,
                     law="plummer")
    g = pos.grad.cpu().numpy()
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= VJP_TOL
