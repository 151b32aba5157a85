"""Slab shares of the forward and adjoint calls (abacus_nf_forces_slab,
abacus_nf_forces_vjp_slab): the sinks of the slabs x in [x_begin, x_end) only,
with sources from their whole stencils (Sec. 3.4.1: one sink slab at a time
with its neighbour slabs resident; Sec. 4.4: a node's range of slabs).

Each slab call must give exactly the bits of the whole-box call on the rows of
its slabs' particles and leave every other row untouched (NaN sentinels).  The
whole-box calls are compared with the oracle by the parity tests.
"""
import sys

import numpy as np
import pytest

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


def slab_rows(bd, boxes, x0, x1):
    """Original indices of the particles in slabs [x0, x1) of every box."""
    off = bd.cell_offsets.cpu().numpy().astype(np.int64)
    perm = bd.perm.cpu().numpy().astype(np.int64)
    rows, cell_base = [], 0
    for b in boxes:
        K = b.cpd
        lo, hi = off[cell_base + x0 * K * K], off[cell_base + x1 * K * K]
        rows.append(perm[lo:hi])
        cell_base += K ** 3
    return np.sort(np.concatenate(rows))


def check_slabs(nf, bd, boxes, cuts, whole, call):
    """Each slab range in `cuts` against the whole-box result; the union of
    the ranges (when they tile [0, K)) reproduces it."""
    n = whole.shape[0]
    union = torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda")
    covered = np.zeros(n, bool)
    for x0, x1 in cuts:
        out = torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda")
        call(x0, x1, out)
        call(x0, x1, union)
        got = out.cpu().numpy()
        rows = slab_rows(bd, boxes, x0, x1)
        mask = np.zeros(n, bool)
        mask[rows] = True
        assert np.array_equal(got[mask].view(np.uint32), whole[mask].view(np.uint32)), (x0, x1)
        assert np.isnan(got[~mask]).all(), (x0, x1)
        covered |= mask
    u = union.cpu().numpy()
    assert np.array_equal(u[covered].view(np.uint32), whole[covered].view(np.uint32))
    assert np.isnan(u[~covered]).all()
    return covered


@pytest.mark.parametrize("accumulation", ["compensated", "chunked", "single"])
def test_forward_slabs_c2(anf, accumulation):
    boxes = synth.config("C2")
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes])
    bd = nf.bin(torch.from_numpy(boxes[0].pos).cuda())
    whole = nf.forces(bd, accumulation)[0].cpu().numpy()
    say(f"[slab] C2 forward {accumulation}: 4 slabs of 8")
    cuts = [(0, 8), (8, 16), (16, 24), (24, 32)]
    covered = check_slabs(nf, bd, boxes, cuts, whole,
                          lambda x0, x1, out: nf.forces_slab(bd, x0, x1, accumulation, out=out))
    assert covered.all()


@pytest.mark.parametrize("law", ["spline", "plummer"])
def test_forward_and_adjoint_slabs_c5(anf, law):
    b = synth.config("C5")[0]
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)], law=law)
    bd = nf.bin(torch.from_numpy(b.pos).cuda())
    w = torch.from_numpy(synth.c5_cotangent()).cuda()
    whole = nf.forces(bd)[0].cpu().numpy()
    whole_g = nf.forces_vjp(bd, w).cpu().numpy()
    say(f"[slab] C5 {law}: uneven slabs, an empty range")
    cuts = [(0, 1), (1, 6), (6, 6), (6, 15), (15, 16)]
    assert check_slabs(nf, bd, [b], cuts, whole,
                       lambda x0, x1, out: nf.forces_slab(bd, x0, x1, out=out)).all()
    assert check_slabs(nf, bd, [b], cuts, whole_g,
                       lambda x0, x1, out: nf.forces_vjp_slab(bd, x0, x1, w, out=out)).all()


def test_slabs_of_a_ragged_batch(anf):
    """One range for every box of a batch (an empty and a one-particle box
    included): each box contributes its own slabs [1, 4)."""
    boxes = [synth.Box(synth.clustered(2500, 6, 8, 13), 1.0, 8, 2, 1 / 500),
             synth.Box(np.zeros((0, 3), np.float32), 1.0, 5, 2, 1 / 500),
             synth.Box(synth.uniform(1, 14), 2.0, 5, 2, 1 / 500),
             synth.Box(synth.clustered(4100, 9, 70, 15), 1.0, 70, 2, 1 / 700),
             synth.Box(synth.uniform(3000, 16, 3.7), 3.7, 11, 2, 3.7 / 640)]
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes])
    pos = torch.from_numpy(np.concatenate([b.pos for b in boxes])).cuda()
    bd = nf.bin(pos)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    w = torch.randn((nf.n_total, 3), generator=gen, dtype=torch.float32, device="cuda")
    whole = nf.forces(bd)[0].cpu().numpy()
    whole_g = nf.forces_vjp(bd, w).cpu().numpy()
    say("[slab] ragged batch: slabs [1, 4) and [0, 1) of every box")
    cuts = [(1, 4), (0, 1)]
    covered = check_slabs(nf, bd, boxes, cuts, whole,
                          lambda x0, x1, out: nf.forces_slab(bd, x0, x1, out=out))
    assert 0 < covered.sum() < nf.n_total
    check_slabs(nf, bd, boxes, cuts, whole_g,
                lambda x0, x1, out: nf.forces_vjp_slab(bd, x0, x1, w, out=out))
