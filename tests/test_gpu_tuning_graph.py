"""GPU checks of the launch-shape tuning and of graph capture.

* Every launch shape sums each sink's pairs in the same order, so forces and
  adjoint must be bit-identical across shapes (and after autotuning).
* The whole step (binning, forces, adjoint) captured in one HIP graph must
  reproduce eager results bit for bit on every replay, with new positions
  written into the captured input buffer between replays and eager work
  interleaved.
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


def bits(t):
    return t.detach().cpu().numpy().view(np.uint32)


FORWARD_SHAPES = [dict(unroll=u, pipeline=p, span=s, grid_mult=g, split=x)
                  for u in (2, 4, 8) for p in (0, 1) for s in (1, 2, 3) for g in (1, 2)
                  for x in (0, 1)
                  if (s == 2 or (u == 4 and p == 0)) and (g == 1 or (u == 4 and s == 2))
                  and (x == 1 or (u == 4 and g == 1))]
ADJOINT_SHAPES = [dict(unroll=u, pipeline=p, span=s, grid_mult=1, split=x)
                  for u in (2, 3, 4) for p in (0, 1) for s in (1, 2, 3) for x in (0, 1)
                  if (s == 2 or (u == 2 and p == 0)) and (x == 1 or (u == 2 and p == 0))]


def test_every_launch_shape_is_bit_identical(anf):
    b = synth.config("C5")[0]
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)])
    pos = torch.from_numpy(b.pos).cuda()
    w = torch.from_numpy(synth.c5_cotangent()).cuda()
    bd = nf.bin(pos)
    ref_a, _, _ = nf.forces(bd)
    ref_g = nf.forces_vjp(bd, w)
    ref_a, ref_g = bits(ref_a), bits(ref_g)
    try:
        for shape in FORWARD_SHAPES:
            say(f"[shape] forward {shape}")
            nf.set_tuning(0, shape)
            a, _, _ = nf.forces(bd)
            assert np.array_equal(bits(a), ref_a), shape
        for shape in ADJOINT_SHAPES:
            say(f"[shape] adjoint {shape}")
            nf.set_tuning(1, shape)
            g = nf.forces_vjp(bd, w)
            assert np.array_equal(bits(g), ref_g), shape
    finally:
        nf.set_tuning(0, None)
        nf.set_tuning(1, None)


def test_autotune_keeps_results(anf):
    b = synth.config("C5")[0]
    nf = anf.NearField([anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)])
    pos = torch.from_numpy(b.pos).cuda()
    w = torch.from_numpy(synth.c5_cotangent()).cuda()
    bd = nf.bin(pos)
    ref_a, _, _ = nf.forces(bd)
    ref_g = nf.forces_vjp(bd, w)
    say("[autotune] C5")
    chosen = nf.autotune(bd)
    say(f"  chosen {chosen}")
    assert nf.get_tuning(0) == chosen["forward"]
    assert nf.get_tuning(1) == chosen["adjoint"]
    a, _, _ = nf.forces(bd)
    g = nf.forces_vjp(bd, w)
    assert np.array_equal(bits(a), bits(ref_a))
    assert np.array_equal(bits(g), bits(ref_g))
    nf.set_tuning(0, None)
    nf.set_tuning(1, None)


def test_graph_replay_matches_eager(anf):
    boxes = synth.config("C4", scale=5)
    specs = [anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes]
    nf = anf.NearField(specs)
    inputs = []
    for seed in range(4):
        parts = [synth.clustered(b.n, max(1, b.n // 1024), b.cpd, 9000 + 10 * seed + k)
                 for k, b in enumerate(boxes)]
        inputs.append(torch.from_numpy(np.concatenate(parts)).cuda())
    w = torch.from_numpy(synth.gaussian_weights(nf.n_total, 31)).cuda()

    # eager references
    refs = []
    for p in inputs:
        bd = nf.bin(p)
        a, m, _ = nf.forces(bd, momentum=True)
        g = nf.forces_vjp(bd, w)
        refs.append((bits(a), m.cpu().numpy(), bits(g)))

    pos = inputs[0].clone()
    binned = nf.alloc_binned()
    acc = torch.empty((nf.n_total, 3), dtype=torch.float32, device="cuda")
    grad = torch.empty_like(acc)
    mom = torch.empty((nf.nboxes, 4), dtype=torch.float64, device="cuda")

    def step():
        nf.bin(pos, out=binned)
        nf.forces(binned, out=acc, momentum_out=mom)
        nf.forces_vjp(binned, w, out=grad)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("[graph] capture")
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(6):
        k = rep % len(inputs)
        pos.copy_(inputs[k])
        graph.replay()
        torch.cuda.synchronize()
        say(f"[graph] replay {rep} input {k}")
        assert np.array_equal(bits(acc), refs[k][0]), rep
        assert np.array_equal(mom.cpu().numpy(), refs[k][1]), rep
        assert np.array_equal(bits(grad), refs[k][2]), rep
        # eager work between replays, on the same workspace
        bd = nf.bin(inputs[(k + 1) % len(inputs)])
        nf.forces(bd)
        torch.cuda.synchronize()


@pytest.mark.parametrize("order", ["original", "cell"])
def test_graph_replay_of_the_widened_rows(anf, order):
    """Binning, forces with the density estimate, the FP64 kernels, slab shares
    of the FP32 forward and adjoint, multipoles (both bases) and kick-drift
    captured in one graph: every replay, with state
    reset and eager work between replays, equals the eager results bit for bit.
    With the particles in their original order and in cell order, so both ways
    of the kick-drift update (chosen on the device) run inside the graph."""
    boxes = synth.config("C4", scale=6)
    specs = [anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer, 0.3 * b.box / b.cpd)
             for b in boxes]
    nf = anf.NearField(specs)
    pos0 = torch.from_numpy(np.concatenate([b.pos for b in boxes])).cuda()
    vel0 = torch.from_numpy(synth.gaussian_weights(nf.n_total, 41) * np.float32(0.01)).cuda()
    if order == "cell":
        sort = nf.bin(pos0).perm.long()
        pos0, vel0 = pos0[sort].contiguous(), vel0[sort].contiguous()
    w64 = torch.from_numpy(synth.gaussian_weights(nf.n_total, 42).astype(np.float64)).cuda()
    grad64 = torch.empty((nf.n_total, 3), dtype=torch.float64, device="cuda")
    pos, vel = pos0.clone(), vel0.clone()
    binned = nf.alloc_binned()
    acc = torch.empty((nf.n_total, 3), dtype=torch.float32, device="cuda")
    acc64 = torch.empty((nf.n_total, 3), dtype=torch.float64, device="cuda")
    rho = torch.empty(nf.n_total, dtype=torch.float32, device="cuda")
    mp_c = torch.empty((nf.cells_total, 165), dtype=torch.float64, device="cuda")
    mp_r = torch.empty((nf.cells_total, 81), dtype=torch.float64, device="cuda")
    w32 = torch.from_numpy(synth.gaussian_weights(nf.n_total, 43)).cuda()
    # rows outside the slabs are never written: NaN throughout, in every replay
    slab_acc = torch.full((nf.n_total, 3), float("nan"), dtype=torch.float32, device="cuda")
    slab_grad = torch.full_like(slab_acc, float("nan"))
    outs = {}

    def step():
        nf.bin(pos, out=binned)
        nf.forces(binned, out=acc, density_out=rho)
        nf.forces_f64(binned, out=acc64)
        nf.forces_vjp_f64(binned, w64, out=grad64)
        nf.forces_slab(binned, 1, 4, out=slab_acc)
        nf.forces_vjp_slab(binned, 2, 6, w32, out=slab_grad)
        nf.multipoles(binned, 8, out=mp_c)
        nf.multipoles(binned, 8, reduced=True, out=mp_r)
        outs["stats"] = nf.kick_drift(binned, pos, vel, acc, 0.01, 0.002, cell_stats=True)

    def snapshot():
        cs, bs = outs["stats"]
        return [t.detach().cpu().numpy().copy() for t in
                (acc, acc64, grad64, rho, mp_c, mp_r, pos, vel, cs, bs, slab_acc, slab_grad)]

    step()                    # eager reference (also allocates the lazy workspaces)
    torch.cuda.synchronize()
    ref = snapshot()
    pos.copy_(pos0)
    vel.copy_(vel0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("[graph] capture of the widened rows")
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        pos.copy_(pos0)
        vel.copy_(vel0)
        graph.replay()
        torch.cuda.synchronize()
        say(f"[graph] widened replay {rep}")
        for k, (x, y) in enumerate(zip(snapshot(), ref)):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), (rep, k)
        bd = nf.bin(pos0)
        nf.multipoles(bd, 4)
        torch.cuda.synchronize()
