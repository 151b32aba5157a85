"""A cell beyond the pair kernels' per-cell limit of 2^28 particles.

Inside one source cell the pair kernels form record offsets (up to 6 floats per
particle) in 32 bits, so the binning flags a cell of more than 2^28 particles
(ABACUS_NF_STATUS_CELLFULL) and the work plan then queues no task.  Both sides
of the limit, on one layout of 2^28 + 1 particles (box 1, K = 3, R = 1):
  * 2^28 particles in the centre cell and one in a corner cell: not flagged
    (only binned: its pair work would be about 7e16 pairs);
  * all 2^28 + 1 in the centre cell: flagged, and forces, the adjoint and the
    FP64 forces return without evaluating a pair.
The flag is checked before any pair kernel is called.
"""
import sys

import pytest

from paper_2110_11392_amd import _lib

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LIMIT = 2 ** 28
N = LIMIT + 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_cell_limit_flag_and_empty_plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd as anf
    nf = anf.NearField([anf.BoxSpec(N, 1.0, 3, 1, 1e-3)])
    say(f"[cell limit] n={N} K=3 R=1; workspace {nf.workspace_bytes / 2 ** 30:.1f} GiB")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    # the centre cell is [1/3, 2/3)^3; [0.4, 0.6) stays clear of its faces
    pos = torch.rand((N, 3), generator=gen, dtype=torch.float32, device="cuda")
    pos.mul_(0.2).add_(0.4)
    pos[N - 1] = torch.tensor([0.9, 0.9, 0.9], device="cuda")  # corner cell (2, 2, 2)
    bd = nf.bin(pos)
    st = int(bd.status.item())
    say(f"  one particle in the corner: status {st}")
    assert st == 0
    assert int(bd.cell_offsets[13 + 1].item()) - int(bd.cell_offsets[13].item()) == LIMIT

    pos[N - 1] = torch.tensor([0.5, 0.5, 0.5], device="cuda")
    bd = nf.bin(pos)
    st = int(bd.status.item())
    say(f"  all in the centre cell: status {st}")
    assert st == _lib.STATUS_CELLFULL
    assert int(bd.cell_offsets[14].item()) - int(bd.cell_offsets[13].item()) == N
    with pytest.raises(ValueError, match="2\\^28"):
        bd.check_status()
    del pos
    torch.cuda.empty_cache()

    acc, _, _ = nf.forces(bd)
    torch.cuda.synchronize()
    say("  forces returned")
    del acc
    w = torch.zeros((N, 3), dtype=torch.float32, device="cuda")
    g = nf.forces_vjp(bd, w)
    torch.cuda.synchronize()
    say("  adjoint returned")
    del g, w
    a64 = nf.forces_f64(bd)
    torch.cuda.synchronize()
    say("  FP64 forces returned")
    del a64
    assert int(bd.status.item()) == _lib.STATUS_CELLFULL
