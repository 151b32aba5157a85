"""Sorted slots far beyond the 32-bit range of the packed source records.

The forward kernel reads 3 floats and the adjoint 6 floats per sorted slot, so
slot offsets above 2^31 / 6 (adjoint) and 2^31 / 3 (forward) need 64-bit
address arithmetic.  A filler box of 720 million uniform particles comes first
in the batch; the checked box (C1, 4096 particles) follows it, so every one of
its sinks and sources sits above slot 7.2e8, where 3 s and 6 s exceed 2^31.
Its binning, forces and adjoint are compared with the oracle on that box alone.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import MEDIAN_TOL, P999_TOL, VJP_TOL, err_stats, frac_err
from paper_2110_11392_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_FILL = 720_000_000
K_FILL = 300          # 27 M cells, about 27 particles per cell


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_checked_box_beyond_slot_2_31_over_3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd as anf
    b = synth.config("C1")[0]
    specs = [anf.BoxSpec(N_FILL, 1.0, K_FILL, 2, 1.0 / (40 * N_FILL ** (1 / 3))),
             anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer)]
    nf = anf.NearField(specs)
    say(f"[large] filler n={N_FILL} K={K_FILL}, checked C1 at slots >= {N_FILL}; "
        f"workspace {nf.workspace_bytes / 2 ** 30:.1f} GiB")
    assert 3 * N_FILL >= 2 ** 31
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2024)
    pos = torch.empty((nf.n_total, 3), dtype=torch.float32, device="cuda")
    w = torch.empty_like(pos)
    step = 60_000_000
    for c0 in range(0, N_FILL, step):
        c1 = min(N_FILL, c0 + step)
        pos[c0:c1] = torch.rand((c1 - c0, 3), generator=gen, dtype=torch.float32, device="cuda")
        w[c0:c1] = torch.randn((c1 - c0, 3), generator=gen, dtype=torch.float32, device="cuda")
    pos[N_FILL:] = torch.from_numpy(b.pos).cuda()
    wb = synth.gaussian_weights(b.n, 31)
    w[N_FILL:] = torch.from_numpy(wb).cuda()
    bd = nf.bin(pos)
    torch.cuda.synchronize()
    bd.check_status()
    say("  binned")
    off = bd.cell_offsets[K_FILL ** 3:].cpu().numpy()
    perm = bd.perm[N_FILL:].cpu().numpy()
    rel = bd.rel[N_FILL:].cpu().numpy()
    _, o_off, o_perm, o_rel = oracle.bin(b.pos, b.box, b.cpd)
    assert np.array_equal(off.astype(np.int64) - N_FILL, o_off)
    assert np.array_equal(perm.astype(np.int64) - N_FILL, o_perm)
    assert np.array_equal(rel.view(np.uint32), o_rel.view(np.uint32))
    acc, _, _ = nf.forces(bd)
    torch.cuda.synchronize()
    say("  forces done")
    a = acc[N_FILL:].cpu().numpy()
    del acc
    g = nf.forces_vjp(bd, w)
    torch.cuda.synchronize()
    say("  adjoint done")
    gg = g[N_FILL:].cpu().numpy()
    ref, _ = oracle.forces(b.pos, b.box, b.cpd, b.radius, b.eps_plummer)
    st = err_stats(frac_err(a, ref))
    gref = oracle.vjp(b.pos, wb, b.box, b.cpd, b.radius, b.eps_plummer)
    rel_g = np.linalg.norm(gg - gref) / np.linalg.norm(gref)
    say(f"  forces {st}; adjoint relative error {rel_g:.3g}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL
    assert rel_g <= VJP_TOL
