"""The largest grid the work plan accepts: K = 644 cells per dimension, R = 2
(K^3 + 2 K^2 + n/64 + 1 stays below 2^28 work items; K = 645 is refused with
ERANGE, checked on the CPU).  267 M cells, 415 k pencils of 645 offsets, 28-bit
cell keys (four radix passes).

65,536 particles: half uniform (almost every one alone in its stencil, so its
force and gradient are exactly zero) and half in 16 clustered blobs of a
fraction of a cell to a few cells (up to a few hundred per cell).  Binning is
compared with the oracle in full (offsets of every cell, permutation, offsets
from the cell centres, bit for bit); forces and the adjoint on 4000 sampled
sinks, mostly from the blobs, at the usual tolerances.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import MEDIAN_TOL, P999_TOL, VJP_TOL, err_stats, frac_err
from paper_2110_11392_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K = 644
EPS_P = 1.0 / (40 * 4096.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_largest_grid_against_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11392_amd as anf
    n_u = n_c = 32768
    pos = np.concatenate([synth.uniform(n_u, 7001), synth.clustered(n_c, 16, K, 7002)])
    n = pos.shape[0]
    nf = anf.NearField([anf.BoxSpec(n, 1.0, K, 2, EPS_P)])
    say(f"[max grid] n={n} K={K} ({K ** 3} cells); "
        f"workspace {nf.workspace_bytes / 2 ** 30:.1f} GiB")
    bd = nf.bin(torch.from_numpy(pos).cuda())
    bd.check_status()
    _, o_off, o_perm, o_rel = oracle.bin(pos, 1.0, K)
    assert np.array_equal(bd.cell_offsets.cpu().numpy(), o_off)
    assert np.array_equal(bd.perm.cpu().numpy(), o_perm)
    assert np.array_equal(bd.rel.cpu().numpy().view(np.uint32), o_rel.view(np.uint32))
    say("  binning bit-exact")

    w = synth.gaussian_weights(n, 11)
    acc = nf.forces(bd)[0].cpu().numpy()
    grad = nf.forces_vjp(bd, torch.from_numpy(w).cuda()).cpu().numpy()
    rng = np.random.default_rng(3)
    sinks = np.concatenate([rng.choice(np.arange(n_u), 1000, replace=False),
                            rng.choice(np.arange(n_u, n), 3000, replace=False)])
    ref, _ = oracle.forces(pos, 1.0, K, 2, EPS_P, sinks=sinks)
    gref = oracle.vjp(pos, w, 1.0, K, 2, EPS_P, sinks=sinks)
    alone = np.linalg.norm(ref, axis=1) == 0
    say(f"  {alone.sum()} sampled sinks without a neighbour in their stencil")
    assert 0 < alone.sum() < sinks.size
    # no neighbour: the only pair is the sink with itself, which adds exactly 0
    assert (acc[sinks[alone]] == 0).all() and (grad[sinks[alone]] == 0).all()
    st = err_stats(frac_err(acc[sinks[~alone]], ref[~alone]))
    rel_g = np.linalg.norm(grad[sinks] - gref) / np.linalg.norm(gref)
    say(f"  forces {st}; adjoint relative error {rel_g:.3g}")
    assert st["median"] <= MEDIAN_TOL and st["p999"] <= P999_TOL
    assert rel_g <= VJP_TOL
