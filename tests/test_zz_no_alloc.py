"""abacus_nf_forces_noalloc against abacus_nf_forces, through the C ABI.

The no-allocation entry point runs the same plan, pair kernel and momentum
reduction with its temporaries in the library's static scratch array, so its
outputs must equal the workspace entry point's bit for bit.  Two calls in a
row, the second on a smaller input, check that the array's leftover contents
from the first call do not leak into the second.  A problem larger than the
scratch must be refused before anything is enqueued.
"""
import ctypes
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
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_11392_amd import _lib
    return _lib


def run_both(_lib, anf, boxes, flags):
    specs = [anf.BoxSpec(b.n, b.box, b.cpd, b.radius, b.eps_plummer) for b in boxes]
    nf = anf.NearField(specs)
    pos = torch.from_numpy(np.ascontiguousarray(np.concatenate([b.pos for b in boxes]))).cuda()
    bd = nf.bin(pos)
    n = nf.n_total
    ref_acc = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    ref_mom = torch.empty((len(boxes), 4), dtype=torch.float64, device="cuda")
    acc = torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda")
    mom = torch.full((len(boxes), 4), float("nan"), dtype=torch.float64, device="cuda")
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cs = bd.cstruct()
    _lib.check(lib.abacus_nf_forces(nf._boxes, nf.nboxes, ctypes.byref(cs),
                                    ctypes.c_void_p(ref_acc.data_ptr()), None,
                                    ctypes.c_void_p(ref_mom.data_ptr()), None, flags,
                                    ctypes.c_void_p(nf.workspace.data_ptr()), nf.workspace_bytes,
                                    stream), "abacus_nf_forces")
    _lib.check(lib.abacus_nf_forces_noalloc(nf._boxes, nf.nboxes, ctypes.byref(cs),
                                            ctypes.c_void_p(acc.data_ptr()), None,
                                            ctypes.c_void_p(mom.data_ptr()), None, flags, stream),
               "abacus_nf_forces_noalloc")
    torch.cuda.synchronize()
    return (ref_acc.cpu().numpy(), ref_mom.cpu().numpy(), acc.cpu().numpy(), mom.cpu().numpy())


@pytest.mark.parametrize("accumulation", ["compensated", "single"])
def test_noalloc_matches_workspace_entry_point(lib, accumulation):
    import paper_2110_11392_amd as anf
    flags = anf.nearfield.ACCUMULATION[accumulation]
    # first a 262144-particle clustered box, then a smaller batch of two boxes
    for label, boxes in (("C5", synth.config("C5")),
                         ("C1 + ragged", synth.config("C1") +
                          [synth.Box(synth.clustered(2500, 6, 8, 13), 1.0, 8, 2, 1 / 500)])):
        say(f"[noalloc] {label} {accumulation}: n={sum(b.n for b in boxes)}")
        ref_acc, ref_mom, acc, mom = run_both(lib, anf, boxes, flags)
        assert np.array_equal(ref_acc.view(np.uint32), acc.view(np.uint32))
        assert np.array_equal(ref_mom.view(np.uint64), mom.view(np.uint64))


def test_noalloc_refuses_what_does_not_fit(lib):
    import paper_2110_11392_amd as anf
    n, K = 16_777_216, 64
    boxes = lib.box_array([(n, 1.0, K, 2, 1.0 / 10240.0, 0.0)])
    fake = lib.Binned(256, 256, 256, 256)
    rc = lib.load().abacus_nf_forces_noalloc(boxes, 1, ctypes.byref(fake), ctypes.c_void_p(256),
                                             None, None, None, 0, None)
    assert rc == lib.ESCRATCH
    assert "scratch" in lib.load().abacus_nf_strerror(rc).decode()
    del anf
