"""The caller's allocator (lp_set_allocator): with torch's caching allocator
installed, clustering, contraction, the cut and batches give exactly the
results of the library's own memory cache, the scratch and the coarse
graph's buffers come from torch, and every block goes back when the calls
and the handle are done."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(lp, G, gs):
    lab = lp.lp_cluster(G, 64, 5, 1)
    C, mp = lp.lp_contract(G, lab)
    cut = lp.lp_edge_cut(G, lab)
    x, a, w, v = lp.lp_decompress(C)
    outs = lp.lp_batch_cluster(gs, [32, 48], 4, [3, 4])
    res = dict(lab=lab.cpu().numpy(), map=mp.cpu().numpy(), cut=cut, x=x.cpu().numpy(), a=a.cpu().numpy(),
               w=w.cpu().numpy(), v=v.cpu().numpy(), batch=[o.cpu().numpy() for o in outs])
    return res, C


def test_torch_allocator_gives_identical_results(lp, synth_mod):
    import torch

    g = synth_mod.rmat_scale(14, 16, seed=2)
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    gs = [lp.lp_compress(h.n, h.xadj.view(np.int64), h.adjncy)
          for h in (synth_mod.rgg2d_16k(seed=1), synth_mod.rmat_scale(12, 8, seed=3))]
    ref, C = _run(lp, G, gs)
    C.free()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    lp.use_torch_allocator(True)
    try:
        got, C = _run(lp, G, gs)
        held = lp.memory_info()["external"]
        assert held > 0  # the coarse graph's buffers came from torch
        assert torch.cuda.memory_allocated() >= before + held
        C.free()
        torch.cuda.synchronize()
        assert lp.memory_info()["external"] == 0  # scratch and handle buffers all returned
    finally:
        lp.use_torch_allocator(False)
    for k in ("lab", "map", "x", "a", "w", "v"):
        assert np.array_equal(ref[k], got[k]), k
    assert ref["cut"] == got["cut"]
    assert all(np.array_equal(p, q) for p, q in zip(ref["batch"], got["batch"]))
    for h in gs:
        h.free()
    G.free()


def test_allocator_argument_errors(lp):
    import ctypes
    bad = lp.lp_allocator(lp._ALLOC_FN(lambda n, s, c: None), lp._FREE_FN(), None)
    assert lp._load().lp_set_allocator(ctypes.byref(bad)) == lp.LP_EINVAL
    assert lp._load().lp_set_allocator(None) == lp.LP_OK
