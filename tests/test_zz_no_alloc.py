"""The allocation-free labeling entry point against the ordinary one.

ccl_label_noalloc labels with the library's static per-GPU scratch instead of
a caller workspace.  Its outputs must equal ccl_label's bit for bit (and the
oracle's), over two calls in a row on one stream, the second on a smaller
input, so nothing left in the scratch by the first call shows in the second.
Named to run last: the round's GPU suite stops at its first failure.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import _lib
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _noalloc(g, mode, sizes):
    """One call through the C ABI with outputs made beforehand."""
    H, W = g.shape
    lab = torch.full((H, W), -7, dtype=torch.int32, device=g.device)
    ncl = torch.full((1,), -7, dtype=torch.int32, device=g.device)
    roots = torch.full((H * W,), -7, dtype=torch.int32, device=g.device) if sizes else None
    szs = torch.full((H * W,), -7, dtype=torch.int32, device=g.device) if sizes else None
    torch.cuda.synchronize()
    st = _lib.lib().ccl_label_noalloc(g.data_ptr(), W, H, sw._MODES[mode], lab.data_ptr(),
                                      roots.data_ptr() if sizes else None, szs.data_ptr() if sizes else None,
                                      ncl.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.SW_OK, _lib.lib().sw_last_error()
    torch.cuda.synchronize()
    return lab, roots, szs, int(ncl.item())


def _compare(inp, mode, sizes):
    H, W = inp.shape
    print(f"noalloc W={W} H={H} mode={mode} sizes={sizes}", flush=True)
    g = torch.from_numpy(inp).cuda()
    lab, roots, szs, n = _noalloc(g, mode, sizes)
    if sizes:
        lab_r, roots_r, szs_r, n_r = sw.ccl_label(g, mode, sizes=True)
        assert n == n_r
        assert torch.equal(roots[:n], roots_r) and torch.equal(szs[:n], szs_r)
    else:
        lab_r = sw.ccl_label(g, mode)
    assert torch.equal(lab, lab_r)
    if mode == "sites_open":
        want, nref = oracle.label_sites(W, H, inp.reshape(-1))
    else:
        want, nref = oracle.label_bonds(W, H, inp.reshape(-1), oracle.PERIODIC)
    assert n == nref
    assert np.array_equal(lab.cpu().numpy().reshape(-1), want)


def test_noalloc_matches_ccl_label_twice_shrinking():
    # the largest square image with sizes that the scratch holds, then a
    # smaller ragged one, then a small bond input without sizes
    _compare(wl.site_image(2048, 2048, 0.5927, seed=71), "sites_open", True)
    _compare(wl.site_image(700, 333, 0.6, seed=72), "sites_open", True)
    _compare(wl.random_bonds(257, 65, 0.5, seed=73), "bonds_periodic", False)


def test_noalloc_refuses_oversize():
    g = torch.zeros((2560, 2560), dtype=torch.uint8, device="cuda")
    lab = torch.empty((2560, 2560), dtype=torch.int32, device="cuda")
    roots = torch.empty(2560 * 2560, dtype=torch.int32, device="cuda")
    szs = torch.empty(2560 * 2560, dtype=torch.int32, device="cuda")
    with pytest.raises(_lib.SwccLError) as e:
        sw.ccl_label_noalloc(g, lab, roots=roots, sizes=szs, mode="sites_open")
    assert e.value.status == _lib.SW_ERR_WORKSPACE
