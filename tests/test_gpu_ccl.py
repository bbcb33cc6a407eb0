"""GPU parity of connected-component labeling against the CPU oracle.

Labels, roots (ascending), sizes and the cluster count must match bit-exactly
for periodic and open bond inputs and for binary images, on shapes that span
many tiles with ragged tails, the degenerate shapes (1 x n, n x 1), empty and
full inputs, and the full-size bond-percolation pass at L = 16384.
"""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = {"bonds_periodic": oracle.PERIODIC, "bonds_open": oracle.OPEN}


def _oracle(inp, mode):
    H, W = inp.shape
    if mode == "sites_open":
        return oracle.label_sites(W, H, inp.reshape(-1))
    return oracle.label_bonds(W, H, inp.reshape(-1), MODES[mode])


def _check(inp, mode, **tile):
    H, W = inp.shape
    print(f"ccl W={W} H={H} mode={mode} {tile}", flush=True)
    g = torch.from_numpy(inp).cuda()
    lab, roots, sizes, n = sw.ccl_label(g, mode, sizes=True, **tile)
    want, nref = _oracle(inp, mode)
    got = lab.cpu().numpy().reshape(-1)
    assert np.array_equal(got, want)
    assert n == nref
    r_ref, s_ref, _ = oracle.cluster_sizes(want)
    assert np.array_equal(roots.cpu().numpy(), r_ref)
    assert np.array_equal(sizes.cpu().numpy(), s_ref)
    lab2 = sw.ccl_label(g, mode, **tile)
    assert torch.equal(lab, lab2)


SHAPES = [(1, 1), (1, 300), (300, 1), (2, 2), (127, 31), (128, 32), (129, 33), (256, 64),
          (1000, 37), (37, 1000), (515, 260), (1024, 1024)]


@pytest.mark.parametrize("mode", ["bonds_periodic", "bonds_open"])
@pytest.mark.parametrize("W,H", SHAPES)
def test_bonds(W, H, mode):
    for k, p in enumerate((0.0, 0.35, 0.5, 0.65, 1.0)):
        _check(wl.random_bonds(W, H, p, seed=1000 + 7 * W + H + k), mode)


@pytest.mark.parametrize("W,H", SHAPES)
def test_sites(W, H):
    for k, p in enumerate((0.0, 0.4, 0.5927, 0.7, 1.0)):
        _check(wl.site_image(W, H, p, seed=2000 + 7 * W + H + k), "sites_open")


@pytest.mark.parametrize("tile_h,merge_waves", [(16, 4), (32, 16), (128, 8), (128, 4)])
@pytest.mark.parametrize("W,H", [(1, 300), (300, 1), (129, 33), (515, 260), (1000, 257)])
def test_tile_shapes(W, H, tile_h, merge_waves):
    """Every tile shape and merge schedule labels bonds and images as the oracle does."""
    for k, p in enumerate((0.35, 0.5, 0.65)):
        seed = 5000 + 7 * W + H + k + tile_h
        _check(wl.random_bonds(W, H, p, seed=seed), "bonds_periodic", tile_h=tile_h, merge_waves=merge_waves)
        _check(wl.random_bonds(W, H, p, seed=seed + 1), "bonds_open", tile_h=tile_h, merge_waves=merge_waves)
    for k, p in enumerate((0.4, 0.5927, 0.7)):
        _check(wl.site_image(W, H, p, seed=6000 + 7 * W + H + k), "sites_open", tile_h=tile_h,
               merge_waves=merge_waves)


def test_structured_inputs():
    W, H = 300, 200
    cb = ((np.add.outer(np.arange(H), np.arange(W)) % 2) == 0).astype(np.uint8)
    _check(cb, "sites_open")
    stripes = np.zeros((H, W), np.uint8)
    stripes[::3, :] = 1  # horizontal lines of right bonds, wrap included
    _check(stripes, "bonds_periodic")
    _check(stripes, "bonds_open")
    spiral = np.zeros((H, W), np.uint8)
    spiral[1:-1, 1] = 2
    spiral[-2, 1:-2] = 1
    spiral[2:-1, -3] = 2
    _check(spiral, "bonds_open")


def test_percolation_16384():
    """Full-size labeling pass: bond percolation at p = 1/2, L = 16384."""
    L = 16384
    inp = wl.percolation_bonds(L, L, seed=wl.SEED_BASE | 3)
    g = torch.from_numpy(inp).cuda()
    lab, roots, sizes, n = sw.ccl_label(g, "bonds_periodic", sizes=True)
    want, nref = oracle.label_bonds(L, L, inp.reshape(-1), oracle.PERIODIC)
    assert n == nref
    assert np.array_equal(lab.cpu().numpy().reshape(-1), want)
    del lab
    r_ref, s_ref, _ = oracle.cluster_sizes(want)
    assert np.array_equal(roots.cpu().numpy(), r_ref)
    assert np.array_equal(sizes.cpu().numpy(), s_ref)
    # exact density of bond-percolation clusters at p = 1/2 is (3 sqrt3 - 5)/2
    assert abs(n / L**2 - (3 * np.sqrt(3) - 5) / 2) < 1e-3


def test_sites_16384():
    """Full-size image labeling: site percolation near its threshold (occupancy
    0.5927), L = 16384, with sizes."""
    L = 16384
    img = wl.site_image(L, L, 0.5927, seed=wl.SEED_BASE | 0x516)
    g = torch.from_numpy(img).cuda()
    print("sites_open 16384^2 with sizes", flush=True)
    lab, roots, sizes, n = sw.ccl_label(g, "sites_open", sizes=True)
    want, nref = oracle.label_sites(L, L, img.reshape(-1))
    assert n == nref
    assert np.array_equal(lab.cpu().numpy().reshape(-1), want)
    del lab
    r_ref, s_ref, _ = oracle.cluster_sizes(want)
    assert np.array_equal(roots.cpu().numpy(), r_ref)
    assert np.array_equal(sizes.cpu().numpy(), s_ref)


def test_percolation_16384_repeated():
    """Eight labelings of the same full-size input all equal the oracle (race guard)."""
    L = 16384
    inp = wl.percolation_bonds(L, L, seed=wl.SEED_BASE | 3)
    want, _ = oracle.label_bonds(L, L, inp.reshape(-1), oracle.PERIODIC)
    want = torch.from_numpy(want.reshape(L, L)).cuda()
    g = torch.from_numpy(inp).cuda()
    ws = torch.empty(sw.ccl_workspace_bytes(L, L) + 256, dtype=torch.uint8, device="cuda")
    for rep in range(8):
        lab = sw.ccl_label(g, "bonds_periodic", workspace=ws)
        bad = int((lab != want).sum().item())
        assert bad == 0, (rep, bad)


def test_side_stream_and_output_checks():
    """ccl_label on a stream other than the current one: a non-contiguous
    input (copied on the current stream first), sizes read back after the side
    stream; results equal the oracle's.  Wrong caller-supplied outputs raise
    before anything is enqueued."""
    W, H = 515, 260
    img = wl.site_image(W, H, 0.5927, seed=2901)
    print(f"ccl side stream W={W} H={H}", flush=True)
    g = torch.from_numpy(np.ascontiguousarray(img.T)).cuda().t()  # (H, W) view, not contiguous
    assert not g.is_contiguous()
    side = torch.cuda.Stream()
    lab, roots, sizes, n = sw.ccl_label(g, "sites_open", sizes=True, stream=side)
    side.synchronize()
    want, nref = _oracle(img, "sites_open")
    assert n == nref
    assert np.array_equal(lab.cpu().numpy().reshape(-1), want)
    r_ref, s_ref, _ = oracle.cluster_sizes(want)
    assert np.array_equal(roots.cpu().numpy(), r_ref)
    assert np.array_equal(sizes.cpu().numpy(), s_ref)
    gc = g.contiguous()
    for bad in (torch.empty((H, W + 1), dtype=torch.int32, device="cuda"),
                torch.empty((H, W), dtype=torch.int64, device="cuda"),
                torch.empty((W, H), dtype=torch.int32, device="cuda").t(),
                torch.empty((H, W), dtype=torch.int32)):
        with pytest.raises(ValueError):
            sw.ccl_label(gc, "sites_open", labels=bad)
    with pytest.raises(ValueError):
        sw.ccl_label(gc, "sites_open", workspace=torch.empty(1 << 24, dtype=torch.uint8))
