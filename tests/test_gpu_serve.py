"""GPU parity of served labeling: every request's labels, roots and sizes equal
the oracle's whether it runs alone or among others, on its own or in a batch
of small requests labeled by shared launches (continuous batching), and
admission never puts more requests in flight than the arena holds."""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pinned(img):
    t = torch.from_numpy(img).pin_memory()
    return t


def _drain(srv, want=None, cap=None):
    """Run the server until it is empty; returns {tag: (labels, roots, sizes, n)} on the host."""
    got = {}
    while srv.pending:
        srv.pump()
        if cap is not None:
            assert len(srv._inflight) <= cap
        for slot, tag in srv.poll():
            lab, roots, sizes, n = srv.result(slot)
            got[tag] = (lab.cpu().numpy().reshape(-1), roots.cpu().numpy(), sizes.cpu().numpy(), n)
            srv.release(slot)
    return got


SHAPES = [(1, 1), (1, 300), (300, 1), (2, 2), (127, 31), (128, 64), (129, 65), (515, 260), (1000, 37),
          (37, 1000), (700, 500), (1024, 1024)]


@pytest.mark.parametrize("batch_px", [0, 1 << 20], ids=["unbatched", "batched"])
def test_server_mix(batch_px):
    srv = sw.CCLServer(1 << 30, mode="sites_open", sizes=True, max_inflight=16, n_streams=3, batch_px=batch_px)
    imgs = {}
    tag = 0
    for k, (W, H) in enumerate(SHAPES):
        for p in (0.4, 0.5927, 0.7):
            imgs[tag] = wl.site_image(W, H, p, seed=4000 + 13 * k + int(p * 100))
            srv.submit(tag, _pinned(imgs[tag]))
            tag += 1
    print(f"server mix: {len(imgs)} requests", flush=True)
    got = _drain(srv)
    assert sorted(got) == sorted(imgs)
    for t, img in imgs.items():
        H, W = img.shape
        want, n = oracle.label_sites(W, H, img.reshape(-1))
        r_ref, s_ref, _ = oracle.cluster_sizes(want)
        lab, roots, sizes, ng = got[t]
        assert ng == n, t
        assert np.array_equal(lab, want), t
        assert np.array_equal(roots, r_ref) and np.array_equal(sizes, s_ref), t
    srv.close()


def test_server_admission_by_footprint():
    """An arena that holds two 1024^2 requests never has more than two in flight."""
    probe = sw.CCLServer(1 << 20, sizes=True, max_inflight=8, n_streams=2)
    fp = probe.footprint(1024, 1024)
    probe.close()
    srv = sw.CCLServer(2 * fp + fp // 2, sizes=True, max_inflight=8, n_streams=2)
    imgs = {t: wl.site_image(1024, 1024, 0.55 + 0.02 * t, seed=5000 + t) for t in range(6)}
    for t, img in imgs.items():
        srv.submit(t, _pinned(img))
    assert len(srv._inflight) == 2
    got = _drain(srv, cap=2)
    for t, img in imgs.items():
        want, n = oracle.label_sites(1024, 1024, img.reshape(-1))
        assert got[t][3] == n and np.array_equal(got[t][0], want), t
    with pytest.raises(sw.SwccLError):
        srv.submit(99, _pinned(wl.site_image(2048, 2048, 0.5, seed=1)))  # larger than the arena
    srv.close()


def test_identical_alone_and_in_mix():
    big = wl.site_image(2048, 2048, 0.5927, seed=6000)
    srv = sw.CCLServer(4 << 30, sizes=True, max_inflight=32, n_streams=4)
    srv.submit(0, _pinned(big))
    alone = _drain(srv)[0]
    others = [wl.site_image(W, H, 0.6, seed=6100 + i) for i, (W, H) in enumerate(SHAPES)]
    for i, img in enumerate(others[:6]):
        srv.submit(100 + i, _pinned(img))
    srv.submit(1, _pinned(big))
    for i, img in enumerate(others[6:]):
        srv.submit(200 + i, _pinned(img))
    mixed = _drain(srv)
    assert np.array_equal(alone[0], mixed[1][0])
    assert np.array_equal(alone[1], mixed[1][1]) and np.array_equal(alone[2], mixed[1][2])
    want, n = oracle.label_sites(2048, 2048, big.reshape(-1))
    assert alone[3] == n and np.array_equal(alone[0], want)
    srv.close()


@pytest.mark.parametrize("batch_px", [0, 1 << 20], ids=["unbatched", "batched"])
def test_server_bonds_mode(batch_px):
    srv = sw.CCLServer(1 << 28, mode="bonds_periodic", sizes=False, max_inflight=4, n_streams=2, batch_px=batch_px)
    imgs = {t: wl.random_bonds(300 + t, 170, 0.5, seed=7000 + t) for t in range(5)}
    for t, img in imgs.items():
        srv.submit(t, _pinned(img))
    got = {}
    while srv.pending:
        srv.pump()
        for slot, tag in srv.poll():
            lab, roots, sizes, n = srv.result(slot)
            assert roots is None and sizes is None
            got[tag] = (lab.cpu().numpy().reshape(-1), n)
            srv.release(slot)
    for t, img in imgs.items():
        H, W = img.shape
        want, n = oracle.label_bonds(W, H, img.reshape(-1), oracle.PERIODIC)
        assert got[t][1] == n and np.array_equal(got[t][0], want), t
    srv.close()


def test_identical_alone_and_in_batched_mix():
    """Continuous batching with an 8192^2 image in the mix: the big image
    (labeled on its own) and a small one (in a batch) give the same results
    alone and among 30 others arriving around them, and every request of the
    mix equals the oracle."""
    srv = sw.CCLServer(6 << 30, sizes=True, max_inflight=64, n_streams=4, batch_px=1 << 20)
    big = wl.site_image(8192, 8192, 0.5927, seed=6500)
    small = wl.site_image(700, 500, 0.6, seed=6501)
    print("served 8192^2 alone", flush=True)
    srv.submit(0, _pinned(big))
    srv.submit(1, _pinned(small))
    alone = _drain(srv)
    imgs = {2: big, 3: small}
    for i in range(30):
        W, H = SHAPES[i % len(SHAPES)]
        imgs[100 + i] = wl.site_image(W, H, 0.4 + 0.01 * i, seed=6600 + i)
    order = [100 + i for i in range(12)] + [2] + [100 + i for i in range(12, 20)] + [3] + \
        [100 + i for i in range(20, 30)]
    print("served mix with batching", flush=True)
    for k, t in enumerate(order):
        srv.submit(t, _pinned(imgs[t]))
        if k % 7 == 6:
            srv.pump()  # batches of those admitted so far
    # a view into a pinned buffer at an odd offset (as the bench's pooled requests are)
    buf = torch.zeros(3 + 300 * 200 + 5, dtype=torch.uint8).pin_memory()
    img_v = wl.site_image(300, 200, 0.59, seed=6700)
    buf[3:3 + 300 * 200] = torch.from_numpy(img_v.reshape(-1))
    imgs[300] = img_v
    srv.submit(300, buf[3:3 + 300 * 200].view(200, 300))
    mixed = _drain(srv)
    for a, m in ((0, 2), (1, 3)):
        assert alone[a][3] == mixed[m][3]
        for j in range(3):
            assert np.array_equal(alone[a][j], mixed[m][j]), (a, j)
    for t, img in imgs.items():
        H, W = img.shape
        want, n = oracle.label_sites(W, H, img.reshape(-1))
        lab, roots, sizes, ng = mixed[t]
        assert ng == n and np.array_equal(lab, want), t
        r_ref, s_ref, _ = oracle.cluster_sizes(want)
        assert np.array_equal(roots, r_ref) and np.array_equal(sizes, s_ref), t
    srv.close()
