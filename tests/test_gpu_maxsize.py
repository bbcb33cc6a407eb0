"""The largest lattice the ABI accepts (W = H = 46340, N = 2,147,395,600 < 2^31),
with ragged last tiles (4 columns, 4 rows).  The oracle cannot hold such a
lattice, so the checks are properties that hold at any size and outputs it
computes site by site: the Philox words of the initial states, bond draws and
flip draws of sampled sites (Sec. II steps 1 and 3)."""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L = 46340
N = L * L
Q = 3
TAG_INIT, TAG_BOND, TAG_FLIP = 0, 1, 2


def _key(seed):
    return (seed & 0xFFFFFFFF, seed >> 32)


def _word(i_block, t, tag, sid, seed, j):
    return int(oracle.philox((i_block & 0xFFFFFFFF, t, tag, sid), _key(seed))[j])


def _state0(i, seed, sid):
    return (_word(i >> 2, 0, TAG_INIT, sid, seed, i & 3) * Q) >> 32


def _flip(r, t, seed, sid):
    return (_word(r >> 2, t, TAG_FLIP, sid, seed, r & 3) * Q) >> 32


def _sample(seed):
    g = wl.rng(seed)
    idx = list(g.integers(0, N, size=1500))
    for y in (0, 1, 63, 64, L - 5, L - 4, L - 1):
        for x in (0, 1, 127, 128, L - 5, L - 4, L - 1):
            idx.append(y * L + x)
    return np.array(sorted(set(int(i) for i in idx)), dtype=np.int64)


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_max_size_no_bonds():
    """K = 0: no bond is active, every site is its own cluster and draws its own state."""
    seed, sid = wl.SEED_BASE | 0x61, 1
    lat = sw.SWLattice(L, L, q=Q, K=0.0, seed=seed, stream_id=sid, ising=False, keep_bonds=True)
    lat.sweep(1)
    o = lat.observables()
    assert o["n_active_bonds"] == 0 and o["n_clusters"] == N
    assert int(torch.count_nonzero(lat.bonds)) == 0
    idx = _sample(seed)
    got = lat.spins.view(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    want = np.array([_flip(int(i), 0, seed, sid) for i in idx])
    assert np.array_equal(got, want)
    del lat
    _free()


def test_max_size_bonds_at_critical_coupling():
    """Critical q = 3: the bonds of sampled sites (wrap bonds of the last row and
    column included) follow from the initial states and the bond draws; the
    active-bond count equals the bond bits."""
    seed, sid = wl.SEED_BASE | 0x62, 2
    K = wl.K_POTTS3_C
    T = oracle.threshold(K)
    lat = sw.SWLattice(L, L, q=Q, K=K, seed=seed, stream_id=sid, ising=False, keep_bonds=True)
    lat.sweep(1)
    o = lat.observables()
    b = lat.bonds.view(-1)
    nbits = int((b & 1).sum(dtype=torch.int64)) + int(((b >> 1) & 1).sum(dtype=torch.int64))
    assert o["n_active_bonds"] == nbits
    idx = _sample(seed)
    got = b[torch.from_numpy(idx).cuda()].cpu().numpy()
    for i, g in zip(idx, got):
        i = int(i)
        y, x = divmod(i, L)
        r = y * L + (x + 1) % L
        d = ((y + 1) % L) * L + x
        s, sr, sd = _state0(i, seed, sid), _state0(r, seed, sid), _state0(d, seed, sid)
        blk = oracle.philox(((i >> 1) & 0xFFFFFFFF, 0, TAG_BOND, sid), _key(seed))
        right = s == sr and int(blk[2 * (i & 1)]) < T
        down = s == sd and int(blk[2 * (i & 1) + 1]) < T
        assert int(g) == (1 if right else 0) | (2 if down else 0), (i, y, x)
    del lat, b
    _free()


def test_max_size_one_cluster():
    """Every bond active between equal spins (K = inf) on a uniform start: one
    cluster, labelled 0, whose draw every site takes."""
    seed, sid = wl.SEED_BASE | 0x63, 3
    spins = torch.zeros((L, L), dtype=torch.uint8, device="cuda")
    lat = sw.SWLattice(L, L, q=Q, K=float("inf"), seed=seed, stream_id=sid, ising=False, spins=spins)
    lat.sweep(1)
    o = lat.observables()
    assert o["n_clusters"] == 1 and o["n_active_bonds"] == 2 * N
    want = _flip(0, 0, seed, sid)
    assert bool(torch.all(lat.spins == want))
    del lat, spins
    _free()


def test_max_size_labeling_extremes():
    """Labeling at the largest size: a full image is one cluster (label 0, size
    N); an empty one has none (labels -1); a checkerboard is N/2 singletons
    labelled by their own index."""
    img = torch.ones((L, L), dtype=torch.uint8, device="cuda")
    lab, roots, sizes, n = sw.ccl_label(img, "sites_open", sizes=True)
    assert n == 1 and int(roots[0]) == 0 and int(sizes[0]) == N
    assert int(torch.count_nonzero(lab)) == 0
    img.zero_()
    lab, roots, sizes, n = sw.ccl_label(img, "sites_open", sizes=True)
    assert n == 0 and bool(torch.all(lab == -1))
    del roots, sizes
    # checkerboard: occupied iff x + y is even (L is even, so no wrap neighbours matter)
    y = torch.arange(L, device="cuda", dtype=torch.int32).view(L, 1)
    x = torch.arange(L, device="cuda", dtype=torch.int32).view(1, L)
    img = ((x + y) % 2 == 0).to(torch.uint8)
    del x, y
    lab = sw.ccl_label(img, "sites_open")
    own = torch.arange(N, device="cuda", dtype=torch.int32).view(L, L)  # N < 2^31
    want = torch.where(img.bool(), own, torch.full_like(own, -1))
    del own
    assert bool(torch.all(lab == want))
    del img, lab, want
    _free()
