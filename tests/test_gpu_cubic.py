"""GPU parity of the simple cubic lattice sweep against the CPU oracle
(bit-exact): packed bonds, canonical labels, spins and the per-sweep records
after every sweep.

Shapes cover one tile with its periodic wraps inside the tile, ragged tiles
along each axis, odd Lx (rows starting at odd site indices), Lx a multiple of
4 with an odd number of rows in a tile (the +z draws shared by lane pairs
over row pairs, and a last single row), the couplings K = 0, K = inf and
1.4 and 0.6 times the critical one,
sweeps on a side stream, extents 1 and 2
(self-bonds and doubled bonds), a restart at a sweep number other than 0,
Lz = 1 against the square-lattice sweep of the same library, the 256^3 and
512^3 Ising lattices at the 3D critical coupling, and the largest accepted
shape class (1024 x 1024 x 2047) by sampled definitions and whole-lattice
counts.
"""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K3 = sw.ising_K(sw.BETA_C_ISING_3D)


def _state(lat):
    s = lat.spins.cpu().numpy().reshape(-1)
    if lat.ising:
        return ((s.astype(np.int16) + 1) // 2).astype(np.uint8)
    return s.astype(np.uint8)


CASES = [
    # Lx, Ly, Lz, q, K, ising
    (16, 8, 8, 2, K3, True),
    (128, 8, 8, 3, 1.0051, False),
    (130, 9, 17, 2, K3, True),
    (257, 11, 9, 2, 0.6, True),
    (5, 3, 7, 3, 1.2, False),
    (1, 1, 6, 2, 1.0, True),
    (2, 2, 2, 2, 0.5, True),
    (1, 40, 3, 4, 1.1, False),
    (300, 1, 2, 2, 0.9, True),
    (64, 64, 64, 2, K3, True),
    (33, 70, 20, 3, 0.8, False),
    (132, 13, 9, 2, K3, True),               # Lx a multiple of 4 (lane pairs share +z blocks), odd tile heights
    (40, 20, 18, 3, 0.0, False),             # K = 0: no bond is active, every site its own cluster
    (40, 20, 18, 2, float("inf"), True),     # K = inf: every bond between equal spins is active
    (160, 64, 48, 2, 1.4 * K3, True),        # ordered phase: one cluster spans the lattice
    (160, 64, 48, 2, 0.6 * K3, True),        # disordered phase: many small clusters
]


@pytest.mark.parametrize("Lx,Ly,Lz,q,K,ising", CASES)
def test_cubic_parity(Lx, Ly, Lz, q, K, ising):
    print(f"cubic Lx={Lx} Ly={Ly} Lz={Lz} q={q} K={K}", flush=True)
    seed, sid = wl.SEED_BASE | 0x3D1, 7
    lat = sw.CubicLattice(Lx, Ly, Lz, q=q, K=K, seed=seed, stream_id=sid, ising=ising, keep_labels=True,
                          keep_bonds=True)
    T = oracle.threshold(K)
    assert lat.threshold == T
    st = oracle.init_states3(Lx, Ly, Lz, q, seed, sid)
    torch.cuda.synchronize()
    assert np.array_equal(_state(lat), st)
    for t in range(5):
        rec = lat.sweep(1, records=True)
        st, bonds, labels, want = oracle.sw3_sweep(Lx, Ly, Lz, q, T, seed, sid, t, st)
        torch.cuda.synchronize()
        assert np.array_equal(lat.bonds.cpu().numpy().reshape(-1), bonds), t
        assert np.array_equal(lat.labels.cpu().numpy().reshape(-1), labels), t
        assert np.array_equal(_state(lat), st), t
        assert [int(v) for v in rec[0].cpu()] == [int(v) for v in want], t


def test_cubic_many_sweeps_per_call_and_restart():
    """Twelve sweeps in one call (records of each), then a lattice restarted
    from the saved spins at t = 12; both follow the oracle."""
    Lx, Ly, Lz, q, seed = 140, 20, 12, 2, wl.SEED_BASE | 0x3D2
    lat = sw.CubicLattice(Lx, Ly, Lz, q=q, K=K3, seed=seed)
    rec = lat.sweep(12, records=True)
    T = oracle.threshold(K3)
    st, want = oracle.sw3_run(Lx, Ly, Lz, q, T, seed, 0, 0, 12, oracle.init_states3(Lx, Ly, Lz, q, seed))
    torch.cuda.synchronize()
    assert np.array_equal(rec.cpu().numpy(), want)
    assert np.array_equal(_state(lat), st)
    lat2 = sw.CubicLattice(Lx, Ly, Lz, q=q, K=K3, seed=seed, spins=lat.spins.clone(), t=12, keep_labels=True)
    lat2.sweep(3)
    st2, _ = oracle.sw3_run(Lx, Ly, Lz, q, T, seed, 0, 12, 2, st)
    st2, _b, labels, _r = oracle.sw3_sweep(Lx, Ly, Lz, q, T, seed, 0, 14, st2)
    torch.cuda.synchronize()
    assert np.array_equal(_state(lat2), st2)
    assert np.array_equal(lat2.labels.cpu().numpy().reshape(-1), labels)


@pytest.mark.parametrize("W,H,q", [(300, 200, 2), (129, 70, 3)])
def test_lz1_equals_square_lattice_on_gpu(W, H, q):
    """A cubic lattice with Lz = 1 follows the square-lattice sweep of the
    same library (its +z bonds join each site to itself)."""
    seed, K = wl.SEED_BASE | 0x3D3, (sw.ising_K(sw.BETA_C_ISING) if q == 2 else 1.0051)
    a = sw.SWLattice(W, H, q=q, K=K, seed=seed, keep_labels=True)
    b = sw.CubicLattice(W, H, 1, q=q, K=K, seed=seed, keep_labels=True)
    for t in range(4):
        a.sweep(1)
        b.sweep(1)
        torch.cuda.synchronize()
        assert torch.equal(a.spins.reshape(-1), b.spins.reshape(-1)), t
        assert torch.equal(a.labels.reshape(-1), b.labels.reshape(-1)), t


@pytest.mark.parametrize("L,sweeps", [(256, 3), (512, 2)])
def test_cubic_full_size(L, sweeps):
    """The 3D Ising lattice at the critical coupling, against the oracle after
    every sweep (spins and records; labels of the last sweep)."""
    seed = wl.SEED_BASE | 0x3D4
    print(f"cubic L={L}^3 Ising at beta_c", flush=True)
    lat = sw.CubicLattice(L, L, L, q=2, K=K3, seed=seed, keep_labels=True)
    T = oracle.threshold(K3)
    st = oracle.init_states3(L, L, L, 2, seed)
    for t in range(sweeps):
        rec = lat.sweep(1, records=True)
        st, _b, labels, want = oracle.sw3_sweep(L, L, L, 2, T, seed, 0, t, st)
        torch.cuda.synchronize()
        assert [int(v) for v in rec[0].cpu()] == [int(v) for v in want], t
        assert np.array_equal(_state(lat), st), t
    assert np.array_equal(lat.labels.cpu().numpy().reshape(-1), labels)


def test_cubic_largest():
    """The largest cubic shape class the library accepts (N just below 2^31,
    ragged along z): one sweep, checked where the oracle cannot run whole.
    At 6000 sampled sites (and the corners): the initial state, the three
    bond bits from the Philox words of the definition, labels that are
    canonical (a root labels itself and is the smallest index seen) and equal
    across every active sampled bond, and the new state drawn at the label;
    over the whole lattice, the recorded state counts, active bonds and
    clusters."""
    Lx, Ly, Lz = 1024, 1024, 2047
    N = Lx * Ly * Lz
    assert N < 2**31
    seed = wl.SEED_BASE | 0x3D7
    print(f"cubic {Lx}x{Ly}x{Lz} (N={N})", flush=True)
    lat = sw.CubicLattice(Lx, Ly, Lz, q=2, K=K3, seed=seed, keep_labels=True, keep_bonds=True)
    before = _state(lat)
    rec = lat.sweep(1, records=True)[0].cpu().numpy()
    torch.cuda.synchronize()
    after = _state(lat)
    bonds = lat.bonds.cpu().numpy().reshape(-1)
    labels = lat.labels.cpu().numpy().reshape(-1)
    del lat
    torch.cuda.empty_cache()
    T = oracle.threshold(K3)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    rng = np.random.default_rng(11)
    sample = [0, Lx - 1, Lx * Ly - 1, N - Lx * Ly, N - 1] + [int(v) for v in rng.integers(0, N, 6000)]
    plane = Lx * Ly
    for i in sample:
        x, y, z = i % Lx, (i // Lx) % Ly, i // plane
        w = oracle.philox([i >> 2, 0, oracle.TAG_INIT, 0], key)[i & 3]
        nbr = [z * plane + y * Lx + (x + 1) % Lx, z * plane + ((y + 1) % Ly) * Lx + x,
               ((z + 1) % Lz) * plane + y * Lx + x]
        b = oracle.philox([i >> 1, 0, oracle.TAG_BOND, 0], key)
        bz = oracle.philox([i >> 2, 0, oracle.TAG_BOND_Z, 0], key)
        words = [int(b[2 * (i & 1)]), int(b[2 * (i & 1) + 1]), int(bz[i & 3])]
        want = sum(1 << k for k in range(3) if before[i] == before[nbr[k]] and words[k] < T)
        assert before[i] == (int(w) * 2) >> 32, i
        assert bonds[i] == want, i
        r = int(labels[i])
        assert 0 <= r <= i and labels[r] == r, i
        for k in range(3):
            if (want >> k) & 1:
                assert labels[nbr[k]] == r, (i, k)
                assert r <= nbr[k]
        f = oracle.philox([r >> 2, 0, oracle.TAG_FLIP, 0], key)[r & 3]
        assert after[i] == (int(f) * 2) >> 32, i
    n1 = int(np.count_nonzero(after))
    assert [int(v) for v in rec[oracle.REC3_COUNTS:oracle.REC3_COUNTS + 2]] == [N - n1, n1]
    active = sum(int(np.count_nonzero(bonds & (1 << k))) for k in range(3))
    assert int(rec[oracle.REC3_ACTIVE]) == active
    roots, step = 0, 1 << 27
    for c0 in range(0, N, step):
        c1 = min(N, c0 + step)
        roots += int(np.count_nonzero(labels[c0:c1] == np.arange(c0, c1, dtype=np.int32)))
    assert int(rec[oracle.REC3_NCLUST]) == roots


def test_cubic_side_stream():
    """Sweeps enqueued on a stream other than the current one follow the
    oracle once that stream is synchronised."""
    Lx, Ly, Lz, seed = 96, 40, 33, wl.SEED_BASE | 0x3D8
    lat = sw.CubicLattice(Lx, Ly, Lz, q=3, K=1.0, seed=seed, ising=False, keep_labels=True)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    rec = lat.sweep(4, records=True, stream=side)
    side.synchronize()
    T = oracle.threshold(1.0)
    st, want = oracle.sw3_run(Lx, Ly, Lz, 3, T, seed, 0, 0, 3, oracle.init_states3(Lx, Ly, Lz, 3, seed))
    st, _b, labels, last = oracle.sw3_sweep(Lx, Ly, Lz, 3, T, seed, 0, 3, st)
    assert np.array_equal(rec.cpu().numpy()[:3], want)
    assert [int(v) for v in rec[3].cpu()] == [int(v) for v in last]
    assert np.array_equal(lat.spins.cpu().numpy().reshape(-1), st)
    assert np.array_equal(lat.labels.cpu().numpy().reshape(-1), labels)


def _bonds3(Lx, Ly, Lz, p, seed, junk=False):
    """Random packed cubic bonds, each bond present with probability p; with
    junk the unused high bits are set at random too."""
    rng = np.random.default_rng(seed)
    N = Lx * Ly * Lz
    b = ((rng.random((N, 3)) < p) * np.array([1, 2, 4])).sum(axis=1).astype(np.uint8)
    if junk:
        b |= (rng.integers(0, 32, N).astype(np.uint8) << 3)
    return b


@pytest.mark.parametrize("Lx,Ly,Lz", [(1, 1, 1), (2, 2, 2), (1, 40, 3), (33, 70, 20), (132, 13, 9), (64, 64, 64),
                                       (257, 11, 17)])
def test_ccl3_parity(Lx, Ly, Lz):
    """Labels and cluster counts of random cubic bonds (several densities,
    junk in the unused bits) against the oracle."""
    print(f"ccl3 Lx={Lx} Ly={Ly} Lz={Lz}", flush=True)
    for k, p in enumerate((0.0, 0.2, 0.2488, 0.4, 1.0)):
        b = _bonds3(Lx, Ly, Lz, p, seed=7000 + k + Lx * 131 + Ly * 7 + Lz, junk=k % 2 == 1)
        labels, n = sw.ccl3_label(torch.from_numpy(b.reshape(Lz, Ly, Lx)).cuda())
        want, nref = oracle.label_bonds3(Lx, Ly, Lz, b & 7)
        assert n == nref, (p, n, nref)
        assert np.array_equal(labels.cpu().numpy().reshape(-1), want), p


def test_ccl3_percolation_512():
    """Bond percolation on the simple cubic lattice 512^3 near its threshold
    (p = 0.2488), against the oracle; a caller workspace reused twice."""
    L = 512
    b = _bonds3(L, L, L, 0.2488, seed=wl.SEED_BASE | 0xCC3)
    g = torch.from_numpy(b.reshape(L, L, L)).cuda()
    ws = torch.empty(sw._lib.lib().ccl3_workspace_bytes(L, L, L) + 256, dtype=torch.uint8, device="cuda")
    ws = ws[(-ws.data_ptr()) % 256:]
    print("ccl3 512^3 bond percolation", flush=True)
    labels, n = sw.ccl3_label(g, workspace=ws)
    want, nref = oracle.label_bonds3(L, L, L, b)
    assert n == nref
    assert np.array_equal(labels.cpu().numpy().reshape(-1), want)
    labels2, n2 = sw.ccl3_label(g, workspace=ws)
    assert n2 == n and torch.equal(labels, labels2)
