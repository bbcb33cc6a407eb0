"""GPU parity of the few-cluster update (Sec. III) against the CPU oracle
(bit-exact): the SW bonds and clusters, one seed per B x B seed tile, every
distinct seeded cluster flipped with probability p_flip.

Each case compares after every sweep: packed bonds, canonical labels, the spins
after the flip and the counters.  The cases cover seed tiles smaller than,
equal to and larger than the labeling tiles, ragged seed and labeling tiles,
B = 1 (every site a seed), one seed for the whole lattice, Ising and q = 2
Potts storage, every tile shape, the reversed tile order, cluster sizes, a
sweep number that comes round again after sw_set_t, and the full 16384^2
lattice.
"""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _state(lat):
    s = lat.spins.cpu().numpy().reshape(-1)
    if lat.ising:
        return ((s.astype(np.int16) + 1) // 2).astype(np.uint8)
    return s.astype(np.uint8)


def _check_obs(lat, rec, st):
    obs = lat.observables()
    nsat, counts = oracle.satisfied(lat.W, lat.H, 2, st)
    assert obs["n_active_bonds"] == rec[oracle.REC_ACTIVE]
    assert obs["n_clusters"] == rec[oracle.REC_NCLUST]
    assert obs["n_sat"] == nsat == rec[oracle.REC_NSAT]
    assert obs["counts"] == [int(c) for c in counts[:2]]


CASES = [
    # W, H, B, p_flip, ising, extra lattice arguments
    (64, 64, 16, 0.5, True, {}),
    (300, 200, 32, 0.9, True, {}),
    (257, 131, 7, 0.7, True, {}),            # odd W, ragged seed and labeling tiles
    (1000, 700, 1, 0.5, True, {}),           # every site a seed
    (130, 66, 200, 0.99, True, {}),          # one seed tile wider than the lattice
    (128, 64, 8, 0.6, False, {}),            # one labeling tile, q = 2 Potts storage
    (16, 2000, 5, 0.8, True, {}),            # thin
    (511, 300, 64, 0.75, True, dict(tile_h=16, merge_waves=4)),
    (511, 300, 13, 0.75, False, dict(tile_h=128, merge_waves=16)),
    (400, 333, 24, 0.6, True, dict(tile_h=32, reverse_tiles=True)),
    (2, 2, 1, 0.5, True, {}),
    (3, 130, 2, 0.5, True, {}),
]


@pytest.mark.parametrize("W,H,B,pf,ising,kw", CASES)
def test_few_parity(W, H, B, pf, ising, kw):
    print(f"case W={W} H={H} B={B} p_flip={pf} ising={ising} {kw}", flush=True)
    seed, sid, K = wl.SEED_BASE | 0xF3, 2, wl.K_ISING_C
    lat = sw.SWLattice(W, H, q=2, K=K, seed=seed, stream_id=sid, ising=ising, keep_labels=True, keep_bonds=True,
                       few_b=B, p_flip=pf, **kw)
    T, Tf = oracle.threshold(K), oracle.prob_threshold(pf)
    st = oracle.init_states(W, H, 2, seed, sid)
    flipped = 0
    for t in range(6):
        lat.sweep(1)
        new, bonds, labels, rec, few = oracle.few_sweep(W, H, T, Tf, B, seed, sid, t, st)
        torch.cuda.synchronize()
        assert np.array_equal(lat.bonds.cpu().numpy().reshape(-1), bonds), t
        assert np.array_equal(lat.labels.cpu().numpy().reshape(-1), labels), t
        assert np.array_equal(_state(lat), new), t
        _check_obs(lat, rec, new)
        flipped += few[1]
        st = new
    if W * H > 4:
        assert flipped > 0  # the cases do flip clusters


def test_few_sizes_and_history():
    W, H, B, pf, seed = 700, 300, 20, 0.5, wl.SEED_BASE | 0xF4
    K = wl.K_ISING_C
    lat = sw.SWLattice(W, H, q=2, K=K, seed=seed, sizes=True, few_b=B, p_flip=pf)
    T, Tf = oracle.threshold(K), oracle.prob_threshold(pf)
    st = oracle.init_states(W, H, 2, seed)
    for t in range(3):
        lat.sweep(1)
        st, _b, labels, rec, _f = oracle.few_sweep(W, H, T, Tf, B, seed, 0, t, st)
        roots, sizes = lat.cluster_sizes()
        r_ref, s_ref, mx = oracle.cluster_sizes(labels)
        assert np.array_equal(roots.cpu().numpy(), r_ref) and np.array_equal(sizes.cpu().numpy(), s_ref)
        assert lat.observables()["max_cluster"] == mx == rec[oracle.REC_MAXCL]
    hist = lat.sweep_history(4)
    for t in range(3, 7):
        st, _b, _l, rec, _f = oracle.few_sweep(W, H, T, Tf, B, seed, 0, t, st)
        assert [int(v) for v in hist[t - 3]] == [int(v) for v in rec], t
    torch.cuda.synchronize()
    assert np.array_equal(_state(lat), st)


def test_few_sweep_number_again_after_set_t():
    """Seed marks carry the sweep number: after sw_set_t moves t back, marks
    left by the first pass over those numbers must not count."""
    W, H, B, pf, seed = 640, 384, 48, 0.9, wl.SEED_BASE | 0xF5
    K = wl.K_ISING_C
    lat = sw.SWLattice(W, H, q=2, K=K, seed=seed, few_b=B, p_flip=pf)
    lat.sweep(6)
    other = oracle.init_states(W, H, 2, seed ^ 0x5A5A, 0)
    lat.spins.copy_(torch.from_numpy((other.astype(np.int16) * 2 - 1).astype(np.int8).reshape(H, W)))
    lat.t = 2
    T, Tf = oracle.threshold(K), oracle.prob_threshold(pf)
    st = other
    for t in range(2, 5):
        lat.sweep(1)
        st, *_ = oracle.few_sweep(W, H, T, Tf, B, seed, 0, t, st)
        torch.cuda.synchronize()
        assert np.array_equal(_state(lat), st), t


def test_few_zero_flip_probability():
    W, H = 512, 256
    lat = sw.SWLattice(W, H, q=2, seed=5, few_b=16, p_flip=0.0, keep_labels=True)
    torch.cuda.synchronize()
    before = lat.spins.clone()
    lat.sweep(3)
    torch.cuda.synchronize()
    assert torch.equal(lat.spins, before)


def test_few_16384():
    """Two few-cluster sweeps of the full 16384^2 Ising lattice at beta_c, seed
    tiles of 64 x 64, against the oracle."""
    L, B, pf, seed = 16384, 64, 0.5, wl.SEED_BASE | 0xF6
    K = wl.K_ISING_C
    print(f"few-cluster L={L} B={B}", flush=True)
    lat = sw.SWLattice(L, L, q=2, K=K, seed=seed, few_b=B, p_flip=pf)
    T, Tf = oracle.threshold(K), oracle.prob_threshold(pf)
    st = oracle.init_states(L, L, 2, seed)
    for t in range(2):
        lat.sweep(1)
        st, _b, _l, rec, few = oracle.few_sweep(L, L, T, Tf, B, seed, 0, t, st)
        torch.cuda.synchronize()
        assert np.array_equal(_state(lat), st), t
        assert few[0] > 0 and few[1] > 0
        _check_obs(lat, rec, st)
