"""GPU parity of batched sweeps: every lattice of a batch follows the oracle's
single-lattice trajectory bit-exactly (spins, bonds, labels, counters)."""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _state(t, ising):
    s = t.cpu().numpy().reshape(-1)
    if ising:
        return ((s.astype(np.int16) + 1) // 2).astype(np.uint8)
    return s.astype(np.uint8)


MIX = [
    dict(W=64, H=64, q=2, K=wl.K_ISING_C, seed=wl.SEED_BASE | 0x31),
    dict(W=257, H=95, q=2, K=wl.K_ISING_C, seed=5),
    dict(W=2, H=2, q=2, K=0.7, seed=6),
    dict(W=130, H=33, q=3, ising=False, K=wl.K_POTTS3_C, seed=7),
    dict(W=300, H=3, q=4, ising=False, K=1.1, seed=8),
    dict(W=33, H=200, q=3, ising=False, K=1.0, seed=9),
    dict(W=1000, H=70, q=8, ising=False, K=1.7, seed=10),
    dict(W=32, H=32, q=2, K=float("inf"), seed=11),
    dict(W=129, H=65, q=255, ising=False, K=3.0, seed=12),
    dict(W=96, H=400, q=2, K=0.0, seed=13),
]


@pytest.mark.parametrize("tile", [{}, dict(tile_h=16, merge_waves=4), dict(tile_h=32), dict(tile_h=128, merge_waves=16),
                                  dict(fused=True), dict(fused=True, tile_h=32, merge_waves=4)],
                         ids=["phases", "phases-h16m4", "phases-h32", "phases-h128m16", "fused", "fused-h32m4"])
def test_batch_mixed_parity(tile):
    specs = [dict(sp, stream_id=j) for j, sp in enumerate(MIX)]
    b = sw.SWBatch(specs, keep_labels=True, keep_bonds=True, **tile)
    st = []
    for sp in b.specs:
        st.append(oracle.init_states(sp["W"], sp["H"], sp["q"], sp["seed"], sp["stream_id"]))
    torch.cuda.synchronize()
    for j, sp in enumerate(b.specs):
        assert np.array_equal(_state(b.spins[j], sp["ising"]), st[j]), j
    for t in range(3):
        b.sweep(1)
        torch.cuda.synchronize()
        for j, sp in enumerate(b.specs):
            W, H, q = sp["W"], sp["H"], sp["q"]
            print(f"batch lattice {j} W={W} H={H} q={q} t={t}", flush=True)
            T = oracle.threshold(sp["K"])
            new, bonds, labels, rec = oracle.sw_sweep(W, H, q, T, sp["seed"], sp["stream_id"], t, st[j])
            assert np.array_equal(b.bonds[j].cpu().numpy().reshape(-1), bonds), (j, t)
            assert np.array_equal(b.labels[j].cpu().numpy().reshape(-1), labels), (j, t)
            assert np.array_equal(_state(b.spins[j], sp["ising"]), new), (j, t)
            o = b.observables(j)
            assert o["t"] == t + 1
            assert o["n_active_bonds"] == rec[oracle.REC_ACTIVE]
            assert o["n_clusters"] == rec[oracle.REC_NCLUST]
            assert o["n_sat"] == rec[oracle.REC_NSAT]
            assert o["digest_spins"] == oracle.digest(new)
            assert o["digest_labels"] == oracle.digest(labels)
            st[j] = new
    assert b.t == 3


@pytest.mark.parametrize("fused", [False, True], ids=["phases", "fused"])
def test_batch256(fused):
    """The batched workload (256 Ising lattices, L = 32..1024): two sweeps, every lattice."""
    specs = wl.batch_specs()
    b = sw.SWBatch(specs, fused=fused)
    b.sweep(2)
    torch.cuda.synchronize()
    for j, sp in enumerate(b.specs):
        W, H = sp["W"], sp["H"]
        st = oracle.init_states(W, H, 2, sp["seed"], sp["stream_id"])
        st, rec = oracle.sw_run(W, H, 2, oracle.threshold(sp["K"]), sp["seed"], sp["stream_id"], 0, 2, st)
        assert np.array_equal(_state(b.spins[j], True), st), j
        if j % 37 == 0:
            o = b.observables(j)
            assert o["n_clusters"] == rec[1, oracle.REC_NCLUST], j
            assert o["n_sat"] == rec[1, oracle.REC_NSAT], j


@pytest.mark.parametrize("fused", [False, True], ids=["phases", "fused"])
def test_batch_graph_replays(fused):
    """Sweeps replayed from a captured HIP graph, mixed with eager sweeps and
    with eager work and synchronisations between the replays: every sweep of
    every lattice matches the oracle."""
    specs = [dict(sp, stream_id=j) for j, sp in enumerate(MIX)]
    b = sw.SWBatch(specs, keep_labels=True, keep_bonds=True, fused=fused)
    st = [oracle.init_states(sp["W"], sp["H"], sp["q"], sp["seed"], sp["stream_id"]) for sp in b.specs]
    for t, graph in enumerate([True, True, False, True, True]):
        print(f"batch graph replay t={t} graph={graph}", flush=True)
        b.sweep(1, graph=graph)
        torch.cuda.synchronize()
        for j, sp in enumerate(b.specs):
            W, H, q = sp["W"], sp["H"], sp["q"]
            T = oracle.threshold(sp["K"])
            new, bonds, labels, rec = oracle.sw_sweep(W, H, q, T, sp["seed"], sp["stream_id"], t, st[j])
            assert np.array_equal(b.bonds[j].cpu().numpy().reshape(-1), bonds), (j, t)
            assert np.array_equal(b.labels[j].cpu().numpy().reshape(-1), labels), (j, t)
            assert np.array_equal(_state(b.spins[j], sp["ising"]), new), (j, t)
            o = b.observables(j)  # eager work between the replays
            assert o["t"] == t + 1
            assert o["n_clusters"] == rec[oracle.REC_NCLUST]
            st[j] = new
    assert b.t == 5


@pytest.mark.parametrize("fused", [False, True], ids=["phases", "fused"])
def test_batch_graph_chunks(fused):
    """Calls of several sweeps replay the eight-sweep graph (then single-sweep
    ones): after calls of 8, 11 and 8 sweeps, with eager work between them,
    every lattice equals the oracle."""
    specs = [dict(sp, stream_id=j) for j, sp in enumerate(MIX)]
    b = sw.SWBatch(specs, fused=fused)
    st = [oracle.init_states(sp["W"], sp["H"], sp["q"], sp["seed"], sp["stream_id"]) for sp in b.specs]
    t = 0
    for n in (8, 11, 8):
        print(f"batch graph chunk t={t} n={n}", flush=True)
        b.sweep(n, graph=True)
        torch.cuda.synchronize()
        for j, sp in enumerate(b.specs):
            T = oracle.threshold(sp["K"])
            st[j], rec = oracle.sw_run(sp["W"], sp["H"], sp["q"], T, sp["seed"], sp["stream_id"], t, n, st[j])
            assert np.array_equal(_state(b.spins[j], sp["ising"]), st[j]), (j, t, n)
            o = b.observables(j)  # eager work between the replays
            assert o["t"] == t + n and o["n_clusters"] == rec[-1, oracle.REC_NCLUST], (j, t, n)
        t += n
    assert b.t == 27
