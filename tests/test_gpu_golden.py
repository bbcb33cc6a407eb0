"""Full-length GPU parity against stored oracle records.

tests/golden/sweeps_<workload>.txt hold, for every sweep of the benchmark
workloads, what the CPU oracle reports (written by
tests/golden/make_sweep_records.py, which calls only oracle/): active bonds,
clusters and the largest cluster of the sweep's bond configuration (SW steps
1-2, Sec. II), satisfied bonds (-H/J, Eq. potts_hamiltonian) and state counts
of the spins after the flip (step 3), and order-independent digests of the
spins, labels and bond bytes.  The library must reproduce every record, sweep
by sweep, over the whole run: 1000 sweeps of Ising L = 64, 200 + 1000 of
Ising L = 4096, the 100 of q = 3 Potts L = 16384 (which covers the sweeps the
benchmark times), every lattice of the batched workload at its
checkpoints, 300 sweeps of the few-cluster update on Ising L = 1024, and 400
sweeps of the simple cubic Ising lattice 128^3.  A digest is a 64-bit sum of
one Philox block per element, so any differing element shows in it.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _records(name):
    path = os.path.join(GOLDEN, f"sweeps_{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_sweep_records.py {name})")
    recs = []
    for ln in open(path):
        if ln.startswith("#"):
            continue
        f = ln.split()
        recs.append(f)
    return recs


def _compare(o, f, q, t, what):
    n = 5 + q
    want = {
        "t": int(f[0]),
        "n_active_bonds": int(f[1]),
        "n_clusters": int(f[2]),
        "max_cluster": int(f[3]),
        "n_sat": int(f[4]),
        "counts": [int(c) for c in f[5:n]][:8],
        "digest_spins": int(f[n], 16),
        "digest_labels": int(f[n + 1], 16),
        "digest_bonds": int(f[n + 2], 16),
    }
    assert want["t"] == t
    got = {k: o[k] for k in want if k != "t"}
    got["t"] = t
    assert got == want, f"{what}: sweep {t}"


def _run_single(name, tile_kw=None):
    c = wl.CONFIGS[name]
    recs = _records(name)
    total = c.warmup + c.sweeps
    assert len(recs) == total
    print(f"golden {name}: {total} sweeps", flush=True)
    lat = sw.SWLattice(c.W, c.H, q=c.q, K=c.K, seed=c.seed, ising=c.ising, keep_labels=True,
                       keep_bonds=True, sizes=True, **(tile_kw or {}))
    for t in range(total):
        lat.sweep(1)
        _compare(lat.observables(), recs[t], c.q, t, name)
        if t % 100 == 0:
            print(f"golden {name}: sweep {t} ok", flush=True)
    lat.close()


def test_ising64_every_sweep():
    _run_single("ising64")


def test_ising64_history_every_sweep():
    """The one-launch small-lattice path (records taken on the device)."""
    c = wl.CONFIGS["ising64"]
    recs = _records("ising64")
    lat = sw.SWLattice(c.W, c.H, q=2, K=c.K, seed=c.seed)
    hist = lat.sweep_history(c.sweeps).cpu().numpy()
    for t in range(c.sweeps):
        f = recs[t]
        assert int(hist[t, 0]) == int(f[1]) and int(hist[t, 1]) == int(f[2]), t
        assert int(hist[t, 3]) == int(f[4]), t
        assert [int(x) for x in hist[t, 4:6]] == [int(f[5]), int(f[6])], t
    o = lat.observables()
    assert o["digest_spins"] == int(recs[-1][7], 16)


def test_ising4096_every_sweep():
    _run_single("ising4096")


@pytest.mark.parametrize("tile", [{}, dict(tile_h=32, merge_waves=16), dict(tile_h=128, merge_waves=4)],
                         ids=["default", "h32m16", "h128m4"])
def test_potts16384_every_sweep(tile):
    _run_single("potts16384", tile)


def test_few1024_every_sweep():
    """The few-cluster update (Sec. III) on an Ising 1024 x 1024 lattice at
    beta_c, 32 x 32 seed tiles, p_flip = 1/2: all 300 recorded sweeps."""
    recs = _records("few1024")
    head = open(os.path.join(GOLDEN, "sweeps_few1024.txt")).readline()
    assert "few_b=32 p_flip=0.5" in head
    L, seed = 1024, wl.SEED_BASE | 0xFE
    lat = sw.SWLattice(L, L, q=2, K=wl.K_ISING_C, seed=seed, keep_labels=True, keep_bonds=True, sizes=True,
                       few_b=32, p_flip=0.5)
    print(f"golden few1024: {len(recs)} sweeps", flush=True)
    for t in range(len(recs)):
        lat.sweep(1)
        _compare(lat.observables(), recs[t], 2, t, "few1024")
        if t % 100 == 0:
            print(f"golden few1024: sweep {t} ok", flush=True)
    lat.close()


@pytest.mark.parametrize("fused", [False, True], ids=["phases", "fused"])
def test_batch256_checkpoints(fused):
    path = os.path.join(GOLDEN, "batch256.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_sweep_records.py batch256)")
    specs = wl.batch_specs()
    stored = {}
    for ln in open(path):
        f = ln.split()
        if not f or f[0] == "#" or ln.startswith("#"):
            continue
        if f[0] == "spec":
            j = int(f[1])
            sp = specs[j]
            assert (int(f[2]), int(f[3]), float(f[4]), int(f[5]), int(f[6])) == (
                sp["W"], sp["H"], sp["K"], sp["seed"], sp["stream_id"]), j
            continue
        stored.setdefault(int(f[1]) + 1, {})[int(f[0])] = f[1:]  # by sweeps done
    b = sw.SWBatch(specs, keep_labels=True, keep_bonds=True, fused=fused)
    done = 0
    for cp in sorted(stored):
        print(f"golden batch256: to sweep {cp}", flush=True)
        b.sweep(cp - done)
        done = cp
        for j in range(len(specs)):
            o = b.observables(j)
            f = stored[cp][j]
            _compare(dict(o, max_cluster=int(f[3])), f, 2, cp - 1, f"batch lattice {j}")


def test_cubic128_every_sweep():
    """The simple cubic Ising lattice 128^3 at its critical coupling: the
    record of every one of 400 sweeps (active bonds, clusters, satisfied
    bonds, state counts; sweeps run 40 to a call) and the spins' digest after
    every 40th sweep, against the oracle's file."""
    path = os.path.join(GOLDEN, "sweeps_cubic128.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_sweep_records.py cubic128)")
    head = open(path).readline()
    L = int(head.split("Lx=Ly=Lz=")[1].split()[0])
    K = float(head.split("K=")[1].split()[0])
    seed = int(head.split("seed=")[1].split()[0], 16)
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    lat = sw.CubicLattice(L, L, L, q=2, K=K, seed=seed)
    print(f"golden cubic128: {len(rows)} sweeps", flush=True)
    for c0 in range(0, len(rows), 40):
        rec = lat.sweep(min(40, len(rows) - c0), records=True).cpu().numpy()
        for k, r in enumerate(rows[c0:c0 + 40]):
            assert int(r[0]) == c0 + k
            assert [int(v) for v in rec[k][:5]] == [int(v) for v in r[1:6]], (c0 + k, rec[k][:5], r)
        s = lat.spins.cpu().numpy().reshape(-1)
        st = ((s.astype(np.int16) + 1) // 2).astype(np.uint8)
        assert oracle.digest(st) == int(rows[c0 + len(rec) - 1][6], 16), c0 + len(rec) - 1
        print(f"golden cubic128: sweep {c0 + len(rec) - 1} ok", flush=True)
