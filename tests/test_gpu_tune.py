"""The autotuner on the device: every candidate is timed, the choice is cached,
and a lattice built with the tuned shape still follows the oracle bit-exactly."""
import numpy as np
import pytest

import oracle
import paper_1105_5804_amd as sw
from paper_1105_5804_amd import tune
from paper_1105_5804_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tune_sweep_and_tuned_lattice(tmp_path, monkeypatch):
    monkeypatch.setenv("SWCCL_TUNE_CACHE", str(tmp_path / "tune.json"))
    W, H, q, seed = 700, 300, 3, wl.SEED_BASE | 0x7E
    print(f"tune sweep W={W} H={H} q={q}", flush=True)
    e = tune.tune_sweep(W, H, q=q, K=wl.K_POTTS3_C, ising=False, reps=3, warmup=2)
    assert tuple(e["choice"]) in tune.CANDIDATES and len(e["timings"]) == len(tune.CANDIDATES)
    assert all(ms > 0 for ms in e["timings"].values())
    assert tune.tune_sweep(W, H, q=q, K=wl.K_POTTS3_C, ising=False) == e  # cached
    lat = tune.tuned_lattice(W, H, q=q, K=wl.K_POTTS3_C, ising=False, seed=seed, keep_labels=True)
    assert [lat.tile_h, lat.merge_waves] == e["choice"]
    T = oracle.threshold(wl.K_POTTS3_C)
    st = oracle.init_states(W, H, q, seed)
    for t in range(2):
        lat.sweep(1)
        st, _b, labels, _r = oracle.sw_sweep(W, H, q, T, seed, 0, t, st)
        torch.cuda.synchronize()
        assert np.array_equal(lat.labels.cpu().numpy().reshape(-1), labels)
        assert np.array_equal(lat.spins.cpu().numpy().reshape(-1), st)


def test_tune_ccl_and_batch(tmp_path, monkeypatch):
    monkeypatch.setenv("SWCCL_TUNE_CACHE", str(tmp_path / "tune.json"))
    img = torch.from_numpy(wl.site_image(900, 700, 0.5927, seed=81)).cuda()
    print("tune ccl 900x700 sites", flush=True)
    e = tune.tune_ccl(img, "sites_open", sizes=True, reps=2)
    assert tuple(e["choice"]) in tune.CANDIDATES
    th, mw = e["choice"]
    lab, roots, sizes, n = sw.ccl_label(img, "sites_open", sizes=True, tile_h=th, merge_waves=mw)
    want, nref = oracle.label_sites(900, 700, img.cpu().numpy().reshape(-1))
    assert n == nref and np.array_equal(lab.cpu().numpy().reshape(-1), want)
    specs = [dict(W=64, H=64, K=wl.K_ISING_C, seed=1, stream_id=0), dict(W=300, H=200, K=wl.K_ISING_C, seed=2,
                                                                        stream_id=1)]
    print("tune batch of 2", flush=True)
    eb = tune.tune_batch(specs, reps=2, warmup=1)
    assert eb["choice"][2] in ("fused", "phases") and len(eb["timings"]) == 24
