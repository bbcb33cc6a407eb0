"""The seeded input recipes: deterministic, in range, and distributed as stated
(closed-form moments checked on large samples, several standard errors wide)."""
import math

import numpy as np

from paper_1105_5804_amd import workloads as wl


def test_configs():
    c = wl.CONFIGS
    assert (c["potts16384"].W, c["potts16384"].H, c["potts16384"].q) == (16384, 16384, 3)
    assert (c["ising4096"].W, c["ising4096"].keep_bonds, c["ising4096"].warmup) == (4096, True, 200)
    assert (c["ising64"].W, c["ising64"].sweeps) == (64, 1000)
    # critical couplings: p_c = sqrt(q) / (1 + sqrt(q)) for K = ln(1 + sqrt(q))
    for K, q in ((wl.K_ISING_C, 2), (wl.K_POTTS3_C, 3)):
        assert math.isclose(-math.expm1(-K), math.sqrt(q) / (1 + math.sqrt(q)), rel_tol=1e-15)
    assert len({cfg.seed for cfg in c.values()}) == len(c)


def test_batch_specs():
    a, b = wl.batch_specs(), wl.batch_specs()
    assert a == b and len(a) == 256
    assert [s["stream_id"] for s in a] == list(range(256))
    assert len({s["seed"] for s in a}) == 256
    bc = 0.5 * wl.K_ISING_C
    for s in a:
        assert s["W"] == s["H"] and s["W"] in (32, 64, 128, 256, 512, 1024)
        assert 2 * bc * 0.9 <= s["K"] <= 2 * bc * 1.1
    # each of the six sides with probability 1/6 (binomial, 4 sigma on 6000 draws)
    big = wl.batch_specs(6000, seed=123)
    counts = np.bincount([int(math.log2(s["W"])) - 5 for s in big], minlength=6)
    assert np.all(np.abs(counts - 1000) < 4 * math.sqrt(6000 * (1 / 6) * (5 / 6)))


def test_served_requests():
    r = wl.served_requests(20000)
    assert r == wl.served_requests(20000)
    N = np.array([x["N"] for x in r], dtype=np.float64)
    assert N.min() >= 64 and N.max() <= 8192
    total = wl.SERVED_POOL_SIDE ** 2
    for x in r[:2000]:
        assert 0 <= x["level"] < wl.SERVED_POOL_LEVELS
        assert 0 <= x["offset"] and x["offset"] + x["N"] ** 2 <= total
    # log-uniform side on [64, 8192]: E[N^2] = (8192^2 - 64^2) / (2 ln 128)
    want = (8192.0 ** 2 - 64.0 ** 2) / (2 * math.log(128))
    assert abs(np.mean(N ** 2) / want - 1) < 0.05
    assert abs(np.mean(np.log(N)) - (math.log(64) + math.log(8192)) / 2) < 0.03
    gaps = np.array([x["gap"] for x in r])
    assert np.all(gaps >= 0) and abs(gaps.mean() - 1) < 0.04  # unit-rate exponential
    levels = np.bincount([x["level"] for x in r], minlength=wl.SERVED_POOL_LEVELS)
    assert np.all(np.abs(levels - 2500) < 4 * math.sqrt(20000 * (1 / 8) * (7 / 8)))
    ps = [wl.served_pool_p(k) for k in range(wl.SERVED_POOL_LEVELS)]
    assert 0.40 < min(ps) and max(ps) < 0.70 and ps == sorted(ps)


def test_random_inputs():
    b = wl.percolation_bonds(512, 384, seed=7)
    assert b.shape == (384, 512) and b.dtype == np.uint8 and b.max() <= 3
    assert np.array_equal(b, wl.percolation_bonds(512, 384, seed=7))
    n = b.size
    for bit in (1, 2):
        assert abs(np.mean((b & bit) != 0) - 0.5) < 4 * math.sqrt(0.25 / n)
    for p in (0.0, 0.3, 1.0):
        rb = wl.random_bonds(300, 200, p, seed=11)
        assert rb.shape == (200, 300) and rb.max() <= 3
        for bit in (1, 2):
            assert abs(np.mean((rb & bit) != 0) - p) <= 4 * math.sqrt(p * (1 - p) / rb.size) + 1e-12
        im = wl.site_image(300, 200, p, seed=12)
        assert im.shape == (200, 300) and set(np.unique(im)) <= {0, 1}
        assert abs(im.mean() - p) <= 4 * math.sqrt(p * (1 - p) / im.size) + 1e-12
