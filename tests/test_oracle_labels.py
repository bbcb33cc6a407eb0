"""Pins of the oracle's connected-component labeling.

* brute-force BFS (a different algorithm) on random small lattices, both
  boundary conditions, W != H, odd sizes, W or H of 1 and 2;
* every bond set of the 2x2 and 3x3 tori against vectorised label propagation;
* closed-form special cases;
* the exact left-right crossing probability 1/2 of bond percolation at p = 1/2
  on the (n+1)-wide, n-tall box (self-duality of the square lattice), exactly
  by enumeration for small n and statistically for larger n.
"""
import numpy as np
import pytest

import oracle
from tests import exact


def _rand_bonds(rng, N, p):
    r = rng.random((N, 2)) < p
    return (r[:, 0] | (r[:, 1] << 1)).astype(np.uint8)


@pytest.mark.parametrize("mode", [oracle.PERIODIC, oracle.OPEN])
def test_bonds_vs_bfs(mode):
    rng = np.random.default_rng(1 + mode)
    shapes = [(1, 1), (1, 5), (5, 1), (2, 2), (2, 3), (3, 2), (4, 4), (7, 5), (9, 13), (16, 16), (31, 17)]
    for W, H in shapes:
        for p in (0.0, 0.3, 0.5, 0.7, 1.0):
            b = _rand_bonds(rng, W * H, p)
            lab, n = oracle.label_bonds(W, H, b, mode)
            ref = exact.bfs_labels(W, H, b, periodic=(mode == oracle.PERIODIC))
            assert np.array_equal(lab, ref), (W, H, p)
            assert n == int((ref == np.arange(W * H)).sum())


def test_sites_vs_bfs():
    rng = np.random.default_rng(7)
    for W, H in [(1, 1), (1, 9), (9, 1), (2, 2), (5, 7), (16, 9), (33, 20)]:
        for p in (0.0, 0.4, 0.6, 1.0):
            occ = (rng.random(W * H) < p).astype(np.uint8)
            lab, n = oracle.label_sites(W, H, occ)
            ref = exact.bfs_site_labels(W, H, occ)
            assert np.array_equal(lab, ref), (W, H, p)
            assert n == int((ref == np.arange(W * H)).sum())


@pytest.mark.parametrize("W,H", [(2, 2), (3, 3)])
def test_torus_exhaustive(W, H):
    packed, _ = exact.all_bond_sets(W, H)
    ref = exact.propagate_labels(W, H, packed)
    for k in range(packed.shape[0]):
        lab, _ = oracle.label_bonds(W, H, packed[k], oracle.PERIODIC)
        if not np.array_equal(lab, ref[k]):
            raise AssertionError((W, H, k, lab, ref[k]))


def test_special_cases():
    W, H = 12, 7
    N = W * H
    lab, n = oracle.label_bonds(W, H, np.zeros(N, np.uint8))
    assert np.array_equal(lab, np.arange(N)) and n == N
    lab, n = oracle.label_bonds(W, H, np.full(N, 3, np.uint8))
    assert np.all(lab == 0) and n == 1
    # open boundary, only wrap bonds set: nothing connects
    b = np.zeros(N, np.uint8)
    b[np.arange(H) * W + W - 1] |= 1
    b[(H - 1) * W + np.arange(W)] |= 2
    lab, n = oracle.label_bonds(W, H, b, oracle.OPEN)
    assert n == N
    # periodic: the same wrap bonds form H row pairs + W column pairs glued at a corner
    lab, n = oracle.label_bonds(W, H, b, oracle.PERIODIC)
    ref = exact.bfs_labels(W, H, b, True)
    assert np.array_equal(lab, ref)
    # a stripe spanning the torus horizontally
    b = np.zeros(N, np.uint8)
    b[3 * W: 4 * W] = 1
    lab, n = oracle.label_bonds(W, H, b)
    assert np.all(lab[3 * W: 4 * W] == 3 * W) and n == N - W + 1
    # images: full, empty, checkerboard
    lab, n = oracle.label_sites(W, H, np.ones(N, np.uint8))
    assert np.all(lab == 0) and n == 1
    lab, n = oracle.label_sites(W, H, np.zeros(N, np.uint8))
    assert np.all(lab == -1) and n == 0
    cb = ((np.arange(N) % W + np.arange(N) // W) % 2 == 0).astype(np.uint8)
    lab, n = oracle.label_sites(W, H, cb)
    assert n == int(cb.sum()) and np.array_equal(lab[cb == 1], np.nonzero(cb)[0])


def _crosses(W, lab):
    H = lab.size // W
    left = set(lab[np.arange(H) * W].tolist())
    right = set(lab[np.arange(H) * W + W - 1].tolist())
    return bool(left & right)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_crossing_probability_exact(n):
    """Exactly half of all relevant bond sets cross (p = 1/2)."""
    W, H = n + 1, n
    rel = exact.crossing_bits(n)
    hits = 0
    total = 1 << len(rel)
    for code in range(total):
        b = np.zeros(W * H, np.uint8)
        for e, (site, bit) in enumerate(rel):
            if (code >> e) & 1:
                b[site] |= bit
        # bonds that cannot change the event (wrap bonds, which open mode
        # ignores, and vertical bonds on the two side columns) are set at random
        rel_set = set(rel)
        for site in range(W * H):
            for bit in (1, 2):
                if (site, bit) not in rel_set and ((code * 2654435761 + 97 * site + bit) >> 7) & 1:
                    b[site] |= bit
        lab, _ = oracle.label_bonds(W, H, b, oracle.OPEN)
        hits += _crosses(W, lab)
    assert 2 * hits == total


def test_crossing_probability_statistical():
    n, samples = 24, 6000
    W, H = n + 1, n
    rng = np.random.default_rng(99)
    hits = 0
    for _ in range(samples):
        b = rng.integers(0, 4, size=W * H, dtype=np.uint8)  # every bond p = 1/2
        lab, _ = oracle.label_bonds(W, H, b, oracle.OPEN)
        hits += _crosses(W, lab)
    frac = hits / samples
    sigma = 0.5 / np.sqrt(samples)
    assert abs(frac - 0.5) < 5 * sigma, frac


def test_cluster_sizes():
    rng = np.random.default_rng(3)
    W, H = 20, 13
    b = _rand_bonds(rng, W * H, 0.55)
    lab, n = oracle.label_bonds(W, H, b)
    roots, sizes, mx = oracle.cluster_sizes(lab)
    assert roots.size == n and np.all(np.diff(roots) > 0)
    assert sizes.sum() == W * H and mx == sizes.max()
    for r, s in zip(roots, sizes):
        assert (lab == r).sum() == s
    occ = (rng.random(W * H) < 0.5).astype(np.uint8)
    lab, n = oracle.label_sites(W, H, occ)
    roots, sizes, _ = oracle.cluster_sizes(lab)
    assert roots.size == n and sizes.sum() == occ.sum()
