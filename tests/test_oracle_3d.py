"""Pins of the oracle's simple cubic lattice sweep (the 3D generalisation of
the SW update of Sec. II: three bonds per site, the same three steps).

What fixes it, independently of the oracle's own code:

* Lz = 1 reduces it to the square lattice: the +z bond joins a site to itself,
  the +x and +y words are the square lattice's, so states, labels and the
  +x/+y bond bits equal the (separately pinned) square-lattice sweep, with N
  extra satisfied bonds and the self-bonds counted as active;
* labels of random 3D bond configurations equal those of a breadth-first
  search over an explicit adjacency list (tests/exact.py), including
  degenerate extents 1 and 2 (self-bonds and doubled bonds);
* the Philox word of every bond, recomputed from rocRAND's independent
  Philox4x32-10 with the counter layout written out;
* satisfied bonds and state counts recounted with numpy rolls;
* the chain's stationary law: long runs on the 2 x 2 x 2 lattice (q = 2 and
  q = 3) give the exact Boltzmann distribution of the satisfied-bond count,
  by enumeration of every spin state, within a chi-square bound.

Copies of the oracle with one plausible mistake planted are compiled and must
fail at least one of these checks.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests.exact import all_states, bfs_labels_cubic, cubic_edges
from tests.test_oracle_philox import _rocrand_blocks

SEED = 0x1105580400003D3D


def _roll_nsat(Lx, Ly, Lz, st):
    s = np.asarray(st).reshape(Lz, Ly, Lx)
    return int(sum((s == np.roll(s, -1, axis=a)).sum() for a in (0, 1, 2)))


# --------------------------------------------------------- Lz = 1 reduction --
def _reduction_mismatches(shapes=((9, 6), (16, 3), (5, 7), (7, 1)), sweeps=4):
    bad = []
    for W, H in shapes:
        for q, K in ((2, 0.8814), (3, 1.0051)):
            T = oracle.threshold(K)
            s2 = oracle.init_states(W, H, q, SEED, 3)
            s3 = oracle.init_states3(W, H, 1, q, SEED, 3)
            if not np.array_equal(s2, s3):
                bad.append(("init", W, H, q))
            for t in range(sweeps):
                s2, b2, l2, r2 = oracle.sw_sweep(W, H, q, T, SEED, 3, t, s2)
                s3, b3, l3, r3 = oracle.sw3_sweep(W, H, 1, q, T, SEED, 3, t, s3)
                ok = (np.array_equal(s2, s3) and np.array_equal(l2, l3) and np.array_equal(b2, b3 & 3)
                      and r3[oracle.REC3_ACTIVE] == r2[oracle.REC_ACTIVE] + int(((b3 >> 2) & 1).sum())
                      and r3[oracle.REC3_NCLUST] == r2[oracle.REC_NCLUST]
                      and r3[oracle.REC3_NSAT] == r2[oracle.REC_NSAT] + W * H
                      and np.array_equal(r3[oracle.REC3_COUNTS:], r2[oracle.REC_COUNTS:]))
                if not ok:
                    bad.append((W, H, q, t))
                    break
    return bad


def test_lz1_is_the_square_lattice():
    assert _reduction_mismatches() == []


# ---------------------------------------------------------------- labels ----
LABEL_SHAPES = [(4, 3, 5), (1, 5, 3), (7, 1, 2), (2, 2, 2), (3, 4, 1), (6, 5, 4), (1, 1, 6), (5, 2, 3)]


def _label_mismatches():
    bad = []
    rng = np.random.default_rng(33)
    for Lx, Ly, Lz in LABEL_SHAPES:
        N = Lx * Ly * Lz
        for dens in (0.2, 0.35, 0.6):
            bonds = ((rng.random((N, 3)) < dens) * np.array([1, 2, 4])).sum(axis=1).astype(np.uint8)
            labels, n = oracle.label_bonds3(Lx, Ly, Lz, bonds)
            want = bfs_labels_cubic(Lx, Ly, Lz, bonds)
            if not np.array_equal(labels, want) or n != len(set(want.tolist())):
                bad.append((Lx, Ly, Lz, dens))
    return bad


def test_labels_match_bfs():
    assert _label_mismatches() == []


# ---------------------------------------------------------------- words -----
def _word_mismatches(Lx=5, Ly=3, Lz=4, t=6, sid=9):
    """Bonds of two-valued spins (most pairs equal) at T = 2^31 against the
    words rocRAND gives for the layout: +x word 2(i&1) and +y word 2(i&1)+1 of
    block(i>>1, t, BOND), +z word i&3 of block(i>>2, t, BOND_Z)."""
    N = Lx * Ly * Lz
    key = [SEED & 0xFFFFFFFF, SEED >> 32]
    ctrs = sorted({(i >> 1, t, oracle.TAG_BOND, sid) for i in range(N)}
                  | {(i >> 2, t, oracle.TAG_BOND_Z, sid) for i in range(N)})
    blk = dict(zip(ctrs, _rocrand_blocks([list(c) + key for c in ctrs])))
    rng = np.random.default_rng(8)
    st = (rng.random(N) < 0.8).astype(np.uint8)
    T = 2**31
    want = np.zeros(N, dtype=np.uint8)
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = (z * Ly + y) * Lx + x
                nb = [(z * Ly + y) * Lx + (x + 1) % Lx, (z * Ly + (y + 1) % Ly) * Lx + x,
                      (((z + 1) % Lz) * Ly + y) * Lx + x]
                b = blk[(i >> 1, t, oracle.TAG_BOND, sid)]
                bz = blk[(i >> 2, t, oracle.TAG_BOND_Z, sid)]
                words = [b[2 * (i & 1)], b[2 * (i & 1) + 1], bz[i & 3]]
                for k in range(3):
                    if st[i] == st[nb[k]] and words[k] < T:
                        want[i] |= 1 << k
    got = oracle.activate_bonds3(Lx, Ly, Lz, st, T, SEED, t, sid)
    return [] if np.array_equal(got, want) else ["bonds"]


def test_bond_words_match_rocrand():
    assert _word_mismatches() == []
    assert _word_mismatches(Lx=8, Ly=2, Lz=3, t=0, sid=0) == []


# ------------------------------------------------------------ observables ----
def _nsat_mismatches():
    bad = []
    rng = np.random.default_rng(5)
    for Lx, Ly, Lz in LABEL_SHAPES:
        for q in (2, 3, 5):
            st = rng.integers(0, q, Lx * Ly * Lz).astype(np.uint8)
            n, counts = oracle.satisfied3(Lx, Ly, Lz, q, st)
            want = np.bincount(st, minlength=8)[:8]
            if n != _roll_nsat(Lx, Ly, Lz, st) or not np.array_equal(counts, want):
                bad.append((Lx, Ly, Lz, q))
    return bad


def test_satisfied_bonds_by_rolls():
    assert _nsat_mismatches() == []


# ------------------------------------------------------ stationary law ------
def _exact_nsat_law(q, K, L=2):
    """P(n_sat = k) under the Boltzmann weight exp(K n_sat) on the periodic
    L^3 lattice, every bond of cubic_edges counted (L = 2 doubles each pair)."""
    N = L**3
    st = all_states(N, q)
    nsat = np.zeros(st.shape[0], dtype=np.int64)
    for i, j, _bit, _owner in cubic_edges(L, L, L):
        nsat += st[:, i] == st[:, j]
    w = np.exp(K * nsat - K * nsat.max())
    law = np.bincount(nsat, weights=w, minlength=3 * N + 1)
    return law / law.sum()


def _chain_chi2(q, K, sweeps=120_000, thin=4, seed=SEED):
    """Chi-square of the chain's n_sat histogram (every thin-th sweep after a
    burn-in) against the exact law; bins with expectation < 5 are pooled."""
    T = oracle.threshold(K)
    st = oracle.init_states3(2, 2, 2, q, seed)
    _, rec = oracle.sw3_run(2, 2, 2, q, T, seed, 0, 0, sweeps, st)
    x = rec[100::thin, oracle.REC3_NSAT]
    law = _exact_nsat_law(q, K)
    obs = np.bincount(x, minlength=law.size)[: law.size].astype(float)
    exp = law * x.size
    order = np.argsort(exp)
    chi2, pool_o, pool_e, dof = 0.0, 0.0, 0.0, -1
    for k in order:  # pool the smallest bins until each holds >= 5 expected
        pool_o += obs[k]
        pool_e += exp[k]
        if pool_e >= 5:
            chi2 += (pool_o - pool_e) ** 2 / pool_e
            pool_o = pool_e = 0.0
            dof += 1
    return chi2, dof


@pytest.mark.parametrize("q,K", [(2, 0.6), (3, 0.9)])
def test_chain_samples_the_boltzmann_law(q, K):
    chi2, dof = _chain_chi2(q, K)
    # thinned sweeps are nearly independent here; 4 dof-standard deviations
    # above the mean leaves a false alarm below 1e-4 for these dof
    assert chi2 < dof + 4 * np.sqrt(2 * dof) + 10, (chi2, dof)


# ------------------------------------------------------- planted mistakes ---
MUTANTS = {
    "+z word from the bond tag": [("block_for(seed, (uint32_t)(i >> 2), t, ORC_TAG_BOND_Z, sid, bz);",
                                   "block_for(seed, (uint32_t)(i >> 2), t, ORC_TAG_BOND, sid, bz);")],
    "+z word index shifted": [("(uint64_t)bz[i & 3] < T", "(uint64_t)bz[(i + 1) & 3] < T")],
    "+z neighbour without wrap": [("int64_t nz = ((int64_t)((z + 1) % Lz) * Ly + y) * Lx + x;",
                                   "int64_t nz = ((int64_t)(z + 1 < Lz ? z + 1 : z) * Ly + y) * Lx + x;")],
    "+z bonds never joined": [("if (bonds[i] & 4) uf_union(parent, i, (((z + 1) % Lz) * Ly + y) * Lx + x);", "")],
    "+y and +z targets swapped in labeling": [
        ("if (bonds[i] & 2) uf_union(parent, i, (z * Ly + (y + 1) % Ly) * Lx + x);",
         "if (bonds[i] & 2) uf_union(parent, i, (((z + 1) % Lz) * Ly + y) * Lx + x);"),
        ("if (bonds[i] & 4) uf_union(parent, i, (((z + 1) % Lz) * Ly + y) * Lx + x);",
         "if (bonds[i] & 4) uf_union(parent, i, (z * Ly + (y + 1) % Ly) * Lx + x);")],
    "+z pairs not counted as satisfied": [
        ("nsat += state[i] == state[((int64_t)((z + 1) % Lz) * Ly + y) * Lx + x];", "")],
    "+x word taken for +z": [("(uint64_t)bz[i & 3] < T", "(uint64_t)b[2 * (i & 1)] < T")],
    "+z bonds at half the probability": [("(uint64_t)bz[i & 3] < T", "(uint64_t)bz[i & 3] < T / 2")],
}


def _all_checks():
    bad = _reduction_mismatches(shapes=((9, 6), (7, 1)), sweeps=2) + _label_mismatches() + _word_mismatches() \
        + _nsat_mismatches()
    if not bad:
        chi2, dof = _chain_chi2(2, 0.6, sweeps=40_000)
        if chi2 >= dof + 4 * np.sqrt(2 * dof) + 10:
            bad.append(("chi2", chi2, dof))
    return bad


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "swccl_oracle.c")).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "swccl_oracle.c")
        with open(c, "w") as f:
            f.write(src)
        so = os.path.join(d, "libmutant.so")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I",
                               os.path.dirname(oracle.__file__), "-o", so, c, "-lm"])
        with oracle.using_library(so):
            assert _all_checks() != [], name
