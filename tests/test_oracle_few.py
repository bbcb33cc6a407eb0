"""Pins of the oracle's few-cluster variant (Sec. III): the SW bond
decomposition, one seed per B x B seed tile, every distinct seeded cluster
flipped with probability p_flip < 1 (q = 2).

Nothing here calls the oracle to compute an expected value:

  - seeds and flip words are computed straight from rocRAND's Philox, with the
    counters written out (seed tile j: block (j, t, SEED, sid), x from word 0
    and y from word 1, each floor(w * extent / 2^32); flip of the cluster with
    canonical root r: word r & 3 of block (r >> 2, t, FEW, sid) below
    floor(p_flip 2^32));
  - clusters come from a breadth-first search written here;
  - the transition matrix of the update is enumerated exactly on a 3 x 2
    torus from the definition alone (bond subsets, seeds, flips): it keeps the
    Boltzmann distribution and obeys detailed balance (the paper's claim for
    this variant), and the oracle's transitions from fixed start states follow
    its rows (a chi-square bound at fixed seeds).

Copies of the oracle with one plausible mistake (a cluster flipped once per
seed, a seed word swapped, the flip keyed on the wrong tag, ragged tiles drawn
as full ones) are compiled and must fail these pins.
"""
import itertools
import os
import subprocess
import tempfile
from collections import deque

import numpy as np
import pytest

import oracle
from tests.test_oracle_philox import _rocrand_blocks

TAG_SEED, TAG_FEW = 3, 4
SEED = 0x1105580400000F3F
SID = 9


def _key():
    return [SEED & 0xFFFFFFFF, SEED >> 32]


def _blocks(ctrs):
    uniq = sorted(set(ctrs))
    ref = _rocrand_blocks([list(c) + _key() for c in uniq])
    return dict(zip(uniq, ref))


def _bfs_labels(W, H, bonds):
    """Canonical labels (minimum site index per cluster), periodic bonds."""
    N = W * H
    adj = [[] for _ in range(N)]
    for y in range(H):
        for x in range(W):
            i = y * W + x
            if bonds[i] & 1:
                j = y * W + (x + 1) % W
                adj[i].append(j)
                adj[j].append(i)
            if bonds[i] & 2:
                j = ((y + 1) % H) * W + x
                adj[i].append(j)
                adj[j].append(i)
    lab = np.full(N, -1, dtype=np.int64)
    for s in range(N):  # ascending: the first site reached of a cluster is its minimum
        if lab[s] >= 0:
            continue
        lab[s] = s
        dq = deque([s])
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if lab[v] < 0:
                    lab[v] = s
                    dq.append(v)
    return lab


def _seeds_ref(W, H, B, t):
    ntx, nty = -(-W // B), -(-H // B)
    blk = _blocks([(j, t, TAG_SEED, SID) for j in range(ntx * nty)])
    out = []
    for ty in range(nty):
        for tx in range(ntx):
            j = ty * ntx + tx
            bw, bh = min(B, W - tx * B), min(B, H - ty * B)
            w = blk[(j, t, TAG_SEED, SID)]
            out.append((ty * B + ((w[1] * bh) >> 32)) * W + tx * B + ((w[0] * bw) >> 32))
    return np.array(out, dtype=np.int64)


def test_prob_threshold_closed_forms():
    assert oracle.prob_threshold(0.0) == 0
    assert oracle.prob_threshold(-0.5) == 0
    assert oracle.prob_threshold(0.5) == 2**31
    assert oracle.prob_threshold(0.25) == 2**30
    assert oracle.prob_threshold(0.75) == 3 * 2**30
    assert oracle.prob_threshold(1.0 - 2.0**-40) == 2**32 - 1  # p < 1 never reaches 2^32


def _few_mismatches(W=21, H=14, B=6, t=3, p_flip=0.6):
    """Differences between the oracle's few-cluster sweep and the definition
    computed here (rocRAND words, BFS clusters)."""
    bad = []
    got_seeds = oracle.few_seeds(W, H, B, SEED, t, SID)
    want_seeds = _seeds_ref(W, H, B, t)
    if not np.array_equal(got_seeds, want_seeds):
        bad.append("seeds")
    rng = np.random.default_rng(11)
    st = (rng.random(W * H) < 0.7).astype(np.uint8)
    T = oracle.threshold(0.9)
    Tf = oracle.prob_threshold(p_flip)
    new, bonds, labels, rec, few = oracle.few_sweep(W, H, T, Tf, B, SEED, SID, t, st)
    # bonds are the SW bonds of the same sweep (their layout is pinned on its own)
    if not np.array_equal(bonds, oracle.activate_bonds(W, H, st, T, SEED, t, SID)):
        bad.append("bonds")
    lab = _bfs_labels(W, H, bonds)
    if not np.array_equal(labels, lab):
        bad.append("labels")
    seeded = sorted(set(int(lab[s]) for s in want_seeds))
    blk = _blocks([(r >> 2, t, TAG_FEW, SID) for r in seeded])
    flipped = {r for r in seeded if blk[(r >> 2, t, TAG_FEW, SID)][r & 3] < Tf}
    want = np.array([1 - v if int(lab[i]) in flipped else v for i, v in enumerate(st)], dtype=np.uint8)
    if not np.array_equal(new, want):
        bad.append("flip")
    if few != (len(seeded), len(flipped)):
        bad.append("counts")
    return bad


def test_few_sweep_matches_definition():
    assert _few_mismatches() == []
    assert _few_mismatches(W=16, H=16, B=16, t=0, p_flip=0.9) == []  # one seed tile
    assert _few_mismatches(W=12, H=10, B=1, t=7, p_flip=0.3) == []   # every site a seed
    assert _few_mismatches(W=13, H=9, B=4, t=2, p_flip=0.999) == []  # ragged tiles


def test_zero_flip_probability_changes_nothing():
    W, H = 30, 20
    st = oracle.init_states(W, H, 2, SEED)
    new, _, _, _, few = oracle.few_sweep(W, H, oracle.threshold(1.2), 0, 5, SEED, 0, 1, st)
    assert np.array_equal(new, st) and few[1] == 0 and few[0] >= 1


# ------------------------------------------------- exact enumeration (3 x 2) --
EW, EH, EB = 3, 2, 2  # seed tiles: 2 x 2 sites and 1 x 2 sites


def _edges():
    e = []
    for y in range(EH):
        for x in range(EW):
            i = y * EW + x
            e.append((i, y * EW + (x + 1) % EW))
            e.append((i, ((y + 1) % EH) * EW + x))
    return e


def _partition(active_edges):
    parent = list(range(EW * EH))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    for a, b in active_edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return [find(i) for i in range(EW * EH)]


def _exact_transitions(K, p_flip):
    """T[s, s'] of the few-cluster update from its definition (states as bit
    masks, bit i = state of site i)."""
    N = EW * EH
    E = _edges()
    p = -np.expm1(-K)
    tiles = []  # the sites of each seed tile
    for ty in range(-(-EH // EB)):
        for tx in range(-(-EW // EB)):
            tiles.append([y * EW + x for y in range(ty * EB, min(EH, ty * EB + EB))
                          for x in range(tx * EB, min(EW, tx * EB + EB))])
    # per active-edge subset: distribution of the flip mask (seeds and flips
    # do not depend on the spins)
    mask_dist = {}
    for sub in range(1 << len(E)):
        lab = _partition([E[k] for k in range(len(E)) if sub >> k & 1])
        dist = {}
        combos = list(itertools.product(*tiles))
        for seeds in combos:
            roots = sorted(set(lab[s] for s in seeds))
            for flips in itertools.product((0, 1), repeat=len(roots)):
                pr = 1.0 / len(combos)
                m = 0
                for r, f in zip(roots, flips):
                    pr *= p_flip if f else 1 - p_flip
                    if f:
                        m |= sum(1 << i for i in range(N) if lab[i] == r)
                dist[m] = dist.get(m, 0.0) + pr
        mask_dist[sub] = dist
    Tm = np.zeros((1 << N, 1 << N))
    for s in range(1 << N):
        sat = [k for k, (a, b) in enumerate(E) if (s >> a & 1) == (s >> b & 1)]
        for bits in range(1 << len(sat)):
            sub = 0
            n_on = 0
            for j, k in enumerate(sat):
                if bits >> j & 1:
                    sub |= 1 << k
                    n_on += 1
            w = p ** n_on * (1 - p) ** (len(sat) - n_on)
            for m, pr in mask_dist[sub].items():
                Tm[s, s ^ m] += w * pr
    return Tm


def _boltzmann(K):
    E = _edges()
    w = np.array([np.exp(K * sum((s >> a & 1) == (s >> b & 1) for a, b in E)) for s in range(1 << (EW * EH))])
    return w / w.sum()


@pytest.fixture(scope="module")
def exact():
    K, pf = 0.8, 0.7
    return K, pf, _exact_transitions(K, pf)


def test_exact_update_keeps_boltzmann_and_detailed_balance(exact):
    K, pf, Tm = exact
    assert np.allclose(Tm.sum(axis=1), 1.0, atol=1e-12)
    pi = _boltzmann(K)
    assert np.allclose(pi @ Tm, pi, atol=1e-12)
    F = pi[:, None] * Tm
    assert np.allclose(F, F.T, atol=1e-13)
    # a flip probability of one would lose ergodicity; below one every state
    # reaches every other (some power of T is positive)
    R = np.linalg.matrix_power((Tm > 0).astype(np.int64), 6)
    assert (R > 0).all()


def _chi2_from(Tm, s0, n=6000, K=0.8, pf=0.7):
    T = oracle.threshold(K)
    Tf = oracle.prob_threshold(pf)
    N = EW * EH
    st0 = np.array([(s0 >> i) & 1 for i in range(N)], dtype=np.uint8)
    counts = np.zeros(1 << N)
    for t in range(n):
        new, *_ = oracle.few_sweep(EW, EH, T, Tf, EB, SEED, 0, t, st0)
        counts[int(sum(int(v) << i for i, v in enumerate(new)))] += 1
    exp = Tm[s0] * n
    assert (counts[exp == 0] == 0).all(), "a transition of probability zero happened"
    live = exp > 0
    return float((((counts - exp) ** 2)[live] / exp[live]).sum()), int(live.sum()) - 1


def test_oracle_transitions_follow_exact_rows(exact):
    _, _, Tm = exact
    for s0 in (0b000000, 0b000111, 0b010101):
        chi2, dof = _chi2_from(Tm, s0)
        # mean dof, sd sqrt(2 dof): 6 sd is far outside chance at these fixed seeds
        assert chi2 < dof + 6 * np.sqrt(2 * dof), (s0, chi2, dof)


MUTANTS = {
    "one flip draw per seed": [("for (int64_t j = 0; j < nseed; ++j) seeded[l[sites[j]]] = 1;",
                                "for (int64_t j = 0; j < nseed; ++j) seeded[l[sites[j]]] ^= 1;")],
    "seed words swapped": [("(int32_t)(((uint64_t)b[0] * (uint64_t)bw) >> 32);",
                            "(int32_t)(((uint64_t)b[1] * (uint64_t)bw) >> 32);"),
                           ("(int32_t)(((uint64_t)b[1] * (uint64_t)bh) >> 32);",
                            "(int32_t)(((uint64_t)b[0] * (uint64_t)bh) >> 32);")],
    "flip keyed on the seed tag": [("(uint32_t)(r >> 2), t, ORC_TAG_FEW", "(uint32_t)(r >> 2), t, ORC_TAG_SEED")],
    "ragged tiles drawn full": [("int32_t bw = W - tx * B < B ? W - tx * B : B;", "int32_t bw = B;"),
                                ("int32_t bh = H - ty * B < B ? H - ty * B : B;", "int32_t bh = B;")],
    "flip word shifted": [("if ((uint64_t)w[r & 3] < Tflip) {", "if ((uint64_t)w[(r + 1) & 3] < Tflip) {")],
}


def _mutant_so(d, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "swccl_oracle.c")).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    c = os.path.join(d, "swccl_oracle.c")
    with open(c, "w") as f:
        f.write(src)
    so = os.path.join(d, "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I",
                           os.path.dirname(oracle.__file__), "-o", so, c, "-lm"])
    return so


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_few_mistakes_are_caught(name):
    with tempfile.TemporaryDirectory() as d:
        so = _mutant_so(d, name)
        with oracle.using_library(so):
            caught = bool(_few_mismatches()) or bool(_few_mismatches(W=13, H=9, B=4, t=2, p_flip=0.999))
            assert caught, name
