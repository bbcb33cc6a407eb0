"""Pins of the oracle's Philox counter layout: which block and which word feed
the initial states, the right and down bonds, and the cluster flips.

The expected values are computed here straight from rocRAND's independent
Philox4x32-10 (its host-callable header, compiled for the CPU), with the
counter (word, t, tag, stream id) and word choice of each step written out:

  init   state_i = (w q) >> 32, w = block(i >> 2, 0, INIT, sid)[i & 3]
  bonds  block(i >> 1, t, BOND, sid): right uses word 2 (i & 1), down word
         2 (i & 1) + 1; a bond between equal spins is active iff w < T
  flip   a cluster with canonical root r takes (w q) >> 32,
         w = block(r >> 2, t, FLIP, sid)[r & 3]

(Sec. II steps 1 and 3 with the keying that fixes the trajectory.)  Copies of
the oracle with one word or counter changed are compiled and must fail this
pin; the -O3 -march=native build must agree with the default one.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests.test_oracle_philox import _rocrand_blocks

TAG_INIT, TAG_BOND, TAG_FLIP = 0, 1, 2
SEED = 0x1105580400000077
SID = 5


def _key():
    return [SEED & 0xFFFFFFFF, SEED >> 32]


def _blocks(ctrs):
    """rocRAND blocks of counters (c0, c1, c2, c3) under the test key, as a dict."""
    uniq = sorted(set(ctrs))
    ref = _rocrand_blocks([list(c) + _key() for c in uniq])
    return dict(zip(uniq, ref))


def _layout_mismatches(W=9, H=6, q=3, t=4):
    """Differences between the oracle and the layout computed from rocRAND."""
    bad = []
    N = W * H
    # init
    blk = _blocks([(i >> 2, 0, TAG_INIT, SID) for i in range(N)])
    want = np.array([(blk[(i >> 2, 0, TAG_INIT, SID)][i & 3] * q) >> 32 for i in range(N)], dtype=np.uint8)
    got = oracle.init_states(W, H, q, SEED, SID)
    if not np.array_equal(got, want):
        bad.append("init")
    # bonds: two spin values only, so most neighbour pairs are equal; T = 2^31
    rng = np.random.default_rng(7)
    st = (rng.random(N) < 0.8).astype(np.uint8)
    T = 2**31
    blk = _blocks([(i >> 1, t, TAG_BOND, SID) for i in range(N)])
    want = np.zeros(N, dtype=np.uint8)
    for y in range(H):
        for x in range(W):
            i = y * W + x
            r, d = y * W + (x + 1) % W, ((y + 1) % H) * W + x
            b = blk[(i >> 1, t, TAG_BOND, SID)]
            right = st[i] == st[r] and b[2 * (i & 1)] < T
            down = st[i] == st[d] and b[2 * (i & 1) + 1] < T
            want[i] = int(right) | (int(down) << 1)
    got = oracle.activate_bonds(W, H, st, T, SEED, t, SID)
    if not np.array_equal(got, want):
        bad.append("bonds")
    # flip: labels of a bond configuration, then the root draws
    labels, _ = oracle.label_bonds(W, H, want)
    roots = sorted(set(int(v) for v in labels))
    blk = _blocks([(r >> 2, t, TAG_FLIP, SID) for r in roots])
    new = {r: (blk[(r >> 2, t, TAG_FLIP, SID)][r & 3] * q) >> 32 for r in roots}
    want_st = np.array([new[int(labels[i])] for i in range(N)], dtype=np.uint8)
    got_st = oracle.flip(W, H, q, labels, st, SEED, t, SID)
    if not np.array_equal(got_st, want_st):
        bad.append("flip")
    return bad


def test_counter_layout_matches_rocrand():
    assert _layout_mismatches() == []
    assert _layout_mismatches(W=16, H=3, q=2, t=0) == []


MUTANTS = {
    "right/down words swapped": [("uint32_t r_right = b[2 * (i & 1)];", "uint32_t r_right = b[2 * (i & 1) + 1];"),
                                 ("uint32_t r_down = b[2 * (i & 1) + 1];", "uint32_t r_down = b[2 * (i & 1)];")],
    "bond block index i>>2": [("block_for(seed, (uint32_t)(i >> 1), t, ORC_TAG_BOND, sid, b);\n"
                               "            uint32_t r_right",
                               "block_for(seed, (uint32_t)(i >> 2), t, ORC_TAG_BOND, sid, b);\n"
                               "            uint32_t r_right")],
    "init word reversed": [("state[i] = state_from_word(b[i & 3], q);", "state[i] = state_from_word(b[3 - (i & 3)], q);")],
    "flip word shifted": [("root_state[r] = state_from_word(b[r & 3], q);",
                           "root_state[r] = state_from_word(b[(r + 1) & 3], q);")],
    "flip keyed on t+1": [("(uint32_t)(r >> 2), t, ORC_TAG_FLIP", "(uint32_t)(r >> 2), t + 1, ORC_TAG_FLIP")],
    "flip with the bond tag": [("(uint32_t)(r >> 2), t, ORC_TAG_FLIP", "(uint32_t)(r >> 2), t, ORC_TAG_BOND")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_layout_mistakes_are_caught(name):
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
            assert _layout_mismatches() != [], name


def test_native_build_matches_default():
    """The -O3 -march=native build (CPU baseline, long fixture runs) gives the
    same sweeps, records and digests as the default -O2 build."""
    W, H, q, seed = 97, 61, 3, 0x1105580400000099
    res = {}
    for fl in ("O2", "native"):
        prev = oracle.flavor()
        oracle.use_flavor(fl)
        try:
            T = oracle.threshold(1.0051)
            st = oracle.init_states(W, H, q, seed)
            out = []
            for t in range(5):
                st, bonds, labels, rec = oracle.sw_sweep(W, H, q, T, seed, 0, t, st)
                out.append((st.copy(), bonds, labels, rec, oracle.digest(st)))
            st2, recs = oracle.sw_run(W, H, q, T, seed, 0, 5, 20, st)
            out.append((st2, recs))
            res[fl] = out
        finally:
            oracle.use_flavor(prev)
    for a, b in zip(res["O2"], res["native"]):
        for x, y in zip(a, b):
            assert np.array_equal(np.asarray(x), np.asarray(y))
