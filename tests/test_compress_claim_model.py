"""Interleaving model of the tile kernel's border claims and compression.

After the unions of a tile (Sec. II.B.2) every site's parent entry holds its
run start, and the run starts form a forest with parents at smaller indices.
Then:

  1. (every thread of the workgroup) the threads of the border sites claim
     their roots: walk to the root (an entry equal to its own index, or
     negative), swing the root's entry from its own index to CLAIMING (-1) by
     compare-and-swap, take the next boundary id k and store -(k + 2);
  2. a barrier;
  3. (per wave, without a barrier between waves) the wave reads its sites'
     entries up front and lists the run starts whose entry is neither their
     own nor negative (linked); its lanes walk the listed run starts up to the
     first entry that is negative (a claimed root, or a start another lane
     already finished) or their own (an unclaimed root) and write the final
     code into the start's entry, encoded as -(code + 2): the boundary id of a
     claimed root, else CAP + the root;
  4. a barrier.

Each site's code is then read in at most one step past its entry (site ->
run start): the decoded negative entry, or CAP + the run start when that is an
unclaimed root.  A seeded random scheduler interleaves every load, store and
compare-and-swap of all threads and lanes; every schedule must give each site
the code of its own root, one id per claimed root and every border root
claimed.  Two mistakes must be caught: claims running beside the compression
(no barrier between them: a walk can encode an interior code for a root that
is claimed afterwards) and a compression that writes the root's index instead
of its final code.
"""
import random

import pytest

CAP = 1 << 20
CLAIMING = -1


def _tile(rng, n):
    """Initial entries: a forest over run starts (parent <= self) and every
    other site pointing at a run start to its left; border sites."""
    P = [0] * n
    starts = []
    for x in range(n):
        if x == 0 or rng.random() < 0.45:
            # a run start: a root, or linked to a smaller run start
            P[x] = x if (not starts or rng.random() < 0.35) else rng.choice(starts)
            starts.append(x)
        else:
            P[x] = rng.choice(starts[-3:])  # the run start of its row segment
    border = sorted(rng.sample(range(n), max(1, n // 3)))
    return P, starts, border


def _root(P0, x):
    while P0[x] != x:
        x = P0[x]
    return x


def _run(P0, border, is_start, n_waves, lanes, rng, mistake=None):
    n = len(P0)
    P = list(P0)
    nb = [0]
    per = (n + n_waves - 1) // n_waves
    claimers = [dict(x=b, pc="walk") for b in border]
    waves = [dict(sites=list(range(w * per, min(n, (w + 1) * per))), stage="read", read=[], list=None,
                  walkers=None) for w in range(n_waves)]

    def step_claim(c):
        if c["pc"] == "walk":
            p = P[c["x"]]
            if p == c["x"] or p < 0:
                c["pc"] = "cas"
            else:
                c["x"] = p
        elif c["pc"] == "cas":
            if P[c["x"]] == c["x"]:
                P[c["x"]] = CLAIMING
                c["pc"] = "store"
            else:
                c["pc"] = "done"  # another thread claims this root
        else:
            k = nb[0]
            nb[0] += 1
            P[c["x"]] = -(k + 2)
            c["pc"] = "done"

    def step_wave(W):
        """One event of wave W's compression; returns False when it has finished."""
        if W["stage"] == "read":  # one up-front load per event
            k = len(W["read"])
            if k < len(W["sites"]):
                x = W["sites"][k]
                W["read"].append(P[x])
                return True
            # linked run starts: entry neither their own nor negative
            W["list"] = [x for x, p in zip(W["sites"], W["read"]) if p >= 0 and p != x and is_start[x]]
            W["walkers"] = [dict(i=L, s0=None, x=None) for L in range(lanes)]
            W["stage"] = "compress"
            return True
        live = [wk for wk in W["walkers"] if wk["i"] < len(W["list"])]
        if not live:
            return False
        wk = rng.choice(live)
        if wk["s0"] is None:
            wk["s0"] = wk["x"] = W["list"][wk["i"]]
            return True
        p = P[wk["x"]]
        if p >= 0 and p != wk["x"]:
            wk["x"] = p
        else:
            if mistake == "root_not_code":
                P[wk["s0"]] = wk["x"]
            else:
                P[wk["s0"]] = p if p < 0 else -(CAP + wk["x"]) - 2
            wk["i"] += lanes
            wk["s0"] = None
        return True

    # claims, then (after a barrier) the waves' compression; with the
    # mistake the two run interleaved
    live_c = list(claimers)
    live_w = list(range(n_waves))
    while live_c or live_w:
        if mistake == "claims_concurrent":
            pick_claim = bool(live_c) and (not live_w or rng.random() < 0.5)
        else:
            pick_claim = bool(live_c)
        if pick_claim:
            c = rng.choice(live_c)
            step_claim(c)
            if c["pc"] == "done":
                live_c.remove(c)
        else:
            w = rng.choice(live_w)
            if not step_wave(waves[w]):
                live_w.remove(w)

    def code_of(x):
        p = P[x]
        if p >= 0 and p != x:
            p = P[p]
        if p < 0:
            c = -p - 2
            return ("id", c) if c < CAP else ("slot", c - CAP)
        return ("slot", p)

    return [code_of(x) for x in range(n)], nb[0]


@pytest.mark.parametrize("mistake", [None, "claims_concurrent", "root_not_code"])
def test_claims_then_encoding_compression(mistake):
    rng = random.Random({None: 5, "claims_concurrent": 6, "root_not_code": 7}[mistake])
    caught = False
    for trial in range(1500):
        n = rng.choice((8, 16, 40))
        P0, starts, border = _tile(rng, n)
        is_start = [False] * n
        for s in starts:
            is_start[s] = True
        codes, n_ids = _run(P0, border, is_start, n_waves=rng.choice((2, 3, 4)), lanes=rng.choice((1, 2, 4)),
                            rng=rng, mistake=mistake)
        roots = [_root(P0, x) for x in range(n)]
        claimed = sorted({roots[b] for b in border})
        try:
            assert n_ids == len(claimed)
            id_of = {}
            for x in range(n):
                kind, v = codes[x]
                if roots[x] in claimed:
                    assert kind == "id", (x, codes[x])
                    assert id_of.setdefault(roots[x], v) == v
                else:
                    assert (kind, v) == ("slot", roots[x]), (x, codes[x])
            assert sorted(id_of.values()) == list(range(n_ids))
        except AssertionError:
            if mistake is None:
                raise
            caught = True
            break
    if mistake is not None:
        assert caught, f"the planted mistake {mistake!r} was not exposed by any schedule"
