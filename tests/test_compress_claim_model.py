"""Interleaving model of the tile kernel's compression and border claims.

After the unions of a tile (Sec. II.B.2) every site's parent entry holds its
run start, and the run starts form a forest with parents at smaller indices.
Then, per wave and without a barrier between waves:

  1. the wave reads its sites' entries up front and lists the run starts whose
     entry is not their own (linked, or a root some other wave has claimed);
  2. its lanes walk the listed run starts to their roots (a walk stops at an
     entry equal to its own index or negative) and point each start straight
     at its root, never writing an entry where the walk ended at its start;
  3. its threads claim the roots of their border sites: find the root, swing
     the root's entry from its own index to CLAIMING (-1) by compare-and-swap,
     take the next boundary id k and store -(k + 2).

After the barrier each site's code is the boundary id of its root if that
root was claimed, else CAP + the root, read in at most two steps (site ->
run start -> root).  A seeded random scheduler interleaves every load, store
and compare-and-swap of all waves' lanes and threads; every schedule must give
each site the code of its own root, one id per claimed root, every border
root claimed.  Dropping the "walk ended at its start" guard must be caught:
a walk that starts at a root claimed before its wave read the entry would
overwrite the claim.
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


def _run(P0, border, n_waves, lanes, rng, mistake=None):
    n = len(P0)
    P = list(P0)
    nb = [0]
    per = (n + n_waves - 1) // n_waves
    # per wave: its sites, its border sites (claim threads), and a program
    waves = []
    for w in range(n_waves):
        sites = list(range(w * per, min(n, (w + 1) * per)))
        claims = [b for k, b in enumerate(border) if k % n_waves == w]
        waves.append(dict(sites=sites, claims=claims, stage="read", read=[], list=None, walkers=None,
                          claimers=None))

    def step_wave(W):
        """One event of wave W; returns False when the wave has finished."""
        if W["stage"] == "read":  # one up-front load per event
            k = len(W["read"])
            if k < len(W["sites"]):
                x = W["sites"][k]
                W["read"].append(P[x])
                return True
            # list linked run starts: entry not its own (claimed roots included);
            # non-start sites never change and are not run starts
            W["list"] = [x for x, p in zip(W["sites"], W["read"]) if p != x and _is_start[x]]
            W["walkers"] = [dict(i=L, s0=None, x=None) for L in range(lanes)]
            W["stage"] = "compress"
            return True
        if W["stage"] == "compress":
            live = [wk for wk in W["walkers"] if wk["i"] < len(W["list"])]
            if not live:
                W["claimers"] = [dict(b=b, x=b, pc="walk") for b in W["claims"]]
                W["stage"] = "claim"
                return True
            wk = rng.choice(live)
            if wk["s0"] is None:
                wk["s0"] = wk["x"] = W["list"][wk["i"]]
                return True
            p = P[wk["x"]]
            if p >= 0 and p != wk["x"]:
                wk["x"] = p
            else:
                if wk["x"] != wk["s0"] or mistake == "no_start_guard":
                    P[wk["s0"]] = wk["x"]
                wk["i"] += lanes
                wk["s0"] = None
            return True
        if W["stage"] == "claim":
            live = [c for c in W["claimers"] if c["pc"] != "done"]
            if not live:
                W["stage"] = "done"
                return False
            c = rng.choice(live)
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
            return True
        return False

    live = list(range(n_waves))
    while live:
        w = rng.choice(live)
        if not step_wave(waves[w]):
            live.remove(w)

    def code_of(x):
        p = P[x]
        x = p if (p >= 0 and p != x) else x
        p = P[x]
        y = p if (p >= 0 and p != x) else x
        p = P[y] if y != x else p
        return ("id", -p - 2) if p < 0 else ("slot", y)

    return [code_of(x) for x in range(n)], nb[0]


_is_start = None


@pytest.mark.parametrize("mistake", [None, "no_start_guard"])
def test_compress_with_concurrent_claims(mistake):
    global _is_start
    rng = random.Random(5 if mistake is None else 6)
    caught = False
    for trial in range(1500):
        n = rng.choice((8, 16, 40))
        P0, starts, border = _tile(rng, n)
        _is_start = [False] * n
        for s in starts:
            _is_start[s] = True
        codes, n_ids = _run(P0, border, n_waves=rng.choice((2, 3, 4)), lanes=rng.choice((1, 2, 4)), rng=rng,
                            mistake=mistake)
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
        assert caught, "the dropped guard was not exposed by any schedule"
