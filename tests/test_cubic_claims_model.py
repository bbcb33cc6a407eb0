"""Interleaving model of the cubic tile kernel's root walks and face claims.

After the unions of a tile (Sec. II.B.2) the parent entries form a forest
(parents at smaller slots, a root's entry its own slot).  Then, with no
barrier between the two steps, every wave

  1. walks each of its sites to the root (loads until an entry equals its own
     slot or is negative) and keeps the roots in registers;
  2. claims the roots of its face sites: compare-and-swap the root's entry
     from its own slot to CLAIMING (-1); the winner takes the next id k and
     stores -(k + 2);

while other waves may already be claiming.  After a barrier every site's code
is the id read at its root (-(entry) - 2) or CAP + the root.  A seeded random
scheduler interleaves the loads, compare-and-swaps and stores of all waves.
Every schedule must give every site its true root, one id per claimed root,
every face root claimed and the codes that follow.  Two mistakes must be
caught: a walk that stops only at an entry equal to its own slot (it follows
a claimed root's negative entry off the table), and claims by a plain load
and store instead of the compare-and-swap (two waves claim one root).
"""
import random

import pytest

CAP = 1 << 20
CLAIMING = -1


def _forest(rng, n):
    P = []
    for x in range(n):
        P.append(x if x == 0 or rng.random() < 0.3 else rng.randrange(x))
    return P


def _root(P0, x):
    while P0[x] != x:
        x = P0[x]
    return x


def _run(P0, face, n_waves, rng, mistake=None):
    n = len(P0)
    P = list(P0)
    nb = [0]
    per = (n + n_waves - 1) // n_waves
    waves = []
    for w in range(n_waves):
        sites = list(range(w * per, min(n, (w + 1) * per)))
        waves.append(dict(sites=sites, k=0, x=None, roots={}, stage="walk", claims=None, c=None))

    def step(W):
        """One shared-memory event of wave W; False when it is done."""
        if W["stage"] == "walk":
            if W["k"] == len(W["sites"]):
                W["stage"] = "claim"
                W["claims"] = [s for s in W["sites"] if face[s]]
                W["k"] = 0
                return True
            s = W["sites"][W["k"]]
            if W["x"] is None:
                W["x"] = s
            x = W["x"]
            assert 0 <= x < n, "walk left the parent table"
            p = P[x]
            stop = p == x if mistake == "no_negative_stop" else (p == x or p < 0)
            if stop:
                W["roots"][s] = x
                W["k"] += 1
                W["x"] = None
            else:
                W["x"] = p
            return True
        if W["stage"] == "claim":
            if W["c"] is not None:  # the winner's id store
                r = W["c"]
                k = nb[0]
                nb[0] += 1
                P[r] = -(k + 2)
                W["c"] = None
                return True
            if W["k"] == len(W["claims"]):
                return False
            s = W["claims"][W["k"]]
            r = W["roots"][s]
            W["k"] += 1
            if mistake == "plain_claim":
                if P[r] == r:      # a load ...
                    W["c"] = r     # ... and later the store: another wave may claim in between
                return True
            if P[r] == r:          # the compare-and-swap, one event
                P[r] = CLAIMING
                W["c"] = r
            return True
        return False

    live = list(range(n_waves))
    while live:
        w = rng.choice(live)
        if not step(waves[w]):
            live.remove(w)
    # after the barrier: codes
    codes = []
    for W in waves:
        for s in W["sites"]:
            r = W["roots"][s]
            pr = P[r]
            codes.append((s, r, -pr - 2 if pr < 0 else CAP + r))
    return codes, nb[0]


@pytest.mark.parametrize("mistake", [None, "no_negative_stop", "plain_claim"])
def test_walks_beside_claims(mistake):
    rng = random.Random({None: 3, "no_negative_stop": 4, "plain_claim": 5}[mistake])
    caught = False
    for _ in range(1500):
        n = rng.choice((8, 20, 48))
        P0 = _forest(rng, n)
        face = [rng.random() < 0.4 for _ in range(n)]
        try:
            codes, n_ids = _run(P0, face, rng.choice((2, 3, 4)), rng, mistake)
            claimed = {_root(P0, s) for s in range(n) if face[s]}
            assert n_ids == len(claimed)
            id_of = {}
            for s, r, c in codes:
                assert r == _root(P0, s)
                if r in claimed:
                    assert c < CAP and id_of.setdefault(r, c) == c
                else:
                    assert c == CAP + r
            assert sorted(id_of.values()) == list(range(n_ids))
        except AssertionError:
            if mistake is None:
                raise
            caught = True
            break
    if mistake is not None:
        assert caught, f"the planted mistake {mistake!r} was not exposed by any schedule"
