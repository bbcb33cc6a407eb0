"""Interleaving model of the cross-tile merge's union-find over boundary ids
(Sec. II.C, tile consolidation).

Each boundary id has a unique key (the site index of its tile-local root) and
starts as its own root.  A union of ids a, b walks both to their roots with
path halving (a node passed over is pointed at its grandparent by a plain
store), then links the root with the larger key below the other by a
compare-and-swap that expects the root still to be its own parent; a failed
swap continues from the parent it found.  A seeded random scheduler
interleaves every load, store and compare-and-swap of all unions.  Every
schedule must keep each parent's key below its child's, end with the exact
partition of the requested unions, and leave each component's minimum key at
its root (the key the flatten reports as the canonical label).  A non-atomic
swap, a link in the wrong key order and a halving store that crosses the two
chains must each be caught.
"""
import random

import pytest


def _want(n, pairs, key):
    f = list(range(n))

    def find(x):
        while f[x] != x:
            x = f[x]
        return x

    for u, v in pairs:
        u, v = find(u), find(v)
        if u != v:
            f[max(u, v)] = min(u, v)
    comp = [find(x) for x in range(n)]
    best = {}
    for x in range(n):
        c = comp[x]
        if c not in best or key[x] < key[best[c]]:
            best[c] = x
    return comp, {c: best[c] for c in best}


def _unite(G, key, a, b, mistake):
    """Generator: one yield per shared-memory event of gunite(a, b)."""

    def find2():
        nonlocal a, b
        pa = G[a]
        yield
        pb = G[b]
        yield
        while pa != a or pb != b:
            ga = G[pa]
            yield
            gb = G[pb]
            yield
            if ga != pa:
                G[a] = gb if mistake == "crossed_halving" else ga
                yield
            if gb != pb:
                G[b] = gb
                yield
            a, b = ga, gb
            pa = G[a]
            yield
            pb = G[b]
            yield

    yield from find2()
    while True:
        if a == b:
            return
        if (key[a] < key[b]) != (mistake == "wrong_order"):
            a, b = b, a
        if mistake == "non_atomic":
            seen = G[a]
            yield
            if seen == a:
                G[a] = b  # written later than read: another link may land in between
                yield
                return
            a = seen
        else:
            cur = G[a]
            if cur == a:
                G[a] = b
                yield
                return
            yield
            a = cur
        yield from find2()


def _run(n, pairs, key, rng, mistake=None):
    G = list(range(n))
    live = [_unite(G, key, a, b, mistake) for a, b in pairs]
    while live:
        k = rng.randrange(len(live))
        try:
            next(live[k])
        except StopIteration:
            live[k] = live[-1]
            live.pop()
            continue
        if mistake is None:
            for x in range(n):
                assert G[x] == x or key[G[x]] < key[x], "parent key above its child's"
    return G


def _check(G, key, comp, best):
    n = len(G)
    root_of = []
    for x in range(n):
        r, steps = x, 0
        while G[r] != r:
            r = G[r]
            steps += 1
            assert steps <= n, "cycle"
        root_of.append(r)
    for x in range(n):
        for y in range(x + 1, n):
            assert (root_of[x] == root_of[y]) == (comp[x] == comp[y]), (x, y)
    for c, m in best.items():
        r = root_of[c]
        assert r == m, f"root {r} of component {c} is not its minimum key holder {m}"


def _case(rng, n, n_pairs):
    key = rng.sample(range(10 * n), n)  # unique keys in arbitrary order
    pairs = [(rng.randrange(n), rng.randrange(n)) for _ in range(n_pairs)]
    return key, pairs


@pytest.mark.parametrize("n,n_pairs", [(4, 6), (10, 12), (30, 40), (80, 60)])
def test_merge_any_interleaving(n, n_pairs):
    rng = random.Random(31 * n + n_pairs)
    for _ in range(300 if n <= 30 else 60):
        key, pairs = _case(rng, n, n_pairs)
        comp, best = _want(n, pairs, key)
        _check(_run(n, pairs, key, rng), key, comp, best)


def test_merge_chain_of_tiles():
    """Unions along a chain (a cluster spanning many tiles), in random order."""
    rng = random.Random(3)
    for _ in range(100):
        n = 40
        key = rng.sample(range(1000), n)
        pairs = [(i, i + 1) for i in range(n - 1)]
        rng.shuffle(pairs)
        comp, best = _want(n, pairs, key)
        _check(_run(n, pairs, key, rng), key, comp, best)


@pytest.mark.parametrize("mistake", ["non_atomic", "wrong_order", "crossed_halving"])
def test_planted_mistakes_are_caught(mistake):
    rng = random.Random(77)
    for _ in range(3000):
        key, pairs = _case(rng, 8, 10)
        comp, best = _want(8, pairs, key)
        try:
            _check(_run(8, pairs, key, rng, mistake=mistake), key, comp, best)
        except AssertionError:
            return
    pytest.fail(f"{mistake}: no schedule in 3000 exposed it")
