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

The GPU runs the merge across eight chiplets whose L2 caches are not kept
coherent with each other inside a launch: a plain load may return any value
the location held earlier in the launch (a stale cache line), and a plain
store may become visible to other work-groups late, after later events of
its own thread.  Only the compare-and-swap acts on the location's current
value.  The weak-memory runs give every plain load and store those
semantics; the same checks must hold, and a mistake that only stale loads
can expose (after a failed swap, continuing from a plain reload of the node
and giving up when that reload still shows it as a root) must be caught.
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


class _Mem:
    """Shared parents.  Sequentially consistent unless weak: then a plain load
    may return any earlier value of the location, and a plain store may be
    held back and applied later (in program order per thread)."""

    def __init__(self, n, rng, weak):
        self.hist = [[x] for x in range(n)]  # every value each location held, oldest first
        self.rng, self.weak = rng, weak
        self.pending = {}  # thread -> list of held-back stores

    def cur(self, x):
        return self.hist[x][-1]

    def __getitem__(self, x):
        h = self.hist[x]
        if self.weak and len(h) > 1 and self.rng.random() < 0.5:
            return h[self.rng.randrange(len(h))]
        return h[-1]

    def store(self, tid, x, v):
        if self.weak and self.rng.random() < 0.5:
            self.pending.setdefault(tid, []).append((x, v))
        else:
            self.flush_thread(tid)  # a thread's stores stay in program order
            self.hist[x].append(v)

    def flush_thread(self, tid):
        for x, v in self.pending.pop(tid, []):
            self.hist[x].append(v)

    def flush_some(self):
        if self.pending:
            self.flush_thread(self.rng.choice(list(self.pending)))

    def cas(self, x, expect, new):
        if self.hist[x][-1] == expect:
            self.hist[x].append(new)
            return True, expect
        return False, self.hist[x][-1]

    def final(self):
        for tid in list(self.pending):
            self.flush_thread(tid)
        return [h[-1] for h in self.hist]


def _unite(G, key, a, b, mistake, tid=0):
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
                G.store(tid, a, gb if mistake == "crossed_halving" else ga)
                yield
            if gb != pb:
                G.store(tid, b, gb)
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
                G.store(tid, a, b)  # written later than read: another link may land in between
                yield
                return
            a = seen
        else:
            ok, cur = G.cas(a, a, b)
            yield
            if ok:
                return
            if mistake == "reload_after_failed_cas":
                cur = G[a]  # a plain reload instead of the value the swap returned
                yield
                if cur == a:
                    return  # "it is still a root, so another lane linked it to b": wrong
            a = cur
        yield from find2()


def _run(n, pairs, key, rng, mistake=None, weak=False):
    G = _Mem(n, rng, weak)
    live = [_unite(G, key, a, b, mistake, tid) for tid, (a, b) in enumerate(pairs)]
    while live:
        if weak and rng.random() < 0.2:
            G.flush_some()
        k = rng.randrange(len(live))
        try:
            next(live[k])
        except StopIteration:
            live[k] = live[-1]
            live.pop()
            continue
        if mistake is None:
            for x in range(n):
                p = G.cur(x)
                assert p == x or key[p] < key[x], "parent key above its child's"
    return G.final()


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


@pytest.mark.parametrize("n,n_pairs", [(4, 6), (10, 12), (30, 40), (80, 60)])
def test_merge_weak_memory(n, n_pairs):
    """Stale plain loads and late plain stores (no coherence across chiplets
    inside a launch): the same partition, minimum-key roots and key order."""
    rng = random.Random(1000 + 31 * n + n_pairs)
    for _ in range(300 if n <= 30 else 60):
        key, pairs = _case(rng, n, n_pairs)
        comp, best = _want(n, pairs, key)
        _check(_run(n, pairs, key, rng, weak=True), key, comp, best)


def test_merge_chain_weak_memory():
    rng = random.Random(5)
    for _ in range(100):
        n = 40
        key = rng.sample(range(1000), n)
        pairs = [(i, i + 1) for i in range(n - 1)]
        rng.shuffle(pairs)
        comp, best = _want(n, pairs, key)
        _check(_run(n, pairs, key, rng, weak=True), key, comp, best)


def _caught(mistake, weak, tries=3000):
    rng = random.Random(77)
    for _ in range(tries):
        key, pairs = _case(rng, 8, 10)
        comp, best = _want(8, pairs, key)
        try:
            _check(_run(8, pairs, key, rng, mistake=mistake, weak=weak), key, comp, best)
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("mistake", ["non_atomic", "wrong_order", "crossed_halving"])
def test_planted_mistakes_are_caught(mistake):
    assert _caught(mistake, weak=False), f"{mistake}: no schedule in 3000 exposed it"


def test_stale_load_mistake_needs_weak_memory():
    """Continuing from a plain reload after a failed swap is right when loads
    are fresh and wrong when they may be stale: only the weak model sees it."""
    assert not _caught("reload_after_failed_cas", weak=False, tries=1500)
    assert _caught("reload_after_failed_cas", weak=True)
