"""Interleaving model of the cubic lattice's merge and resolve passes
(Sec. II.C, tile consolidation, on the simple cubic lattice).

The merge is the square lattice's union-find over boundary ids (walks with
path halving, a compare-and-swap link that expects the root to be its own
parent, a failed swap continuing from the parent it returned), with one
change: roots are ordered by a fixed random priority of the ids (a bijective
hash) instead of by key, so the root of a component is not its minimum-key
id.  The resolve pass that follows (a new launch: it sees the merge's final
parents) points every id at its root and gathers each component's minimum key
at its root: an id reads the root's key with a plain load (a stale read shows
an earlier, larger value, since keys only decrease) and issues an atomic
minimum only when its own key is smaller.

The merge is run under the interleavings and the weak-memory semantics of
tests/test_merge_model.py (plain loads may return earlier values, plain
stores may land late); the resolve under a random interleaving of its loads,
stores and atomic minima, plain loads of a key returning any value the key
held in the launch.  Every schedule must leave every id pointing at its
component's root and the root's key equal to the component's minimum key.  A
key gathered with a plain store (a lost update), an inverted test before the
atomic, and a resolve that takes the id's own key instead of the root's must
each be caught.
"""
import random

import pytest

from tests.test_merge_model import _Mem, _unite, _want


def _prio(x: int) -> int:
    """The kernel's id priority: a bijection of the 32-bit integers."""
    h = (x * 0x9E3779B1) & 0xFFFFFFFF
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    return h


def _merge(n, pairs, rng, weak):
    """Final parents after the merge: the root of lower priority is linked
    below the other (the model's union links the larger 'key' below, so its
    key is the negated priority)."""
    order = [-_prio(x) for x in range(n)]
    G = _Mem(n, rng, weak)
    live = [_unite(G, order, a, b, None, tid) for tid, (a, b) in enumerate(pairs)]
    while live:
        if weak and rng.random() < 0.2:
            G.flush_some()
        k = rng.randrange(len(live))
        try:
            next(live[k])
        except StopIteration:
            live[k] = live[-1]
            live.pop()
    return G.final()


def _resolve(parent, key, rng, mistake=None):
    """Generator-interleaved resolve: one thread per id."""
    n = len(parent)
    G = [[p] for p in parent]   # values each parent entry held in this launch
    K = [[k] for k in key]      # values each key held in this launch

    def load(h):
        return h[rng.randrange(len(h))] if len(h) > 1 and rng.random() < 0.5 else h[-1]

    def thread(i):
        x = i
        p = load(G[x])
        yield
        while p != x:
            x = p
            p = load(G[x])
            yield
        if x == i:
            return
        G[i].append(x)
        yield
        own = key[i]  # not a root: its key never changes
        seen = load(K[x])
        yield
        take = (own > seen) if mistake == "inverted_test" else (own < seen)
        if take:
            if mistake == "plain_store":
                K[x].append(own)  # written from the value read: a smaller key may be overwritten
            else:
                K[x].append(min(K[x][-1], own))
            yield

    live = [thread(i) for i in range(n)]
    while live:
        k = rng.randrange(len(live))
        try:
            next(live[k])
        except StopIteration:
            live[k] = live[-1]
            live.pop()
    return [h[-1] for h in G], [h[-1] for h in K]


def _check(n, pairs, key, par, gkey, mistake=None):
    comp, _ = _want(n, pairs, key)
    roots = {}
    for x in range(n):
        assert par[par[x]] == par[x], "an id does not point at a root"
        roots.setdefault(comp[x], set()).add(par[x])
    for c, rs in roots.items():
        assert len(rs) == 1, "a component has two roots"
    for c in roots:
        r = next(iter(roots[c]))
        want = min(key[x] for x in range(n) if comp[x] == c)
        got = key[r] if mistake == "own_key" else gkey[r]
        assert got == want, f"root key {got} is not the component's minimum {want}"


def _case(rng, n, n_pairs):
    key = rng.sample(range(10 * n), n)
    pairs = [(rng.randrange(n), rng.randrange(n)) for _ in range(n_pairs)]
    return key, pairs


@pytest.mark.parametrize("weak", [False, True], ids=["sc", "weak"])
@pytest.mark.parametrize("n,n_pairs", [(6, 8), (20, 30), (60, 80)])
def test_priority_merge_then_resolve(n, n_pairs, weak):
    rng = random.Random(1000 * n + n_pairs + weak)
    for _ in range(150 if n <= 20 else 40):
        key, pairs = _case(rng, n, n_pairs)
        par = _merge(n, pairs, rng, weak)
        par, gkey = _resolve(par, key, rng)
        _check(n, pairs, key, par, gkey)


@pytest.mark.parametrize("mistake", ["plain_store", "inverted_test", "own_key"])
def test_planted_mistakes_are_caught(mistake):
    rng = random.Random({"plain_store": 1, "inverted_test": 2, "own_key": 3}[mistake])
    for _ in range(3000):
        n = rng.choice((6, 12, 24))
        key, pairs = _case(rng, n, 2 * n)
        par = _merge(n, pairs, rng, False)
        par, gkey = _resolve(par, key, rng, None if mistake == "own_key" else mistake)
        try:
            _check(n, pairs, key, par, gkey, mistake if mistake == "own_key" else None)
        except AssertionError:
            return
    pytest.fail(f"the planted mistake {mistake!r} was not exposed")


def test_priority_is_a_bijection_on_a_sample():
    xs = random.Random(5).sample(range(1 << 31), 20000)
    assert len({_prio(x) for x in xs}) == len(xs)
