"""Independent reference computations used to pin the oracle.

Nothing here calls the oracle or the GPU library.  These are different
algorithms for the same mathematical objects:

* ``bfs_labels`` -- breadth-first search over an explicit adjacency list
  (a different algorithm from the oracle's union-find);
* ``propagate_labels`` -- vectorised minimum-label propagation over many bond
  configurations at once (used for exhaustive enumeration of tiny tori);
* ``potts_exact`` -- exact Boltzmann averages by enumerating every spin state;
* ``fk_exact`` -- exact random-cluster (Fortuin-Kasteleyn) expectations by
  enumerating every bond set of a tiny torus, Eq. random_cluster;
* ``cubic_edges`` / ``bfs_labels_cubic`` -- the bonds of a periodic simple
  cubic lattice and BFS labels of a packed 3D bond configuration.
"""
from __future__ import annotations

from collections import deque
from fractions import Fraction
import itertools

import numpy as np


def lattice_edges(W: int, H: int, periodic: bool = True):
    """List of (i, j, bit, owner) for every bond: owner site i, bit 1 = right, 2 = down."""
    edges = []
    for y in range(H):
        for x in range(W):
            i = y * W + x
            if periodic or x + 1 < W:
                edges.append((i, y * W + (x + 1) % W, 1, i))
            if periodic or y + 1 < H:
                edges.append((i, ((y + 1) % H) * W + x, 2, i))
    return edges


def bfs_labels(W: int, H: int, bonds: np.ndarray, periodic: bool = True) -> np.ndarray:
    """Canonical labels (minimum site index per component) by BFS."""
    N = W * H
    adj = [[] for _ in range(N)]
    for i, j, bit, owner in lattice_edges(W, H, periodic):
        if bonds[owner] & bit:
            adj[i].append(j)
            adj[j].append(i)
    labels = np.full(N, -1, dtype=np.int64)
    for s in range(N):
        if labels[s] >= 0:
            continue
        comp = [s]
        labels[s] = s
        dq = deque([s])
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if labels[v] < 0:
                    labels[v] = s
                    comp.append(v)
                    dq.append(v)
        m = min(comp)
        for v in comp:
            labels[v] = m
    return labels


def bfs_site_labels(W: int, H: int, occ: np.ndarray) -> np.ndarray:
    """Canonical labels of 4-connected occupied pixels, open boundary, background -1."""
    occ = np.asarray(occ).reshape(-1) != 0
    N = W * H
    labels = np.full(N, -2, dtype=np.int64)
    labels[~occ] = -1
    for s in range(N):
        if labels[s] != -2:
            continue
        comp = [s]
        labels[s] = s
        dq = deque([s])
        while dq:
            u = dq.popleft()
            ux, uy = u % W, u // W
            for vx, vy in ((ux + 1, uy), (ux - 1, uy), (ux, uy + 1), (ux, uy - 1)):
                if 0 <= vx < W and 0 <= vy < H:
                    v = vy * W + vx
                    if labels[v] == -2:
                        labels[v] = s
                        comp.append(v)
                        dq.append(v)
        m = min(comp)
        for v in comp:
            labels[v] = m
    return labels


def all_bond_sets(W: int, H: int):
    """Every bond configuration of the W x H torus as packed bytes, shape (2^E, N)."""
    edges = lattice_edges(W, H, True)
    E = len(edges)
    codes = np.arange(1 << E, dtype=np.int64)
    packed = np.zeros((1 << E, W * H), dtype=np.uint8)
    for e, (i, j, bit, owner) in enumerate(edges):
        on = ((codes >> e) & 1).astype(np.uint8)
        packed[:, owner] |= on * bit
    return packed, edges


def propagate_labels(W: int, H: int, packed: np.ndarray, periodic: bool = True) -> np.ndarray:
    """Min-label propagation for a batch of configurations (rows of ``packed``)."""
    B, N = packed.shape
    labels = np.tile(np.arange(N, dtype=np.int64), (B, 1))
    edges = lattice_edges(W, H, periodic)
    changed = True
    while changed:
        changed = False
        for i, j, bit, owner in edges:
            act = (packed[:, owner] & bit) != 0
            m = np.minimum(labels[:, i], labels[:, j])
            upd = act & ((labels[:, i] != m) | (labels[:, j] != m))
            if upd.any():
                changed = True
                labels[upd, i] = m[upd]
                labels[upd, j] = m[upd]
    return labels


def cluster_stats(labels: np.ndarray):
    """(n_clusters, max_size) per row of a batch of canonical labelings."""
    B, N = labels.shape
    idx = np.arange(N)
    ncl = (labels == idx).sum(axis=1)
    counts = np.zeros((B, N), dtype=np.int64)
    np.add.at(counts, (np.repeat(np.arange(B), N), labels.reshape(-1)), 1)
    return ncl, counts.max(axis=1)


def all_states(N: int, q: int) -> np.ndarray:
    """Every spin configuration of N sites with q states, shape (q^N, N), uint8."""
    codes = np.arange(q ** N, dtype=np.int64)
    out = np.zeros((q ** N, N), dtype=np.uint8)
    for s in range(N):
        out[:, s] = (codes // q ** s) % q
    return out


def potts_exact(W: int, H: int, q: int, K: float):
    """Exact averages of the periodic W x H q-state Potts model, weight exp(K n_sat).

    n_sat counts satisfied bonds (Eq. potts_hamiltonian with -H/J = n_sat).
    Returns a dict with <n_sat>, and for q == 2 the Ising magnetisation moments
    <|m|>, <m^2>, <m^4> (m = M/N, s = 2*state - 1), plus <max_k n_k>/N.
    """
    N = W * H
    st = all_states(N, q)
    nsat = np.zeros(st.shape[0], dtype=np.int64)
    for i, j, _bit, _owner in lattice_edges(W, H, True):
        nsat += st[:, i] == st[:, j]
    logw = K * nsat
    w = np.exp(logw - logw.max())
    Z = w.sum()
    out = {"nsat": float((w * nsat).sum() / Z)}
    counts = np.stack([(st == k).sum(axis=1) for k in range(q)], axis=1)
    out["maxfrac"] = float((w * counts.max(axis=1)).sum() / Z / N)
    if q == 2:
        m = (2.0 * counts[:, 1] - N) / N
        out["absm"] = float((w * np.abs(m)).sum() / Z)
        out["m2"] = float((w * m ** 2).sum() / Z)
        out["m4"] = float((w * m ** 4).sum() / Z)
    return out


def fk_exact(W: int, H: int, q: int, p: float):
    """Exact random-cluster expectations on the W x H torus (Eq. random_cluster).

    Weight of a bond set with b active bonds and n components:
    p^b (1-p)^(E-b) q^n.  Returns E[n], E[b], E[max cluster size].
    """
    packed, edges = all_bond_sets(W, H)
    E = len(edges)
    labels = propagate_labels(W, H, packed)
    ncl, mx = cluster_stats(labels)
    nb = np.zeros(packed.shape[0], dtype=np.int64)
    for e in range(E):
        nb += (np.arange(packed.shape[0]) >> e) & 1
    logw = nb * np.log(p) + (E - nb) * np.log1p(-p) + ncl * np.log(q)
    w = np.exp(logw - logw.max())
    Z = w.sum()
    return {
        "nclust": float((w * ncl).sum() / Z),
        "active": float((w * nb).sum() / Z),
        "maxcl": float((w * mx).sum() / Z),
    }


def crossing_bits(n: int):
    """Relevant bonds of the (n+1)-wide x n-tall open box for a left-right crossing.

    Horizontal bonds everywhere and vertical bonds off the two side columns
    (those on the sides cannot change whether a crossing exists).  Returns a list
    of (owner_site, bit) for W = n+1, H = n.
    """
    W, H = n + 1, n
    rel = []
    for y in range(H):
        for x in range(W):
            i = y * W + x
            if x + 1 < W:
                rel.append((i, 1))
            if y + 1 < H and 0 < x < W - 1:
                rel.append((i, 2))
    return rel


def binned_error(x: np.ndarray, nbins: int = 50) -> float:
    """Standard error of the mean of a correlated series by binning."""
    x = np.asarray(x, dtype=np.float64)
    m = (x.size // nbins) * nbins
    b = x[:m].reshape(nbins, -1).mean(axis=1)
    return float(b.std(ddof=1) / np.sqrt(nbins))


__all__ = [
    "Fraction",
    "itertools",
    "lattice_edges",
    "bfs_labels",
    "bfs_site_labels",
    "all_bond_sets",
    "propagate_labels",
    "cluster_stats",
    "all_states",
    "potts_exact",
    "fk_exact",
    "crossing_bits",
    "binned_error",
]


def cubic_edges(Lx: int, Ly: int, Lz: int):
    """List of (i, j, bit, owner) for every bond of the periodic Lx x Ly x Lz
    simple cubic lattice, site i = (z Ly + y) Lx + x: bit 1 = +x, 2 = +y, 4 = +z."""
    edges = []
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = (z * Ly + y) * Lx + x
                edges.append((i, (z * Ly + y) * Lx + (x + 1) % Lx, 1, i))
                edges.append((i, (z * Ly + (y + 1) % Ly) * Lx + x, 2, i))
                edges.append((i, (((z + 1) % Lz) * Ly + y) * Lx + x, 4, i))
    return edges


def bfs_labels_cubic(Lx: int, Ly: int, Lz: int, bonds: np.ndarray) -> np.ndarray:
    """Canonical labels (minimum site index per component) of packed cubic
    bonds, by BFS over an explicit adjacency list."""
    N = Lx * Ly * Lz
    adj = [[] for _ in range(N)]
    for i, j, bit, owner in cubic_edges(Lx, Ly, Lz):
        if bonds[owner] & bit:
            adj[i].append(j)
            adj[j].append(i)
    labels = np.full(N, -1, dtype=np.int64)
    for s in range(N):
        if labels[s] >= 0:
            continue
        comp = [s]
        labels[s] = s
        dq = deque([s])
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if labels[v] < 0:
                    labels[v] = s
                    comp.append(v)
                    dq.append(v)
        m = min(comp)
        for v in comp:
            labels[v] = m
    return labels
