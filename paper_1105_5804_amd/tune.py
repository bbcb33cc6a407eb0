"""Autotuner for the tile shape and the merge schedule.

The labeling splits into a local phase on 128 x tile_h tiles and a global
phase over the clusters that touch tile borders; the tile size moves work
between the two (the paper's tile-size trade-off, Sec. II.E, Eqs.
optimaltile1-2).  Which split is fastest depends on the lattice shape, on the
number of states and the coupling (cluster structure), and on the device, so
it is measured: every candidate (tile_h in 16, 32, 64, 128; merge_waves, the
tiles per merge workgroup, in 4, 8, 16; for batches also the fused or the
per-phase engine) is timed with HIP events on the device, and the fastest is
kept in a JSON cache keyed on (gfx arch, W, H, q, mode).  Outputs never depend
on the choice; only time does.

The cache file is ``$SWCCL_TUNE_CACHE`` or ``~/.cache/swccl/tune.json``.
"""
from __future__ import annotations

import json
import os
import tempfile

TILE_HEIGHTS = (16, 32, 64, 128)
MERGE_WAVES = (4, 8, 16)
CANDIDATES = tuple((th, mw) for th in TILE_HEIGHTS for mw in MERGE_WAVES)


def cache_path() -> str:
    return os.environ.get("SWCCL_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "swccl",
                                                              "tune.json")


def cache_key(arch: str, W: int, H: int, q: int, mode: str) -> str:
    """(gfx arch, W, H, q, mode) as one string; mode names the workload kind
    ("sweep", "sweep_sizes", "batch", "bonds_periodic", "bonds_open", "sites_open")."""
    return f"{arch}|{int(W)}x{int(H)}|q{int(q)}|{mode}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    """Add one entry to the cache file (written to a temporary file, then renamed)."""
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    d = os.path.dirname(path) or "."
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune.", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(times: dict) -> tuple:
    """The fastest candidate of {candidate: ms}; ties go to the first listed."""
    if not times:
        raise ValueError("no candidate was timed")
    best = None
    for cand, ms in times.items():
        if best is None or ms < times[best]:
            best = cand
    return best


def tune(key: str, candidates, timer, force: bool = False, path: str | None = None) -> dict:
    """The cached entry for `key`, or time every candidate with `timer(candidate)
    -> ms`, cache the fastest and return its entry."""
    if not force:
        hit = load_cache(path).get(key)
        if hit is not None:
            return hit
    times = {}
    for cand in candidates:
        times[tuple(cand)] = float(timer(tuple(cand)))
    best = pick(times)
    entry = {"choice": list(best), "ms": times[best],
             "timings": {"/".join(map(str, c)): round(ms, 5) for c, ms in times.items()}}
    store(key, entry, path)
    return entry


# ---------------------------------------------------------------- device --

def _arch(torch) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _event_ms(torch, fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_sweep(W: int, H: int, q: int = 2, K: float | None = None, ising: bool | None = None,
               sizes: bool = False, reps: int = 5, warmup: int = 3, seed: int = 1, force: bool = False,
               candidates=CANDIDATES, path: str | None = None) -> dict:
    """Tile shape and merge schedule for sweeps of one W x H lattice (timed
    after `warmup` sweeps from a random start, so near the equilibrium cluster
    structure of the coupling K)."""
    import torch

    from . import SWLattice

    key = cache_key(_arch(torch), W, H, q, "sweep_sizes" if sizes else "sweep")

    def timer(cand):
        th, mw = cand
        lat = SWLattice(W, H, q=q, K=K, seed=seed, ising=ising, sizes=sizes, tile_h=th, merge_waves=mw)
        lat.sweep(warmup)
        ms = _event_ms(torch, lambda: lat.sweep(1), reps)
        lat.close()
        return ms

    return tune(key, candidates, timer, force, path)


def tuned_lattice(W: int, H: int, q: int = 2, K: float | None = None, ising: bool | None = None, **kw):
    """An SWLattice with the cached (or freshly tuned) tile shape and merge schedule."""
    from . import SWLattice

    e = tune_sweep(W, H, q=q, K=K, ising=ising, sizes=kw.get("sizes", False))
    th, mw = e["choice"]
    return SWLattice(W, H, q=q, K=K, ising=ising, tile_h=th, merge_waves=mw, **kw)


def tune_ccl(inp, mode: str = "bonds_periodic", sizes: bool = False, reps: int = 5, force: bool = False,
             candidates=CANDIDATES, path: str | None = None) -> dict:
    """Tile shape and merge schedule for labeling inputs like `inp` (an (H, W)
    uint8 GPU tensor; its statistics, e.g. the occupancy, steer the choice)."""
    import torch

    from . import ccl_label, ccl_workspace_bytes

    H, W = inp.shape
    key = cache_key(_arch(torch), W, H, 0, mode + ("_sizes" if sizes else ""))
    labels = torch.empty((H, W), dtype=torch.int32, device=inp.device)

    def timer(cand):
        th, mw = cand
        ws = torch.empty(ccl_workspace_bytes(W, H, mode, tile_h=th) + 256, dtype=torch.uint8, device=inp.device)
        ms = _event_ms(torch, lambda: ccl_label(inp, mode, sizes=sizes, workspace=ws, labels=labels, tile_h=th,
                                                merge_waves=mw), reps)
        del ws
        return ms

    return tune(key, candidates, timer, force, path)


def tune_batch(specs, reps: int = 5, warmup: int = 2, force: bool = False, path: str | None = None) -> dict:
    """Tile shape, merge schedule and engine (fused persistent launch or one
    launch per phase) for a batch of lattices; keyed on the batch's lattice
    count and total sites."""
    import torch

    from . import SWBatch

    nsite = sum(int(sp["W"]) * int(sp["H"]) for sp in specs)
    q = max(int(sp.get("q", 2)) for sp in specs)
    key = cache_key(_arch(torch), len(specs), nsite, q, "batch")
    cands = [(th, mw, eng) for th in TILE_HEIGHTS for mw in MERGE_WAVES for eng in ("phases", "fused")]

    def timer(cand):
        th, mw, eng = cand
        b = SWBatch(specs, tile_h=th, merge_waves=mw, fused=(eng == "fused"))
        b.sweep(warmup)
        ms = _event_ms(torch, lambda: b.sweep(1), reps)
        b.close()
        return ms

    return tune(key, cands, timer, force, path)
