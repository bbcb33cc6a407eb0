#!/usr/bin/env python3
"""Benchmark of the Swendsen-Wang sweep on one MI355X.

A step is one full sweep (bond activation + tile labeling, cross-tile merge,
flatten + flip) of the q=3 Potts lattice L=16384 at its critical coupling
(``potts16384``), with inputs resident in HBM.  Prints one JSON line with:

* value: ns per spin per sweep over the timed steps (lower is better);
* phases: per-phase device time from HIP events on the launch stream;
* roofline: the dominant kernel against the HBM and ALU ceilings;
* ccl: the labeling-only pass on bond percolation at p = 1/2, same L
  (labeled sites/s);
* cpu_baseline: the CPU oracle on the machine's host, one sweep of the same lattice.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CUS, CLOCK_GHZ, LANES_PER_CU_CLK = 256, 2.4, 64
# Algorithmic bytes per site (a sweep needs the spin read and written once and
# one int32 label per site written and read back across the tile/merge split).
SWEEP_BYTES_PER_SITE = 10
TILE_BYTES_PER_SITE = 5   # spin in (1) + label out (4)
FLIP_BYTES_PER_SITE = 5   # label in (4) + spin out (1)
CCL_BYTES_PER_SITE = 13   # input (1) + label write, read and canonical write (3 x 4)
SERVE_BATCH_PX = 1 << 20  # the batched leg: requests of at most 1024^2 pixels share launches


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="potts16384")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ccl", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-few", action="store_true")
    ap.add_argument("--no-cubic", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--study", action="store_true",
                    help="instead of the bench line: sweep time and phases over couplings and q at L=16384")
    ap.add_argument("--few-scan", action="store_true",
                    help="few-cluster sweep time over L and the seed-tile edge B, beside the oracle")
    ap.add_argument("--size-scan", action="store_true",
                    help="per-phase sweep time per spin over L = 64 .. 16384 (q = 2 at beta_c), beside the oracle")
    ap.add_argument("--tile-scan", action="store_true",
                    help="instead of the bench line: sweep time and phases over tile shapes and merge schedules")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (calibrates HBM byte counters)")
    return ap.parse_args()


VALU_ISSUE_PEAK = CUS * CLOCK_GHZ * 1e9  # wave64 VALU instructions per second (1 per CU per clock)


def _profile(kernel: str):
    """Counter figures for `kernel` from the committed rocprofv3 summary, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_potts16384.json")
    src = os.path.join(ROOT, "paper_1105_5804_amd", "csrc", "kernels.hpp")
    try:
        prof = json.load(open(path))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if prof.get("kernels_hpp_sha256_16") != h:
        return None
    for name, v in prof.get("kernels", {}).items():
        if name.startswith(kernel):
            return v
    return None


def _served(args, torch, sw, wl, batch_px: int = 0, closed_loop_only: bool = False) -> dict:
    """Open-loop image-segmentation requests through the labeling server.

    Pool buffers (one per occupancy level, i.i.d. pixels) sit in pinned host
    memory; a request is N*N consecutive pixels of one, taken as an N x N
    image and copied to the device as part of the request.  Capacity is measured closed-loop on the first requests of the
    same mix; the open-loop run then offers Poisson arrivals at 0.8 x capacity.
    Latency: arrival -> completion of labels, roots and sizes in device memory,
    as seen by the host polling loop."""
    import numpy as np

    side = wl.SERVED_POOL_SIDE
    pool = []
    for lev in range(wl.SERVED_POOL_LEVELS):
        g = torch.Generator(device="cuda")
        g.manual_seed((wl.SEED_BASE | 5) + lev)
        img = (torch.rand((side, side), generator=g, device="cuda") < wl.served_pool_p(lev)).to(torch.uint8)
        host = torch.empty((side, side), dtype=torch.uint8, pin_memory=True)
        host.copy_(img)
        pool.append(host)
        del img
    torch.cuda.synchronize()
    reqs = wl.served_requests(args.serve_requests)
    flat = [p.view(-1) for p in pool]
    views = [flat[r["level"]][r["offset"]:r["offset"] + r["N"] * r["N"]].view(r["N"], r["N"]) for r in reqs]
    px = [r["N"] * r["N"] for r in reqs]
    srv = sw.CCLServer(32 << 30, mode="sites_open", sizes=True, max_inflight=256, n_streams=8, batch_px=batch_px)

    def run(order, arrivals):
        lat = {}
        t0 = time.perf_counter()
        i, n = 0, len(order)
        while len(lat) < n:
            now = time.perf_counter() - t0
            while i < n and arrivals[i] <= now:
                srv.submit(i, views[order[i]])
                i += 1
            srv.pump()
            for slot, tag in srv.poll():
                lat[tag] = time.perf_counter() - t0 - arrivals[tag]
                srv.release(slot)
        return lat, time.perf_counter() - t0

    # warm-up, then closed loop: every request offered at t = 0
    run(list(range(min(50, len(reqs)))), [0.0] * min(50, len(reqs)))
    nc = min(2000, len(reqs))
    _, tc = run(list(range(nc)), [0.0] * nc)
    cap = nc / tc
    if closed_loop_only:
        srv.close()
        return {"batch_px": batch_px, "closed_loop_req_per_s": round(cap, 1),
                "closed_loop_px_per_s": round(sum(px[:nc]) / tc, 1)}
    lam = 0.8 * cap
    arr, t = [], 0.0
    for r in reqs:
        t += r["gap"] / lam
        arr.append(t)
    lat, wall = run(list(range(len(reqs))), arr)
    srv.close()
    ms = np.array([lat[k] for k in range(len(reqs))]) * 1e3
    # the host -> device link alone: one pool image (1 byte per pixel) copied
    # from pinned memory, the bound on pixels per second of any served mix
    dst = torch.empty_like(pool[0], device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(pool[0], non_blocking=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(pool[0], non_blocking=True)
    ev1.record()
    torch.cuda.synchronize()
    h2d_gbs = 5 * pool[0].numel() / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del dst
    return {"workload": f"{len(reqs)} site-percolation images, side 64..8192 log-uniform, p 0.40..0.70, "
                        f"Poisson arrivals at 0.8 x closed-loop capacity; H2D from pinned host memory included",
            "batch_px": batch_px,
            "closed_loop_req_per_s": round(cap, 1),
            "closed_loop_px_per_s": round(sum(px[:nc]) / tc, 1),
            "offered_req_per_s": round(lam, 1),
            "p50_ms": round(float(np.percentile(ms, 50)), 4), "p99_ms": round(float(np.percentile(ms, 99)), 4),
            "mean_ms": round(float(ms.mean()), 4),
            "labeled_px_per_s": round(sum(px) / wall, 1), "wall_s": round(wall, 3),
            "h2d_pinned_gbs": round(h2d_gbs, 1)}


def _study(args) -> int:
    """Sweep time and per-phase split of the tiled path over the paper's variant
    axes: coupling off the critical point (0.6, 1.0, 1.4 x beta_c) and the
    number of states (q = 2, 3, 4), L = 16384, after equilibration."""
    import numpy as np
    import torch

    import paper_1105_5804_amd as sw

    L = 16384
    rows = []
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    for q in (2, 3, 4):
        kc = math.log1p(math.sqrt(q))
        for f in (0.6, 1.0, 1.4):
            lat = sw.SWLattice(L, L, q=q, K=kc * f, seed=(0x1105580400000000 | 0x57) + q, ising=False)
            lat.sweep(max(args.warmup, 20))
            torch.cuda.synchronize()
            evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
            for k in range(args.steps):
                evs[k][0].record(stream)
                for ph in range(3):
                    lat.sweep_phase(ph)
                    evs[k][ph + 1].record(stream)
            torch.cuda.synchronize()
            ph_ms = [float(np.mean([evs[k][p].elapsed_time(evs[k][p + 1]) for k in range(args.steps)])) for p in range(3)]
            o = lat.observables()
            rows.append({"q": q, "beta_over_beta_c": f, "K": round(kc * f, 6), "ms_per_sweep": round(sum(ph_ms), 4),
                         "tile_ms": round(ph_ms[0], 4), "merge_ms": round(ph_ms[1], 4), "flip_ms": round(ph_ms[2], 4),
                         "clusters_per_site": round(o["n_clusters"] / (L * L), 5),
                         "active_bonds_per_site": round(o["n_active_bonds"] / (L * L), 5)})
            print(json.dumps(rows[-1]), flush=True)
            del lat
            torch.cuda.empty_cache()
    return 0


def _size_scan(args) -> int:
    """Sweep time per spin and its split into the three phases over the
    lattice size (the q = 2 model at beta_c, Ising storage), beside the oracle
    on one host core: the analogue of the paper's breakdown and speed-up over
    L (Sec. II.E).  Whole sweeps go through sw_sweep (one-tile lattices take the
    fused whole-in-LDS kernel); the phase split comes from per-phase launches."""
    import numpy as np
    import torch

    import oracle
    import paper_1105_5804_amd as sw
    from paper_1105_5804_amd import workloads as wl

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    oracle.use_flavor("native")
    oracle.init_states(4, 4, 2, 1)  # builds the native oracle outside the timed calls
    K = wl.K_ISING_C
    for L in (64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384):
        N = L * L
        steps = max(args.steps, min(400, (1 << 26) // N))
        lat = sw.SWLattice(L, L, q=2, K=K, seed=wl.SEED_BASE | 0x5C)
        lat.sweep(max(args.warmup, 30))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.sweep(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        for k in range(steps):
            evs[k][0].record(stream)
            for ph in range(3):
                lat.sweep_phase(ph)
                evs[k][ph + 1].record(stream)
        torch.cuda.synchronize()
        ph_ms = [float(np.mean([evs[k][p].elapsed_time(evs[k][p + 1]) for k in range(steps)])) for p in range(3)]
        st = ((lat.spins.cpu().numpy().reshape(-1).astype(np.int16) + 1) // 2).astype(np.uint8)
        del lat
        torch.cuda.empty_cache()
        cpu_ns = None
        if N <= 8192 * 8192:  # one sweep of the oracle from the equilibrated spins, bounded in time
            c = time.perf_counter()
            oracle.sw_run(L, L, 2, oracle.threshold(K), wl.SEED_BASE | 0x5C, 0, 10**6, 1, st)
            cpu_ns = (time.perf_counter() - c) * 1e9 / N
        row = {"L": L, "sweeps": steps, "ms_per_sweep": round(ms, 5), "ns_per_spin": round(ms * 1e6 / N, 5),
               "tile_ns_per_spin": round(ph_ms[0] * 1e6 / N, 5), "merge_ns_per_spin": round(ph_ms[1] * 1e6 / N, 5),
               "flip_ns_per_spin": round(ph_ms[2] * 1e6 / N, 5),
               "phases_ns_per_spin": round(sum(ph_ms) * 1e6 / N, 5),
               "cpu_oracle_ns_per_spin": None if cpu_ns is None else round(cpu_ns, 3),
               "speedup_vs_oracle": None if cpu_ns is None else round(cpu_ns / (ms * 1e6 / N), 1)}
        print(json.dumps(row), flush=True)
    oracle.use_flavor("O2")
    return 0


def _few_scan(args) -> int:
    """Few-cluster sweeps (Sec. III; q = 2 at beta_c, p_flip = 1/2) over the
    lattice size and the seed-tile edge B, from SW-equilibrated spins, beside
    the oracle's few-cluster sweep on one host core: the analogue of the
    paper's speed-up of the few-cluster variant over L with the best B."""
    import numpy as np
    import torch

    import oracle
    import paper_1105_5804_amd as sw
    from paper_1105_5804_amd import workloads as wl

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    oracle.use_flavor("native")
    oracle.init_states(4, 4, 2, 1)  # builds the native oracle outside the timed calls
    K, seed = wl.K_ISING_C, wl.SEED_BASE | 0xF8
    for L in (256, 1024, 4096, 16384):
        N = L * L
        steps = max(args.steps, min(200, (1 << 26) // N))
        base = sw.SWLattice(L, L, q=2, K=K, seed=seed)
        base.sweep(max(args.warmup, 30))
        torch.cuda.synchronize()
        start = base.spins.clone()
        del base
        for B in (8, 32, 128, 512):
            if B > L:
                continue
            lat = sw.SWLattice(L, L, q=2, K=K, seed=seed, few_b=B, p_flip=0.5, spins=start.clone(), t=1000)
            lat.sweep(2)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.sweep(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            del lat
            cpu_ns = None
            if N <= 4096 * 4096:
                st = ((start.cpu().numpy().reshape(-1).astype(np.int16) + 1) // 2).astype(np.uint8)
                c = time.perf_counter()
                oracle.few_sweep(L, L, oracle.threshold(K), oracle.prob_threshold(0.5), B, seed, 0, 1000, st)
                cpu_ns = (time.perf_counter() - c) * 1e9 / N
            row = {"L": L, "B": B, "seeds": ((L + B - 1) // B) ** 2, "sweeps": steps, "ms_per_sweep": round(ms, 5),
                   "ns_per_spin": round(ms * 1e6 / N, 5),
                   "cpu_oracle_ns_per_spin": None if cpu_ns is None else round(cpu_ns, 3),
                   "speedup_vs_oracle": None if cpu_ns is None else round(cpu_ns / (ms * 1e6 / N), 1)}
            print(json.dumps(row), flush=True)
        del start
        torch.cuda.empty_cache()
    oracle.use_flavor("O2")
    return 0


def _batched(args, torch, sw, wl, stream) -> dict:
    """The batched workload (256 Ising lattices, L = 32..1024, own couplings
    and seeds): sweeps of the fused persistent launch (eager and as graph
    replays), of the one-launch-per-phase engine, and of the plain path that
    sweeps each lattice with its own launch sequence."""
    specs = wl.batch_specs()
    nsite = sum(sp["W"] * sp["H"] for sp in specs)
    reps = 16  # batched calls of 16 sweeps: two replays of the eight-sweep graph
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, n=1):
        fn()
        torch.cuda.synchronize()
        c0.record(stream)
        for _ in range(reps // n):
            fn()
        c1.record(stream)
        torch.cuda.synchronize()
        return c0.elapsed_time(c1) / reps

    res = {}
    for name, fused in (("fused", True), ("phases", False)):
        b = sw.SWBatch(specs, fused=fused)
        b.sweep(2)
        res[name] = timed(lambda: b.sweep(reps), reps)
        res[name + "_graph"] = timed(lambda: b.sweep(reps, graph=True), reps)
        del b
    lats = [sw.SWLattice(sp["W"], sp["H"], q=2, K=sp["K"], seed=sp["seed"], stream_id=sp["stream_id"])
            for sp in specs]
    for lat in lats:
        lat.sweep(2)

    def plain():
        for lat in lats:
            lat.sweep(1)

    res["plain"] = timed(plain)
    del lats
    torch.cuda.empty_cache()
    best = min(res["fused"], res["fused_graph"], res["phases"], res["phases_graph"])
    return {"workload": f"{len(specs)} Ising lattices, L in 32..1024, {nsite} sites",
            "ms_per_sweep": round(best, 4), "spins_per_s": round(nsite / (best * 1e-3), 1),
            "fused_ms_per_sweep": round(res["fused"], 4), "fused_graph_ms_per_sweep": round(res["fused_graph"], 4),
            "phases_ms_per_sweep": round(res["phases"], 4),
            "phases_graph_ms_per_sweep": round(res["phases_graph"], 4),
            "plain_ms_per_sweep": round(res["plain"], 4),
            "plain_spins_per_s": round(nsite / (res["plain"] * 1e-3), 1),
            "speedup_vs_plain": round(res["plain"] / best, 3),
            "frac_of_hbm_roofline": round(SWEEP_BYTES_PER_SITE * nsite / (best * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def _cpu_sweep_job(args):
    """One worker of the multi-core legs: n sweeps of one batch lattice."""
    import oracle

    oracle.use_flavor("native")
    W, H, K, seed, sid, n = args
    st = oracle.init_states(W, H, 2, seed, sid)
    t0 = time.perf_counter()
    oracle.sw_run(W, H, 2, oracle.threshold(K), seed, sid, 0, n, st)
    return time.perf_counter() - t0


def _cpu_label_job(args):
    """One worker of the served leg: label one site-percolation request image."""
    import oracle
    from paper_1105_5804_amd import workloads as wl

    oracle.use_flavor("native")
    N, p, seed = args
    img = wl.site_image(N, N, p, seed=seed).reshape(-1)
    t0 = time.perf_counter()
    oracle.label_sites(N, N, img)
    return time.perf_counter() - t0


def _cpu_baseline(cfg, wl) -> dict:
    """The CPU oracle (-O3 -march=native, built on this host) on bounded
    samples of the same workloads: sweeps of the benchmark lattice and the
    labeling pass on one thread, the batched and served mixes over every host
    core (one process per lattice or request)."""
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    import oracle

    oracle.use_flavor("native")
    N = cfg.W * cfg.H
    cores = _host_cores()
    st = oracle.init_states(cfg.W, cfg.H, cfg.q, cfg.seed)
    T = oracle.threshold(cfg.K)
    n_sw, t_sw = 0, 0.0
    while n_sw < 5 and t_sw < 15.0:  # sweeps 0, 1, ... from the seeded start, one call each
        c = time.perf_counter()
        st, _ = oracle.sw_run(cfg.W, cfg.H, cfg.q, T, cfg.seed, 0, n_sw, 1, st)
        t_sw += time.perf_counter() - c
        n_sw += 1
    del st
    out = {"value": round(t_sw * 1e9 / (n_sw * N), 3), "unit": "ns/spin/sweep", "cores": 1, "kind": "oracle",
           "sample": f"sweeps 0-{n_sw - 1} of the same {cfg.W}x{cfg.H} q={cfg.q} lattice from its seeded start, "
                     f"single thread, oracle built -O3 -march=native",
           "cpu_model": _cpu_model(), "host_cores": cores, "threads_of_host": f"1 of {cores}"}
    inp = wl.percolation_bonds(cfg.W, cfg.H, seed=wl.SEED_BASE | 3).reshape(-1)
    c = time.perf_counter()
    oracle.label_bonds(cfg.W, cfg.H, inp, oracle.PERIODIC)
    dt = time.perf_counter() - c
    del inp
    out["ccl"] = {"labeled_sites_per_s": round(N / dt, 1), "cores": 1,
                  "sample": f"one labeling of the {cfg.W}x{cfg.H} bond-percolation input (p = 1/2, periodic)"}
    specs = wl.batch_specs()
    jobs = [(sp["W"], sp["H"], sp["K"], sp["seed"], sp["stream_id"], 2) for sp in specs]
    nsite = sum(sp["W"] * sp["H"] for sp in specs)
    with ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_cpu_sweep_job, [(64, 64, specs[0]["K"], 1, 0, 1)] * cores))  # workers started, oracle built
        c = time.perf_counter()
        list(ex.map(_cpu_sweep_job, sorted(jobs, key=lambda j: -j[0] * j[1])))
        wall = time.perf_counter() - c
        out["batched"] = {"spins_per_s": round(2 * nsite / wall, 1), "cores": cores,
                          "sample": f"2 sweeps of each of the {len(specs)} batch lattices, one process per lattice"}
        reqs = wl.served_requests(400)
        rjobs = [(r["N"], wl.served_pool_p(r["level"]), 7000 + k) for k, r in enumerate(reqs)]
        px = sum(r["N"] * r["N"] for r in reqs)
        busy = sum(ex.map(_cpu_label_job, rjobs))
        out["served"] = {"labeled_px_per_s": round(cores * px / busy, 1), "labeled_px_per_s_per_core": round(px / busy, 1),
                         "cores": cores,
                         "sample": "the first 400 requests of the served mix (same sides and occupancies), one "
                                   "process per request; each labeling timed in its process (image generation "
                                   "excluded), aggregate = per-core rate x cores"}
    # the few-cluster update: one sweep of the Ising L = 4096 lattice at beta_c, seed tiles of 64 x 64
    Lf = 4096
    stf = oracle.init_states(Lf, Lf, 2, wl.SEED_BASE | 0xF7)
    c = time.perf_counter()
    oracle.few_sweep(Lf, Lf, oracle.threshold(wl.K_ISING_C), oracle.prob_threshold(0.5), 64, wl.SEED_BASE | 0xF7,
                     0, 0, stf)
    dt = time.perf_counter() - c
    del stf
    out["few_cluster"] = {"ns_per_spin_per_sweep": round(dt * 1e9 / (Lf * Lf), 3), "cores": 1,
                          "sample": f"one few-cluster sweep (64 x 64 seed tiles, p_flip 0.5) of an Ising "
                                    f"{Lf}x{Lf} lattice at beta_c from its seeded start, single thread"}
    # the simple cubic lattice: one sweep of an Ising 256^3 lattice at its critical coupling
    import paper_1105_5804_amd as sw3

    Lc = 256
    stc = oracle.init_states3(Lc, Lc, Lc, 2, wl.SEED_BASE | 0x3D5)
    c = time.perf_counter()
    oracle.sw3_sweep(Lc, Lc, Lc, 2, oracle.threshold(sw3.ising_K(sw3.BETA_C_ISING_3D)), wl.SEED_BASE | 0x3D5, 0, 0,
                     stc)
    dt = time.perf_counter() - c
    del stc
    out["cubic"] = {"ns_per_spin_per_sweep": round(dt * 1e9 / Lc**3, 3), "cores": 1,
                    "sample": f"one sweep of an Ising {Lc}^3 simple cubic lattice at beta_c from its seeded start, "
                              f"single thread"}
    out["paper_cpu_context"] = {"ns_per_spin_per_sweep": {"q2_L8192_Core2_Q6700": 77.39, "q2_L16384_Xeon_E5620": 152.1,
                                                          "q3_L8192_Core2_Q6700": 70.73},
                                "note": "serial CPU timings the paper lists beside its GPU ones (Table of results)"}
    oracle.use_flavor("O2")
    return out


def _phase_times(torch, lat, steps, stream):
    """Mean per-phase device time (tile, merge, flatten + flip) over `steps` sweeps."""
    import numpy as np

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps):
        evs[k][0].record(stream)
        for ph in range(3):
            lat.sweep_phase(ph)
            evs[k][ph + 1].record(stream)
    torch.cuda.synchronize()
    return [float(np.mean([evs[k][p].elapsed_time(evs[k][p + 1]) for k in range(steps)])) for p in range(3)]


def _few_cluster(args, torch, sw, wl, stream) -> dict:
    """Few-cluster sweeps (one seed per B x B seed tile, p_flip = 1/2) of the
    Ising L = 16384 lattice at beta_c for several B, beside the SW sweep of the
    same lattice.  Every update starts from the same SW-equilibrated spins
    (the few-cluster update alone would take many sweeps to leave the random
    start), so all rows time the same cluster structure; phases are timed as
    in the main leg."""
    import numpy as np

    L, K, seed = 16384, wl.K_ISING_C, wl.SEED_BASE | 0xF7
    steps = max(5, args.steps // 2)

    def timed(lat):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps * 3 + 1)]
        evs[0].record(stream)
        for k in range(steps):
            for ph in range(3):
                lat.sweep_phase(ph)
                evs[k * 3 + ph + 1].record(stream)
        torch.cuda.synchronize()
        ms = evs[0].elapsed_time(evs[-1]) / steps
        ph = [float(np.mean([evs[k * 3 + p].elapsed_time(evs[k * 3 + p + 1]) for k in range(steps)]))
              for p in range(3)]
        return {"ms_per_sweep": round(ms, 4), "ns_per_spin": round(ms * 1e6 / (L * L), 6),
                "tile_ms": round(ph[0], 4), "merge_ms": round(ph[1], 4), "seed_flip_ms": round(ph[2], 4),
                "energy_per_site_after": round(lat.observables()["energy_per_site"], 4)}

    base = sw.SWLattice(L, L, q=2, K=K, seed=seed)
    base.sweep(max(20, args.warmup))
    torch.cuda.synchronize()
    start = base.spins.clone()
    rows = [dict(update="sw", seed_tile=0, **timed(base))]
    del base
    for B in (16, 64, 256):
        lat = sw.SWLattice(L, L, q=2, K=K, seed=seed, few_b=B, p_flip=0.5, spins=start.clone(), t=1000)
        rows.append(dict(update="few", seed_tile=B, **timed(lat)))
        del lat
        torch.cuda.empty_cache()
    return {"workload": f"Ising {L}x{L} at beta_c from SW-equilibrated spins; few-cluster rows: one seed per "
                        f"B x B seed tile, p_flip 0.5", "rows": rows}


def _cubic(args, torch, sw, wl, stream) -> dict:
    """SW sweeps of the simple cubic Ising lattice (L = 512, 134 M sites) at
    its critical coupling, after equilibration sweeps: time per sweep, with
    and without per-sweep records, and the mean energy per site over the
    recorded sweeps.  The same 10 B/site model as the square lattice (spin in
    and out, a label carried across the local/global split) gives the HBM
    roofline fraction."""
    L = 512
    N = L**3
    K = sw.ising_K(sw.BETA_C_ISING_3D)
    lat = sw.CubicLattice(L, L, L, q=2, K=K, seed=wl.SEED_BASE | 0x3D5)
    lat.sweep(max(20, args.warmup))
    torch.cuda.synchronize()
    steps = max(5, args.steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    lat.sweep(steps)
    ev[1].record(stream)
    rec = lat.sweep(steps, records=True)
    ev[2].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    ms_rec = ev[1].elapsed_time(ev[2]) / steps
    e = -(2.0 * rec[:, 2].double() - 3.0 * N) / N
    # labeling alone: bond percolation near the simple cubic threshold (p = 0.2488)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(wl.SEED_BASE & 0xFFFFFFFF)
    on = torch.rand((3, L, L, L), device="cuda", generator=gen) < 0.2488
    bonds = (on[0].to(torch.uint8) | (on[1].to(torch.uint8) << 1) | (on[2].to(torch.uint8) << 2)).contiguous()
    del on
    sw.ccl3_label(bonds)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    _labels, _n = sw.ccl3_label(bonds)
    c1.record(stream)
    torch.cuda.synchronize()
    ccl_ms = c0.elapsed_time(c1)
    del bonds, _labels
    out = {"workload": f"Ising {L}^3 simple cubic at beta_c = {sw.BETA_C_ISING_3D}, {max(20, args.warmup)} "
                       f"equilibration sweeps, then {steps} timed",
           "ccl3_labeled_sites_per_s": round(N / (ccl_ms * 1e-3), 1),
           "ccl3_workload": "bond percolation on the same lattice at p = 0.2488 (labels and count, one call)",
           "ms_per_sweep": round(ms, 4), "ns_per_spin": round(ms * 1e6 / N, 6),
           "ms_per_sweep_with_records": round(ms_rec, 4),
           "mean_energy_per_site": round(float(e.mean()), 5),
           "hbm_frac_10B_per_site": round(SWEEP_BYTES_PER_SITE * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "mean_clusters_per_site": round(float(rec[:, 1].double().mean()) / N, 5)}
    del lat, rec
    torch.cuda.empty_cache()
    return out


def _tile_scan(args) -> int:
    """Sweep time and per-phase split against the tile shape (128 x tile_h) and
    the merge schedule (tiles per merge workgroup), on the benchmark lattice
    (q = 3 Potts, L = 16384, critical coupling) and on bond-percolation
    labeling of the same size: the local/global trade-off of the tile size."""
    import torch

    import paper_1105_5804_amd as sw
    from paper_1105_5804_amd import workloads as wl

    cfg = wl.CONFIGS["potts16384"]
    N = cfg.W * cfg.H
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    inp = torch.from_numpy(wl.percolation_bonds(cfg.W, cfg.H, seed=wl.SEED_BASE | 3)).cuda()
    labels = torch.empty((cfg.H, cfg.W), dtype=torch.int32, device="cuda")
    for th in (16, 32, 64, 128):
        for mw in (4, 8, 16):
            lat = sw.SWLattice(cfg.W, cfg.H, q=cfg.q, K=cfg.K, seed=cfg.seed, ising=False, tile_h=th, merge_waves=mw)
            lat.sweep(max(args.warmup, 5))
            torch.cuda.synchronize()
            ph = _phase_times(torch, lat, args.steps, stream)
            del lat
            torch.cuda.empty_cache()
            ws = torch.empty(sw.ccl_workspace_bytes(cfg.W, cfg.H, tile_h=th) + 256, dtype=torch.uint8, device="cuda")
            for _ in range(2):
                sw.ccl_label(inp, "bonds_periodic", workspace=ws, labels=labels, tile_h=th, merge_waves=mw)
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            for _ in range(args.steps):
                sw.ccl_label(inp, "bonds_periodic", workspace=ws, labels=labels, tile_h=th, merge_waves=mw)
            c1.record(stream)
            torch.cuda.synchronize()
            ccl_ms = c0.elapsed_time(c1) / args.steps
            del ws
            torch.cuda.empty_cache()
            row = {"tile": f"128x{th}", "merge_waves": mw, "ms_per_sweep": round(sum(ph), 4),
                   "ns_per_spin": round(sum(ph) * 1e6 / N, 6), "tile_ms": round(ph[0], 4),
                   "merge_ms": round(ph[1], 4), "flip_ms": round(ph[2], 4), "ccl_ms": round(ccl_ms, 4)}
            print(json.dumps(row), flush=True)
    return 0


def main() -> int:
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(a lattice would shard into row strips, one per GPU, exchanging one halo row and one gather of "
              "strip-crossing cluster pairs per sweep)", file=sys.stderr)
        return 2

    if args.study:
        return _study(args)
    if args.tile_scan:
        return _tile_scan(args)
    if args.size_scan:
        return _size_scan(args)
    if args.few_scan:
        return _few_scan(args)

    import numpy as np
    import torch

    import paper_1105_5804_amd as sw
    from paper_1105_5804_amd import workloads as wl

    cfg = wl.CONFIGS[args.workload]
    N = cfg.W * cfg.H
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    lat = sw.SWLattice(cfg.W, cfg.H, q=cfg.q, K=cfg.K, seed=cfg.seed, ising=cfg.ising,
                       keep_bonds=cfg.keep_bonds)
    for _ in range(args.warmup):
        lat.sweep(1)
    torch.cuda.synchronize()

    # ---- timed region: K full sweeps, an event between every two phases ----
    # (the phases are the sweep's three launches; the events add no work and
    # give the per-phase times of the same sweeps that are timed)
    nph = 3
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps * nph + 1)]
    t_wall0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        for ph in range(nph):
            lat.sweep_phase(ph)
            evs[k * nph + ph + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    ms_total = evs[0].elapsed_time(evs[-1])
    ms_step = ms_total / args.steps
    ns_spin = ms_step * 1e6 / N
    phase_ms = [float(np.mean([evs[k * nph + ph].elapsed_time(evs[k * nph + ph + 1]) for k in range(args.steps)]))
                for ph in range(nph)]
    names = ["tile", "merge", "flatten_flip"]
    obs = lat.observables()

    dom = int(np.argmax(phase_ms))
    dom_ms = phase_ms[dom]
    kname = {0: "swccl::k_tile<0", 1: "swccl::k_merge", 2: "swccl::k_flatten<0"}[dom]
    dom_bytes = [TILE_BYTES_PER_SITE, 0, FLIP_BYTES_PER_SITE][dom] * N
    achieved_gbs = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_bytes else 0.0
    prof = _profile(kname)
    roofline = {
        "kernel": kname.split("::")[-1].split("<")[0],
        "bound": "hbm",
        "achieved": round(achieved_gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
        "traffic": (prof["fetch_bytes"] + prof["write_bytes"]) if prof else None,
        "bytes_per_site": [TILE_BYTES_PER_SITE, 0, FLIP_BYTES_PER_SITE][dom],
        "sweep_frac_of_hbm_roofline": round(SWEEP_BYTES_PER_SITE * N / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    if prof and prof.get("valu_insts"):
        # the secondary (instruction-issue) ceiling: wave64 VALU instructions per
        # launch from the counters over this launch's time, against one per CU
        # per clock; valu_busy is the counters' own busy fraction
        rate = prof["valu_insts"] / (dom_ms * 1e-3)
        roofline["alu"] = {"achieved": round(rate / 1e9, 1), "peak": round(VALU_ISSUE_PEAK / 1e9, 1),
                           "unit": "G wave64 VALU instr/s", "frac": round(rate / VALU_ISSUE_PEAK, 4),
                           "valu_busy": prof.get("valu_busy")}
        roofline["binds"] = "alu" if rate / VALU_ISSUE_PEAK > roofline["frac"] else "hbm"
    if dom == 0:
        # the bond RNG alone: half a Philox4x32-10 block per site at ~62 lane-cycles per block
        roofline["philox_floor_ms"] = round(N * 31 / (CUS * LANES_PER_CU_CLK * CLOCK_GHZ * 1e9) * 1e3, 4)

    out = {
        "metric": "ns/spin per SW sweep at L=16384; labeled sites/s; batched/served vs plain",
        "value": round(ns_spin, 6),
        "unit": "ns/spin/sweep",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": cfg.name, "W": cfg.W, "H": cfg.H, "q": cfg.q, "K": cfg.K,
                   "spins": "int8" if cfg.ising else "uint8", "seed": hex(cfg.seed)},
        "spins_per_s": round(N / (ms_step * 1e-3), 1),
        "wall_s_timed": round(wall, 4),
        "phases_ms": {n: round(v, 4) for n, v in zip(names, phase_ms)},
        "roofline": roofline,
        "final_obs": {"t": obs["t"], "energy_per_site": obs["energy_per_site"],
                      "n_clusters": obs["n_clusters"], "n_active_bonds": obs["n_active_bonds"]},
    }
    del lat
    torch.cuda.empty_cache()

    # ---- labeling-only pass: bond percolation p = 1/2, same L ----
    if not args.no_ccl:
        inp = torch.from_numpy(wl.percolation_bonds(cfg.W, cfg.H, seed=wl.SEED_BASE | 3)).cuda()
        ws = torch.empty(sw.ccl_workspace_bytes(cfg.W, cfg.H) + 256, dtype=torch.uint8, device="cuda")
        labels = torch.empty((cfg.H, cfg.W), dtype=torch.int32, device="cuda")
        for _ in range(2):
            sw.ccl_label(inp, "bonds_periodic", workspace=ws, labels=labels)
        torch.cuda.synchronize()
        reps = max(3, args.steps // 2)
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(reps):
            sw.ccl_label(inp, "bonds_periodic", workspace=ws, labels=labels)
        c1.record(stream)
        torch.cuda.synchronize()
        ms = c0.elapsed_time(c1) / reps
        gbs = CCL_BYTES_PER_SITE * N / (ms * 1e-3) / 1e9
        out["ccl"] = {"workload": "bond percolation p=1/2, periodic", "ms": round(ms, 4),
                      "labeled_sites_per_s": round(N / (ms * 1e-3), 1),
                      "bytes_per_site": CCL_BYTES_PER_SITE, "achieved_gbs": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
        del inp, ws, labels

    # ---- batched sweeps of 256 mixed-size lattices vs one launch sequence each ----
    if not args.no_batch:
        out["batched"] = _batched(args, torch, sw, wl, stream)

    # ---- a one-tile lattice (Ising L=64, 1000 sweeps): fused launch vs tiled path ----
    if not args.no_batch:
        c = wl.CONFIGS["ising64"]
        res = {}
        for name in ("fused", "tiled"):
            lat = sw.SWLattice(c.W, c.H, q=2, K=c.K, seed=c.seed)
            torch.cuda.synchronize()
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            if name == "fused":
                lat.sweep_history(c.sweeps)
            else:
                for _ in range(c.sweeps):
                    for ph in range(3):
                        lat.sweep_phase(ph)
            c1.record(stream)
            torch.cuda.synchronize()
            res[name] = c0.elapsed_time(c1) * 1e3 / c.sweeps
            del lat
        out["small"] = {"workload": f"Ising {c.W}x{c.H}, {c.sweeps} sweeps with per-sweep records",
                        "us_per_sweep": round(res["fused"], 3),
                        "us_per_sweep_tiled_launches": round(res["tiled"], 3)}

    # ---- Ising L=4096, packed bonds kept: 200 + 1000 sweeps, without and with per-sweep records ----
    if not args.no_batch:
        c = wl.CONFIGS["ising4096"]
        lat = sw.SWLattice(c.W, c.H, q=2, K=c.K, seed=c.seed, keep_bonds=c.keep_bonds)
        lat.sweep(c.warmup)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        lat.sweep(c.sweeps)
        ev[1].record(stream)
        hist = lat.sweep_history(c.sweeps)
        ev[2].record(stream)
        torch.cuda.synchronize()
        ms_plain = ev[0].elapsed_time(ev[1]) / c.sweeps
        ms_rec = ev[1].elapsed_time(ev[2]) / c.sweeps
        e = -(2.0 * hist[:, 3].double() - 2.0 * c.W * c.H) / (c.W * c.H)
        out["ising4096"] = {"workload": f"Ising {c.W}x{c.H} at beta_c, packed bonds kept, "
                                        f"{c.warmup} + {c.sweeps} sweeps",
                            "ms_per_sweep": round(ms_plain, 4),
                            "ns_per_spin": round(ms_plain * 1e6 / (c.W * c.H), 6),
                            "ms_per_sweep_with_records": round(ms_rec, 4),
                            "mean_energy_per_site": round(float(e.mean()), 6)}
        del lat, hist
        torch.cuda.empty_cache()

    # ---- few-cluster update (Sec. III) on Ising L=16384 at beta_c, against the SW sweep ----
    if not args.no_few:
        out["few_cluster"] = _few_cluster(args, torch, sw, wl, stream)

    # ---- the same sweep on the simple cubic lattice ----
    if not args.no_cubic:
        out["cubic"] = _cubic(args, torch, sw, wl, stream)

    # ---- served labeling ----
    if not args.no_serve:
        out["served"] = _served(args, torch, sw, wl)
        # continuous batching of the small requests: more throughput closed-loop
        out["served"]["batched"] = _served(args, torch, sw, wl, batch_px=SERVE_BATCH_PX, closed_loop_only=True)
        torch.cuda.empty_cache()

    # ---- CPU oracle on the host cores: bounded samples of the same workloads ----
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(cfg, wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
