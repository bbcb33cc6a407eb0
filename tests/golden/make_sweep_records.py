#!/usr/bin/env python3
"""Write per-sweep oracle records of the benchmark workloads to tests/golden/.

Calls only the CPU oracle (and the seeded parameter sets of
paper_1105_5804_amd.workloads, which hold none of the method's arithmetic).
One line per recorded sweep t:

    t active n_clusters max_cluster n_sat counts[0..q-1] digest_spins digest_labels digest_bonds

with the counters of Sec. II's three steps as the oracle reports them (active
bonds, clusters and the largest cluster of the sweep's bond configuration;
satisfied bonds (-H/J, Eq. potts_hamiltonian) and state counts of the spins
after the flip) and the order-independent array digests (spins after the flip;
labels and bond bytes of the sweep, before the flip), in hexadecimal.

    python tests/golden/make_sweep_records.py ising64 ising4096 potts16384 batch256 few1024 cubic128

ising64 / ising4096 / potts16384 record every sweep (1000, 200 + 1000 and 100
sweeps); batch256 records every lattice of the batched workload after sweeps
1, 10, 100 and 1000; few1024 records every sweep of the few-cluster update
(Sec. III) on an Ising 1024 x 1024 lattice at beta_c with 32 x 32 seed tiles
and p_flip = 1/2 (the FEW parameters below); cubic128 records every sweep of
the SW update on the simple cubic Ising lattice 128^3 at its critical
coupling (the CUBIC parameters below; lines "t active n_clusters n_sat
counts[0..1] digest_spins").  The oracle is built with -O3 -march=native for
speed; a CPU test checks that this build agrees with the default one.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1105_5804_amd import workloads as wl  # noqa: E402

BATCH_CHECKPOINTS = (1, 10, 100, 1000)
# the few-cluster record: L, seed tile edge, p_flip, sweeps, seed
FEW = dict(L=1024, B=32, p_flip=0.5, sweeps=300, seed=wl.SEED_BASE | 0xFE)
# the cubic-lattice record: L, sweeps, seed; K = 2 beta_c of the 3D Ising model
CUBIC = dict(L=128, sweeps=400, seed=wl.SEED_BASE | 0x3DC, K=2 * 0.22165455)


def _line(t, rec, q, d_spins, d_labels, d_bonds) -> str:
    counts = " ".join(str(int(c)) for c in rec[oracle.REC_COUNTS:oracle.REC_COUNTS + min(q, 8)])
    return (f"{t} {int(rec[oracle.REC_ACTIVE])} {int(rec[oracle.REC_NCLUST])} {int(rec[oracle.REC_MAXCL])} "
            f"{int(rec[oracle.REC_NSAT])} {counts} {d_spins:016x} {d_labels:016x} {d_bonds:016x}")


def single(name: str) -> None:
    """Every sweep of one single-lattice workload."""
    cfg = wl.CONFIGS[name]
    T = oracle.threshold(cfg.K)
    st = oracle.init_states(cfg.W, cfg.H, cfg.q, cfg.seed)
    total = cfg.warmup + cfg.sweeps
    out = os.path.join(HERE, f"sweeps_{name}.txt")
    pool = ThreadPoolExecutor(max_workers=3)  # the three digests of a sweep run beside the next sweep
    pending = []
    t0 = time.time()
    with open(out + ".tmp", "w") as f:
        f.write(f"# {name}: W={cfg.W} H={cfg.H} q={cfg.q} K={cfg.K!r} seed={cfg.seed:#x} stream_id=0, "
                f"sweeps t=0..{total - 1}\n")
        f.write("# written by tests/golden/make_sweep_records.py from the CPU oracle only\n")
        f.write("# t active n_clusters max_cluster n_sat counts[0..q-1] digest_spins digest_labels digest_bonds\n")
        for t in range(total):
            st, bonds, labels, rec = oracle.sw_sweep(cfg.W, cfg.H, cfg.q, T, cfg.seed, 0, t, st)
            futs = [pool.submit(oracle.digest, a) for a in (st.copy(), labels, bonds)]
            pending.append((t, rec, futs))
            while pending and (len(pending) > 2 or t == total - 1):
                tt, rr, ff = pending.pop(0)
                f.write(_line(tt, rr, cfg.q, *[x.result() for x in ff]) + "\n")
                f.flush()
            if t % 10 == 0:
                print(f"{name}: sweep {t} of {total} ({time.time() - t0:.0f} s)", flush=True)
    os.replace(out + ".tmp", out)
    print(f"{name}: wrote {out}", flush=True)


def _batch_lattice(args):
    j, sp = args
    oracle.use_flavor("native")
    q = 2
    T = oracle.threshold(sp["K"])
    st = oracle.init_states(sp["W"], sp["H"], q, sp["seed"], sp["stream_id"])
    lines, done = [], 0
    for cp in BATCH_CHECKPOINTS:
        if cp - 1 > done:
            st, _ = oracle.sw_run(sp["W"], sp["H"], q, T, sp["seed"], sp["stream_id"], done, cp - 1 - done, st)
        st, bonds, labels, rec = oracle.sw_sweep(sp["W"], sp["H"], q, T, sp["seed"], sp["stream_id"], cp - 1, st)
        done = cp
        lines.append(f"{j} " + _line(cp - 1, rec, q, oracle.digest(st), oracle.digest(labels), oracle.digest(bonds)))
    return j, lines


def batch() -> None:
    """Every lattice of the batched workload at the checkpoints."""
    specs = wl.batch_specs()
    out = os.path.join(HERE, "batch256.txt")
    res = {}
    t0 = time.time()
    # largest lattices first so the pool drains evenly
    order = sorted(enumerate(specs), key=lambda js: -js[1]["W"] * js[1]["H"])
    with ProcessPoolExecutor(max_workers=max(1, (os.cpu_count() or 2) - 2)) as ex:
        for j, lines in ex.map(_batch_lattice, order):
            res[j] = lines
            if len(res) % 16 == 0:
                print(f"batch256: {len(res)} of {len(specs)} lattices ({time.time() - t0:.0f} s)", flush=True)
    with open(out + ".tmp", "w") as f:
        f.write(f"# batch256: the {len(specs)} lattices of workloads.batch_specs(), records after sweeps "
                f"{', '.join(map(str, BATCH_CHECKPOINTS))}\n")
        f.write("# written by tests/golden/make_sweep_records.py from the CPU oracle only\n")
        f.write("# spec: j W H K seed stream_id\n")
        for j, sp in enumerate(specs):
            f.write(f"spec {j} {sp['W']} {sp['H']} {sp['K']!r} {sp['seed']} {sp['stream_id']}\n")
        f.write("# j t active n_clusters max_cluster n_sat counts[0..1] digest_spins digest_labels digest_bonds\n")
        for j in range(len(specs)):
            for ln in res[j]:
                f.write(ln + "\n")
    os.replace(out + ".tmp", out)
    print(f"batch256: wrote {out}", flush=True)


def few() -> None:
    """Every sweep of the few-cluster update on the FEW lattice."""
    L, B, pf, n, seed = FEW["L"], FEW["B"], FEW["p_flip"], FEW["sweeps"], FEW["seed"]
    K = wl.K_ISING_C
    T, Tf = oracle.threshold(K), oracle.prob_threshold(pf)
    st = oracle.init_states(L, L, 2, seed)
    out = os.path.join(HERE, "sweeps_few1024.txt")
    with open(out + ".tmp", "w") as f:
        f.write(f"# few1024: W={L} H={L} q=2 K={K!r} seed={seed:#x} stream_id=0 few_b={B} p_flip={pf!r}, "
                f"sweeps t=0..{n - 1}\n")
        f.write("# written by tests/golden/make_sweep_records.py from the CPU oracle only\n")
        f.write("# t active n_clusters max_cluster n_sat counts[0..1] digest_spins digest_labels digest_bonds\n")
        for t in range(n):
            st, bonds, labels, rec, _ = oracle.few_sweep(L, L, T, Tf, B, seed, 0, t, st)
            f.write(_line(t, rec, 2, oracle.digest(st), oracle.digest(labels), oracle.digest(bonds)) + "\n")
    os.replace(out + ".tmp", out)
    print(f"few1024: wrote {out}", flush=True)


def cubic() -> None:
    """Every sweep of the SW update on the CUBIC lattice."""
    L, n, seed, K = CUBIC["L"], CUBIC["sweeps"], CUBIC["seed"], CUBIC["K"]
    T = oracle.threshold(K)
    st = oracle.init_states3(L, L, L, 2, seed)
    out = os.path.join(HERE, "sweeps_cubic128.txt")
    t0 = time.time()
    with open(out + ".tmp", "w") as f:
        f.write(f"# cubic128: Lx=Ly=Lz={L} q=2 K={K!r} seed={seed:#x} stream_id=0, sweeps t=0..{n - 1}\n")
        f.write("# written by tests/golden/make_sweep_records.py from the CPU oracle only\n")
        f.write("# t active n_clusters n_sat counts[0..1] digest_spins\n")
        for t in range(n):
            st, _b, _l, rec = oracle.sw3_sweep(L, L, L, 2, T, seed, 0, t, st)
            f.write(f"{t} {int(rec[oracle.REC3_ACTIVE])} {int(rec[oracle.REC3_NCLUST])} {int(rec[oracle.REC3_NSAT])} "
                    f"{int(rec[oracle.REC3_COUNTS])} {int(rec[oracle.REC3_COUNTS + 1])} {oracle.digest(st):016x}\n")
            if t % 20 == 0:
                print(f"cubic128: sweep {t} of {n} ({time.time() - t0:.0f} s)", flush=True)
    os.replace(out + ".tmp", out)
    print(f"cubic128: wrote {out}", flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+", choices=["ising64", "ising4096", "potts16384", "batch256", "few1024",
                                                 "cubic128"])
    args = ap.parse_args()
    oracle.use_flavor("native")
    for w in args.which:
        if w == "batch256":
            batch()
        elif w == "few1024":
            few()
        elif w == "cubic128":
            cubic()
        else:
            single(w)
    return 0


if __name__ == "__main__":
    sys.exit(main())
