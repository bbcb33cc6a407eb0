"""Seeded synthetic workloads shaped like the paper's benchmarks.

This module only produces parameter sets and random inputs; it contains none of
the method's arithmetic, and both the GPU path and the CPU oracle consume what
it produces.  Random inputs come from numpy's PCG64.

Workloads (Sec. II.E and Table tab:results study critical Potts models and
percolation on periodic square lattices):
  ising64      q=2 Ising, L=64, beta_c, 1000 sweeps, energy/|m| per sweep
  ising4096    q=2 Ising, L=4096, beta_c, packed bonds kept, 200 + 1000 sweeps
  potts16384   q=3 Potts, L=16384, beta_c = ln(1+sqrt3) (Potts normalisation),
               100 sweeps; plus a labeling pass on bond percolation at p = 1/2
  batch256     256 independent Ising lattices of mixed size L in {32, ..., 1024}
               and couplings near beta_c (replicas / temperatures), swept
               together
  served       image-segmentation requests (Sec. I): square binary images of
               side N log-uniform in [64, 8192], site occupancy p uniform in
               [0.40, 0.70] (straddling site percolation, p_c ~ 0.5927),
               Poisson arrivals
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 0x1105580400000000

K_ISING_C = math.log1p(math.sqrt(2.0))   # K = 2 beta_c J for +-1 spins
K_POTTS3_C = math.log1p(math.sqrt(3.0))  # K = beta_c J for q = 3


@dataclass(frozen=True)
class SWConfig:
    name: str
    W: int
    H: int
    q: int
    ising: bool
    K: float
    seed: int
    sweeps: int
    warmup: int = 0
    keep_bonds: bool = False


CONFIGS = {
    "ising64": SWConfig("ising64", 64, 64, 2, True, K_ISING_C, SEED_BASE | 1, 1000),
    "ising4096": SWConfig("ising4096", 4096, 4096, 2, True, K_ISING_C, SEED_BASE | 2, 1000, 200, True),
    "potts16384": SWConfig("potts16384", 16384, 16384, 3, False, K_POTTS3_C, SEED_BASE | 3, 100),
}


def batch_specs(n: int = 256, seed: int = SEED_BASE | 4) -> list[dict]:
    """Lattice specs of the batched workload: lattice j has side L_j uniform over
    {32, 64, ..., 1024}, beta_j = beta_c (0.9 + 0.2 u_j) (K = 2 beta J for +-1
    spins), its own 64-bit seed and stream id j."""
    g = rng(seed)
    sides = 32 << g.integers(0, 6, size=n)
    u = g.random(n)
    seeds = g.integers(0, 2**63, size=n, dtype=np.int64)
    beta_c = 0.5 * K_ISING_C
    return [dict(W=int(L), H=int(L), q=2, ising=True, K=2.0 * beta_c * (0.9 + 0.2 * float(uj)),
                 seed=int(sd), stream_id=j)
            for j, (L, uj, sd) in enumerate(zip(sides, u, seeds))]


SERVED_POOL_SIDE = 8192
SERVED_POOL_LEVELS = 8


def served_pool_p(level: int) -> float:
    """Occupancy of pool image `level`: SERVED_POOL_LEVELS values spanning [0.40, 0.70]."""
    return 0.40 + 0.30 * (level + 0.5) / SERVED_POOL_LEVELS


def served_requests(n: int, seed: int = SEED_BASE | 5) -> list[dict]:
    """Parameters of n served requests: side N = round(exp(ln 64 + ln 128 u)),
    an occupancy level (a pool buffer of SERVED_POOL_SIDE^2 pixels of that p),
    the offset of the request's N*N pixels in that buffer (taken as a
    contiguous N x N image), and a unit-rate exponential inter-arrival gap
    (scaled by 1/lambda by the caller).  Every pool pixel is occupied
    independently, so every request is an i.i.d. site-percolation image."""
    g = rng(seed)
    u = g.random((n, 4))
    out = []
    total = SERVED_POOL_SIDE * SERVED_POOL_SIDE
    for r in range(n):
        N = int(round(math.exp(math.log(64) + math.log(128) * u[r, 0])))
        N = min(max(N, 1), SERVED_POOL_SIDE)
        lev = min(int(u[r, 1] * SERVED_POOL_LEVELS), SERVED_POOL_LEVELS - 1)
        span = total - N * N
        out.append(dict(N=N, level=lev, offset=int(u[r, 2] * (span + 1)), gap=-math.log1p(-u[r, 3])))
    return out


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def percolation_bonds(W: int, H: int, seed: int) -> np.ndarray:
    """Packed bond bytes (bit0 right, bit1 down), every bond open with p = 1/2."""
    return (rng(seed).integers(0, 256, size=(H, W), dtype=np.uint8) & 3).astype(np.uint8)


def random_bonds(W: int, H: int, p: float, seed: int) -> np.ndarray:
    """Packed bond bytes with every bond open independently with probability p."""
    r = rng(seed).random((H, W, 2)) < p
    return (r[..., 0].astype(np.uint8) | (r[..., 1].astype(np.uint8) << 1)).astype(np.uint8)


def site_image(W: int, H: int, p: float, seed: int) -> np.ndarray:
    """Binary image: each pixel occupied (1) with probability p."""
    return (rng(seed).random((H, W)) < p).astype(np.uint8)
