"""CPU oracle for the Swendsen-Wang sweep and connected-component labeling.

TEST INFRASTRUCTURE ONLY.  This package wraps the plain sequential C reference
in ``swccl_oracle.c``.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the GPU library never does,
and the two share no code.

Every function takes and returns numpy arrays.  Potts states are 0..q-1; the
Ising conversion (s = 2*state - 1) is done by the caller.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swccl_oracle.c")
_HDR = os.path.join(_HERE, "swccl_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

TAG_INIT, TAG_BOND, TAG_FLIP, TAG_SEED, TAG_FEW, TAG_BOND_Z = 0, 1, 2, 3, 4, 5
PERIODIC, OPEN = 0, 1
REC_ACTIVE, REC_NCLUST, REC_MAXCL, REC_NSAT, REC_COUNTS, REC_LEN = 0, 1, 2, 3, 4, 12
REC3_ACTIVE, REC3_NCLUST, REC3_NSAT, REC3_COUNTS, REC3_LEN = 0, 1, 2, 3, 11


def build(force: bool = False) -> str:
    """Compile the oracle into ``liboracle.so`` with gcc (plain -O2 C11) when
    forced, missing, or older than its source or header."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = f"{_LIB}.tmp{os.getpid()}"  # one per process: parallel test workers may build at once
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


NATIVE_FLAGS = ["-O3", "-march=native", "-std=c11"]


def build_native() -> str:
    """Compile the same source with -O3 -march=native for the host that runs
    this process (the CPU-baseline timing and long fixture runs).  Built into a
    fresh temporary directory every time: a library tuned for one host's CPU
    must never be loaded on another."""
    d = tempfile.mkdtemp(prefix="swccl_oracle_native_")
    out = os.path.join(d, "liboracle_native.so")
    subprocess.check_call(["gcc", *NATIVE_FLAGS, "-fPIC", "-shared", "-o", out, _SRC, "-lm"])
    return out


_libs: dict = {}
_flavor = "O2"


def use_flavor(flavor: str) -> None:
    """Select the build the functions below call: "O2" (the default, built
    in-tree) or "native" (-O3 -march=native, built for this host on first
    use).  Both compile the same source; a CPU test checks that they agree."""
    global _flavor
    if flavor not in ("O2", "native"):
        raise ValueError(f"unknown oracle build flavor {flavor!r}")
    _flavor = flavor


def flavor() -> str:
    return _flavor


def _load(which: str | None = None):
    which = which or _flavor
    if which not in _libs:
        _libs[which] = _declare(ctypes.CDLL(build() if which == "O2" else build_native()))
    return _libs[which]


@contextlib.contextmanager
def using_library(path: str):
    """Route every call below to another build of the oracle (tests that plant
    a mistake in a copy of the source check that the pins catch it)."""
    global _flavor
    key = f"path:{path}"
    _libs[key] = _declare(ctypes.CDLL(path))
    prev, _flavor = _flavor, key
    try:
        yield
    finally:
        _flavor = prev
        _libs.pop(key, None)


def _declare(lib):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    c_i32, c_u32, c_u64, c_i64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_threshold.argtypes = [ctypes.c_double]
    lib.orc_threshold.restype = c_u64
    lib.orc_init_states.argtypes = [c_i32, c_i32, c_i32, c_u64, c_u32, u8p]
    lib.orc_init_states.restype = None
    lib.orc_activate_bonds.argtypes = [c_i32, c_i32, u8p, c_u64, c_u64, c_u32, c_u32, u8p]
    lib.orc_activate_bonds.restype = None
    lib.orc_label_bonds.argtypes = [c_i32, c_i32, u8p, c_i32, i32p]
    lib.orc_label_bonds.restype = c_i64
    lib.orc_label_sites.argtypes = [c_i32, c_i32, u8p, i32p]
    lib.orc_label_sites.restype = c_i64
    lib.orc_cluster_sizes.argtypes = [c_i64, i32p, i32p, i32p, i64p]
    lib.orc_cluster_sizes.restype = c_i64
    lib.orc_flip.argtypes = [c_i32, c_i32, c_i32, i32p, c_u64, c_u32, c_u32, u8p]
    lib.orc_flip.restype = None
    lib.orc_satisfied.argtypes = [c_i32, c_i32, c_i32, u8p, i64p]
    lib.orc_satisfied.restype = c_i64
    lib.orc_sw_sweep.argtypes = [c_i32, c_i32, c_i32, c_u64, c_u64, c_u32, c_u32,
                                 u8p, u8p, i32p, i64p]
    lib.orc_sw_sweep.restype = None
    lib.orc_sw_run.argtypes = [c_i32, c_i32, c_i32, c_u64, c_u64, c_u32, c_u32, c_i32,
                               u8p, i64p]
    lib.orc_sw_run.restype = None
    lib.orc_prob_threshold.argtypes = [ctypes.c_double]
    lib.orc_prob_threshold.restype = c_u64
    lib.orc_few_seeds.argtypes = [c_i32, c_i32, c_i32, c_u64, c_u32, c_u32, i32p]
    lib.orc_few_seeds.restype = c_i64
    lib.orc_few_sweep.argtypes = [c_i32, c_i32, c_u64, c_u64, c_i32, c_u64, c_u32, c_u32,
                                  u8p, u8p, i32p, i64p, i64p]
    lib.orc_few_sweep.restype = None
    lib.orc3_activate_bonds.argtypes = [c_i32, c_i32, c_i32, u8p, c_u64, c_u64, c_u32, c_u32, u8p]
    lib.orc3_activate_bonds.restype = None
    lib.orc3_label_bonds.argtypes = [c_i32, c_i32, c_i32, u8p, i32p]
    lib.orc3_label_bonds.restype = c_i64
    lib.orc3_satisfied.argtypes = [c_i32, c_i32, c_i32, c_i32, u8p, i64p]
    lib.orc3_satisfied.restype = c_i64
    lib.orc3_sw_sweep.argtypes = [c_i32, c_i32, c_i32, c_i32, c_u64, c_u64, c_u32, c_u32, u8p, u8p, i32p, i64p]
    lib.orc3_sw_sweep.restype = None
    lib.orc3_sw_run.argtypes = [c_i32, c_i32, c_i32, c_i32, c_u64, c_u64, c_u32, c_u32, c_i32, u8p, i64p]
    lib.orc3_sw_run.restype = None
    lib.orc_digest_u8.argtypes = [c_i64, u8p]
    lib.orc_digest_u8.restype = c_u64
    lib.orc_digest_i32.argtypes = [c_i64, i32p]
    lib.orc_digest_i32.restype = c_u64
    return lib


def _p(a: np.ndarray | None, ct):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ct))
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u8(a):
    return _p(a, ctypes.c_uint8)


def _i32(a):
    return _p(a, ctypes.c_int32)


def _i64(a):
    return _p(a, ctypes.c_int64)


# ------------------------------------------------------------------ Philox --
def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one counter (4 words) and key (2 words)."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def threshold(K: float) -> int:
    """T = floor((1 - exp(-K)) 2^32): a bond between equal spins is active iff r < T."""
    return int(_load().orc_threshold(float(K)))


# ----------------------------------------------------------------- SW steps --
def init_states(W: int, H: int, q: int, seed: int, sid: int = 0) -> np.ndarray:
    st = np.zeros(W * H, dtype=np.uint8)
    _load().orc_init_states(W, H, q, seed, sid, _u8(st))
    return st


def activate_bonds(W, H, state, T, seed, t, sid=0) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.uint8).reshape(-1)
    bonds = np.zeros(W * H, dtype=np.uint8)
    _load().orc_activate_bonds(W, H, _u8(st), T, seed, t, sid, _u8(bonds))
    return bonds


def label_bonds(W, H, bonds, mode=PERIODIC):
    """(labels, n_clusters) of a packed bond array (bit0 right, bit1 down)."""
    b = np.ascontiguousarray(bonds, dtype=np.uint8).reshape(-1)
    labels = np.zeros(W * H, dtype=np.int32)
    n = _load().orc_label_bonds(W, H, _u8(b), mode, _i32(labels))
    return labels, int(n)


def label_sites(W, H, occ):
    """(labels, n_clusters) of a binary image, 4-connected, open; background -1."""
    o = np.ascontiguousarray(occ, dtype=np.uint8).reshape(-1)
    labels = np.zeros(W * H, dtype=np.int32)
    n = _load().orc_label_sites(W, H, _u8(o), _i32(labels))
    return labels, int(n)


def cluster_sizes(labels):
    """(roots ascending, sizes, max_size)."""
    lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    N = lab.size
    roots = np.zeros(max(N, 1), dtype=np.int32)
    sizes = np.zeros(max(N, 1), dtype=np.int32)
    mx = np.zeros(1, dtype=np.int64)
    n = _load().orc_cluster_sizes(N, _i32(lab), _i32(roots), _i32(sizes), _i64(mx))
    return roots[:n].copy(), sizes[:n].copy(), int(mx[0])


def digest(a) -> int:
    """Check-sum of an array: sum of lo64(Philox((i, a_i, 0xD16E57, 0), key 0)) mod 2^64.
    uint8 arrays (states, bond bytes) and int32 arrays (labels) are accepted."""
    a = np.asarray(a).reshape(-1)
    if a.dtype == np.uint8:
        a = np.ascontiguousarray(a)
        return int(_load().orc_digest_u8(a.size, _u8(a)))
    if a.dtype == np.int32:
        a = np.ascontiguousarray(a)
        return int(_load().orc_digest_i32(a.size, _i32(a)))
    raise TypeError(f"digest of {a.dtype} arrays is not defined")


def flip(W, H, q, labels, state, seed, t, sid=0) -> np.ndarray:
    lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    st = np.array(state, dtype=np.uint8).reshape(-1)
    _load().orc_flip(W, H, q, _i32(lab), seed, t, sid, _u8(st))
    return st


def satisfied(W, H, q, state):
    """(n_sat, counts[8])."""
    st = np.ascontiguousarray(state, dtype=np.uint8).reshape(-1)
    counts = np.zeros(8, dtype=np.int64)
    n = _load().orc_satisfied(W, H, q, _u8(st), _i64(counts))
    return int(n), counts


def sw_sweep(W, H, q, T, seed, sid, t, state):
    """One sweep; returns (new_state, bonds, labels, record)."""
    st = np.array(state, dtype=np.uint8).reshape(-1)
    bonds = np.zeros(W * H, dtype=np.uint8)
    labels = np.zeros(W * H, dtype=np.int32)
    rec = np.zeros(REC_LEN, dtype=np.int64)
    _load().orc_sw_sweep(W, H, q, T, seed, sid, t, _u8(st), _u8(bonds), _i32(labels), _i64(rec))
    return st, bonds, labels, rec


def sw_run(W, H, q, T, seed, sid, t0, n, state):
    """n sweeps in C; returns (final_state, records[n, REC_LEN])."""
    st = np.array(state, dtype=np.uint8).reshape(-1)
    rec = np.zeros((max(n, 1), REC_LEN), dtype=np.int64)
    _load().orc_sw_run(W, H, q, T, seed, sid, t0, n, _u8(st), _i64(rec))
    return st, rec[:n]


# ------------------------------------------------------------- few-cluster --
def prob_threshold(p: float) -> int:
    """floor(p 2^32) for p in [0, 1): an event of probability p happens iff a
    uniform 32-bit word is below it."""
    return int(_load().orc_prob_threshold(float(p)))


def few_seeds(W, H, B, seed, t, sid=0) -> np.ndarray:
    """Seed sites of sweep t, one per B x B seed tile (tiles in raster order)."""
    n = ((W + B - 1) // B) * ((H + B - 1) // B)
    sites = np.zeros(max(n, 1), dtype=np.int32)
    _load().orc_few_seeds(W, H, B, seed, t, sid, _i32(sites))
    return sites[:n].copy()


def few_sweep(W, H, T, Tflip, B, seed, sid, t, state):
    """One few-cluster sweep of a q = 2 lattice; returns (new_state, bonds,
    labels, record, (seeded clusters, flipped clusters))."""
    st = np.array(state, dtype=np.uint8).reshape(-1)
    bonds = np.zeros(W * H, dtype=np.uint8)
    labels = np.zeros(W * H, dtype=np.int32)
    rec = np.zeros(REC_LEN, dtype=np.int64)
    few = np.zeros(2, dtype=np.int64)
    _load().orc_few_sweep(W, H, T, Tflip, B, seed, sid, t, _u8(st), _u8(bonds), _i32(labels), _i64(rec),
                          _i64(few))
    return st, bonds, labels, rec, (int(few[0]), int(few[1]))


# ---------------------------------------------------------- cubic lattices --
# Lx x Ly x Lz, periodic, site i = (z Ly + y) Lx + x; bond bits +x, +y, +z.
def init_states3(Lx, Ly, Lz, q, seed, sid=0) -> np.ndarray:
    """Initial states: those of the square lattice at the same site index."""
    return init_states(Lx, Ly * Lz, q, seed, sid)


def activate_bonds3(Lx, Ly, Lz, state, T, seed, t, sid=0) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.uint8).reshape(-1)
    bonds = np.zeros(Lx * Ly * Lz, dtype=np.uint8)
    _load().orc3_activate_bonds(Lx, Ly, Lz, _u8(st), T, seed, t, sid, _u8(bonds))
    return bonds


def label_bonds3(Lx, Ly, Lz, bonds):
    """(labels, n_clusters) of packed 3D bond bytes (bit0 +x, bit1 +y, bit2 +z)."""
    b = np.ascontiguousarray(bonds, dtype=np.uint8).reshape(-1)
    labels = np.zeros(Lx * Ly * Lz, dtype=np.int32)
    n = _load().orc3_label_bonds(Lx, Ly, Lz, _u8(b), _i32(labels))
    return labels, int(n)


def satisfied3(Lx, Ly, Lz, q, state):
    """(n_sat over the 3N bonds, counts[8])."""
    st = np.ascontiguousarray(state, dtype=np.uint8).reshape(-1)
    counts = np.zeros(8, dtype=np.int64)
    n = _load().orc3_satisfied(Lx, Ly, Lz, q, _u8(st), _i64(counts))
    return int(n), counts


def sw3_sweep(Lx, Ly, Lz, q, T, seed, sid, t, state):
    """One sweep of the cubic lattice; returns (new_state, bonds, labels, record)."""
    N = Lx * Ly * Lz
    st = np.array(state, dtype=np.uint8).reshape(-1)
    bonds = np.zeros(N, dtype=np.uint8)
    labels = np.zeros(N, dtype=np.int32)
    rec = np.zeros(REC3_LEN, dtype=np.int64)
    _load().orc3_sw_sweep(Lx, Ly, Lz, q, T, seed, sid, t, _u8(st), _u8(bonds), _i32(labels), _i64(rec))
    return st, bonds, labels, rec


def sw3_run(Lx, Ly, Lz, q, T, seed, sid, t0, n, state):
    """n sweeps of the cubic lattice in C; returns (final_state, records[n, REC3_LEN])."""
    st = np.array(state, dtype=np.uint8).reshape(-1)
    rec = np.zeros((max(n, 1), REC3_LEN), dtype=np.int64)
    _load().orc3_sw_run(Lx, Ly, Lz, q, T, seed, sid, t0, n, _u8(st), _i64(rec))
    return st, rec[:n]
