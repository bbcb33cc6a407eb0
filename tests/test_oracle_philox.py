"""Pins of the oracle's Philox4x32-10 and bond threshold.

Philox is pinned against rocRAND's own implementation of the published
generator (its host-callable header, compiled here for the CPU), which shares
nothing with the oracle.  The threshold is pinned against closed forms of the
critical bond probabilities.
"""
import atexit
import math
import os
import shutil
import subprocess
import tempfile
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle

_ROCRAND_HELPER = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = ((unsigned long long)c0 | ((unsigned long long)c1 << 32)) * 4ull;
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    uint4 v = rocrand4(&st);
    printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
"""


_HELPER = {}


def _rocrand_exe():
    """The helper program, compiled once per test session."""
    if "exe" not in _HELPER:
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        hdr = "/opt/rocm/include/rocrand/rocrand_kernel.h"
        if not (os.path.exists(hipcc) and os.path.exists(hdr)):
            pytest.skip("hipcc or rocRAND headers not available")
        d = tempfile.mkdtemp(prefix="swccl_rocrand_")
        atexit.register(shutil.rmtree, d, True)
        src = os.path.join(d, "rr.cpp")
        exe = os.path.join(d, "rr")
        with open(src, "w") as f:
            f.write(_ROCRAND_HELPER)
        subprocess.check_call([hipcc, "-O1", "-o", exe, src],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        _HELPER["exe"] = exe
    return _HELPER["exe"]


def _rocrand_blocks(rows):
    inp = "\n".join(" ".join("%08x" % v for v in r) for r in rows) + "\n"
    out = subprocess.run([_rocrand_exe()], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand():
    rng = np.random.default_rng(20110531)
    rows = []
    # rocRAND's offset route takes counter words 0-1 as a 64-bit block index
    # times 4, so word 1 is kept below 2^30 to avoid overflow there.
    for _ in range(1500):
        c = rng.integers(0, 2**32, size=6, dtype=np.uint64)
        c[1] %= 2**30
        rows.append([int(v) for v in c])
    # counters shaped like the ones the sweep uses: (index word, t, tag, stream)
    for w in (0, 1, 2, 3, 2**29, 2**31 - 1, 2**32 - 1):
        for t in (0, 1, 999):
            for tag in (0, 1, 2):
                rows.append([w, t, tag, 7, 0x00000000, 0x11055804])
    rows.append([0, 0, 0, 0, 0, 0])
    ref = _rocrand_blocks(rows)
    assert len(ref) == len(rows)
    for r, want in zip(rows, ref):
        got = oracle.philox(r[:4], r[4:])
        assert [int(v) for v in got] == want, r


def _floor_pow32(p: Decimal) -> int:
    return int((p * (Decimal(2) ** 32)).to_integral_value(rounding="ROUND_FLOOR"))


def test_threshold_closed_forms():
    getcontext().prec = 60
    # Ising at beta_c: K = 2 beta_c J = ln(1+sqrt2) -> p = 1 - 1/(1+sqrt2) = 2 - sqrt2
    assert oracle.threshold(math.log1p(math.sqrt(2.0))) == _floor_pow32(2 - Decimal(2).sqrt())
    # q=3 Potts at K = ln(1+sqrt3) -> p = sqrt3/(1+sqrt3) = (3 - sqrt3)/2
    assert oracle.threshold(math.log1p(math.sqrt(3.0))) == _floor_pow32((3 - Decimal(3).sqrt()) / 2)
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(-1.0) == 0
    assert oracle.threshold(float("inf")) == 2**32
    assert oracle.threshold(100.0) == 2**32
    assert oracle.threshold(math.log(2.0)) in (2**31 - 1, 2**31)
    # monotone in K
    Ks = np.linspace(0.01, 5, 200)
    Ts = [oracle.threshold(k) for k in Ks]
    assert all(a <= b for a, b in zip(Ts, Ts[1:]))


def test_oracle_ctypes_match_header():
    """The oracle wrapper's ctypes declarations equal the C prototypes of
    swccl_oracle.h (return type, arity, parameter types; arrays are pointers)."""
    import ctypes
    import os
    import re

    hdr = open(os.path.join(os.path.dirname(oracle.__file__), "swccl_oracle.h")).read()
    hdr = re.sub(r"/\*.*?\*/", " ", hdr, flags=re.S)
    scalars = {"int32_t": ctypes.c_int32, "uint32_t": ctypes.c_uint32, "int64_t": ctypes.c_int64,
               "uint64_t": ctypes.c_uint64, "uint8_t": ctypes.c_uint8, "double": ctypes.c_double}
    lib = oracle._load()
    protos = re.findall(r"(\w+)\s+(orc_\w+)\s*\(([^)]*)\)\s*;", hdr)
    assert {p[1] for p in protos} == set(re.findall(r"\b(orc_\w+)\s*\(", hdr))  # every prototype parsed
    for ret, name, params in protos:
        fn = getattr(lib, name)
        assert (fn.restype is None) if ret == "void" else (fn.restype is scalars[ret]), name
        plist = [p.strip() for p in params.split(",") if p.strip() and p.strip() != "void"]
        assert len(plist) == len(fn.argtypes), name
        for p, py in zip(plist, fn.argtypes):
            p = re.sub(r"(\w+)\s*\[\d*\]$", r"* \1", p)  # an array parameter is a pointer
            base = " ".join(re.sub(r"\b\w+$", "", p).replace("const", " ").replace("*", " ").split())
            want = ctypes.POINTER(scalars[base]) if "*" in p else scalars[base]
            assert py is want, (name, p, py)
