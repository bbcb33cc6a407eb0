"""Stored values under tests/golden/ and what they pin.

critical_couplings.txt: the bond thresholds T of the critical points
K_c = ln(1 + sqrt q) (Sec. II.B.3 for q = 2), written from the closed form by
make_critical_couplings.py.  The oracle's threshold and the library's host-side
threshold (no device needed) must both give them from K in double precision."""
import importlib.util
import math
import os

import oracle
from paper_1105_5804_amd import _lib

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows():
    out = {}
    for line in open(os.path.join(HERE, "critical_couplings.txt")):
        if line.strip() and not line.startswith("#"):
            q, T = line.split()
            out[int(q)] = int(T)
    return out


def test_fixture_matches_its_generator():
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "make_critical_couplings.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    rows = _rows()
    assert sorted(rows) == [2, 3, 4, 8]
    for q, T in rows.items():
        assert mk.threshold(q) == T


def test_thresholds_at_critical_points():
    L = _lib.lib()
    for q, T in _rows().items():
        K = math.log1p(math.sqrt(q))
        assert oracle.threshold(K) == T, q
        assert L.sw_threshold(K) == T, q
