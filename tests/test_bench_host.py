"""Host logic of bench.py that runs without a GPU: the gate that reports
counter traffic only for the kernel source it was measured on, and the
refusal of multi-GPU runs."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports nothing GPU-side at module level)


def _tree(tmp_path, kernels_src: bytes):
    """A minimal copy of the files the gate reads, with the given kernel source."""
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1105_5804_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "traffic_potts16384.json"), tmp_path / "profiles")
    (tmp_path / "paper_1105_5804_amd" / "csrc" / "kernels.hpp").write_bytes(kernels_src)
    return str(tmp_path)


def test_profile_gate_matches_source(tmp_path, monkeypatch):
    src = open(os.path.join(ROOT, "paper_1105_5804_amd", "csrc", "kernels.hpp"), "rb").read()
    prof = json.load(open(os.path.join(ROOT, "profiles", "traffic_potts16384.json")))
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path, src))
    got = bench._profile("swccl::k_tile<0")
    if prof["kernels_hpp_sha256_16"] != hashlib.sha256(src).hexdigest()[:16]:
        # counters taken on another kernel source: the bench must report no traffic
        assert got is None
        return
    assert got is not None
    assert got["fetch_bytes"] > 0 and got["write_bytes"] > 0 and got["valu_insts"] > 0
    assert bench._profile("swccl::no_such_kernel") is None


def test_profile_gate_rejects_changed_source(tmp_path, monkeypatch):
    src = open(os.path.join(ROOT, "paper_1105_5804_amd", "csrc", "kernels.hpp"), "rb").read()
    monkeypatch.setattr(bench, "ROOT", _tree(tmp_path, src + b"\n// changed\n"))
    assert bench._profile("swccl::k_tile<0") is None


def test_profile_gate_without_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._profile("swccl::k_tile<0") is None


@pytest.mark.parametrize("argv", [["--gpus", "2"], ["--gpus", "8", "--steps", "1"]])
def test_multi_gpu_refused(argv):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
