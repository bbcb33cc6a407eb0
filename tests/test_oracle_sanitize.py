"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only): a C program calls every oracle function on small, ragged and
degenerate shapes with exactly sized heap buffers; any report aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_exercise")
    flags = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    subprocess.run([gcc, *flags, "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "sanitize", "oracle_exercise.c"),
                    os.path.join(ROOT, "oracle", "swccl_oracle.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, timeout=120)
    # verify_asan_link_order=0: run even if the environment preloads a library ahead of the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr
