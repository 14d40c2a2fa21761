"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) passes every pin: no out-of-bounds access or undefined
behaviour in the reference the GPU path is checked against."""
import os
import shutil
import subprocess
import sys

import pytest

import oracle
import pins

ORACLE_SRC = os.path.join(os.path.dirname(oracle.__file__), "spmv_oracle.c")


def _libasan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(shutil.which("gcc") is None or _libasan() is None, reason="gcc/libasan missing")
def test_pins_under_sanitizers(tmp_path):
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fno-fast-math", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-shared", "-fPIC", "-o", so,
                           ORACLE_SRC, "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = _libasan() + ((" " + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(pins.__file__), "pins.py"), so],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ALL-PASS" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
