"""The host runtime (the rt_*.cpp units) built with AddressSanitizer and
UndefinedBehaviorSanitizer, host code only, linked with the regular objects
of the HIP sources: every host-side interface test must pass with no
sanitizer report.
Runs without a GPU (only the paths that fail before touching the device)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1106_5908_amd", "_build")
def _device_objects():
    from paper_1106_5908_amd import build as b

    return [os.path.splitext(src)[0] + ".o" for src in b.SOURCES if src.endswith(".hip")]


def _host_sources():
    from paper_1106_5908_amd import build as b

    return [src for src in b.SOURCES if src.endswith(".cpp")]


def _lib(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("g++") is None or _lib("libasan.so") is None
                    or not os.path.isdir("/opt/rocm/include"), reason="toolchain missing")
def test_host_runtime_under_sanitizers(tmp_path):
    objs = [os.path.join(BUILD, o) for o in _device_objects()]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("device objects not built (run the package build first)")
    so = str(tmp_path / "libspmv_san.so")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    host_objs = []
    for src in _host_sources():
        o = str(tmp_path / (os.path.splitext(src)[0] + "_san.o"))
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                               "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), *san,
                               "-c", os.path.join(ROOT, "paper_1106_5908_amd", "csrc", src), "-o", o])
        host_objs.append(o)
    subprocess.check_call(["g++", "-shared", *san, "-o", so, *host_objs, *objs, "-L/opt/rocm/lib",
                           "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ)
    pre = [_lib("libasan.so"), _lib("libubsan.so")]
    env["LD_PRELOAD"] = " ".join([p for p in pre if p] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["SPMV_LIBRARY"] = so
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_host.py"),
                        "-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu"],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
