"""The serving loop's scheduling core on the host, with a fake executor in
place of the GPU (tests/serve_core_test.cpp): admission by memory budget,
FIFO order, max_batch per launch, arrivals sharing the next launch, failure
and shutdown paths, nearest-rank percentiles, and many threads at once.
Built with g++, and with clang++ under the address + undefined-behaviour and
the thread sanitizers (host code only; clang's thread sanitizer understands
the steady-clock timed waits of the engine loop)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_core_test.cpp")
INC = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1310_7297_amd", "csrc")]
CLANG = "/opt/rocm/llvm/bin/clang++"

VARIANTS = {
    "gcc": ("g++", ["-O2"]),
    "asan_ubsan": (CLANG, ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer"]),
    "tsan": (CLANG, ["-O1", "-g", "-fsanitize=thread"]),
}


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_serve_core(variant, tmp_path):
    cxx, flags = VARIANTS[variant]
    if shutil.which(cxx) is None:
        pytest.skip(f"{cxx} not available")
    exe = str(tmp_path / f"serve_core_{variant}")
    cmd = [cxx, "-std=c++17", "-Wall", "-Wextra", "-Werror", "-pthread"] + flags + INC + [SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
