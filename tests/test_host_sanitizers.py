"""The host planning code of libdmp (csrc/plan.cpp) under the address and
undefined-behaviour sanitizers and, separately, the thread sanitizer: a
host-only driver (tests/host/host_stress.cpp) plans, carves and fills the
descriptors of random batches from eight threads at once, writes every
carved region of a workspace allocated at exactly the planned size, and
shares one keyed cache and the purification lock between the threads.
No GPU is involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2407_13299_amd", "csrc")
SRC = [os.path.join(HERE, "host", "host_stress.cpp"), os.path.join(CSRC, "plan.cpp")]

SANITIZERS = {
    "address_undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
    "thread": ["-fsanitize=thread"],
}


@pytest.mark.parametrize("name", sorted(SANITIZERS))
def test_host_planning_under_sanitizer(name, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / f"host_stress_{name}"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"), *SANITIZERS[name],
           *SRC, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in (r.stderr or ""):
        pytest.skip(f"sanitizer runtime for {name} not installed")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([str(exe), "8", "15"], capture_output=True, text=True, env=env,
                         timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "host planning ok" in run.stdout
    assert "WARNING" not in run.stderr and "runtime error" not in run.stderr, run.stderr
