"""The slice GEMM's loads straight into LDS are inline assembly that sets m0
(the LDS address of the fragment) right before each load.  m0 is a register
the compiler reserves and does not expect to change, so this is only sound
while nothing else in the compiled kernels reads m0.  The test compiles
ozgemm.hip to gfx950 assembly (host only, no GPU) and checks that every m0
reference is one of those writes, immediately followed by its load."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_13299_amd", "csrc")


def test_m0_only_feeds_the_lds_loads(tmp_path):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hipcc = os.path.join(rocm, "bin", "hipcc")
    if not os.path.exists(hipcc):
        hipcc = shutil.which("hipcc")
    if not hipcc:
        pytest.skip("no hipcc")
    out = tmp_path / "ozgemm.s"
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O3", "-S",
           "--cuda-device-only", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-Wno-inline-asm",
           os.path.join(CSRC, "ozgemm.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l.strip() for l in out.read_text().splitlines()]
    writes = 0
    for i, line in enumerate(lines):
        if line.startswith(";") or "m0" not in line.replace("m0_", ""):
            continue
        assert line.startswith("s_mov_b32 m0,"), f"other use of m0: {line}"
        nxt = lines[i + 1]
        assert nxt.startswith("buffer_load_dwordx4") and nxt.endswith(" lds"), (line, nxt)
        writes += 1
    assert writes > 0
