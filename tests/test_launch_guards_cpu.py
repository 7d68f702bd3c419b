"""Host-only checks of the level-major launch geometry and the launchers'
empty-range guards: tests/native/launch_guards.hip, compiled with hipcc and
linked against the built library, run on the CPU (it launches no kernel)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "launch_guards.hip")
LIBDIR = os.path.join(ROOT, "paper_2304_10516_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(os.path.join(LIBDIR, "libdvnr.so")) or not shutil.which(HIPCC),
                    reason="needs hipcc and the built library")
def test_level_major_mapping_and_empty_launches(tmp_path):
    exe = str(tmp_path / "launch_guards")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", SRC, "-o", exe, f"-L{LIBDIR}", "-ldvnr", f"-Wl,-rpath,{LIBDIR}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "launch guards ok" in r.stdout
