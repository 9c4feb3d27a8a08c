"""The host-side mesh preprocessing (csrc/mesh.cpp) built with
AddressSanitizer and UndefinedBehaviorSanitizer by the system g++ and run on
valid meshes (invariants: permutation, mutual neighbours, boundary types,
tile halos) and on invalid inputs that must be refused with a message.  No
GPU and no HIP: the file is plain C++."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2307_14302_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_mesh_preprocessing_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "mesh_host_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{CSRC}", os.path.join(HERE, "native", "mesh_host_check.cpp"),
           os.path.join(CSRC, "mesh.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
