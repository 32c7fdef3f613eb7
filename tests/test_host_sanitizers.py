"""Host code of the library (charge aggregation, binned estimate, layout
conversion) and the C oracle built for the host with ROCm's clang (which
knows _Float16 on x86) under AddressSanitizer and UndefinedBehaviorSanitizer
and run on the CPU; no GPU code is built."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")


@pytest.mark.skipif(not os.path.exists(CLANGXX) or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs ROCm's clang and the HIP headers")
def test_host_code_under_sanitizers(tmp_path):
    exe = tmp_path / "host_checks"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    csrc = os.path.join(ROOT, "paper_1403_0711_amd", "csrc")
    oracle_c = tmp_path / "oracle.o"
    r = subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-fopenmp", *san, "-c",
                        os.path.join(ROOT, "oracle", "heatbath_oracle.c"), "-o", str(oracle_c)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([CLANGXX, "-O1", "-g", "-std=c++17", "-fopenmp", *san, "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), "-I", csrc,
                        os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                        os.path.join(csrc, "runtime_common.cpp"), str(oracle_c),
                        "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", "-o", str(exe)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2",
               LD_LIBRARY_PATH=os.path.join(ROCM, "lib") + os.pathsep + os.environ.get("LD_LIBRARY_PATH", ""))
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
