"""The runtime's host code (plans, submission, tickets, check bookkeeping,
batch tables) under AddressSanitizer and UBSan, on the CPU: it is built with
g++ from the library's own sources against a stand-in HIP header and stub
launchers (tests/host_runtime/), and driven through the C ABI.  Includes the
regression test for polling: a pending sse_poll must not make the next
submission report a launch failure.  The persistent launchers' stand-ins run
the kernels' tile-pull code for simulated workgroups in a scrambled order
(grids of 1 to the plan's size, batches that leave work queues empty): every
tile must come out exactly once.  The two C oracles run under the same
sanitizers (with OpenMP) through each of their paths."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
H = os.path.join(ROOT, "tests", "host_runtime")
CSRC = os.path.join(ROOT, "paper_1912_08810_amd", "csrc")


def test_runtime_host_code_under_sanitizers(tmp_path):
    exe = os.path.join(tmp_path, "runtime_host_test")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-x", "c++", "-I", H, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(CSRC, "sse_runtime.hip"), os.path.join(CSRC, "sse_geometry.hip"),
           os.path.join(H, "launch_stubs.cpp"), os.path.join(H, "driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and "OK" in r.stdout, (r.stdout[-2000:], r.stderr[-3000:])


def test_phonon_geometry_fits_the_kernel_layout(tmp_path):
    """pi_geometry against the phonon kernel's LDS layout and task mapping over
    orbital, neighbour and frequency counts and four shift-table shapes."""
    exe = os.path.join(tmp_path, "pi_geometry_check")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-x", "c++", "-I", H, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(CSRC, "sse_geometry.hip"),
           os.path.join(H, "pi_geometry_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-500:])
    assert r.returncode == 0 and "OK" in r.stdout, (r.stdout[-2000:], r.stderr[-3000:])


def test_oracles_under_sanitizers(tmp_path):
    """Both C oracles built with AddressSanitizer, UBSan and OpenMP, driven
    through the full, block-list and stacked-block (gslot) paths and their
    error returns; block-list and gslot results must equal the full
    evaluation bit for bit."""
    exe = os.path.join(tmp_path, "oracle_driver")
    odir = os.path.join(ROOT, "oracle")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", os.path.join(odir, "sse_oracle.c"),
           os.path.join(odir, "pi_oracle.c"), os.path.join(H, "oracle_driver.c"), "-lm",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1", OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-500:])
    assert r.returncode == 0 and "OK" in r.stdout, (r.stdout[-2000:], r.stderr[-3000:])
