"""One HIP runtime per process: the bindings load PyTorch's HIP runtime before
their own libraries, whatever the caller imports first (CPU only: loading a
library and mapping its runtime needs no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import sys
sys.path.insert(0, {root!r})
{first}
import torch
maps = open("/proc/self/maps").read()
rts = sorted({{l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}})
print(len(rts), rts)
"""


def run(first):
    code = PROBE.format(root=ROOT, first=first)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout


def test_library_imported_before_torch_shares_torchs_runtime():
    out = run("from paper_1912_08810_amd import sse")
    assert out.startswith("1 "), out


def test_generator_device_library_shares_torchs_runtime():
    out = run("import ssegen; ssegen._devlib()")
    assert out.startswith("1 "), out


def test_serving_module_first():
    out = run("from paper_1912_08810_amd import serving")
    assert out.startswith("1 "), out
