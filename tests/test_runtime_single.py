"""The binding must leave one HIP runtime in the process whatever the import
order (torch's device pointers are only valid in torch's runtime)."""

import subprocess
import sys
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import sys
sys.path.insert(0, {root!r})
import paper_2212_11403_amd as ls
ls.load()
import torch
maps = open('/proc/self/maps').read().splitlines()
print(len({{l.split()[-1] for l in maps if 'libamdhip64' in l}}))
"""


def test_one_hip_runtime_when_library_loads_first():
    pytest.importorskip("torch")
    lib = os.path.join(ROOT, "paper_2212_11403_amd", "libls.so")
    if not os.path.exists(lib):
        pytest.skip("libls.so not built")
    out = subprocess.run([sys.executable, "-c", PROBE.format(root=ROOT)], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
