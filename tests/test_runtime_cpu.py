"""The binding loads the library against the HIP runtime that torch loaded,
so that one process holds one HIP runtime (CPU check: no device needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_shares_torchs_hip_runtime():
    code = (
        "import paper_2305_03284_amd as D\n"
        "D.lib()\n"
        "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
        "print(len(libs))\n"
    )
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=ROOT)
    if out.returncode != 0:
        pytest.fail(out.stderr[-2000:])
    assert out.stdout.strip().splitlines()[-1] == "1"
