"""CPU audit of the fused kernel's LDS layouts (host planning code only):
every layout the library would use for a sweep of filters, scale counts,
reference and pulse lengths keeps each access inside its region."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fused_layouts_pass_bounds_audit(tmp_path):
    cxx = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not cxx:
        pytest.skip("hipcc not available")
    exe = tmp_path / "layout_check"
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "layout_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "violations: 0" in r.stdout
