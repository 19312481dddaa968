"""Host tables of the affine-lattice face kernel (CPU only).

At P2/P3 the face kernel forms the tangential averaged gradient and the
averaged BR2 lifting {r} (Sec. 2.1, the face term of the viscous flux) from the
two traces at the face points.  The point maps must reproduce the modal maps
they replace: d/dx_t of the trace of every mode (exact, the face Gauss grid
resolves the trace polynomial) and the modal averaged-lifting map (the same
face quadrature).  A small C++ program built against the library's host
sources checks every entry.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1809_00866_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC), reason="needs g++ and ROCm headers")
def test_face_point_maps_reproduce_the_modal_maps(tmp_path):
    exe = str(tmp_path / "face_point_maps")
    cmd = ["g++", "-std=c++17", "-O1", "-w", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(HERE, "host_checks", "face_point_maps.cpp"), os.path.join(CSRC, "host_setup.cpp"),
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60, check=True).stdout.split("\n")
    rows = [l.split() for l in out if l.startswith("order")]
    assert [int(r[1]) for r in rows] == [2, 3]
    for _, order, derr, lerr, scale in rows:
        assert float(scale) > 1.0
        assert float(derr) <= 1e-12 * float(scale), (order, derr)
        assert float(lerr) <= 1e-12 * float(scale), (order, lerr)
