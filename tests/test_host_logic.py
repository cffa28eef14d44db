"""Host-side logic of the HIP sources, compiled for the host only.

The pass orders of the staged-gather and batched sweeps (batch::Slabs, the
incremental batch::SlabWalk the kernels use, and kpm::FastDiv) are
__host__ __device__ code; tests/host/pass_order.cpp checks them exhaustively
on small lattices.  The batched solver's gather offsets, derived from a row's
lattice site (batch::gather_offsets), are checked against the builder's
column rule by tests/host/gather_offsets.cpp.  The pencil order of the
staged-gather sweep (TileGeom, batch::TileWalk) is checked to cover every row
exactly once in whole passes by tests/host/tile_walk.cpp.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1410_5242_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_pass_order(tmp_path):
    exe = str(tmp_path / "pass_order")
    cmd = [HIPCC, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", CSRC,
           os.path.join(HERE, "host", "pass_order.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith(", 0 bad")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_batched_gather_offsets_follow_the_builder(tmp_path):
    exe = str(tmp_path / "gather_offsets")
    cmd = [HIPCC, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", CSRC,
           os.path.join(HERE, "host", "gather_offsets.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith(", 0 bad")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_pencil_order_covers_every_row_once(tmp_path):
    exe = str(tmp_path / "tile_walk")
    cmd = [HIPCC, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", CSRC,
           os.path.join(HERE, "host", "tile_walk.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith(", 0 bad")
