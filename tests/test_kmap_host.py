"""Host-side check of the block-sparse product maps (``csrc/blocks.cpp``)
without a device: ``tests/kmap_check.cpp`` is compiled against the map
builder alone and checks by brute force, on random charge lists (sorted and
unsorted, short K and long K that the builder splits), that every nonzero
term of C = A B under U(1) charges is computed exactly once, that an unsplit
map writes every output once and flags only sub-blocks sharing no charge as
empty, that split parts partition each sub-block's K range as tinfo records,
and that the upload order is the stable non-increasing order of K lengths."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_06104_amd", "csrc")


def _hipcc():
    return shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


def test_block_sparse_maps_cover_every_nonzero_term_once(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "kmap_check"
    cmd = [hipcc, "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "kmap_check.cpp"), os.path.join(CSRC, "blocks.cpp"),
           "-o", str(exe), "-lrocprofiler-sdk-roctx"]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-4000:] + r.stderr[-2000:]
