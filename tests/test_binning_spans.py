"""The binning's per-splat tile spans against the per-entry tile test (host
build of the kernels' helpers, no GPU): the count kernel tabulates, once per
splat, the tile columns each tile row keeps and shrinks the splat's tile
rectangle to them; the emission builds each coarse entry's tile mask from
that.  For random splats at 8-, 16- and 32-pixel tiles every super-tile of the
splat's square gets the same mask either way (the shrunk rectangle leaves out
only super-tiles whose mask is empty), and the shrunk rectangles hold fewer
coarse entries.  (Conservative culling, reading of Alg. 1's DuplicateWithKeys;
the GPU tests check the kernels' lists, images and dropped pairs.)"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_tabulated_spans_give_the_per_entry_masks(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "spans_check")
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-Wno-unused-command-line-argument", os.path.join(HERE, "spans_check.hip"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    out = subprocess.run([exe, "60000"], check=True, capture_output=True, text=True, timeout=600).stdout
    rows = [ln.split() for ln in out.splitlines() if ln.startswith("tile ")]
    assert [int(r[1]) for r in rows] == [8, 16, 32]
    for r in rows:
        mismatches, square, shrunk = int(r[3]), int(r[5]), int(r[6])
        assert mismatches == 0, out
        assert 0 < shrunk < 0.8 * square, out
