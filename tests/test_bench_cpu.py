"""Host-side parts of bench.py: the one-GPU guard and the count of tiles the
symmetric sampled product (the density matrix on the pattern of H) forms, which
the report's issued rate is computed over."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_symmetric_formed_tiles_on_a_symmetric_pattern():
    # block rows 0..2, tridiagonal block pattern: (0,0) (0,1) / (1,0) (1,1) (1,2) / (2,1) (2,2)
    rowptr = [0, 2, 5, 7]
    tcol = [0, 1, 0, 1, 2, 1, 2]
    f = bench.symmetric_formed_tiles(rowptr, tcol)
    assert f.tolist() == [True, True, False, True, True, False, True]
    assert int(f.sum()) == (len(tcol) + 3) // 2       # diagonal + one of each mirror pair


def test_symmetric_formed_tiles_keeps_an_unmirrored_lower_tile():
    # (2,0) has no mirror (0,2): the product forms it itself
    rowptr = [0, 1, 2, 4]
    tcol = [0, 1, 0, 2]
    f = bench.symmetric_formed_tiles(rowptr, tcol)
    assert f.tolist() == [True, True, True, True]


def test_symmetric_formed_tiles_on_the_lattice_pattern():
    # tile pattern of a 12^3 lattice at h <= 4 in 4x4x4 site blocks: every block
    # row holds the blocks within one block in each direction
    nb = 3
    rowptr, tcol = [0], []
    for bx in range(nb):
        for by in range(nb):
            for bz in range(nb):
                cols = sorted((cx * nb + cy) * nb + cz
                              for cx in range(max(0, bx - 1), min(nb, bx + 2))
                              for cy in range(max(0, by - 1), min(nb, by + 2))
                              for cz in range(max(0, bz - 1), min(nb, bz + 2)))
                tcol += cols
                rowptr.append(len(tcol))
    f = bench.symmetric_formed_tiles(np.array(rowptr), np.array(tcol))
    assert int(f.sum()) == (len(tcol) + nb ** 3) // 2
