"""CPU check of the partial-sum buffer layout (csrc/partials.h) with the block counts of the
configured workloads: every launch that writes per-block partial sums fits the buffer."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _blocks(wl):
    """(colour-schedule apply blocks, owner-computes apply blocks) of a workload, computed from its
    mesh the way the library counts them: 256 // nh columns per block; the owner-computes face pass
    has one block per 256 shared nodes and per chunk of 8 node levels."""
    import numpy as np
    m = wl.mesh
    nh = m.nh
    cpb = 256 // nh
    col_blocks = -(-m.n_eh // cpb)
    counts = np.bincount(m.eh_nodes.ravel(), minlength=m.n_s)
    n_shared = int((counts > 1).sum())
    face = -(-n_shared // 256) * -(-(m.p * m.nz + 1) // 8)
    return 4 * col_blocks, col_blocks + face     # at most one partially filled block per colour (<= 4 + slack)


def test_partial_layout_holds_every_launch(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "partials_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_2506_09435_amd", "csrc"),
                    os.path.join(ROOT, "tests", "partials_check.cpp"), "-o", exe], check=True)
    from workloads import configs
    args = []
    for wl in (configs.c1(), configs.c2(n=10), configs.small_box(nx=4, ny=3, nz=2, p=1),
               configs.small_box(nx=5, ny=4, nz=3, p=8)):
        args += [str(v) for v in _blocks(wl)]
    r = subprocess.run([exe] + args, capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
