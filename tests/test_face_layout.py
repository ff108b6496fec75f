"""CPU check of the tile assembly tables of the owner-computes apply and geometry (representatives,
LDS exchange entries, tile face slots, the geometry's face layout), built by the library's host
set-up code and checked by tests/face_layout_check.cpp on the configured meshes and on degree and
tiling extremes."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc to compile the host set-up code")
    exe = str(tmp_path_factory.mktemp("face") / "face_layout_check")
    csrc = os.path.join(ROOT, "paper_2506_09435_amd", "csrc")
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "face_layout_check.cpp"), os.path.join(csrc, "setup.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def _write(mesh, d):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "meta.txt"), "w") as f:
        f.write(f"{mesh.dim} {mesh.p} {mesh.nz} {mesh.n_eh} {mesh.n_s}\n")
    np.ascontiguousarray(mesh.eh_nodes, dtype=np.int32).tofile(os.path.join(d, "nodes.bin"))
    np.ascontiguousarray(mesh.eh_corner, dtype=np.float64).tofile(os.path.join(d, "corner.bin"))
    np.ascontiguousarray(mesh.eh_face_tag, dtype=np.int32).tofile(os.path.join(d, "tag.bin"))
    arc = np.zeros(0) if mesh.eh_arc is None else mesh.eh_arc
    np.ascontiguousarray(arc, dtype=np.float64).tofile(os.path.join(d, "arc.bin"))
    layer = np.zeros(0) if mesh.layer_s is None else mesh.layer_s
    np.ascontiguousarray(layer, dtype=np.float64).tofile(os.path.join(d, "layer.bin"))


def _meshes():
    from workloads import configs
    from workloads import mesh as wm
    out = [("C2", configs.c2().mesh), ("C3", configs.c3().mesh), ("C4", configs.c4().mesh)]
    for p in (1, 2, 6, 8):
        box = wm.structured_box(7, 5, 0.0, 1.0, 0.0, 1.0, False, False, p=p, nz=2)
        out.append((f"box p{p}", box))
        out.append((f"box p{p} shared-first", wm.renumber_blocked(box, shared_first=True)))
        per = wm.structured_box(6, 4, 0.0, 1.0, 0.0, 1.0, True, True, p=p, nz=1)
        out.append((f"periodic box p{p}", wm.renumber_blocked(per, shared_first=True)))
    # one column, and a row of columns shorter than a tile
    out.append(("one column", wm.structured_box(1, 1, 0.0, 1.0, 0.0, 1.0, False, False, p=3, nz=1)))
    out.append(("a row", wm.structured_box(3, 1, 0.0, 1.0, 0.0, 1.0, False, False, p=6, nz=1)))
    return out


@pytest.mark.parametrize("name,mesh", _meshes(), ids=lambda v: v if isinstance(v, str) else "")
def test_tile_tables(checker, tmp_path, name, mesh):
    d = str(tmp_path / "mesh")
    _write(mesh, d)
    r = subprocess.run([checker, d], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), name + ": " + r.stdout + r.stderr
