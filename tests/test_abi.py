"""CPU checks of the C ABI: every declared symbol is exported, host-side entry points agree
with the oracle, and argument validation rejects bad meshes before any HIP call."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.gll import gll as oracle_gll
from paper_2506_09435_amd import fnpf
from workloads import configs, mesh as wm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fnpf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fnpf_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fnpf.lib()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every declared entry point
    assert set(names) <= set(fnpf.SIGNATURES)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_matches_oracle(p):
    x, w, D = fnpf.gll(p)
    xo, wo, Do = oracle_gll(p)
    np.testing.assert_allclose(x, xo, atol=2e-16 * p)
    np.testing.assert_allclose(w, wo, rtol=1e-14)
    np.testing.assert_allclose(D, Do, atol=1e-13 * p * p)


def test_gll_rejects_bad_degree():
    assert fnpf.lib().fnpf_gll(0, None, None, None) == 1
    assert fnpf.lib().fnpf_gll(9, None, None, None) == 1


def _create(mesh, **over):
    nodes = np.ascontiguousarray(over.pop("eh_nodes", mesh.eh_nodes), dtype=np.int32)
    corner = np.ascontiguousarray(over.pop("eh_corner", mesh.eh_corner), dtype=np.float64)
    tags = np.ascontiguousarray(mesh.eh_face_tag, dtype=np.int32)
    d = fnpf.MeshDesc(dim=mesh.dim, p=mesh.p, nz=mesh.nz, n_eh=mesh.n_eh, n_s=mesh.n_s,
                      eh_nodes=nodes.ctypes.data, eh_corner=corner.ctypes.data, eh_arc=None,
                      eh_face_tag=tags.ctypes.data, layer_s=None, g=9.81)
    for k, v in over.items():
        setattr(d, k, v)
    h = C.c_void_p()
    st = fnpf.lib().fnpf_create(C.byref(d), C.byref(h))
    return st, fnpf.lib().fnpf_last_error(None).decode(), h


def test_create_validation_without_gpu():
    m = configs.c1().mesh
    st, msg, h = _create(m, p=0)
    assert st == 1 and "p <= 8" in msg and not h.value
    st, msg, _ = _create(m, nz=0)
    assert st == 1
    bad = m.eh_nodes.copy()
    bad[2, 1] = m.n_s + 5
    st, msg, _ = _create(m, eh_nodes=bad)
    assert st == 1 and "out of range" in msg
    st, msg, _ = _create(m, n_s=m.n_s + 1)
    assert st == 1 and "not used" in msg
    rev = m.eh_corner[:, ::-1].copy()
    st, msg, _ = _create(m, eh_corner=rev)
    assert st == 1 and "Jacobian" in msg
    m3 = wm.structured_box(3, 3, 0, 1, 0, 1, False, False, p=2, nz=1)
    cw = m3.eh_corner[:, ::-1].copy()
    st, msg, _ = _create(m3, eh_corner=cw)
    assert st == 1 and "Jacobian" in msg
    assert fnpf.lib().fnpf_create(None, None) == 1
    # empty meshes are rejected before any device work
    for over in (dict(n_eh=0), dict(n_s=0), dict(p=9), dict(dim=4)):
        st, msg, h = _create(m, **over)
        assert st == 1 and "invalid mesh header" in msg and not h.value


def test_null_context_calls():
    L = fnpf.lib()
    assert L.fnpf_destroy(None) == 1
    assert L.fnpf_geom(None, None, None, None) == 1
    assert L.fnpf_solve(None, None, None, None, None, None, None) == 1
    assert L.fnpf_multigrid_info(None, None, None, None, 0) == 1
    assert L.fnpf_status_string(4).decode().startswith("geometry")
    o = fnpf.default_opts()
    assert (o.precision, o.precond, o.rtol, o.check_every, o.cheb_degree, o.extrapolate) == (0, 2, 1e-8, 8, 2, 4)
    assert o.inner_rtol == 1e-6


def test_binding_pointer_checks():
    """The binding is the only guard against undersized or mistyped device arrays (the C ABI takes
    bare pointers): element count and dtype are checked before anything reaches the library."""
    torch = pytest.importorskip("torch")
    t = torch.zeros(5, dtype=torch.float64)
    with pytest.raises(ValueError, match="expected 6 elements"):
        fnpf._ptr(t, torch.float64, n=6)
    with pytest.raises(TypeError):
        fnpf._ptr(t, torch.float32, n=5)
    with pytest.raises(ValueError, match="device tensor"):
        fnpf._ptr(t, torch.float64, n=5)
    assert fnpf._ptr(None, torch.float64, n=5) is None
