"""GPU parity at the ends of the supported degree range (p = 1, 2, 7, 8), slices and boxes:
geometry, apply against the oracle's assembled matrix, the solve with every preconditioner
(the multigrid hierarchy is 1 level at p = 1, 8 -> 4 -> 2 -> 1 at p = 8), and one ERK4 step in
FP64 and mixed precision.  Tolerances as in the other parity tests (FP64 path 1e-10, mixed
1e-8; single kernels at the FP64 rounding level of their sums)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import geometry as geo
from oracle import operator as op
from oracle import solve as sv
from oracle import timestep as ts
from paper_2506_09435_amd import fnpf
from workloads import configs, mesh as wm


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(name):
    kind, p = name.rsplit("_p", 1)
    p = int(p)
    if kind == "slice":
        wl = configs.small_slice(nx=4, nz=2, p=p, periodic=True)
    elif kind == "box":
        wl = configs.small_box(nx=3, ny=3, nz=2 if p < 7 else 1, p=p, periodic=(True, False))
    elif kind == "column":
        # a single walled column: no node is shared, so no face slots and no exchange at all
        wl = configs.small_box(nx=1, ny=1, nz=3, p=p, periodic=(False, False))
    else:
        raise KeyError(name)
    return wl


CASES = ["slice_p1", "slice_p8", "box_p1", "box_p2", "box_p7", "box_p8", "column_p4"]


def _setup(name):
    wl = _case(name)
    m = wl.mesh
    x, y = geo.node_xy(m)
    h = np.asarray(wl.depth(x, y), dtype=np.float64)
    eta = np.asarray(wl.eta0(x, y), dtype=np.float64)
    phis = np.asarray(wl.phi0(x, y), dtype=np.float64)
    return wl, m, h, eta, phis


@pytest.mark.parametrize("name", CASES)
def test_geometry_apply_and_solve(name):
    wl, m, h, eta, phis = _setup(name)
    ctx = fnpf.Context(m, g=wl.g)
    ctx.enable_fp32()
    ctx.geom(dev(eta), dev(h))
    G, _, _ = geo.factors(m, eta, h)
    A = op.assemble_dense(m, G)
    _, diag = ctx.export_geometry(fnpf.F64)
    assert rel(host(diag), np.diag(A)) < 1e-13
    rng = np.random.default_rng(m.p)
    u = rng.standard_normal(m.n_v)
    ya = A @ u
    assert rel(host(ctx.laplace_apply(dev(u))), ya) < 1e-13
    assert rel(host(ctx.laplace_apply(dev(u).float())), ya) < 2e-6
    phio = sv.solve_dense(m, A, phis)
    for precond in (0, 1, 2):
        phi, info = ctx.solve(dev(phis), opts=fnpf.default_opts(rtol=1e-13, precond=precond, check_every=5))
        assert info["status"] == "OK", (precond, info)
        assert rel(host(phi), phio) < 1e-10, precond


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_rk4_step(name, precision):
    wl, m, h, eta, phis = _setup(name)
    ctx = fnpf.Context(m, g=wl.g)
    md = ts.Model(wl, solver="dense")
    e1, p1 = md.rk4_step(eta, phis, 0.0, 0.02)
    e, p = dev(eta), dev(phis)
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-12, inner_rtol=1e-3)
    infos = ctx.rk4_step(e, p, dev(h), 0.0, 0.02, opts=opts)
    assert all(i["rel_res"] <= opts.rtol for i in infos)
    tol = 1e-10 if precision == 0 else 1e-8
    assert rel(host(e), e1) < tol and rel(host(p), p1) < tol
